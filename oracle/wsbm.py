"""Weakly singular Burton-Miller (WSBM) Nystrom matrix, right-hand side, far
field and dense solve -- the plain definition the HIP path must reproduce.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper:
  * Sec. II: layer potentials S_k, D_k, and their normal derivatives D*_k, N_k;
    k_j = omega sqrt(eps_j mu_j); n is the outward normal; q is the scaled
    normal derivative of u;
  * Eq. (3): the WSBM operator
        [ D_k1 + I/2                  , -eps1 S_k1                                     ]
        [ D_k0 - I/2 + a(N_k0 - N_k1) , -eps0 S_k0 - a(eps0 D*_k0 - eps1 D*_k1) - a(eps0+eps1) I/2 ]
    with a = alpha = i/k0 (stated after Eq. (2)), right-hand side
    (0, -u_in - alpha du_in/dn);
  * Eq. (5): the same 2x2 structure holds for every block A_ij of the
    partitioned system, with Kronecker deltas on the identity terms;
  * Sec. I/II: Nystrom discretisation by the trapezoidal rule in which only the
    diagonal entries are corrected (one-point corrected quadrature);
  * Sec. IV: plane wave propagating along x1 (general angle allowed).

Readings (the paper does not write these out):
  R1  G_k(x, y) = (i/4) H0^(1)(k|x-y|)  (time convention e^{-i w t}, consistent
      with alpha = i/k0);
  R2  D_k has kernel dG/dn_y, D*_k has kernel dG/dn_x, N_k has kernel
      d2G/dn_x dn_y (with n outward, the +-I/2 terms of Eq. (3) are the jump
      relations of these operators);
  R3  q = (1/eps_j) du/dn on side j (TE interface conditions);
  R4  one-point correction: the log-singular part of a kernel is integrated by
      the punctured trapezoidal rule plus h g(t_i) ln(h/2pi) (zeta correction,
      -2 zeta'(0) = ln 2pi); the bounded kernels D, D* use their continuous
      limit -kappa/(4 pi) on the diagonal.  The resulting diagonal entries are
        S_k[i,i]         = -(w_i/2pi) (L_k - i pi/2),   L_k = ln(k w_i/4pi) + gamma
        D_k[i,i] = D*_k[i,i] = -kappa_i w_i / (4 pi)
        (N_k0 - N_k1)[i,i] = -(w_i/4pi) [k0^2 (L_k0 - 1/2 - i pi/2) - k1^2 (L_k1 - 1/2 - i pi/2)]
  R5  unknowns are node-interleaved: column 2j is u_j, column 2j+1 is q_j; row 2i
      is the first row of Eq. (3) at node i, row 2i+1 the second row;
  R6  several disjoint scatterers: the interior (k1) operators act only
      between nodes of the same closed curve; the exterior (k0) operators couple
      all nodes.
N_k0 - N_k1 is evaluated here as the plain difference of the two hypersingular
kernels (off the diagonal); the Hankel functions come from SciPy (AMOS),
H2 directly as hankel1(2, .).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
from scipy.special import hankel1

from .geometry import Nodes

EULER_GAMMA = float(np.euler_gamma)


def _kernels(tx, tn, sx, sn, sw, k):
    """Off-diagonal kernels at wavenumber k for every (target, source) pair.

    Returns S, D, Ds, N (each (nt, ns) complex), already multiplied by the
    source weight sw_j.  Coincident points must not be passed."""
    rho = tx[:, None, :] - sx[None, :, :]
    r = np.sqrt(rho[..., 0] ** 2 + rho[..., 1] ** 2)
    a = rho[..., 0] * tn[:, None, 0] + rho[..., 1] * tn[:, None, 1]   # rho . n_target
    b = rho[..., 0] * sn[None, :, 0] + rho[..., 1] * sn[None, :, 1]   # rho . n_source
    c = tn[:, None, 0] * sn[None, :, 0] + tn[:, None, 1] * sn[None, :, 1]
    z = k * r
    h0 = hankel1(0, z)
    h1 = hankel1(1, z)
    h2 = hankel1(2, z)
    w = sw[None, :]
    S = 0.25j * h0 * w
    D = 0.25j * k * h1 * (b / r) * w
    Ds = -0.25j * k * h1 * (a / r) * w
    N = 0.25j * k * (h1 * c / r - k * h2 * a * b / r**2) * w
    return S, D, Ds, N


def _combine(S0, D0, Ds0, ND, S1, D1, Ds1, media, delta):
    """Eq. (5): the 2x2 block structure from the layer-potential blocks.

    ``delta`` is the Kronecker delta of the identity terms (array or 0)."""
    e0, e1 = media.eps0, media.eps1
    alpha = 1j / media.k0
    out = np.empty(S0.shape[:1] + (2,) + S0.shape[1:] + (2,), dtype=np.complex128)
    out[:, 0, :, 0] = D1 + 0.5 * delta
    out[:, 0, :, 1] = -e1 * S1
    out[:, 1, :, 0] = D0 - 0.5 * delta + alpha * ND
    out[:, 1, :, 1] = -e0 * S0 - alpha * (e0 * Ds0 - e1 * Ds1) - alpha * (e0 + e1) * 0.5 * delta
    return out


def pair_blocks(tx, tn, sx, sn, sw, media, interior=None):
    """2x2 WSBM blocks (Eq. (5), off-diagonal: no identity terms) between
    arbitrary target points (tx, tn) and source points (sx, sn, sw), e.g. nodes
    against proxy points.  Coincident points must not be passed.

    ``interior`` (nt, ns) bool: where False the k1 operators are dropped (R6).
    Returns complex array (nt, 2, ns, 2)."""
    S0, D0, Ds0, N0 = _kernels(tx, tn, sx, sn, sw, media.k0)
    S1, D1, Ds1, N1 = _kernels(tx, tn, sx, sn, sw, media.k1)
    if interior is not None:
        m = interior.astype(np.float64)
        S1, D1, Ds1, N1 = S1 * m, D1 * m, Ds1 * m, N1 * m
    return _combine(S0, D0, Ds0, N0 - N1, S1, D1, Ds1, media, 0.0)


def _grid(nodes: Nodes, rows, cols):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    same = rows[:, None] == cols[None, :]
    return rows, cols, same


def layer_operators(nodes: Nodes, rows, cols, k):
    """Discrete S_k, D_k, D*_k (weighted by w_j) on node index lists, with the
    one-point corrected diagonal of reading R4.  Returns (S, D, Ds), each
    (len(rows), len(cols)) complex."""
    rows, cols, same = _grid(nodes, rows, cols)
    with np.errstate(divide="ignore", invalid="ignore"):
        S, D, Ds, _ = _kernels(nodes.x[rows], nodes.n[rows], nodes.x[cols], nodes.n[cols],
                               nodes.w[cols], k)
    if same.any():
        ti, tj = np.nonzero(same)
        i = rows[ti]
        w, kap = nodes.w[i], nodes.kappa[i]
        L = np.log(k * w / (4 * np.pi)) + EULER_GAMMA
        S[ti, tj] = -(w / (2 * np.pi)) * (L - 0.5j * np.pi)
        D[ti, tj] = -kap * w / (4 * np.pi)
        Ds[ti, tj] = -kap * w / (4 * np.pi)
    return S, D, Ds


def n_difference(nodes: Nodes, rows, cols, k0, k1):
    """Discrete N_k0 - N_k1 (weighted by w_j) with the corrected diagonal of R4."""
    rows, cols, same = _grid(nodes, rows, cols)
    args = (nodes.x[rows], nodes.n[rows], nodes.x[cols], nodes.n[cols], nodes.w[cols])
    with np.errstate(divide="ignore", invalid="ignore"):
        N0 = _kernels(*args, k0)[3]
        N1 = _kernels(*args, k1)[3]
    ND = N0 - N1
    if same.any():
        ti, tj = np.nonzero(same)
        w = nodes.w[rows[ti]]
        L0 = np.log(k0 * w / (4 * np.pi)) + EULER_GAMMA
        L1 = np.log(k1 * w / (4 * np.pi)) + EULER_GAMMA
        ND[ti, tj] = -(w / (4 * np.pi)) * (k0**2 * (L0 - 0.5 - 0.5j * np.pi)
                                           - k1**2 * (L1 - 0.5 - 0.5j * np.pi))
    return ND


def system_blocks(nodes: Nodes, media, rows, cols):
    """Blocks A(rows, cols) of the WSBM Nystrom matrix for node index lists
    (Eq. (5)); pairs with row node == column node carry the identity terms and
    the corrected diagonal entries.  Returns complex (len(rows), 2, len(cols), 2);
    reshape to (2 nr, 2 nc) for the node-interleaved matrix of R5."""
    rows, cols, same = _grid(nodes, rows, cols)
    interior = (nodes.curve[rows][:, None] == nodes.curve[cols][None, :]).astype(np.float64)
    S0, D0, Ds0 = layer_operators(nodes, rows, cols, media.k0)
    S1, D1, Ds1 = layer_operators(nodes, rows, cols, media.k1)
    if not interior.all():
        # R6: across scatterers only the exterior operators remain, so the
        # difference N_k0 - N_k1 reduces to N_k0 there.
        args = (nodes.x[rows], nodes.n[rows], nodes.x[cols], nodes.n[cols], nodes.w[cols])
        with np.errstate(divide="ignore", invalid="ignore"):
            N0 = _kernels(*args, media.k0)[3]
        ND = np.where(interior > 0, n_difference(nodes, rows, cols, media.k0, media.k1), N0)
        S1, D1, Ds1 = S1 * interior, D1 * interior, Ds1 * interior
    else:
        ND = n_difference(nodes, rows, cols, media.k0, media.k1)
    return _combine(S0, D0, Ds0, ND, S1, D1, Ds1, media, same.astype(np.float64))


def assemble_dense(nodes: Nodes, media) -> np.ndarray:
    """The full 2N x 2N node-interleaved WSBM matrix (Eq. (3), R5)."""
    idx = np.arange(nodes.size)
    return system_blocks(nodes, media, idx, idx).reshape(2 * nodes.size, 2 * nodes.size)


def assemble_rows(nodes: Nodes, media, rows) -> np.ndarray:
    """Rows 2i, 2i+1 for each node i in `rows` (all columns): (2 len(rows), 2N)."""
    rows = np.asarray(rows, dtype=np.int64)
    out = system_blocks(nodes, media, rows, np.arange(nodes.size))
    return out.reshape(2 * len(rows), 2 * nodes.size)


def rhs_plane_wave(nodes: Nodes, media, theta: float) -> np.ndarray:
    """b[2i] = 0, b[2i+1] = -u_in(x_i) - alpha du_in/dn(x_i) with
    u_in = exp(i k0 d.x), d = (cos theta, sin theta)  (Eq. (3), Sec. IV)."""
    d = np.array([np.cos(theta), np.sin(theta)])
    uin = np.exp(1j * media.k0 * (nodes.x @ d))
    dn_uin = 1j * media.k0 * (nodes.n @ d) * uin
    b = np.zeros(2 * nodes.size, dtype=np.complex128)
    b[1::2] = -uin - (1j / media.k0) * dn_uin
    return b


def rhs_incident(nodes: Nodes, media, uin: np.ndarray, dn_uin: np.ndarray) -> np.ndarray:
    """The right-hand side of Eq. (3) for an arbitrary incident field given by
    its values u_in and outward normal derivatives du_in/dn at the nodes:
    b[2i] = 0, b[2i+1] = -u_in - alpha du_in/dn, alpha = i/k0."""
    b = np.zeros(2 * nodes.size, dtype=np.complex128)
    b[1::2] = -np.asarray(uin) - (1j / media.k0) * np.asarray(dn_uin)
    return b


def point_source_field(nodes: Nodes, k0: float, src) -> tuple:
    """u_in = H0^(1)(k0 |x - x_s|) of a point source at x_s outside the
    scatterers, and du_in/dn = -k0 H1^(1)(k0 R) ((x - x_s).n)/R, R = |x - x_s|."""
    d = nodes.x - np.asarray(src, dtype=np.float64)[None, :]
    R = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    uin = hankel1(0, k0 * R)
    dn = -k0 * hankel1(1, k0 * R) * (d[:, 0] * nodes.n[:, 0] + d[:, 1] * nodes.n[:, 1]) / R
    return uin, dn


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """phi = A^{-1} b by LU with partial pivoting (LAPACK zgetrf/zgetrs)."""
    lu, piv = scipy.linalg.lu_factor(A, check_finite=False)
    return scipy.linalg.lu_solve((lu, piv), b, check_finite=False)


def solve_dense_inplace(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The same solve for a matrix too large to copy: A (C-ordered) is
    destroyed.  Its memory, read in Fortran order, is A^T, which LAPACK
    factors in place (P L U = A^T); the solve then applies the transposed
    factors (zgetrs with trans = 'T'), i.e. solves A phi = b."""
    assert A.flags.c_contiguous and A.shape[0] == A.shape[1]
    lu, piv = scipy.linalg.lu_factor(A.T, overwrite_a=True, check_finite=False)
    return scipy.linalg.lu_solve((lu, piv), b, trans=1, check_finite=False)


def assemble_dense_parallel(nodes: Nodes, media, mapper=map, chunk: int = 64) -> np.ndarray:
    """assemble_dense for large N: the rows are generated in chunks of `chunk`
    nodes by assemble_rows (mapper, e.g. a process pool's imap, may run the
    chunks in parallel; it must return them in order) and copied into one
    preallocated matrix."""
    n = nodes.size
    A = np.empty((2 * n, 2 * n), dtype=np.complex128)
    jobs = [(nodes, media, np.arange(s, min(n, s + chunk))) for s in range(0, n, chunk)]
    for (_, _, rows), blk in zip(jobs, mapper(_rows_job, jobs)):
        A[2 * rows[0]:2 * rows[-1] + 2] = blk
    return A


def _rows_job(args):
    nodes, media, rows = args
    return assemble_rows(nodes, media, rows)


def far_field(nodes: Nodes, media, phi: np.ndarray, angles) -> np.ndarray:
    """Far-field pattern u_inf(xhat) of the scattered field, defined by
    u_sc(x) ~ exp(i k0 |x|)/sqrt(|x|) u_inf(xhat), from the exterior integral
    representation u_sc = D_k0[u] - S_k0[eps0 q] (Sec. II, remark after Eq. (3))
    and the large-argument form of H0^(1)/H1^(1):
        u_inf(xhat) = e^{i pi/4}/sqrt(8 pi k0) sum_j [-i k0 (xhat.n_j) u_j - eps0 q_j]
                      exp(-i k0 xhat.x_j) w_j."""
    angles = np.atleast_1d(np.asarray(angles, dtype=np.float64))
    u = phi[0::2]
    q = phi[1::2]
    xh = np.stack([np.cos(angles), np.sin(angles)], axis=1)
    k0 = media.k0
    ph = np.exp(-1j * k0 * (xh @ nodes.x.T))                       # (nang, N)
    dens = (-1j * k0 * (xh @ nodes.n.T)) * u[None, :] - media.eps0 * q[None, :]
    return np.exp(0.25j * np.pi) / np.sqrt(8 * np.pi * k0) * np.sum(dens * ph * nodes.w[None, :], axis=1)


def far_field_weights(nodes: Nodes, media, angle: float) -> np.ndarray:
    """The weights g (2N complex) with u_inf(angle) = sum_k g_k phi_k, i.e. the
    far_field formula above written per unknown:
        g[2j]   = c (-i k0 xhat.n_j) exp(-i k0 xhat.x_j) w_j,
        g[2j+1] = c (-eps0)          exp(-i k0 xhat.x_j) w_j,
    c = e^{i pi/4}/sqrt(8 pi k0)."""
    xh = np.array([np.cos(angle), np.sin(angle)])
    k0 = media.k0
    c = np.exp(0.25j * np.pi) / np.sqrt(8 * np.pi * k0)
    ph = c * np.exp(-1j * k0 * (nodes.x @ xh)) * nodes.w
    g = np.empty(2 * nodes.size, dtype=np.complex128)
    g[0::2] = -1j * k0 * (nodes.n @ xh) * ph
    g[1::2] = -media.eps0 * ph
    return g
