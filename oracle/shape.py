"""Shape derivative of a far-field objective of the WSBM Nystrom solution -- the
plain definition the HIP adjoint path must reproduce.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper solves the transmission problem for a fixed boundary; differentiating
it with respect to the boundary is an extension of this project, so every
definition here is a reading (listed under "Readings" below), built only from
the paper's discrete system:
  * the boundary is r(t) = 1 + sum_{j=1..M} (a_j cos jt + b_j sin jt), sampled
    at N equispaced parameter values (Sec. II, trapezoidal Nystrom nodes);
  * phi solves the dense WSBM system A phi = b of Eq. (3) with the one-point
    corrected diagonal and the plane-wave right-hand side (Sec. IV);
  * u_inf(xhat) is the far field of the exterior representation (remark after
    Eq. (3)), and the objective is the backscattered intensity
    J = |u_inf(-d)|^2 for the incident direction d.

Two evaluations of dJ/dc for the coefficient vector c = (a_1..a_M, b_1..b_M):
  gradient_fd            central differences of J itself with one Richardson
                         step, D(h) = (J(c + h e) - J(c - h e)) / 2h and
                         dJ = (4 D(h/2) - D(h)) / 3 (error O(h^4)): the plain
                         definition of a derivative, for small N;
  directional_derivative the derivative along one direction v for large N from
                         a single dense LU: differentiating A phi = b gives
                         du_inf = dg^T phi + lam^T (db - dA phi), A^T lam = g,
                         with g the far-field weights (u_inf = g^T phi) and dA phi,
                         db, dg the same Richardson central differences of the
                         matrix-vector product, the right-hand side and the
                         weights; dJ = 2 Re(conj(u_inf) du_inf).

Readings:
  S1  the objective is J = |u_inf(-d)|^2 for one incident plane wave, the
      derivative is that of the discrete J (nodes moved with the curve);
  S2  the M coefficients are a_1..a_M followed by b_1..b_M, radius 1, centre 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

import scatterers as sc

from .geometry import discretize
from . import wsbm


def nodes_of(coef: np.ndarray, n: int):
    """Nodes of the curve with coefficients coef = (a_1..a_M, b_1..b_M) (reading S2)."""
    coef = np.asarray(coef, dtype=np.float64)
    m = coef.size // 2
    crv = sc.fourier_curve(coef[:m], coef[m:])
    xyd, sizes = sc.sample_curves([crv], [n])
    return discretize(xyd, sizes)


def backscatter(coef, n: int, media, theta_inc: float):
    """(u_inf(-d), J) with J = |u_inf(-d)|^2, from a dense solve (reading S1)."""
    nd = nodes_of(coef, n)
    A = wsbm.assemble_dense(nd, media)
    phi = wsbm.solve_dense(A, wsbm.rhs_plane_wave(nd, media, theta_inc))
    u = wsbm.far_field(nd, media, phi, [theta_inc + np.pi])[0]
    return u, abs(u) ** 2


def _richardson(f, h):
    """(4 D(h/2) - D(h)) / 3 with D(s) = (f(s) - f(-s)) / 2s; f(s) may be an array."""
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def gradient_fd(coef, n: int, media, theta_inc: float, h: float = 1e-4) -> np.ndarray:
    """dJ/dc_m for every coefficient by Richardson-extrapolated central differences."""
    coef = np.asarray(coef, dtype=np.float64)
    g = np.empty(coef.size)
    for m in range(coef.size):
        e = np.zeros(coef.size)
        e[m] = 1.0
        g[m] = _richardson(lambda s: backscatter(coef + s * e, n, media, theta_inc)[1], h)
    return g


def _row_block(args):
    """Rows of A for the node range [r0, r1) (times x when x is given)."""
    nd, media, r0, r1, x = args
    blk = wsbm.assemble_rows(nd, media, np.arange(r0, r1))
    return blk if x is None else blk @ x


def _row_jobs(nd, media, x, chunk):
    return [(nd, media, r0, min(nd.size, r0 + chunk), x) for r0 in range(0, nd.size, chunk)]


def _matvec_rows(nd, media, x, chunk=256, mapper=map):
    """A x assembled a block of rows at a time (nothing of size N^2 is kept)."""
    return np.concatenate(list(mapper(_row_block, _row_jobs(nd, media, x, chunk))))


def directional_derivative(coef, v, n: int, media, theta_inc: float, h: float = 1e-4,
                           chunk: int = 256, mapper=map):
    """(u_inf, J, dJ.v) from one dense LU and differentiated pieces (see the module
    docstring).  Assembly goes by blocks of rows, so N in the thousands fits;
    `mapper` (e.g. a process pool's map) may evaluate the blocks in parallel."""
    coef = np.asarray(coef, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    obs = theta_inc + np.pi
    nd = nodes_of(coef, n)
    A = np.empty((2 * n, 2 * n), dtype=np.complex128)
    for (_, _, r0, r1, _), blk in zip(_row_jobs(nd, media, None, chunk),
                                      mapper(_row_block, _row_jobs(nd, media, None, chunk))):
        A[2 * r0:2 * r1] = blk
    b = wsbm.rhs_plane_wave(nd, media, theta_inc)
    g = wsbm.far_field_weights(nd, media, obs)
    lu = scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
    del A
    phi = scipy.linalg.lu_solve(lu, b, check_finite=False)
    lam = scipy.linalg.lu_solve(lu, g, trans=1, check_finite=False)   # A^T lam = g
    del lu
    u = g @ phi

    def moved(s):
        return nodes_of(coef + s * v, n)

    d_gphi = _richardson(lambda s: wsbm.far_field_weights(moved(s), media, obs) @ phi, h)
    d_b = _richardson(lambda s: wsbm.rhs_plane_wave(moved(s), media, theta_inc), h)
    d_aphi = _richardson(lambda s: _matvec_rows(moved(s), media, phi, chunk, mapper), h)
    du = d_gphi + lam @ (d_b - d_aphi)
    return u, abs(u) ** 2, 2.0 * np.real(np.conj(u) * du)
