"""Pins of the CPU oracle against things other than itself (closed forms,
invariants and brute force), CPU only.

Each pin is chosen so that a plausible mistake in the oracle fails it:
  * geometry         -- closed forms on the circle (normal, weight, curvature);
  * circle spectra   -- every discrete operator S, D, D*, N_k0-N_k1 against its
                        eigenvalue from Graf's addition theorem: a wrong sign or
                        factor gives an O(1) error, a wrong diagonal correction
                        breaks the O(h^3) rate; on the circle rho.n_j = -rho.n_i,
                        so a swapped normal flips the sign of D;
  * Green identities -- S and D on a star (no symmetry) with point sources
                        inside/outside: catches geometry mix-ups a circle hides;
  * kernel symmetry  -- D*_k[i,j]/w_j = D_k[j,i]/w_i (dG/dn_x(x,y) = dG/dn_y(y,x))
                        on a star: catches a transposed normal in D*;
  * Mie series       -- the whole 2x2 system (block placement, eps, alpha, the
                        +-I/2 jumps, the right-hand side, the far field);
  * optical theorem, reciprocity -- the whole system on stars, including two
                        scatterers (the interior/exterior coupling rule);
  * brute force      -- 30-digit mpmath entries, including near-diagonal pairs
                        where N_k0 - N_k1 cancels.
"""
import json
import os

import numpy as np
import pytest

import scatterers as sc
from oracle import brute, geometry, mie, wsbm

HERE = os.path.dirname(os.path.abspath(__file__))


def nodes_for(curves, sizes):
    xyd, s = sc.sample_curves(curves, sizes)
    return geometry.discretize(xyd, s)


def test_geometry_circle_closed_forms():
    a, N = 1.7, 96
    nd = nodes_for([sc.circle(a)], [N])
    t = 2 * np.pi * np.arange(N) / N
    np.testing.assert_allclose(nd.n, np.stack([np.cos(t), np.sin(t)], 1), atol=1e-15)
    np.testing.assert_allclose(nd.w, 2 * np.pi * a / N, rtol=1e-14)
    np.testing.assert_allclose(nd.kappa, 1 / a, rtol=1e-14)


def test_geometry_star_perimeter_and_outward_normals():
    from scipy.integrate import quad
    crv = sc.star(0.3, 5)
    nd = nodes_for([crv], [512])

    def speed(t):
        r = 1 + 0.3 * np.cos(5 * t)
        dr = -1.5 * np.sin(5 * t)
        return np.hypot(r, dr)

    perim = quad(speed, 0, 2 * np.pi, limit=400, epsabs=1e-13, epsrel=1e-13)[0]
    assert abs(nd.w.sum() - perim) < 1e-12 * perim       # trapezoidal rule is spectral here
    assert np.all(np.einsum("ij,ij->i", nd.n, nd.x) > 0)  # outward (star-shaped about 0)


def _spectrum_error(N, m, k0, k1, which):
    nd = nodes_for([sc.circle(1.0)], [N])
    idx = np.arange(N)
    t = 2 * np.pi * idx / N
    phi = np.exp(1j * m * t)
    if which == "S":
        A, lam = wsbm.layer_operators(nd, idx, idx, k0)[0], mie.eig_single(k0, m)
    elif which == "D":
        A, lam = wsbm.layer_operators(nd, idx, idx, k0)[1], mie.eig_double(k0, m)
    elif which == "Ds":
        A, lam = wsbm.layer_operators(nd, idx, idx, k1)[2], mie.eig_double(k1, m)
    else:
        A = wsbm.n_difference(nd, idx, idx, k0, k1)
        lam = mie.eig_hypersingular(k0, m) - mie.eig_hypersingular(k1, m)
    return np.max(np.abs(A @ phi - lam * phi)) / abs(lam)


@pytest.mark.parametrize("which,bound", [("S", 3e-5), ("D", 2e-6), ("Ds", 4e-6), ("ND", 2e-5)])
def test_circle_operator_spectra_third_order(which, bound):
    errs = {N: max(_spectrum_error(N, m, 10.0, 15.0, which) for m in (0, 3, 7)) for N in (256, 512)}
    assert errs[512] < bound
    ratio = errs[256] / errs[512]
    assert 7.0 < ratio < 9.0, (which, errs, ratio)


def _point_source(k, x, n, z):
    from scipy.special import hankel1
    d = x - z[None, :]
    r = np.hypot(d[:, 0], d[:, 1])
    v = 0.25j * hankel1(0, k * r)
    dv = -0.25j * k * hankel1(1, k * r) * np.einsum("ij,ij->i", d, n) / r
    return v, dv


@pytest.mark.parametrize("k", [10.0, 15.0])
def test_green_identities_on_star(k):
    res = {}
    for N in (512, 1024):
        nd = nodes_for([sc.star(0.3, 5)], [N])
        idx = np.arange(N)
        S, D, _ = wsbm.layer_operators(nd, idx, idx, k)
        for label, z, sign in (("out", np.array([2.0, 0.5]), +1), ("in", np.array([0.1, 0.2]), -1)):
            v, dv = _point_source(k, nd.x, nd.n, z)
            r = D @ v + sign * 0.5 * v - S @ dv
            res[(label, N)] = np.max(np.abs(r)) / np.max(np.abs(v))
    for label in ("out", "in"):
        assert res[(label, 1024)] < 2e-5
        assert 6.5 < res[(label, 512)] / res[(label, 1024)] < 9.5, res


def test_double_layer_transpose_symmetry_on_star():
    nd = nodes_for([sc.star(0.3, 5)], [200])
    idx = np.arange(200)
    _, D, Ds = wsbm.layer_operators(nd, idx, idx, 12.0)
    lhs = Ds / nd.w[None, :]
    rhs = (D / nd.w[None, :]).T
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())
    # the double layer itself is not symmetric on a star (a transposed normal would show)
    assert np.abs(D / nd.w[None, :] - (D / nd.w[None, :]).T).max() > 1e-2 * np.abs(D / nd.w).max()


def _mie_errors(media, sizes):
    errs = {}
    for N in sizes:
        nd = nodes_for([sc.circle(1.0)], [N])
        A = wsbm.assemble_dense(nd, media)
        phi = wsbm.solve_dense(A, wsbm.rhs_plane_wave(nd, media, 0.0))
        t = 2 * np.pi * np.arange(N) / N
        u, q = mie.boundary_values(media, t)
        ang = np.linspace(0, 2 * np.pi, 64, endpoint=False)
        ff, ffx = wsbm.far_field(nd, media, phi, ang), mie.far_field(media, ang)
        errs[N] = (np.linalg.norm(phi[0::2].real - u.real) / np.linalg.norm(u.real),
                   np.linalg.norm(phi[1::2] - q) / np.linalg.norm(q),
                   np.linalg.norm(ff - ffx) / np.linalg.norm(ffx))
    return errs


def test_mie_circle_plain_dense_workload():
    """Circle radius 1, k_ext = 10, n = 1.5, plane wave at angle 0."""
    media = sc.media_from_index(10.0, 1.5)
    errs = _mie_errors(media, (256, 512))
    assert errs[512][0] < 3.5e-5 and errs[512][1] < 1.5e-5 and errs[512][2] < 2e-5
    for c in range(3):
        assert 7.5 < errs[256][c] / errs[512][c] < 8.7


def test_mie_circle_table1_parameters():
    with open(os.path.join(HERE, "golden", "table1_parameters.json")) as f:
        t1 = json.load(f)
    media = sc.table1_media()
    assert media.eps0 == t1["eps0"] and media.eps1 == t1["eps1"]
    assert media.k0 == pytest.approx(t1["omega"] * np.sqrt(t1["eps0"] * t1["mu0"]))
    assert media.k1 == pytest.approx(t1["omega"] * np.sqrt(t1["eps1"] * t1["mu1"]))
    errs = _mie_errors(media, (256, 512))
    order = np.log2(errs[256][0] / errs[512][0])
    assert abs(order - t1["claimed_convergence_order_wsbm"]) < 0.15
    assert errs[512][0] < 3e-4


def _star_far_fields(curves, sizes, media, theta):
    nd = nodes_for(curves, sizes)
    phi = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_plane_wave(nd, media, theta))
    return lambda ang: wsbm.far_field(nd, media, phi, ang)


def _optical_defect(curves, sizes, media, theta):
    ff = _star_far_fields(curves, sizes, media, theta)
    ang = 2 * np.pi * np.arange(512) / 512
    lhs = np.sum(np.abs(ff(ang)) ** 2) * 2 * np.pi / 512
    rhs = -np.sqrt(8 * np.pi / media.k0) * np.real(np.exp(0.25j * np.pi) * ff([theta])[0])
    return abs(lhs - rhs) / abs(rhs)


def test_optical_theorem_star():
    media = sc.media_from_index(10.0, 1.5)
    d = {N: _optical_defect([sc.star(0.3, 5)], [N], media, 0.0) for N in (256, 512)}
    assert d[512] < 5e-5 and 6.5 < d[256] / d[512] < 9.5


def test_optical_theorem_two_scatterers():
    media = sc.media_from_index(10.0, 1.5)
    crv = [sc.star(0.2, 4, 1.0, (0.0, 0.0)), sc.star(0.25, 3, 1.0, (3.0, 0.5))]
    d = {N: _optical_defect(crv, [N, N], media, 0.3) for N in (256, 512)}
    assert d[512] < 5e-5 and 6.5 < d[256] / d[512] < 9.5


def test_cross_scatterer_blocks_have_no_interior_terms():
    media = sc.media_from_index(10.0, 1.5)
    nd = nodes_for([sc.circle(1.0), sc.circle(1.0, (4.0, 0.0))], [32, 32])
    A = wsbm.system_blocks(nd, media, np.arange(32), np.arange(32, 64))
    assert np.all(A[:, 0, :, :] == 0)            # first row of Eq. (3) is interior only
    assert np.all(np.abs(A[:, 1, :, :]) > 0)


def test_reciprocity_star():
    media = sc.media_from_index(10.0, 1.5)
    t1, t2 = 0.7, 2.1
    f1 = _star_far_fields([sc.star(0.3, 5)], [512], media, t1)([t2])[0]
    f2 = _star_far_fields([sc.star(0.3, 5)], [512], media, t2 + np.pi)([t1 + np.pi])[0]
    assert abs(f1 - f2) / abs(f1) < 1e-3


def test_brute_force_tiny_star_and_two_curves():
    media = sc.media_from_index(7.0, 1.6)
    for curves, sizes in (([sc.star(0.3, 5)], [16]),
                          ([sc.star(0.2, 3), sc.circle(0.5, (3.0, 1.0))], [10, 6])):
        nd = nodes_for(curves, sizes)
        A = wsbm.assemble_dense(nd, media)
        B = brute.system_matrix(nd, media)
        assert np.abs(A - B).max() < 1e-13 * np.abs(B).max()


def test_brute_force_near_diagonal_cancellation():
    """Neighbouring nodes at N = 16384 on the star with k0 = 50, k1 = 75: the
    hypersingular parts of N_k0 and N_k1 cancel to a few digits."""
    media = sc.media_from_index(50.0, 1.5)
    nd = nodes_for([sc.star(0.3, 5)], [16384])
    rows = np.array([0, 1, 4000])
    cols = np.array([0, 1, 2, 3, 16383, 3999, 4000, 4001, 8000])
    A = wsbm.system_blocks(nd, media, rows, cols)
    B = brute.system_blocks(nd, media, rows, cols)
    scale = np.abs(B).max(axis=(0, 2), keepdims=True)
    assert np.all(np.abs(A - B) <= 1e-11 * scale)


def test_large_matrix_helpers_match_the_plain_assembly_and_solve():
    """The chunked assembly and the in-place (transposed-factor) LU used for the
    N = 16384 dense golden reproduce assemble_dense and solve_dense (Mie-pinned
    above) on a small two-curve problem; a dropped row chunk or a solve with the
    untransposed factors fails."""
    media = sc.media_from_index(12.0, 1.4)
    nd = nodes_for([sc.star(0.3, 5), sc.circle(0.5, (3.0, 0.5))], [150, 50])
    A = wsbm.assemble_dense(nd, media)
    Ap = wsbm.assemble_dense_parallel(nd, media, chunk=37)
    assert np.array_equal(A, Ap)
    b = wsbm.rhs_plane_wave(nd, media, 0.4)
    x = wsbm.solve_dense(A, b)
    y = wsbm.solve_dense_inplace(Ap, b)
    assert np.linalg.norm(x - y) < 1e-12 * np.linalg.norm(x)


def test_point_source_incidence_against_mie():
    """An incident field other than a plane wave: a point source at distance 3
    from a dielectric circle (k0 = 10, n = 1.5).  The right-hand side built from
    its values and normal derivatives (rhs_incident) and the dense solve must
    reproduce the separation-of-variables solution (Graf's addition theorem for
    the incident coefficients) at the O(h^3) rate; a wrong sign of alpha, a
    wrong normal derivative or a swapped u/q row fails the rate."""
    media = sc.media_from_index(10.0, 1.5)
    rho, th = 3.0, 0.8
    src = (rho * np.cos(th), rho * np.sin(th))
    errs = {}
    for N in (256, 512):
        nd = nodes_for([sc.circle(1.0)], [N])
        uin, dn = wsbm.point_source_field(nd, media.k0, src)
        phi = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_incident(nd, media, uin, dn))
        t = 2 * np.pi * np.arange(N) / N
        u, q = mie.boundary_values(media, t, theta_inc=th, src=rho)
        errs[N] = (np.linalg.norm(phi[0::2] - u) / np.linalg.norm(u), np.linalg.norm(phi[1::2] - q) / np.linalg.norm(q))
    assert errs[512][0] < 1e-4 and errs[512][1] < 1e-4
    for c in range(2):
        assert 7.0 < errs[256][c] / errs[512][c] < 9.0, errs


def test_rhs_incident_of_a_plane_wave_is_the_plane_wave_rhs():
    media = sc.media_from_index(20.0, 1.3)
    nd = nodes_for([sc.star(0.3, 5)], [300])
    d = np.array([np.cos(1.1), np.sin(1.1)])
    uin = np.exp(1j * media.k0 * (nd.x @ d))
    dn = 1j * media.k0 * (nd.n @ d) * uin
    assert np.allclose(wsbm.rhs_incident(nd, media, uin, dn), wsbm.rhs_plane_wave(nd, media, 1.1), rtol=1e-14, atol=0)
