"""Closed forms for a dielectric circle of radius a centred at the origin.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper (Sec. IV) verifies its solver on a circle because the transmission
problem has an explicit solution there.  We write that solution by separation
of variables from the problem statement of Sec. II, independently of the
integral-equation machinery:
  * incident plane wave (Jacobi-Anger)
        u_in = sum_m i^m J_m(k0 r) e^{i m (theta - theta_inc)}
  * interior field  u = sum_m c_m J_m(k1 r) e^{i m (theta - theta_inc)}
  * scattered field u_sc = sum_m b_m H_m(k0 r) e^{i m (theta - theta_inc)}
  * interface conditions (reading R3 of oracle.wsbm): u and (1/eps) du/dn are
    continuous across r = a.
For each m the two conditions form a 2x2 linear system for (c_m, b_m), solved
numerically here.

It also gives the eigenvalues of the continuous layer potentials on the circle
(Graf's addition theorem for H0(k|x-y|)): on the density e^{i m theta},
  S_k   -> (i pi a / 2) J_m(ka) H_m(ka)
  D_k   -> (i pi k a / 4) (J_m(ka) H_m'(ka) + J_m'(ka) H_m(ka))   (= D*_k)
  N_k   -> (i pi k^2 a / 2) J_m'(ka) H_m'(ka)
so that the discrete operators can be checked one by one.
"""
from __future__ import annotations

import numpy as np
from scipy.special import h1vp, hankel1, jv, jvp


def _orders(media, a, extra=40):
    mmax = int(np.ceil(max(media.k0, media.k1) * a)) + extra
    return np.arange(-mmax, mmax + 1)


def coefficients(media, a=1.0, src=None):
    """(m, c_m, b_m) for theta_inc = 0.  src = rho_s > a: instead of the plane
    wave, the field of a point source at distance rho_s on the axis theta = 0,
    u_in = H0^(1)(k0 |x - x_s|) = sum_m H_m(k0 rho_s) J_m(k0 r) e^{i m theta}
    for r < rho_s (Graf's addition theorem), i.e. the incident coefficient
    H_m(k0 rho_s) in place of i^m."""
    k0, k1, e0, e1 = media.k0, media.k1, media.eps0, media.eps1
    m = _orders(media, a)
    if src is not None:
        assert src > a
        m = np.arange(-(int(np.ceil(k0 * src)) + 40), int(np.ceil(k0 * src)) + 41)
    c = np.empty(m.shape, dtype=np.complex128)
    b = np.empty(m.shape, dtype=np.complex128)
    for idx, mm in enumerate(m):
        M = np.array([[jv(mm, k1 * a), -hankel1(mm, k0 * a)],
                      [(k1 / e1) * jvp(mm, k1 * a), -(k0 / e0) * h1vp(mm, k0 * a)]])
        inc = (1j ** mm) if src is None else hankel1(mm, k0 * src)
        rhs = inc * np.array([jv(mm, k0 * a), (k0 / e0) * jvp(mm, k0 * a)])
        c[idx], b[idx] = np.linalg.solve(M, rhs)
    return m, c, b


def boundary_values(media, theta_nodes, a=1.0, theta_inc=0.0, src=None):
    """Exact u and q = (1/eps1) du/dn (interior side) at boundary angles;
    src = rho_s: for a point source at (rho_s cos theta_inc, rho_s sin theta_inc)."""
    m, c, _ = coefficients(media, a, src)
    e = np.exp(1j * np.outer(np.asarray(theta_nodes) - theta_inc, m))
    u = e @ (c * jv(m, media.k1 * a))
    q = e @ (c * (media.k1 / media.eps1) * jvp(m, media.k1 * a))
    return u, q


def far_field(media, angles, a=1.0, theta_inc=0.0):
    """u_inf(phi) with u_sc ~ e^{i k0 r}/sqrt(r) u_inf (large-argument H_m)."""
    m, _, b = coefficients(media, a)
    e = np.exp(1j * np.outer(np.asarray(angles) - theta_inc, m))
    return np.sqrt(2.0 / (np.pi * media.k0)) * np.exp(-0.25j * np.pi) * (e @ (b * (-1j) ** m))


def eig_single(k, m, a=1.0):
    return 0.5j * np.pi * a * jv(m, k * a) * hankel1(m, k * a)


def eig_double(k, m, a=1.0):
    z = k * a
    return 0.25j * np.pi * k * a * (jv(m, z) * h1vp(m, z) + jvp(m, z) * hankel1(m, z))


def eig_hypersingular(k, m, a=1.0):
    z = k * a
    return 0.5j * np.pi * k * k * a * jvp(m, z) * h1vp(m, z)
