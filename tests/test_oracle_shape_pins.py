"""Pins of the oracle's shape derivative (oracle/shape.py), CPU only.

The oracle defines dJ/dc as the derivative of the discrete backscatter
intensity J = |u_inf(-d)|^2 with respect to the Fourier coefficients of the
boundary.  J itself is pinned by the Mie, optical-theorem and reciprocity tests
of the system; these tests pin the derivative machinery and the coefficient
convention against facts that hold independently of it:
  * two formulas        -- Richardson differences of J and the adjoint identity
                           du = dg.phi + lam.(db - dA phi) must agree: a wrong
                           step scale, sign or transpose in either shows;
  * mirror symmetry     -- with b = 0 and incidence along x the node set is
                           mirror symmetric (t_j -> t_{N-j}), so J is exactly
                           even in every b_m: dJ/db_m = 0;
  * discrete rotation   -- rotating the curve by one node spacing multiple
                           beta permutes the nodes, so J(R c, th) = J(c, th - beta)
                           exactly and dJ(R c, th).(R v) = dJ(c, th - beta).v: a
                           swapped a/b or shifted mode index breaks it;
  * translation         -- on the circle, a_1 moves the curve rigidly to first
                           order and |u_inf| does not change under translation,
                           so dJ/da_1 -> 0 at the O(h^3) rate of the method;
  * far-field weights   -- g.phi reproduces the (Mie-pinned) far field.
"""
import numpy as np

import scatterers as sc
from oracle import geometry, shape, wsbm

MEDIA = sc.media_from_index(10.0, 1.5)


def unit(m, size):
    e = np.zeros(size)
    e[m] = 1.0
    return e


def test_far_field_weights_match_far_field():
    xyd, s = sc.sample_curves([sc.star(0.2, 3)], [96])
    nd = geometry.discretize(xyd, s)
    rng = np.random.default_rng(0)
    phi = rng.standard_normal(192) + 1j * rng.standard_normal(192)
    for ang in (0.0, 1.3, 4.0):
        g = wsbm.far_field_weights(nd, MEDIA, ang)
        ref = wsbm.far_field(nd, MEDIA, phi, [ang])[0]
        assert abs(g @ phi - ref) <= 1e-13 * abs(ref)


def test_fd_and_adjoint_forms_agree():
    rng = np.random.default_rng(1)
    coef = rng.normal(0.0, 0.02, 6)
    g = shape.gradient_fd(coef, 96, MEDIA, 0.4)
    for _ in range(2):
        v = rng.standard_normal(6)
        d = shape.directional_derivative(coef, v, 96, MEDIA, 0.4)[2]
        assert abs(d - g @ v) <= 1e-8 * np.abs(g).max() * np.abs(v).sum()
    assert np.abs(g).max() > 0.1


def test_mirror_symmetry_b_derivatives_vanish():
    rng = np.random.default_rng(2)
    M = 4
    coef = np.concatenate([rng.normal(0.0, 0.03, M), np.zeros(M)])
    d = np.array([shape.directional_derivative(coef, unit(m, 2 * M), 96, MEDIA, 0.0)[2]
                  for m in range(2 * M)])
    scale = np.abs(d[:M]).max()
    assert scale > 0.1
    assert np.abs(d[M:]).max() <= 1e-9 * scale


def test_discrete_rotation_covariance():
    rng = np.random.default_rng(3)
    M, N, shift = 4, 128, 5
    beta = 2 * np.pi * shift / N
    j = np.arange(1, M + 1)

    def rot(c):
        a, b = c[:M], c[M:]
        return np.concatenate([a * np.cos(j * beta) - b * np.sin(j * beta),
                               a * np.sin(j * beta) + b * np.cos(j * beta)])

    coef = rng.normal(0.0, 0.03, 2 * M)
    v = rng.standard_normal(2 * M)
    u1, J1, d1 = shape.directional_derivative(rot(coef), rot(v), N, MEDIA, 0.3)
    u2, J2, d2 = shape.directional_derivative(coef, v, N, MEDIA, 0.3 - beta)
    assert abs(J1 - J2) <= 1e-12 * J2
    assert abs(d1 - d2) <= 1e-9 * abs(d2)
    assert abs(d2) > 1.0


def test_translation_mode_derivative_vanishes_at_third_order():
    d = {}
    for N in (128, 256):
        d[N] = [shape.directional_derivative(np.zeros(4), unit(m, 4), N, MEDIA, 0.0)[2]
                for m in range(2)]
    scale = abs(d[256][1])          # dJ/da_2: a genuine shape change
    assert scale > 1.0
    assert abs(d[128][0]) <= 2e-3 * scale
    assert abs(d[256][0]) <= abs(d[128][0]) / 6      # ~ 2^3 for O(h^3)
