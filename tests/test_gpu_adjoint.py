"""GPU tests of the shape-derivative (adjoint) path through the C-ABI:
the transposed HSS solve, the far-field weights, the per-node derivative of
L = g.phi + lam.(b - A phi), the Fourier boundary and its chain rule, and the
torch.autograd.Function that strings them together.

References: the oracle's dense transpose solve (LAPACK), its far-field weights,
Richardson central differences of the oracle's L and J (oracle/shape.py), and,
at the full differentiation workload (N = 8192), central differences of the
GPU's own J with step 1e-6."""
import math
import sys

import numpy as np
import pytest
import scipy.linalg

import scatterers as sc
from oracle import geometry, shape, wsbm

pytestmark = pytest.mark.gpu

HSS_BAR = 1e-7


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cplx(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def bodies_problem(bm, bodies):
    """bodies: list of (curves, sizes, media) -> GPU problem, per-body xyd/sizes, node offsets."""
    curves, sizes, boc, media, parts, lo = [], [], [], [], [], [0]
    for b, (cv, sz, md) in enumerate(bodies):
        curves += cv
        sizes += sz
        boc += [b] * len(cv)
        media.append((md.k0, md.k1, md.eps0, md.eps1))
        parts.append(sc.sample_curves(cv, sz))
        lo.append(lo[-1] + sum(sz))
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create_bodies(g, boc, media)
    return p, parts, lo


@pytest.mark.parametrize("sketch", [0, 128, -1])   # -1: the tuned options (with the stop rule)
def test_hss_solve_transpose_matches_dense(gpu_lib, sketch):
    """A^T x = b on a forest of three bodies (one too small to compress)."""
    import torch
    bm = gpu_lib
    note(f"adjoint: transposed HSS solve, three bodies, sketch={sketch}")
    bodies = [([sc.star(0.3, 5)], [1500], sc.media_from_index(30.0, 1.5)),
              ([sc.circle(1.0)], [96], sc.media_from_index(10.0, 2.0)),
              ([sc.star(0.2, 3), sc.circle(0.3, (3.0, 0.0))], [700, 200], sc.media_from_index(20.0, 1.8))]
    p, parts, lo = bodies_problem(bm, bodies)
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=sketch,
                        max_rank_ratio=-1.0 if sketch == -1 else 0.0)
    rng = np.random.default_rng(3)
    B = np.stack([cplx(rng, 2 * lo[-1]) for _ in range(2)])
    X = bm.bm_hss_solve_transpose(h, torch.from_numpy(B).cuda().contiguous()).cpu().numpy()
    for q, (_, _, md) in enumerate(bodies):
        sl = slice(2 * lo[q], 2 * lo[q + 1])
        A = wsbm.assemble_dense(geometry.discretize(*parts[q]), md)
        lu = scipy.linalg.lu_factor(A)
        for r in range(2):
            ref = scipy.linalg.lu_solve(lu, B[r, sl], trans=1)
            err = np.linalg.norm(X[r, sl] - ref) / np.linalg.norm(ref)
            note(f"  body {q} rhs {r}: relative error {err:.2e}")
            assert err < HSS_BAR
    # in place (x aliasing b) gives the same result
    Bt = torch.from_numpy(B).cuda().contiguous()
    bm.bm_hss_solve_transpose(h, Bt, out=Bt)
    assert np.array_equal(Bt.cpu().numpy(), X)


def test_far_field_weights_match_oracle(gpu_lib):
    import torch
    bm = gpu_lib
    note("adjoint: far-field weights, two bodies")
    bodies = [([sc.star(0.3, 5)], [400], sc.media_from_index(25.0, 1.5)),
              ([sc.star(0.2, 3), sc.circle(0.3, (3.0, 0.0))], [300, 64], sc.media_from_index(12.0, 2.0))]
    p, parts, lo = bodies_problem(bm, bodies)
    for ang in (0.0, 2.2):
        g = bm.bm_far_field_weights(p, ang).cpu().numpy()
        for q, (_, _, md) in enumerate(bodies):
            ref = wsbm.far_field_weights(geometry.discretize(*parts[q]), md, ang)
            got = g[2 * lo[q]:2 * lo[q + 1]]
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fourier_curve_and_chain(gpu_lib):
    import torch
    bm = gpu_lib
    note("adjoint: Fourier boundary samples and their chain rule, M = 32, n = 1000")
    rng = np.random.default_rng(4)
    M, n = 32, 1000
    coef = rng.normal(0.0, 0.01, 2 * M)
    xyd = bm.bm_fourier_curve(torch.from_numpy(coef).cuda(), n).cpu().numpy()
    ref, _ = sc.sample_curves([sc.fourier_curve(coef[:M], coef[M:])], [n])
    assert np.abs(xyd - ref).max() <= 1e-13 * np.abs(ref).max()
    # the samples are affine in the coefficients, so a difference is an exact
    # Jacobian-vector product: out . v = grad . (xyd(c + v) - xyd(c))
    grad = rng.standard_normal((6, n))
    out = bm.bm_fourier_chain(torch.from_numpy(grad).cuda().contiguous(), M).cpu().numpy()
    for _ in range(3):
        v = rng.standard_normal(2 * M)
        moved, _ = sc.sample_curves([sc.fourier_curve(coef[:M] + v[:M], coef[M:] + v[M:])], [n])
        jvp = np.sum(grad * (moved - ref))
        assert abs(out @ v - jvp) <= 1e-10 * np.abs(grad).sum() * np.abs(moved - ref).max()


def _richardson(f, h):
    return (4 * (f(h / 2) - f(-h / 2)) / h - (f(h) - f(-h)) / (2 * h)) / 3


def test_shape_derivative_matches_oracle_per_sample(gpu_lib):
    """grad[q, i] = Re(coef_b dL_b/d xyd[q, i]) for random phi, lam (not
    solutions), two bodies, one of them two curves; checked against Richardson
    differences of the oracle's L on sampled nodes, including the first and
    last node of every curve."""
    import torch
    bm = gpu_lib
    note("adjoint: per-sample shape derivative vs oracle differences")
    bodies = [([sc.star(0.2, 3), sc.circle(0.3, (2.5, 0.0))], [48, 40], sc.media_from_index(8.0, 1.5)),
              ([sc.star(0.25, 5)], [56], sc.media_from_index(12.0, 2.0))]
    p, parts, lo = bodies_problem(bm, bodies)
    n = lo[-1]
    rng = np.random.default_rng(5)
    phi, lam = cplx(rng, 2 * n), cplx(rng, 2 * n)
    coef = cplx(rng, 2)
    inc, obs = 0.7, 2.9
    grad = bm.bm_shape_derivative(p, torch.from_numpy(phi).cuda(), torch.from_numpy(lam).cuda(), inc, obs,
                                  coef=torch.from_numpy(coef).cuda()).cpu().numpy()
    assert grad.shape == (6, n)
    for q, (_, sizes, md) in enumerate(bodies):
        xyd0, s = parts[q]
        sl = slice(2 * lo[q], 2 * lo[q + 1])

        def L(xyd):
            nd = geometry.discretize(xyd, s)
            g = wsbm.far_field_weights(nd, md, obs)
            b = wsbm.rhs_plane_wave(nd, md, inc)
            return g @ phi[sl] + lam[sl] @ (b - wsbm.assemble_dense(nd, md) @ phi[sl])

        ends = np.cumsum([0] + sizes)
        picks = sorted(set(rng.choice(ends[-1], 8, replace=False).tolist()
                           + ends[:-1].tolist() + (ends[1:] - 1).tolist()))
        ref = np.zeros((6, len(picks)))
        for a, i in enumerate(picks):
            for r in range(6):
                def f(h, r=r, i=i):
                    x = xyd0.copy()
                    x[r, i] += h
                    return L(x)
                ref[r, a] = np.real(coef[q] * _richardson(f, 1e-5 if r < 4 else 1e-3))
        got = grad[:, lo[q] + np.array(picks)]
        scale = np.abs(ref).max()
        note(f"  body {q}: max |grad| {scale:.3e}, max error {np.abs(got - ref).max() / scale:.2e}")
        assert np.abs(got - ref).max() <= 1e-7 * scale


def test_shape_derivative_default_weight_is_backscatter(gpu_lib):
    """coef = NULL uses 2 conj(u_inf,b(obs)) of phi itself."""
    import torch
    bm = gpu_lib
    bodies = [([sc.star(0.3, 5)], [300], sc.media_from_index(15.0, 1.5)),
              ([sc.star(0.2, 3)], [200], sc.media_from_index(10.0, 1.8))]
    p, parts, lo = bodies_problem(bm, bodies)
    rng = np.random.default_rng(6)
    phi = torch.from_numpy(cplx(rng, 2 * lo[-1])).cuda()
    lam = torch.from_numpy(cplx(rng, 2 * lo[-1])).cuda()
    u = bm.bm_far_field(p, phi, torch.tensor([3.5], dtype=torch.float64))
    g1 = bm.bm_shape_derivative(p, phi, lam, 0.4, 3.5)
    g2 = bm.bm_shape_derivative(p, phi, lam, 0.4, 3.5, coef=(2 * u.conj()).contiguous())
    d = (g1 - g2).abs().max().item()
    assert d <= 1e-12 * g2.abs().max().item()


def test_autograd_gradient_matches_oracle_small(gpu_lib):
    """dJ/dc of the backscatter intensity (HSS forward, adjoint backward) against
    the oracle's Richardson differences of the dense J: N = 192, 8 coefficients."""
    import torch
    bm = gpu_lib
    note("adjoint: autograd gradient vs oracle, N = 192, M = 4, k0 = 10")
    md = sc.media_from_index(10.0, 1.5)
    rng = np.random.default_rng(7)
    c0 = rng.normal(0.0, 0.03, 8)
    coef = torch.from_numpy(c0).cuda().requires_grad_(True)
    J = bm.backscatter_intensity(coef, 192, md.k0, md.k1, md.eps0, md.eps1, theta_inc=0.3, leaf=32,
                                 proxy_ratio=1.5, proxy_points=64, id_tol=1e-12)
    J.backward()
    got = coef.grad.cpu().numpy()
    u_ref, J_ref = shape.backscatter(c0, 192, md, 0.3)
    ref = shape.gradient_fd(c0, 192, md, 0.3)
    note(f"  J {J.item():.12e} (oracle {J_ref:.12e}); grad error {np.abs(got - ref).max() / np.abs(ref).max():.2e}")
    assert abs(J.item() - J_ref) <= 1e-8 * J_ref
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def _full_workload():
    wl = sc.fourier_workload()
    crv = wl.curves[0]
    return wl, np.concatenate([crv.a, crv.b])


# The differentiation workload is solved with id_tol 1e-12: at 1e-10 the HSS
# backscatter intensity is off by ~5e-7 relative, which central differences with
# step 1e-6 amplify to ~1e-3 of the gradient; at 1e-12 J is accurate to ~1e-9
# and the differences resolve the gradient to ~1e-8.
FULL_OPTS = dict(leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-12)
# the same with the library's tuned build options (Gaussian-sketch ID, stop rule),
# the benchmark's configuration
TUNED_OPTS = dict(FULL_OPTS, sketch=-1, max_rank_ratio=-1)
FULL_CASES = [pytest.param(FULL_OPTS, id="cpqr"), pytest.param(TUNED_OPTS, id="tuned")]


@pytest.mark.parametrize("opts", FULL_CASES)
def test_autograd_gradient_full_workload_central_differences(gpu_lib, opts):
    """The differentiation workload: r = 1 + sum_{j<=32} (a_j cos jt + b_j sin jt),
    coefficients ~ N(0, 0.01^2), N = 8192, k0 = 40, n = 1.5, J = |u_inf(-d)|^2:
    all 64 gradient entries against central differences of the GPU's J with
    step 1e-6."""
    import torch
    bm = gpu_lib
    wl, c0 = _full_workload()
    md, n = wl.media, wl.n
    note(f"adjoint: full workload N={n}, 64 coefficients, central differences step 1e-6")
    coef = torch.from_numpy(c0).cuda().requires_grad_(True)
    J = bm.backscatter_intensity(coef, n, md.k0, md.k1, md.eps0, md.eps1, theta_inc=wl.theta_inc, **opts)
    J.backward()
    got = coef.grad.cpu().numpy()
    h = 1e-6
    fd = np.empty(64)

    def jv(c):
        with torch.no_grad():
            return bm.backscatter_intensity(torch.from_numpy(c).cuda(), n, md.k0, md.k1, md.eps0, md.eps1,
                                            theta_inc=wl.theta_inc, **opts).item()

    for m in range(64):
        e = np.zeros(64)
        e[m] = h
        fd[m] = (jv(c0 + e) - jv(c0 - e)) / (2 * h)
    err = np.abs(got - fd).max() / np.abs(fd).max()
    note(f"  J {J.item():.12e}, max |grad| {np.abs(fd).max():.3e}, max error vs differences {err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("opts", FULL_CASES)
def test_autograd_gradient_full_workload_dense_oracle(gpu_lib, opts):
    """J and directional derivatives dJ.v at the full differentiation workload
    against the dense oracle (one LU of the 16384 x 16384 system, values stored
    by tests/golden/make_shape_golden.py)."""
    import json
    import os
    import torch
    bm = gpu_lib
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "shape_fourier8192.json")) as f:
        gold = json.load(f)
    wl, c0 = _full_workload()
    md, n = wl.media, wl.n
    assert (gold["n"], gold["k0"], gold["k1"], gold["theta_inc"]) == (n, md.k0, md.k1, wl.theta_inc)
    coef = torch.from_numpy(c0).cuda().requires_grad_(True)
    J = bm.backscatter_intensity(coef, n, md.k0, md.k1, md.eps0, md.eps1, theta_inc=wl.theta_inc, **opts)
    J.backward()
    g = coef.grad.cpu().numpy()
    note(f"adjoint: full workload vs dense oracle: J {J.item():.12e} (oracle {gold['J']:.12e})")
    assert abs(J.item() - gold["J"]) <= 2e-8 * gold["J"]
    for case in gold["cases"]:
        v = np.array(case["v"])
        d = g @ v
        note(f"  dJ.v {d:.12e} (oracle {case['dJ_dv']:.12e})")
        assert abs(d - case["dJ_dv"]) <= 1e-6 * np.linalg.norm(g)
