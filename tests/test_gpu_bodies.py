"""GPU tests of problems made of independent bodies (the batched workload):
every body has its own curves and media, pairs in different bodies are zero
blocks, and the HSS build factors the bodies as a forest, one tree per body,
with the levels of all trees compressed together.

The oracle has no notion of bodies: each body is checked against the oracle's
single-body system of the same curves and media, and the cross-body blocks
must be exactly zero."""
import sys

import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, wsbm

from parity import assert_parity

pytestmark = pytest.mark.gpu

HSS_BAR = 1e-7


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bodies_problem(bm, bodies):
    """bodies: list of (curves, sizes, media).  Returns the GPU problem, the
    per-body oracle node sets and the node offsets of the bodies."""
    curves, sizes, boc, media, nds, lo = [], [], [], [], [], [0]
    for b, (cv, sz, md) in enumerate(bodies):
        curves += cv
        sizes += sz
        boc += [b] * len(cv)
        media.append((md.k0, md.k1, md.eps0, md.eps1))
        xyd_b, s_b = sc.sample_curves(cv, sz)
        nds.append(geometry.discretize(xyd_b, s_b))
        lo.append(lo[-1] + sum(sz))
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create_bodies(g, boc, media)
    return p, nds, lo


def three_bodies():
    return [([sc.star(0.3, 5)], [300], sc.media_from_index(20.0, 1.5)),
            ([sc.star(0.2, 3), sc.circle(0.3, (2.5, 0.0))], [257, 64], sc.media_from_index(12.0, 2.0)),
            ([sc.circle(1.0)], [129], sc.media_from_index(35.0, 1.2))]


def test_bodies_dense_block_diagonal(gpu_lib):
    import torch
    bm = gpu_lib
    note("bodies: dense matrix of three bodies (ragged, one with two curves)")
    bodies = three_bodies()
    p, nds, lo = bodies_problem(bm, bodies)
    n = lo[-1]
    A = bm.bm_assemble_dense(p).cpu().numpy()
    assert A.shape == (2 * n, 2 * n)
    for b, (_, _, md) in enumerate(bodies):
        r = slice(2 * lo[b], 2 * lo[b + 1])
        ref = wsbm.assemble_dense(nds[b], md)
        assert_parity(A[r, r], ref)
        mask = np.ones(2 * n, bool)
        mask[r] = False
        assert np.all(A[r][:, mask] == 0)


def test_bodies_rhs_matvec_far_field(gpu_lib):
    import torch
    bm = gpu_lib
    note("bodies: RHS, matvec and far field per body")
    bodies = three_bodies()
    p, nds, lo = bodies_problem(bm, bodies)
    n = lo[-1]
    rhs = bm.bm_rhs_plane_wave(p, 0.7).cpu().numpy()
    rng = np.random.default_rng(5)
    xh = rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)
    y = bm.bm_matvec(p, torch.from_numpy(xh).cuda()).cpu().numpy()
    ang = np.linspace(0, 2 * np.pi, 7, endpoint=False)
    uinf = bm.bm_far_field(p, torch.from_numpy(xh).cuda(), torch.from_numpy(ang)).cpu().numpy()
    assert uinf.shape == (3 * ang.size,)
    for b, (_, _, md) in enumerate(bodies):
        r = slice(2 * lo[b], 2 * lo[b + 1])
        np.testing.assert_allclose(rhs[r], wsbm.rhs_plane_wave(nds[b], md, 0.7), rtol=1e-12, atol=1e-13)
        yb = wsbm.assemble_dense(nds[b], md) @ xh[r]
        assert np.abs(y[r] - yb).max() <= 1e-10 * np.abs(yb).max()
        fb = wsbm.far_field(nds[b], md, xh[r], ang)
        got = uinf[b * ang.size:(b + 1) * ang.size]
        assert np.abs(got - fb).max() <= 1e-10 * np.abs(fb).max()


@pytest.mark.parametrize("sketch", [0, 128, -1])   # -1: the tuned options (with the stop rule)
def test_bodies_hss_forest(gpu_lib, sketch):
    """Five bodies of uneven size, wavenumber and index, leaf 64: trees of
    different depth compressed together, one body too small to compress."""
    import torch
    bm = gpu_lib
    note(f"bodies: HSS forest of five bodies, sketch={sketch}")
    bodies = [([sc.star(0.3, 5)], [1500], sc.media_from_index(30.0, 1.5)),
              ([sc.star(0.15, 4)], [700], sc.media_from_index(15.0, 1.8)),
              ([sc.star(0.25, 7)], [2100], sc.media_from_index(40.0, 1.3)),
              ([sc.circle(1.0)], [96], sc.media_from_index(10.0, 2.0)),
              ([sc.star(0.2, 3)], [1024], sc.media_from_index(25.0, 1.6))]
    p, nds, lo = bodies_problem(bm, bodies)
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=sketch,
                        max_rank_ratio=-1.0 if sketch == -1 else 0.0)
    st = bm.bm_hss_stats(h)
    note(f"  stats {st}")
    for l in range(st["compressed_levels"]):
        note(f"  iteration {l}: {bm.bm_hss_level(h, l)}")
    assert st["compressed_levels"] >= (1 if sketch == -1 else 3)   # the stop rule may end bodies early
    b = bm.bm_rhs_plane_wave(p, 0.4)
    B = torch.stack([b, bm.bm_rhs_plane_wave(p, 2.0)]).contiguous()
    X = bm.bm_hss_solve(h, B).cpu().numpy()
    for r, ang in enumerate([0.4, 2.0]):
        for q, (_, _, md) in enumerate(bodies):
            sl = slice(2 * lo[q], 2 * lo[q + 1])
            ref = wsbm.solve_dense(wsbm.assemble_dense(nds[q], md), wsbm.rhs_plane_wave(nds[q], md, ang))
            err = np.linalg.norm(X[r, sl] - ref) / np.linalg.norm(ref)
            note(f"  rhs {r} body {q}: relative error {err:.2e}")
            assert err < HSS_BAR, (r, q, err)


def test_bodies_rejects_bad_body_lists(gpu_lib):
    bm = gpu_lib
    xyd, s = sc.sample_curves([sc.circle(), sc.circle(0.5, (3, 0)), sc.circle(0.5, (0, 3))], [64, 64, 64])
    g = bm.bm_geom_create(s, xyd)
    m = (10.0, 15.0, 1.0, 2.25)
    for boc, media in (([0, 2, 2], [m, m, m]), ([1, 1, 1], [m, m]), ([0, 1, 0], [m, m]),
                       ([0, 0, 1], [m]), ([0, 1, 1], [m, (10.0, -1.0, 1.0, 1.0)])):
        with pytest.raises(bm.BmError):
            bm.bm_problem_create_bodies(g, boc, media)
