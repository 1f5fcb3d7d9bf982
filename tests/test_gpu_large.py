"""GPU test of the large single-GPU workload at its full size: 16 stars on a
4 x 4 grid of spacing 3 in one body, 16384 nodes each (N = 262144), k0 = 200,
n = 2, leaf 128, 96 proxy points (adaptive), tol 1e-10, Gaussian-sketch ID and
the rank-ratio stop rule -- the configuration `bench.py --mode large` times.

The dense oracle cannot solve this size, so the solution is checked by
properties that hold at any size: the residual |A x - b| / |b| through the
GPU's matrix-free product, and sampled rows of A x - b assembled one by one by
the oracle (both stars' media, all 262144 columns)."""
import sys

import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, wsbm

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_large_workload_full_size_residuals(gpu_lib):
    import torch
    bm = gpu_lib
    wl = sc.grid_of_stars_workload()
    note(f"large: {wl.name}, N={wl.n}")
    xyd, s = wl.xyd()
    g = bm.bm_geom_create(s, torch.from_numpy(xyd).cuda())
    md = wl.media
    p = bm.bm_problem_create(g, md.k0, md.k1, md.eps0, md.eps1)
    h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                        id_tol=wl.id_tol, sketch=128, proxy_adapt=True, max_rank_ratio=0.8)
    st = bm.bm_hss_stats(h)
    note(f"  build {st['seconds_total']:.1f} s, {st['compressed_levels']} levels, root {st['root_size']}")
    b = bm.bm_rhs_plane_wave(p, wl.theta_inc)
    x = bm.bm_hss_solve(h, b)
    del h
    res = (torch.linalg.vector_norm(bm.bm_matvec(p, x) - b) / torch.linalg.vector_norm(b)).item()
    note(f"  matrix-free residual {res:.2e}")
    assert res < 1e-6
    # sampled rows through the oracle: the first and last node of two stars and one node in between
    nd = geometry.discretize(xyd, s)
    rows = np.array([0, 16383, 5 * 16384 + 7000, 15 * 16384, 15 * 16384 + 16383])
    xh = x.cpu().numpy()
    bh = wsbm.rhs_plane_wave(nd, md, wl.theta_inc)
    ax = wsbm.assemble_rows(nd, md, rows) @ xh
    for q, i in enumerate(rows):
        r = ax[2 * q:2 * q + 2] - bh[2 * i:2 * i + 2]
        note(f"  node {i}: |(A x - b)_i| = {np.abs(r).max():.2e}, |b_i| = {np.abs(bh[2 * i + 1]):.2e}")
        assert np.abs(r).max() <= 1e-6 * np.abs(bh).max()
