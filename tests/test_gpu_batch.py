"""GPU test of the batched workload: 256 independent stars (a ~ U[0.1, 0.3],
m ~ U{3..8}, N ~ U{1024..8192}, k0 ~ U[10, 80], n ~ U[1.2, 2.0], drawn per
star in that order) in ONE problem of 256 bodies, factored as one HSS forest
and solved for a plane wave each, checked star by star against rows of the
oracle's own system matrix (Eq. (3)/(5)) at three nodes per star: the first,
one in the middle and the last.

Bars, relative to the largest |b| of the star: 1e-7 for the FP64 build at
tolerance 1e-10 (the tuned options, adaptive proxy counts; the measured
per-star 2-norm residuals are below 2e-8).  FP32 proxy blocks are meant for
tolerances at or above their rounding noise (~1e-7 per entry): at tolerance
1e-6 their worst sampled residual must stay within 5 times that of the FP64
proxies at the same tolerance (or 5 tol), the criterion of the one-body FP32
test; the FP32 build's distance from the FP64 solutions is reported per
star."""
import sys

import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, wsbm

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_batched_256_stars_vs_oracle_rows(gpu_lib):
    import torch
    bm = gpu_lib
    wls = sc.batched_star_workloads(256)
    curves, sizes, boc, media = [], [], [], []
    for q, w in enumerate(wls):
        curves += w.curves
        sizes += w.sizes
        boc += [q] * len(w.curves)
        media.append((w.media.k0, w.media.k1, w.media.eps0, w.media.eps1))
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create_bodies(g, boc, media)
    n = g.n
    lo = np.concatenate([[0], np.cumsum([sum(w.sizes) for w in wls])])
    note(f"batch: 256 stars, {n} nodes in one problem")
    b = bm.bm_rhs_plane_wave(p, 0.0)
    bh = b.cpu().numpy()
    sols = {}
    for name, opts in (("fp64_tol1e-10", dict(id_tol=1e-10, sketch=-1, max_rank_ratio=-1.0)),
                       ("fp64_tol1e-6", dict(id_tol=1e-6, sketch=-1, max_rank_ratio=-1.0)),
                       ("fp32proxies_tol1e-6", dict(id_tol=1e-6, sketch=-1, max_rank_ratio=-1.0, proxy_fp32=True))):
        h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, proxy_adapt=True, **opts)
        st = bm.bm_hss_stats(h)
        sols[name] = bm.bm_hss_solve(h, b).cpu().numpy()
        note(f"  {name}: {st['compressed_levels']} iterations, roots {st['root_size']} unknowns in total, "
             f"build {st['seconds_total']:.2f} s")
        del h
    worst = {k: 0.0 for k in sols}
    dist = []
    for q, w in enumerate(wls):
        nq = sum(w.sizes)
        xq, sq = sc.sample_curves(w.curves, w.sizes)
        nd = geometry.discretize(xq, sq)
        bq = wsbm.rhs_plane_wave(nd, w.media, 0.0)
        assert np.abs(bh[2 * lo[q]:2 * lo[q + 1]] - bq).max() <= 1e-12 * np.abs(bq).max()
        rows = np.array([0, nq // 2 + 1, nq - 1])
        A = wsbm.assemble_rows(nd, w.media, rows)
        brow = bq[np.ravel(np.column_stack([2 * rows, 2 * rows + 1]))]
        for name, x in sols.items():
            r = A @ x[2 * lo[q]:2 * lo[q + 1]] - brow
            worst[name] = max(worst[name], np.abs(r).max() / np.abs(bq).max())
        x64 = sols["fp64_tol1e-10"][2 * lo[q]:2 * lo[q + 1]]
        dist.append([np.linalg.norm(sols[k][2 * lo[q]:2 * lo[q + 1]] - x64) / np.linalg.norm(x64)
                     for k in ("fp64_tol1e-6", "fp32proxies_tol1e-6")])
    dist = np.array(dist)
    note(f"  worst sampled residual / max|b| per star: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    note(f"  distance from the tol-1e-10 solution per star: FP64 proxies at 1e-6 max {dist[:, 0].max():.2e} "
         f"median {np.median(dist[:, 0]):.2e}; FP32 proxies at 1e-6 max {dist[:, 1].max():.2e} "
         f"median {np.median(dist[:, 1]):.2e}")
    assert worst["fp64_tol1e-10"] <= 1e-7
    assert worst["fp32proxies_tol1e-6"] <= 5 * max(worst["fp64_tol1e-6"], 1e-6)
