#!/usr/bin/env python3
"""Benchmark of the Burton-Miller entry generation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode hss|dense]

Workload: the star r = 1 + 0.3 cos 5 theta, N = 16384 nodes, k_ext = 50,
n = 1.5, plane wave at a seeded angle; HSS leaf 64, proxy circle 1.5 x box
radius with 64 points, ID tolerance 1e-10, FP64 throughout.

mode "hss" (default): a step is the whole hot path -- HSS build (all entry
generation: near, proxy, diagonal and skeleton blocks; ID; factorisation),
plane-wave right-hand side and solve.  value = matrix entries generated per
second of step time; ms_per_step is the HSS build+solve time.
mode "dense": a step is one full sweep of the 2N x 2N matrix: N^2 pairs, 4 N^2
complex entries written to HBM (17.2 GB).

Prints ONE JSON line (rank 0).  The timed region is bracketed by
torch.cuda.synchronize() and measured with HIP events recorded on the stream
the kernels are launched on; inputs are resident in HBM before it starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TF = 78.6      # MI355X FP64 vector, TFLOP/s
BYTES_PER_PAIR = 64             # 4 complex128 entries written per (target, source) pair


def cpu_baseline(wl, rows: int = 256):
    """Oracle (NumPy/SciPy, single thread) on a bounded sample: `rows` target
    nodes against all N sources of the same workload."""
    import numpy as np
    from oracle import geometry, wsbm
    xyd, sizes = wl.xyd()
    nd = geometry.discretize(xyd, sizes)
    idx = np.linspace(0, wl.n - 1, rows).astype(np.int64)
    t0 = time.perf_counter()
    wsbm.assemble_rows(nd, wl.media, idx)
    dt = time.perf_counter() - t0
    entries = 4 * rows * wl.n
    return {"value": entries / dt / 1e9, "unit": "Gentries/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} target rows x {wl.n} sources of the same star workload "
                      f"({rows * wl.n} pairs, {dt:.1f} s; NumPy/SciPy elementwise, one thread)"}


def run_dense(args):
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    g = bm.bm_geom_create(sizes, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    n = wl.n
    A = torch.empty((2 * n, 2 * n), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bm.bm_assemble_dense(p, out=A)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        bm.bm_assemble_dense(p, out=A)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    pairs = n * n
    entries = 4 * pairs
    gbs = BYTES_PER_PAIR * pairs / (ms * 1e-3) / 1e9
    out = {
        "metric": "Gentries/s Burton-Miller blocks (frac FP64 peak); HSS build+solve s at N=16384",
        "value": entries / (ms * 1e-3) / 1e9,
        "unit": "Gentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dense WSBM sweep, {wl.name}", "n_nodes": n, "pairs": pairs,
                   "entries": entries, "theta_inc": wl.theta_inc},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_dense",
                     "avg_launch_ms": ms},
    }
    return out, wl


def run_hss(args):
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    g = bm.bm_geom_create(sizes, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    stream = torch.cuda.current_stream()
    b = torch.empty(2 * wl.n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)

    def step():
        h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio,
                            proxy_points=wl.proxy_points, id_tol=wl.id_tol)
        bm.bm_rhs_plane_wave(p, wl.theta_inc, out=b)
        bm.bm_hss_solve(h, b, out=x)
        return bm.bm_hss_stats(h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stats = []
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        stats.append(step())
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    st = stats[-1]
    gen_s = sum(q["seconds_generate"] for q in stats) / len(stats)
    entries = st["entries"]
    gen_gbs = 16 * entries / gen_s / 1e9
    out = {
        "metric": "Gentries/s Burton-Miller blocks (frac FP64 peak); HSS build+solve s at N=16384",
        "value": entries / (ms * 1e-3) / 1e9,
        "unit": "Gentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"HSS build+solve, {wl.name}", "n_nodes": wl.n, "leaf": wl.leaf,
                   "proxy_points": wl.proxy_points, "proxy_ratio": wl.proxy_ratio,
                   "id_tol": wl.id_tol, "theta_inc": wl.theta_inc},
        "hss_build_solve_s": ms * 1e-3,
        "hss": {"entries": entries, "pairs": st["pairs"], "levels": st["levels"],
                "compressed_levels": st["compressed_levels"], "root_size": st["root_size"],
                "max_rank": st["max_rank"],
                "seconds_generate": gen_s,
                "seconds_compress": sum(q["seconds_compress"] for q in stats) / len(stats),
                "seconds_factor": sum(q["seconds_factor"] for q in stats) / len(stats),
                "generation_Gentries_s": entries / gen_s / 1e9},
        "roofline": {"bound": "hbm", "achieved": gen_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gen_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_gen_jobs"},
    }
    return out, wl


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["hss", "dense"], default="hss")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the run, copy this many MiB device-to-device once (a plain copy "
                         "kernel of known size, to scale HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        return 2
    if args.calib_copy_mib > 0:
        import torch
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out, wl = run_hss(args) if args.mode == "hss" else run_dense(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
