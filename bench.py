#!/usr/bin/env python3
"""Benchmark of the Burton-Miller entry generation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode hss|dense|matvec|batch|adjoint]

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
# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (separate
# runs), scaled by what the same counters read for a plain 1 GiB device copy
# (FETCH x 2.0, WRITE x 1.0); profiles/pmc_counters_star16384.txt.  Valid for
# the kernels and workloads those counters were taken on.
# FP64 operations per pair of the entry kernel, from rocprofv3 --pmc
# SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 over the dense sweep (FMA counted as 2)
FLOP_PER_PAIR = 313.9
# the same for the generate-and-reduce kernel (entries times x, block sums)
FLOP_PER_PAIR_MATVEC = 349.9
MEASURED_TRAFFIC = {
    # one sweep: one launch
    "k_dense": (2.0 * 48516.6 + 16864326) * 1024,
    # two HSS builds with the tuned options (gaussian sketch, unknowns + 8 rows; stop
    # ratio 0.6; the root inverted by panels on one stream): 256 launches of the
    # matrix-core class (k_gemm_t16 x154, k_gemm x46, k_gemm_t64 x8 and the panel
    # steps k_gauss_jordan_blk_panel x48), 10 of k_cpqr_fused
    ("k_gemm", 8, 0.6): (2.0 * (770917.0625 + 1994889.8125 + 386684.3125 + 1506995.0625)
                         + (249421.8125 + 735561.28125 + 305524.125 + 1821347.71875)) * 1024 / 256,
    ("k_cpqr_fused", 8, 0.6): (2.0 * (37028.375 + 78610.0625 + 6049.75)
                               + (72882.375 + 156152.59375 + 10894.5)) * 1024 / 10,
}


def _cpu_rows(args):
    """Oracle rows for a chunk of target nodes (one worker of the baseline pool)."""
    from oracle import geometry, wsbm
    xyd, sizes, media, rows = args
    nd = geometry.discretize(xyd, sizes)
    wsbm.assemble_rows(nd, media, rows)
    return len(rows)


def cpu_baseline_run(chunks: int = 2, chunk_rows: int = 64, lu_n: int = 6144):
    """The oracle on the host (run in a child process that never touches the
    GPU): (a) the dense assembly of the benchmark star, a process pool over row
    chunks, every worker assembling `chunk_rows` target nodes against all N
    sources, `chunks` chunks per core; (b) the dense LU (LAPACK zgetrf through
    SciPy, BLAS threads = cores) of an lu_n x lu_n complex matrix, timed and
    extrapolated by n^3 to the benchmark's 2N x 2N system.  Cores: the host's,
    at most 16 (the host share of one GPU)."""
    import multiprocessing as mp
    import numpy as np
    import scipy.linalg
    from threadpoolctl import threadpool_limits
    import scatterers as sc
    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    cores = max(1, min(os.cpu_count() or 1, 16))
    nrows = cores * chunks * chunk_rows
    starts = np.linspace(0, wl.n - chunk_rows, cores * chunks).astype(np.int64)
    jobs = [(xyd, sizes, wl.media, np.arange(s0, s0 + chunk_rows)) for s0 in starts]
    # the LU first: OpenBLAS's thread pool is not safe to start again in a
    # process that has forked workers
    rng = np.random.default_rng(0)
    A = rng.standard_normal((lu_n, lu_n)) + 1j * rng.standard_normal((lu_n, lu_n))
    A = np.asfortranarray(A)
    with threadpool_limits(cores):
        t0 = time.perf_counter()
        scipy.linalg.lu_factor(A, overwrite_a=True, check_finite=False)
        t_lu = time.perf_counter() - t0
    del A
    with threadpool_limits(1):
        with mp.get_context("fork").Pool(cores) as pool:
            pool.map(_cpu_rows, jobs[:cores])   # warm-up: imports, geometry
            t0 = time.perf_counter()
            done = sum(pool.map(_cpu_rows, jobs))
            t_asm = time.perf_counter() - t0
    pairs = done * wl.n
    rate = pairs / t_asm
    n2 = 2 * wl.n
    lu_full = t_lu * (n2 / lu_n) ** 3
    asm_full = wl.n * wl.n / rate
    return {"value": 4 * rate / 1e9, "unit": "Gentries/s", "cores": cores, "kind": "oracle",
            "sample": f"(a) assembly: {done} target rows x {wl.n} sources of the benchmark star ({pairs} pairs, "
                      f"{t_asm:.1f} s, a pool of {cores} processes over row chunks, NumPy/SciPy elementwise); "
                      f"(b) dense LU of a {lu_n} x {lu_n} complex matrix ({t_lu:.1f} s, LAPACK with {cores} "
                      f"BLAS threads), extrapolated by n^3 to 2N = {n2}",
            "assembly_Gentries_s": 4 * rate / 1e9, "assembly_pairs_s": rate,
            "assembly_seconds_full_matrix": asm_full,
            "lu_n": lu_n, "lu_seconds": t_lu, "lu_seconds_2N_extrapolated": lu_full,
            "dense_solve_seconds_estimate": asm_full + lu_full,
            "note": "the oracle has no HSS solver: its build+solve equivalent is dense assembly + LU of the "
                    "2N x 2N system (dense_solve_seconds_estimate = full assembly at the measured rate + the "
                    "extrapolated LU)"}


def cpu_baseline(wl):
    """cpu_baseline_run in a child process (it forks a process pool; the
    benchmark process itself has initialised the GPU)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only"], capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"value": None, "unit": "Gentries/s", "cores": None, "kind": "oracle",
                "sample": "failed: " + r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def fma_probe(blocks, iters, out):
    """The FP64 FMA-rate probe of the benchmark-only library libbmhss_probe.so
    (16 independent FMA chains per thread, blocks x 256 threads)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2607_00790_amd", "libbmhss_probe.so"))
    lib.fma_probe.restype = ctypes.c_int
    lib.fma_probe.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    rc = lib.fma_probe(ctypes.c_void_p(out.data_ptr()), int(blocks), int(iters),
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"fma_probe: HIP error {rc}")
    return out


def entry_kernel_rates(p, n):
    """The entry kernels on the benchmark star, outside the timed HSS step: the
    dense sweep (N^2 pairs written to HBM) and the generate-and-reduce product
    (the same entries, nothing stored), each as Gentries/s and as a fraction of
    the published FP64 peak and of the FP64 FMA rate this device sustains
    (measured by the benchmark's FMA probe in the same run)."""
    import torch
    import paper_2607_00790_amd as bm
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    blocks, iters = 256 * 32, 2048
    buf = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    probe_ms = timed(lambda: fma_probe(blocks, iters, buf), 5)
    measured = 2.0 * 16 * iters * 256 * blocks / (probe_ms * 1e-3) / 1e12
    pairs = n * n
    out = {"fp64_fma_probe_tflops": measured, "fp64_spec_peak_tflops": FP64_VECTOR_PEAK_TF}
    A = torch.empty((2 * n, 2 * n), dtype=torch.complex128, device="cuda")
    dense_ms = timed(lambda: bm.bm_assemble_dense(p, out=A), 3)
    del A
    x = bm.bm_rhs_plane_wave(p, 0.3)
    y = torch.empty_like(x)
    mv_ms = timed(lambda: bm.bm_matvec(p, x, out=y), 3)
    for name, ms, fpp in (("dense", dense_ms, FLOP_PER_PAIR), ("matvec", mv_ms, FLOP_PER_PAIR_MATVEC)):
        tf = fpp * pairs / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "Gentries_s": 4 * pairs / (ms * 1e-3) / 1e9, "flop_per_pair": fpp, "tflops": tf,
                     "frac_spec_peak": tf / FP64_VECTOR_PEAK_TF, "frac_measured_peak": tf / measured}
    out["dense"]["hbm_GBs"] = BYTES_PER_PAIR * pairs / (dense_ms * 1e-3) / 1e9
    out["dense"]["hbm_frac"] = out["dense"]["hbm_GBs"] / HBM_PEAK_GBS
    return out


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
    tf = FLOP_PER_PAIR * pairs / (ms * 1e-3) / 1e12
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
                     "frac": gbs / HBM_PEAK_GBS, "traffic": MEASURED_TRAFFIC.get("k_dense"),
                     "kernel": "k_dense", "avg_launch_ms": ms,
                     "algorithmic_bytes_per_launch": BYTES_PER_PAIR * pairs},
        "fp64": {"flop_per_pair": FLOP_PER_PAIR, "tflops": tf, "peak_tflops": FP64_VECTOR_PEAK_TF,
                 "frac": tf / FP64_VECTOR_PEAK_TF},
    }
    return out, wl


def run_matvec(args):
    """Generate-and-reduce: y = A x with every entry evaluated on the fly and
    nothing written but y (the entry kernel's arithmetic roof)."""
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    g = bm.bm_geom_create(sizes, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    n = wl.n
    x = bm.bm_rhs_plane_wave(p, wl.theta_inc)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bm.bm_matvec(p, x, out=y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        bm.bm_matvec(p, x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    pairs = n * n
    entries = 4 * pairs
    tf = FLOP_PER_PAIR_MATVEC * pairs / (ms * 1e-3) / 1e12
    out = {
        "metric": "Gentries/s Burton-Miller blocks (frac FP64 peak); HSS build+solve s at N=16384",
        "value": entries / (ms * 1e-3) / 1e9,
        "unit": "Gentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"matrix-free y = A x (generate and reduce), {wl.name}", "n_nodes": n,
                   "pairs": pairs, "entries": entries},
        "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s",
                     "frac": tf / FP64_VECTOR_PEAK_TF, "traffic": None, "kernel": "k_matvec_partial",
                     "flop_per_pair": FLOP_PER_PAIR_MATVEC, "avg_launch_ms": ms},
    }
    return out, wl


def run_batch(args):
    """The batched workload: independent stars of uneven N, wavenumber and index
    in one problem, factored as a forest (every level of every tree in one
    launch per kernel) and solved for one plane wave each.  The same stars are
    then built one by one through the plain one-body path, for comparison."""
    import numpy as np
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    wls = sc.batched_star_workloads(args.batch)
    curves, sizes, boc, media = [], [], [], []
    for b, w in enumerate(wls):
        curves += w.curves
        sizes += w.sizes
        boc += [b] * len(w.curves)
        media.append((w.media.k0, w.media.k1, w.media.eps0, w.media.eps1))
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create_bodies(g, boc, media)
    n = g.n
    opts = dict(leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=args.sketch,
                proxy_adapt=bool(args.proxy_adapt), max_rank_ratio=args.max_rank_ratio)
    stream = torch.cuda.current_stream()
    b = torch.empty(2 * n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)

    def step():
        h = bm.bm_hss_build(p, **opts)
        bm.bm_rhs_plane_wave(p, 0.0, out=b)
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
    # residual of every body through the matrix-free product (block diagonal)
    r = (bm.bm_matvec(p, x) - b).cpu().numpy()
    bh = b.cpu().numpy()
    lo = np.concatenate([[0], np.cumsum([sum(w.sizes) for w in wls])])
    res = [np.linalg.norm(r[2 * lo[q]:2 * lo[q + 1]]) / np.linalg.norm(bh[2 * lo[q]:2 * lo[q + 1]])
           for q in range(len(wls))]
    # the plain path: one problem and one build per star
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for w in wls:
        xw, sw = sc.sample_curves(w.curves, w.sizes)
        gw = bm.bm_geom_create(sw, torch.from_numpy(xw).cuda())
        pw = bm.bm_problem_create(gw, w.media.k0, w.media.k1, w.media.eps0, w.media.eps1)
        hw = bm.bm_hss_build(pw, **opts)
        bm.bm_hss_solve(hw, bm.bm_rhs_plane_wave(pw, 0.0))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t1
    out = {
        "metric": "Gentries/s Burton-Miller blocks (frac FP64 peak); HSS build+solve s at N=16384",
        "value": st["entries"] / (ms * 1e-3) / 1e9,
        "unit": "Gentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(wls)} independent stars (batched, one forest)", "bodies": len(wls),
                   "n_nodes": n, "leaf": 64, "proxy_points": 64, "proxy_ratio": 1.5, "id_tol": 1e-10,
                   "id": "cpqr" if st["sketch"] == 0 else f"gaussian sketch, unknowns+{st['sketch']} rows",
                   "max_rank_ratio": st["max_rank_ratio"],
                   "proxy_points_rule": "max(64, ceil(2 k R_p) + 32)" if args.proxy_adapt else "64"},
        "batch": {"entries": st["entries"], "iterations": st["compressed_levels"], "roots_total": st["root_size"],
                  "max_rank": st["max_rank"], "max_body_residual": max(res), "median_body_residual": float(np.median(res)),
                  "plain_per_body_builds_s": plain_s, "speedup_vs_plain": plain_s / (ms * 1e-3),
                  "seconds_cpqr": st["seconds_cpqr"], "seconds_factor": st["seconds_factor"]},
    }
    return out, wls[0]


def run_large(args):
    """The large single-GPU workload: 16 stars on a 4 x 4 grid of spacing 3 in
    ONE body (coupled through the exterior medium; the interior operators act
    within each star only), 16384 nodes each (N = 262144), k0 = 200, n = 2,
    leaf 128, 96 proxy points (adaptive: max(96, ceil(2 k R_p) + 32)), tol 1e-10.
    A step is one HSS build + plane-wave right-hand side + solve; the
    residual |A x - b| / |b| comes from the matrix-free product."""
    import numpy as np
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    os.environ.setdefault("BMHSS_VERBOSE", "1")   # progress lines on stderr during the long build
    wl = sc.grid_of_stars_workload(per_curve=args.per_curve)
    xyd, s = wl.xyd()
    g = bm.bm_geom_create(s, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    n = g.n
    opts = dict(leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points, id_tol=wl.id_tol,
                sketch=args.sketch, proxy_adapt=True, max_rank_ratio=args.max_rank_ratio)
    stream = torch.cuda.current_stream()
    b = torch.empty(2 * n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)
    levels = []

    def step():
        h = bm.bm_hss_build(p, **opts)
        st = bm.bm_hss_stats(h)
        print(f"large: build {st['seconds_total']:.2f} s, root {st['root_size']}, max rank {st['max_rank']}",
              file=sys.stderr, flush=True)
        bm.bm_rhs_plane_wave(p, wl.theta_inc, out=b)
        bm.bm_hss_solve(h, b, out=x)
        if not levels:
            levels.extend(bm.bm_hss_level(h, l) for l in range(st["compressed_levels"]))
        return st

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
    t1 = time.perf_counter()
    r = bm.bm_matvec(p, x) - b
    torch.cuda.synchronize()
    mv_s = time.perf_counter() - t1
    res = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    out = {
        "metric": "Gentries/s Burton-Miller blocks (frac FP64 peak); HSS build+solve s at N=16384",
        "value": st["entries"] / (ms * 1e-3) / 1e9,
        "unit": "Gentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"HSS build+solve, {wl.name} (one body of {len(wl.curves)} curves)",
                   "n_nodes": n, "k0": wl.media.k0, "k1": wl.media.k1, **opts,
                   "proxy_points_rule": f"max({wl.proxy_points}, ceil(2 k R_p) + 32)"},
        "large": {"entries": st["entries"], "pairs": st["pairs"], "levels": st["levels"],
                  "compressed_levels": st["compressed_levels"], "root_size": st["root_size"],
                  "max_rank": st["max_rank"], "seconds_build_wall": st["seconds_total"],
                  "seconds_generate": st["seconds_generate"], "seconds_compress": st["seconds_compress"],
                  "seconds_cpqr": st["seconds_cpqr"], "seconds_factor": st["seconds_factor"],
                  "residual": res, "matvec_s": mv_s, "per_level": levels},
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

    levels = []

    def step():
        # the build records the one-right-hand-side solve graph while the GPU
        # inverts the root; the step's solve replays it
        h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio,
                            proxy_points=wl.proxy_points, id_tol=wl.id_tol, sketch=args.sketch,
                            max_rank_ratio=args.max_rank_ratio)
        bm.bm_rhs_plane_wave(p, wl.theta_inc, out=b)
        if args.solve == "graph":
            bm.bm_hss_solve_graph(h, b, out=x)
        else:
            bm.bm_hss_solve(h, b, out=x)
        st = bm.bm_hss_stats(h)
        if not levels:
            levels.extend(bm.bm_hss_level(h, l) for l in range(st["compressed_levels"]))
        return st

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

    def avg(key):
        return sum(q[key] for q in stats) / len(stats)

    # the solve alone: eager (descriptors staged per call, synchronises) and
    # replayed from the HIP graph captured on its first call
    # the HSS build below (kernel_timing) also times every batched GEMM and
    # Gauss-Jordan launch with HIP events (an event pair per launch, so it is
    # kept out of the timed steps)
    h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                        id_tol=wl.id_tol, sketch=args.sketch, max_rank_ratio=args.max_rank_ratio,
                        kernel_timing=True)
    kst = bm.bm_hss_stats(h)
    bm.bm_hss_solve_graph(h, b, out=x)
    solve_ms = {}
    for name, fn in (("eager", lambda: bm.bm_hss_solve(h, b, out=x)),
                     ("graph", lambda: bm.bm_hss_solve_graph(h, b, out=x))):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        solve_ms[name] = (time.perf_counter() - t1) / 20 * 1e3
    del h

    entry = entry_kernel_rates(p, wl.n)

    gen_s = avg("seconds_generate")
    entries = st["entries"]
    # the step-wise CPQR of the levels too large for the whole-box kernel
    launches = st["cpqr_launches"]
    cq_s = avg("seconds_cpqr")
    cq_bytes = st["cpqr_bytes"]
    cq_gbs = cq_bytes / cq_s / 1e9 if cq_s > 0 else None
    sk, ratio = st["sketch"], st["max_rank_ratio"]
    # every kernel class of the step with its launch time (HIP events): the
    # batched GEMM, Gauss-Jordan, sketch and entry-generation launches are
    # event-timed one by one in the extra build above, the CPQR per level in
    # every build.  Each class carries its bound and its algorithmic work.
    kern = {
        # the matrix-core products, with the root's panel steps (each inverts a
        # diagonal block and applies the previous panel's trailing update; its
        # work is both, 8 K^2 b + 8 b^3 flops)
        "k_gemm": dict(seconds=kst["seconds_gemm"], launches=kst["gemm_launches"], work=kst["gemm_flops"],
                       bound="mfma", unit="TFLOP/s", peak=FP64_VECTOR_PEAK_TF,
                       kernels=["k_gemm_t16", "k_gemm", "k_gemm_t64", "k_gauss_jordan_blk_panel"]),
        "k_gauss_jordan": dict(seconds=kst["seconds_inv"], launches=kst["inv_launches"], work=kst["inv_flops"],
                               bound="alu", unit="TFLOP/s", peak=FP64_VECTOR_PEAK_TF,
                               kernels=["k_gauss_jordan_blk", "k_gauss_jordan_pairs<8>", "k_gauss_jordan_32"]),
        "k_sketch": dict(seconds=kst["seconds_sketch"], launches=kst["sketch_launches"],
                         work=kst["sketch_flops"], bound="alu", unit="TFLOP/s", peak=FP64_VECTOR_PEAK_TF),
        "k_gen_jobs": dict(seconds=kst["seconds_gen"], launches=kst["gen_launches"],
                           work=kst["gen_pairs"] * FLOP_PER_PAIR, bound="alu", unit="TFLOP/s",
                           peak=FP64_VECTOR_PEAK_TF),
        "k_cpqr_step_reg": dict(seconds=kst["seconds_cpqr"], launches=kst["cpqr_launches"],
                                work=kst["cpqr_bytes"], bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS),
        "k_cpqr_fused": dict(seconds=kst["seconds_cpqr_fused"], launches=kst["cpqr_fused_launches"],
                             work=kst["cpqr_fused_bytes"], bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS),
    }
    for v in kern.values():
        scale = 1e12 if v["unit"] == "TFLOP/s" else 1e9
        v["achieved"] = v["work"] / v["seconds"] / scale if v["seconds"] > 0 else None
        v["frac"] = v["achieved"] / v["peak"] if v["achieved"] else None
        v["avg_launch_ms"] = v["seconds"] / max(v["launches"], 1) * 1e3
    # the HSS build's own entry generator, beside the dense sweep and the matrix-free product
    g_s, g_pairs = kst["seconds_gen"], kst["gen_pairs"]
    if g_s > 0:
        g_tf = FLOP_PER_PAIR * g_pairs / g_s / 1e12
        entry["gen_jobs"] = {"seconds_per_build": g_s, "launches": kst["gen_launches"], "pairs": g_pairs,
                             "Gpairs_s": g_pairs / g_s / 1e9, "flop_per_pair": FLOP_PER_PAIR, "tflops": g_tf,
                             "frac_spec_peak": g_tf / FP64_VECTOR_PEAK_TF,
                             "frac_measured_peak": g_tf / entry["fp64_fma_probe_tflops"]}
    dom = max(kern, key=lambda k: kern[k]["seconds"])
    d = kern[dom]
    d_work = d["work"] / max(d["launches"], 1)
    traffic = MEASURED_TRAFFIC.get((dom, sk, ratio))
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
                   "id_tol": wl.id_tol, "theta_inc": wl.theta_inc,
                   "id": "cpqr" if sk == 0 else f"gaussian sketch, unknowns+{sk} rows",
                   "max_rank_ratio": ratio, "solve": args.solve},
        "hss_build_solve_s": ms * 1e-3,
        "hss": {"entries": entries, "pairs": st["pairs"], "levels": st["levels"],
                "compressed_levels": st["compressed_levels"], "root_size": st["root_size"],
                "max_rank": st["max_rank"],
                "seconds_build_wall": avg("seconds_total"),
                "seconds_generate": gen_s,
                "seconds_compress": avg("seconds_compress"),
                "seconds_cpqr": cq_s,
                "seconds_cpqr_fused": avg("seconds_cpqr_fused"),
                "cpqr_fused_launches": st["cpqr_fused_launches"],
                "cpqr_fused_bytes": st["cpqr_fused_bytes"],
                "seconds_factor": avg("seconds_factor"),
                "generation_Gentries_s": entries / gen_s / 1e9,
                "solve_ms_eager": solve_ms["eager"], "solve_ms_graph": solve_ms["graph"],
                "kernels_event_timed": kern,
                "cpqr_step": {"seconds": cq_s, "launches": launches,
                              "algorithmic_GBs": cq_gbs,
                              "traffic_per_launch": MEASURED_TRAFFIC.get(("k_cpqr_step_reg", sk, ratio))},
                "per_level": levels},
        "entry_generation": entry,
        # the kernel class with the largest launch time in the step; achieved =
        # its algorithmic work per launch / its average event-timed launch time
        "roofline": {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                     "frac": d["frac"], "traffic": traffic, "kernel": dom,
                     "kernels": d.get("kernels", [dom]), "launches": d["launches"],
                     ("algorithmic_flops_per_launch" if d["unit"] == "TFLOP/s" else "algorithmic_bytes_per_launch"):
                         d_work,
                     "avg_launch_ms": d["avg_launch_ms"]},
    }
    return out, wl


# FP64 operations per ordered pair of the shape-derivative pair kernel, from
# rocprofv3 --pmc SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 (FMA counted as 2),
# profiles/pmc_counters_fourier8192.txt
FLOP_PER_PAIR_ADJOINT = 729.6


def run_adjoint(args):
    """Shape gradient of the backscatter intensity J = |u_inf(-d)|^2 with respect
    to the 64 Fourier coefficients of r = 1 + sum_{j<=32} (a_j cos jt + b_j sin jt)
    (coefficients ~ N(0, 0.01^2), N = 8192, k0 = 40, n = 1.5): a step is the
    forward solve (boundary samples, geometry, HSS build, solve, far field) and
    the backward pass (far-field weights, transposed HSS solve, pair-derivative
    contraction, chain rule to the coefficients), through the autograd Function."""
    import numpy as np
    import torch
    import scatterers as sc
    import paper_2607_00790_amd as bm

    wl = sc.fourier_workload()
    crv = wl.curves[0]
    c0 = torch.from_numpy(np.concatenate([crv.a, crv.b])).cuda()
    md, n = wl.media, wl.n
    opts = dict(leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=args.id_tol, sketch=args.sketch,
                max_rank_ratio=args.max_rank_ratio)
    stream = torch.cuda.current_stream()

    def step():
        coef = c0.clone().requires_grad_(True)
        J = bm.backscatter_intensity(coef, n, md.k0, md.k1, md.eps0, md.eps1, theta_inc=wl.theta_inc, **opts)
        J.backward()
        return coef.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    # the phases of one step, each timed alone with events on the same stream
    xyd = bm.bm_fourier_curve(c0, n)
    g = bm.bm_geom_create([n], xyd)
    p = bm.bm_problem_create(g, md.k0, md.k1, md.eps0, md.eps1)
    obs = wl.theta_inc + np.pi

    def timed(fn, reps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, r

    build_ms, h = timed(lambda: bm.bm_hss_build(p, **opts), 2)
    hst = bm.bm_hss_stats(h)
    used = dict(opts, sketch=hst["sketch"], max_rank_ratio=hst["max_rank_ratio"])
    rhs = bm.bm_rhs_plane_wave(p, wl.theta_inc)
    solve_ms, phi = timed(lambda: bm.bm_hss_solve(h, rhs), 3)
    gw = bm.bm_far_field_weights(p, obs)
    tsolve_ms, lam = timed(lambda: bm.bm_hss_solve_transpose(h, gw), 3)
    g6 = torch.empty((6, n), dtype=torch.float64, device="cuda")
    deriv_ms, _ = timed(lambda: bm.bm_shape_derivative(p, phi, lam, wl.theta_inc, obs, out=g6), 5)
    pairs = n * (n - 1)
    out = {
        "metric": "shape gradients/s of the backscatter intensity (64 Fourier coefficients, N=8192)",
        "value": 1e3 / ms,
        "unit": "gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"shape gradient, {wl.name}, J = |u_inf(-d)|^2", "n_nodes": n,
                   "coefficients": 64, "k0": md.k0, "k1": md.k1, "theta_inc": wl.theta_inc, **used},
        "phases_ms": {"hss_build": build_ms, "hss_solve": solve_ms, "hss_solve_transpose": tsolve_ms,
                      "shape_derivative": deriv_ms},
    }
    roof = {"bound": "alu", "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s", "traffic": None,
            "kernel": "k_shape_pairs", "pairs": pairs, "avg_launch_ms": deriv_ms,
            "note": "launch time of bm_shape_derivative (zeroing, pair kernel, node kernel)"}
    if FLOP_PER_PAIR_ADJOINT:
        tf = FLOP_PER_PAIR_ADJOINT * pairs / (deriv_ms * 1e-3) / 1e12
        roof.update(achieved=tf, frac=tf / FP64_VECTOR_PEAK_TF, flop_per_pair=FLOP_PER_PAIR_ADJOINT)
    else:
        roof.update(achieved=None, frac=None, flop_per_pair=None,
                    pairs_per_s=pairs / (deriv_ms * 1e-3))
    out["roofline"] = roof
    return out, wl


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["hss", "dense", "matvec", "batch", "adjoint", "large"], default="hss")
    ap.add_argument("--id-tol", type=float, default=1e-12, help="adjoint mode: HSS ID tolerance")
    ap.add_argument("--per-curve", type=int, default=16384, help="large mode: nodes per star")
    ap.add_argument("--max-rank-ratio", type=float, default=None,
                    help="HSS: a body stops compressing once a level keeps more than this fraction of its "
                         "unknowns (0: never; -1: the library's tuned value; default: -1 in hss, adjoint and "
                         "batch modes, 0.8 in large mode, 0 otherwise)")
    ap.add_argument("--batch", type=int, default=256, help="batch mode: number of stars")
    ap.add_argument("--proxy-adapt", type=int, choices=[0, 1], default=1,
                    help="batch mode: proxy points per circle max(64, ceil(2 k R_p) + 32)")
    ap.add_argument("--sketch", type=int, default=None,
                    help="HSS: p > 0 runs the ID on a Gaussian sketch with unknowns + p rows (0: plain "
                         "CPQR; -1: the library's tuned value; default: -1 in hss, adjoint and batch modes, "
                         "128 in large mode, 0 otherwise)")
    ap.add_argument("--solve", choices=["graph", "eager"], default="graph",
                    help="hss mode: the step's solve replays the graph the build records, or runs eagerly")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the run, copy this many MiB device-to-device once (a plain copy "
                         "kernel of known size, to scale HBM traffic counters)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_run()), flush=True)
        return 0
    if args.max_rank_ratio is None:
        args.max_rank_ratio = {"hss": -1.0, "adjoint": -1.0, "batch": -1.0, "large": 0.8}.get(args.mode, 0.0)
    if args.sketch is None:
        args.sketch = {"hss": -1, "adjoint": -1, "batch": -1, "large": 128}.get(args.mode, 0)
    if args.gpus != 1:
        print("the library runs on one GPU (it has no multi-GPU path); --gpus must be 1", file=sys.stderr)
        return 2
    if args.calib_copy_mib > 0:
        import torch
        src = torch.ones(args.calib_copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out, wl = {"hss": run_hss, "dense": run_dense, "matvec": run_matvec, "batch": run_batch,
               "adjoint": run_adjoint, "large": run_large}[args.mode](args)
    if not args.no_cpu_baseline and args.mode in ("hss", "dense", "matvec"):
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
