"""Autotuner of the HSS build for the GPU it runs on.

    python -m paper_2607_00790_amd.autotune [--out FILE] [--steps 5] [--repeats 2]

Stage 1 (one child process) picks the build options that bm_hss_opts value -1
selects: the sketch size p (0 = plain CPQR) and the rank ratio above which a
body stops compressing (0 = never).  For every pair it builds and solves the
benchmark workload (the N = 16384 star of bench.py's default mode) several
times, keeps the median time, and checks the relative residual |A x - b|/|b|
through the matrix-free product: a candidate is admissible only if its
residual is no larger than that of plain CPQR on every level.  The fastest
admissible pair wins.

Stage 2 then times, with the chosen options, every pair (Gauss-Jordan base
block 32 / 64 / 128, rocBLAS threshold 1e8 / 4e8 / 2e9 flops): a child
process of this module per candidate (the library reads BMHSS_TUNE_INV_BASE /
BMHSS_TUNE_BLAS_FLOPS once per process) runs warm-up steps and then times
`steps` build + right-hand side + solve steps with HIP events, and the median
step time over the repeats is kept.

The result is a tuned_params.h that makes the winners the compiled defaults,
with every measurement in its comments.  Copy it to csrc/tuned_params.h and
rebuild to adopt it.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

BASES = (32, 64, 128)
FLOPS = (1e8, 4e8, 2e9)
SKETCHES = (0, 8, 16, 32)
RATIOS = (0.0, 0.55, 0.6, 0.65, 0.7, 0.8)


def build_options_sweep(builds: int) -> list:
    """Stage 1, run in a child process: (median ms, sketch, ratio, residual, root size) per pair."""
    import time
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import scatterers as sc
    import paper_2607_00790_amd as bm
    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    g = bm.bm_geom_create(sizes, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    b = bm.bm_rhs_plane_wave(p, wl.theta_inc)
    rows = []
    for sk, ratio in itertools.product(SKETCHES, RATIOS):
        ts = []
        for _ in range(builds):
            torch.cuda.synchronize()
            t = time.perf_counter()
            h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                                id_tol=wl.id_tol, sketch=sk, max_rank_ratio=ratio)
            x = bm.bm_hss_solve(h, b)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
            root = bm.bm_hss_stats(h)["root_size"]
            del h
        res = (torch.linalg.vector_norm(bm.bm_matvec(p, x) - b) / torch.linalg.vector_norm(b)).item()
        med = statistics.median(ts)
        rows.append((med, sk, ratio, res, root))
        print(f"autotune: sketch {sk:2d}, stop ratio {ratio:.2f}: median {med:.3f} ms, residual {res:.2e}, "
              f"root {root}", file=sys.stderr, flush=True)
    return rows


def stage1(builds: int) -> list:
    """Stage 1 in a child process, so that this process never initialises the GPU."""
    out = subprocess.run([sys.executable, "-m", "paper_2607_00790_amd.autotune", "--stage1-child",
                          "--builds", str(builds)], cwd=ROOT, stdout=subprocess.PIPE, text=True,
                         check=True).stdout
    return [tuple(r) for r in json.loads([l for l in out.splitlines() if l.startswith("[")][-1])]


def time_steps(steps: int, sketch: int, ratio: float) -> float:
    """Stage 2, run in a child process: ms per build + right-hand side + solve
    step on the benchmark workload (2 warm-up steps, then `steps` timed with
    HIP events on the current stream)."""
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import scatterers as sc
    import paper_2607_00790_amd as bm
    wl = sc.star_workload()
    xyd, sizes = wl.xyd()
    g = bm.bm_geom_create(sizes, torch.from_numpy(xyd).cuda())
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    b = torch.empty(2 * wl.n, dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)

    def step():
        h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                            id_tol=wl.id_tol, sketch=sketch, max_rank_ratio=ratio)
        bm.bm_rhs_plane_wave(p, wl.theta_inc, out=b)
        bm.bm_hss_solve(h, b, out=x)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure(base: int, flops: float, steps: int, sketch: int, ratio: float) -> float:
    env = dict(os.environ, BMHSS_TUNE_INV_BASE=str(base), BMHSS_TUNE_BLAS_FLOPS=repr(flops))
    cmd = [sys.executable, "-m", "paper_2607_00790_amd.autotune", "--stage2-child", "--steps", str(steps),
           "--sketch", str(sketch), "--ratio", repr(ratio)]
    out = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, check=True).stdout
    return json.loads([l for l in out.splitlines() if l.strip()][-1])


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned_params.h"))
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--builds", type=int, default=6, help="stage 1: builds per option pair")
    ap.add_argument("--stage1-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--stage2-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--sketch", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--ratio", type=float, default=0.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.stage1_child:
        print(json.dumps(build_options_sweep(args.builds)), flush=True)
        return 0
    if args.stage2_child:
        print(json.dumps(time_steps(args.steps, args.sketch, args.ratio)), flush=True)
        return 0
    opts = stage1(args.builds)
    ref = [r for r in opts if r[1] == 0 and r[2] == 0.0][0]
    ok = [r for r in opts if r[3] <= ref[3]]
    best_o = min(ok)
    print(f"autotune: options sketch {best_o[1]}, stop ratio {best_o[2]} ({best_o[0]:.3f} ms, residual "
          f"{best_o[3]:.2e} <= {ref[3]:.2e})", flush=True)
    rows = []
    for base, flops in itertools.product(BASES, FLOPS):
        ms = [measure(base, flops, args.steps, best_o[1], best_o[2]) for _ in range(args.repeats)]
        med = statistics.median(ms)
        rows.append((med, base, flops, ms))
        print(f"autotune: base {base:3d}, blas flops {flops:.0e}: median {med:.3f} ms "
              f"({', '.join(f'{m:.3f}' for m in ms)})", flush=True)
    best = min(rows)
    t_opts = "\n".join(f"//   sketch {s:2d}  ratio {r:.2f}  median {m:8.3f} ms  residual {e:.2e}  root {q}"
                       f"{'' if e <= ref[3] else '  (residual above plain CPQR: excluded)'}"
                       for m, s, r, e, q in opts)
    t_inv = "\n".join(f"//   base {b:3d}  blas {f:.0e}  median {m:8.3f} ms" for m, b, f, _ in rows)
    text = f"""// Tuned parameters of the HSS build on gfx950, written by
// paper_2607_00790_amd/autotune.py on the benchmark workload (star
// r = 1 + 0.3 cos 5t, N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy points,
// tol 1e-10).
// Stage 1, build options: median of {args.builds} build+solve runs per pair; the
// residual |A x - b| / |b| may not exceed that of plain CPQR on every level:
{t_opts}
// Stage 2, with those options: median step time (build + right-hand side +
// solve, {args.steps} steps after 2 warm-up steps, {args.repeats} runs each):
{t_inv}
#pragma once

namespace bm {{
namespace tuned {{

// Largest block inverted directly by Gauss-Jordan (32, 64 or 128); larger
// blocks go through the 2 x 2 Schur-complement recursion.
constexpr int kInvBase = {best[1]};
// Products of at least this many real flops go to rocBLAS ZGEMM.
constexpr double kBlasFlops = {best[2]:.0e};
// HSS build options selected by bm_hss_opts value -1 (sketch rows beyond the
// unknowns; level rank ratio above which a body stops compressing).
constexpr long kSketchRows = {best_o[1]};
constexpr double kStopRankRatio = {best_o[2]};

}}  // namespace tuned
}}  // namespace bm
"""
    with open(args.out, "w") as f:
        f.write(text)
    print(f"autotune: best base {best[1]}, blas flops {best[2]:.0e} ({best[0]:.3f} ms) -> {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
