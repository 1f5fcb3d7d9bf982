"""Autotuner of the HSS factorisation parameters for the GPU it runs on.

    python -m paper_2607_00790_amd.autotune [--out FILE] [--steps 5] [--repeats 3]

For every candidate pair (Gauss-Jordan base block 32 / 64 / 128, rocBLAS
threshold 1e8 / 4e8 / 2e9 flops) it runs the benchmark's HSS build+solve (the
N = 16384 star of bench.py's default mode) in a child process with the
candidate in BMHSS_TUNE_INV_BASE / BMHSS_TUNE_BLAS_FLOPS, keeps the median step
time over the repeats, and writes a tuned_params.h that makes the fastest pair
the compiled default (with every measurement in its comments).  Copy the file
to csrc/tuned_params.h and rebuild to adopt it.
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


def measure(base: int, flops: float, steps: int) -> float:
    env = dict(os.environ, BMHSS_TUNE_INV_BASE=str(base), BMHSS_TUNE_BLAS_FLOPS=repr(flops))
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", str(steps), "--warmup", "2",
           "--no-cpu-baseline"]
    out = subprocess.run(cmd, env=env, capture_output=True, text=True, check=True).stdout
    line = [l for l in out.splitlines() if l.startswith("{")][-1]
    return json.loads(line)["ms_per_step"]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned_params.h"))
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()
    rows = []
    for base, flops in itertools.product(BASES, FLOPS):
        ms = [measure(base, flops, args.steps) for _ in range(args.repeats)]
        med = statistics.median(ms)
        rows.append((med, base, flops, ms))
        print(f"autotune: base {base:3d}, blas flops {flops:.0e}: median {med:.3f} ms "
              f"({', '.join(f'{m:.3f}' for m in ms)})", flush=True)
    best = min(rows)
    table = "\n".join(f"//   base {b:3d}  blas {f:.0e}  median {m:8.3f} ms" for m, b, f, _ in rows)
    text = f"""// Tuned parameters of the HSS factorisation on gfx950, written by
// paper_2607_00790_amd/autotune.py: median HSS build+solve step of the benchmark
// (star r = 1 + 0.3 cos 5t, N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy points,
// tol 1e-10; bench.py --steps {args.steps} --warmup 2, {args.repeats} runs each):
{table}
#pragma once

namespace bm {{
namespace tuned {{

// Largest block inverted directly by Gauss-Jordan (32, 64 or 128); larger
// blocks go through the 2 x 2 Schur-complement recursion.
constexpr int kInvBase = {best[1]};
// Products of at least this many real flops go to rocBLAS ZGEMM.
constexpr double kBlasFlops = {best[2]:.0e};

}}  // namespace tuned
}}  // namespace bm
"""
    with open(args.out, "w") as f:
        f.write(text)
    print(f"autotune: best base {best[1]}, blas flops {best[2]:.0e} ({best[0]:.3f} ms) -> {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
