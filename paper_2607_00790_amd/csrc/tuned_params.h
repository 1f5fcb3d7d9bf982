// Tuned parameters of the HSS build on gfx950, written by
// paper_2607_00790_amd/autotune.py on the benchmark workload (star
// r = 1 + 0.3 cos 5t, N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy points,
// tol 1e-10).
// Stage 1, build options: median of 6 build+solve runs per pair; the
// residual |A x - b| / |b| may not exceed that of plain CPQR on every level:
//   sketch  0  ratio 0.00  median   21.903 ms  residual 2.73e-07  root 935
//   sketch  0  ratio 0.55  median   20.040 ms  residual 1.98e-09  root 2327
//   sketch  0  ratio 0.60  median   17.631 ms  residual 7.03e-09  root 1550
//   sketch  0  ratio 0.65  median   17.568 ms  residual 7.03e-09  root 1550
//   sketch  0  ratio 0.70  median   19.178 ms  residual 3.16e-08  root 1132
//   sketch  0  ratio 0.80  median   21.883 ms  residual 2.73e-07  root 935
//   sketch  8  ratio 0.00  median   16.613 ms  residual 2.44e-07  root 916
//   sketch  8  ratio 0.55  median   15.370 ms  residual 5.69e-09  root 2289
//   sketch  8  ratio 0.60  median   12.907 ms  residual 2.34e-08  root 1526
//   sketch  8  ratio 0.65  median   12.960 ms  residual 2.34e-08  root 1526
//   sketch  8  ratio 0.70  median   14.093 ms  residual 6.47e-08  root 1120
//   sketch  8  ratio 0.80  median   16.568 ms  residual 2.44e-07  root 916
//   sketch 16  ratio 0.00  median   16.520 ms  residual 5.29e-07  root 918  (residual above plain CPQR: excluded)
//   sketch 16  ratio 0.55  median   15.351 ms  residual 6.13e-09  root 2292
//   sketch 16  ratio 0.60  median   12.999 ms  residual 2.54e-08  root 1531
//   sketch 16  ratio 0.65  median   12.921 ms  residual 2.54e-08  root 1531
//   sketch 16  ratio 0.70  median   14.127 ms  residual 6.48e-08  root 1118
//   sketch 16  ratio 0.80  median   16.538 ms  residual 5.29e-07  root 918  (residual above plain CPQR: excluded)
//   sketch 32  ratio 0.00  median   16.823 ms  residual 3.27e-07  root 919  (residual above plain CPQR: excluded)
//   sketch 32  ratio 0.55  median   15.643 ms  residual 4.03e-09  root 2297
//   sketch 32  ratio 0.60  median   13.206 ms  residual 2.72e-08  root 1526
//   sketch 32  ratio 0.65  median   13.212 ms  residual 2.72e-08  root 1526
//   sketch 32  ratio 0.70  median   14.412 ms  residual 5.87e-08  root 1122
//   sketch 32  ratio 0.80  median   17.092 ms  residual 3.27e-07  root 919  (residual above plain CPQR: excluded)
// Stage 2, with those options: median bench.py step (--steps 5 --warmup 2,
// 2 runs each):
//   base  32  blas 1e+08  median   14.339 ms
//   base  32  blas 4e+08  median   14.387 ms
//   base  32  blas 2e+09  median   14.715 ms
//   base  64  blas 1e+08  median   13.035 ms
//   base  64  blas 4e+08  median   13.042 ms
//   base  64  blas 2e+09  median   13.336 ms
//   base 128  blas 1e+08  median   14.359 ms
//   base 128  blas 4e+08  median   14.368 ms
//   base 128  blas 2e+09  median   14.726 ms
#pragma once

namespace bm {
namespace tuned {

// Largest block inverted directly by Gauss-Jordan (32, 64 or 128); larger
// blocks go through the 2 x 2 Schur-complement recursion.
constexpr int kInvBase = 64;
// Products of at least this many real flops go to rocBLAS ZGEMM.
constexpr double kBlasFlops = 1e+08;
// HSS build options selected by bm_hss_opts value -1 (sketch rows beyond the
// unknowns; level rank ratio above which a body stops compressing).
constexpr long kSketchRows = 8;
constexpr double kStopRankRatio = 0.6;

}  // namespace tuned
}  // namespace bm
