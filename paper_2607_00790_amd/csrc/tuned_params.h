// Tuned parameters of the HSS factorisation on gfx950, written by
// paper_2607_00790_amd/autotune.py: median HSS build+solve step of the benchmark
// (star r = 1 + 0.3 cos 5t, N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy points,
// tol 1e-10; bench.py --steps 5 --warmup 2, 3 runs each):
//   base  32  blas 1e+08  median   26.560 ms
//   base  32  blas 4e+08  median   26.542 ms
//   base  32  blas 2e+09  median   26.767 ms
//   base  64  blas 1e+08  median   25.218 ms
//   base  64  blas 4e+08  median   25.739 ms
//   base  64  blas 2e+09  median   25.445 ms
//   base 128  blas 1e+08  median   26.320 ms
//   base 128  blas 4e+08  median   26.132 ms
//   base 128  blas 2e+09  median   27.076 ms
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
