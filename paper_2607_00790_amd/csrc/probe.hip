// Device diagnostics: the FP64 FMA rate this device actually sustains, the
// reference the entry kernels' FP64 fraction is also reported against (the
// published peak assumes the full clock, which a device may not hold).
#include "internal.hpp"

namespace bm {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 16;   // independent FMA chains per thread: enough to hide the FMA latency

__global__ void __launch_bounds__(kProbeThreads)
k_fma_probe(double* __restrict__ out, int64_t iters) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    const double x = 1.0 + 1e-9 * static_cast<double>(t & 1023);
    const double y = 1e-12 * static_cast<double>(threadIdx.x);
    double a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = 1e-3 * static_cast<double>(c + 1);
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    out[t] = s;
}

}  // namespace

}  // namespace bm

extern "C" int bm_fp64_fma_probe(double* out, int64_t blocks, int64_t iters, hipStream_t stream) {
    bm::clear_error();
    if (!out) return bm::fail(BM_EINVAL, "bm_fp64_fma_probe: null argument");
    if (blocks < 1 || blocks > (int64_t{1} << 24) - 1 || iters < 1)
        return bm::fail(BM_EINVAL, "bm_fp64_fma_probe: need 1 <= blocks < 2^24, iters >= 1");
    hipLaunchKernelGGL(bm::k_fma_probe, dim3(static_cast<unsigned>(blocks)), dim3(bm::kProbeThreads), 0, stream,
                       out, iters);
    BM_HIP(hipGetLastError());
    return BM_OK;
}
