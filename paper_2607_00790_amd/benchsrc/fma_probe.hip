// Benchmark-only diagnostic, built into libbmhss_probe.so (not the product
// library): the FP64 FMA rate this device actually sustains, the reference the
// entry kernels' FP64 fraction is also reported against (the published peak
// assumes the full clock, which a device may not hold).
//
// fma_probe(out, blocks, iters, stream): blocks x 256 threads, each running
// 16 independent chains a <- a x + y of `iters` fused multiply-adds (2 * 16 *
// iters real flops per thread) from a_c = 1e-3 (c + 1), x = 1 + 1e-9 (t mod
// 1024), y = 1e-12 (t mod 256), writing the sum of its chains to out[t]
// (device, blocks * 256 doubles).  Returns the HIP error code of the launch.
#include <hip/hip_runtime.h>

#include <cstdint>

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

extern "C" int fma_probe(double* out, int64_t blocks, int64_t iters, hipStream_t stream) {
    if (!out || blocks < 1 || blocks > (int64_t{1} << 24) - 1 || iters < 1) return static_cast<int>(hipErrorInvalidValue);
    hipLaunchKernelGGL(k_fma_probe, dim3(static_cast<unsigned>(blocks)), dim3(kProbeThreads), 0, stream, out, iters);
    return static_cast<int>(hipGetLastError());
}
