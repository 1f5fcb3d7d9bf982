// Entry-generation kernels for the WSBM Nystrom matrix (paper Eq. (3)/(5)),
// plus the boundary discretisation, plane-wave right-hand side, matrix-free
// product and far field.
//
// Layout choices for gfx950 (64-wide wavefronts):
//  * lanes run along the SOURCE index j, so a wavefront writes 64 consecutive
//    2x2 blocks = two contiguous 2 KiB row segments (rows 2i and 2i+1) of the
//    row-major complex matrix: fully coalesced 16-byte stores;
//  * a workgroup covers one TARGET i and kThreads consecutive sources; the
//    target's node data are wave-uniform and come through the scalar cache,
//    each lane loads its own source node.  No LDS staging is needed: the only
//    shared operand is the uniform target.
//  * one pair per thread and no loop: the ~120 FP64 polynomial coefficients of
//    the Bessel functions stay scalar operands materialised at their use
//    (a loop lets the compiler hoist them into vector registers, which drops
//    the occupancy to one wave per SIMD).
#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "internal.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;   // 4 wavefronts

__global__ void __launch_bounds__(kThreads)
k_geometry(const double* __restrict__ xyd, const int64_t* __restrict__ offsets, int ncurves,
           int64_t n, double* __restrict__ soa, int32_t* __restrict__ curve) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= n) return;
    int c = 0;
    while (c + 1 < ncurves && offsets[c + 1] <= j) ++c;
    const double nc = static_cast<double>(offsets[c + 1] - offsets[c]);
    const double dx = xyd[2 * n + j], dy = xyd[3 * n + j];
    const double ddx = xyd[4 * n + j], ddy = xyd[5 * n + j];
    const double s = sqrt(dx * dx + dy * dy);
    const double is = 1.0 / s;
    soa[j] = xyd[j];
    soa[n + j] = xyd[n + j];
    soa[2 * n + j] = dy * is;
    soa[3 * n + j] = -dx * is;
    soa[4 * n + j] = (2.0 * kPi / nc) * s;
    soa[5 * n + j] = (dx * ddy - dy * ddx) * is * is * is;
    curve[j] = c;
}

__device__ __forceinline__ void store_block(double* __restrict__ out, int64_t ld, int64_t row,
                                            int64_t col, const Block& b) {
    // complex (row, col) lives at doubles 2*(row*ld + col)
    double2* r0 = reinterpret_cast<double2*>(out) + (2 * row) * ld + 2 * col;
    double2* r1 = r0 + ld;
    r0[0] = make_double2(b.v[0], b.v[1]);
    r0[1] = make_double2(b.v[2], b.v[3]);
    r1[0] = make_double2(b.v[4], b.v[5]);
    r1[1] = make_double2(b.v[6], b.v[7]);
}

// Off-diagonal pair written row by row: row 2i needs only the interior (k1)
// kernels, so it is stored before the exterior (k0) Bessel functions are
// evaluated and its write overlaps the rest of the arithmetic.
__device__ __forceinline__ void emit_pair(double* __restrict__ out, int64_t ld, int64_t row,
                                          int64_t col, double tx, double ty, double tnx, double tny,
                                          double sx, double sy, double snx, double sny, double sw,
                                          const Media& m, bool interior) {
    const PairGeom g = pair_geom(tx, ty, tnx, tny, sx, sy, snx, sny);
    const Hankel01 h1 = pair_interior(g, m, interior);
    double o[4];
    pair_row0(g, h1, sw, m, o);
    double2* r0 = reinterpret_cast<double2*>(out) + (2 * row) * ld + 2 * col;
    r0[0] = make_double2(o[0], o[1]);
    r0[1] = make_double2(o[2], o[3]);
    pair_row1(g, interior_terms(h1, m), sw, m, o);
    double2* r1 = reinterpret_cast<double2*>(out) + (2 * row + 1) * ld + 2 * col;
    r1[0] = make_double2(o[0], o[1]);
    r1[1] = make_double2(o[2], o[3]);
}

__device__ __forceinline__ int body_of(const NodeView& v, int64_t i) { return v.body ? v.body[i] : 0; }

// The media of a body with the coefficient table taken from a kernel argument.
// Every Media holds the same table pointer, but one read from device memory
// leaves the compiler with a generic pointer, and the coefficient loads through
// it then ran at half speed on some devices (the generate-and-reduce product:
// 8.1 ms against 3.8 ms with the pointer as a kernel argument).
__device__ __forceinline__ Media with_table(Media m, const BesselTable* __restrict__ tab) {
    m.tab = tab;
    return m;
}

// Zero 2x2 block (a pair in two different bodies).
__device__ __forceinline__ void store_zero(double* __restrict__ out, int64_t ld, int64_t row, int64_t col) {
    double2* r0 = reinterpret_cast<double2*>(out) + (2 * row) * ld + 2 * col;
    double2* r1 = r0 + ld;
    const double2 z = make_double2(0.0, 0.0);
    r0[0] = z;
    r0[1] = z;
    r1[0] = z;
    r1[1] = z;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// Block-wide sum of NV values per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV]) {
    __shared__ double red[NV][kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0;
            for (int w = 0; w < kThreads / 64; ++w) s += red[q][w];
            acc[q] = s;
        }
    }
}

// Full matrix: workgroup b covers target i = b / ntj and sources
// [jt*kThreads, (jt+1)*kThreads), jt = b % ntj.
__global__ void __launch_bounds__(kThreads, kPairWavesPerSimd)
k_dense(NodeView v, int64_t n, int64_t ntj, const Media* __restrict__ media, double* __restrict__ A,
        int64_t ld, const BesselTable* __restrict__ tab) {
    const int64_t i = blockIdx.x / ntj;
    const int64_t j = (blockIdx.x % ntj) * kThreads + threadIdx.x;
    if (j >= n) return;
    const int bi = body_of(v, i);   // wave-uniform: the media come through the scalar cache
    const Media m = with_table(media[bi], tab);
    if (body_of(v, j) != bi) {
        store_zero(A, ld, i, j);
    } else if (i == j) {
        store_block(A, ld, i, j, diag_block(v.w[j], v.kappa[j], m));
    } else {
        emit_pair(A, ld, i, j, v.x[i], v.y[i], v.nx[i], v.ny[i], v.x[j], v.y[j], v.nx[j], v.ny[j],
                  v.w[j], m, v.curve[i] == v.curve[j]);
    }
}

__global__ void __launch_bounds__(kThreads)
k_rhs_plane_wave(NodeView v, int64_t n, const Media* __restrict__ media, double dx, double dy,
                 double2* __restrict__ rhs) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const Media m = media[body_of(v, i)];
    double s, c;
    sincos(m.k0 * (dx * v.x[i] + dy * v.y[i]), &s, &c);
    // -u_in - alpha du_in/dn = -u_in (1 + (i/k0)(i k0 d.n)) = -u_in (1 - d.n)
    const double f = -(1.0 - (dx * v.nx[i] + dy * v.ny[i]));
    rhs[2 * i] = make_double2(0.0, 0.0);
    rhs[2 * i + 1] = make_double2(f * c, f * s);
}

// Right-hand side of Eq. (3) for a given incident field: rhs[2i] = 0,
// rhs[2i+1] = -u_in(x_i) - alpha du_in/dn(x_i), alpha = i/k0 of the node's body.
__global__ void __launch_bounds__(kThreads)
k_rhs_incident(NodeView v, int64_t n, const Media* __restrict__ media, const double2* __restrict__ uin,
               const double2* __restrict__ dn_uin, double2* __restrict__ rhs) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const double ik0 = media[body_of(v, i)].ik0;
    const double2 u = uin[i], du = dn_uin[i];
    // alpha du = (i/k0)(du.x + i du.y) = (-du.y + i du.x)/k0
    rhs[2 * i] = make_double2(0.0, 0.0);
    rhs[2 * i + 1] = make_double2(-u.x + ik0 * du.y, -u.y - ik0 * du.x);
}

// y = A x, stage 1: workgroup b covers target i = b / ntj and one tile of
// kMvSources * kThreads sources (each thread takes kMvSources of them, kThreads
// apart, so that the block reduction is paid once per kMvSources pairs); it
// writes the tile's partial sums of rows 2i, 2i+1 to part[b] (4 doubles).
constexpr int kMvSources = 8;
constexpr int kMvWavesPerSimd = 4;

__global__ void __launch_bounds__(kThreads, kMvWavesPerSimd)
k_matvec_partial(NodeView v, const int64_t* __restrict__ body_lo, int64_t ntj, int64_t i0,
                 const Media* __restrict__ media, const double2* __restrict__ x,
                 double4* __restrict__ part, const BesselTable* __restrict__ tab) {
    // tiles run over the target's own body only (the system is block diagonal);
    // the launch covers targets i0, i0 + 1, ...
    const int64_t i = i0 + blockIdx.x / ntj;
    const int bi = body_of(v, i);
    const int64_t jend = body_lo[bi + 1];
    const int64_t j0 = body_lo[bi] + (blockIdx.x % ntj) * (kThreads * kMvSources) + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const Media m = with_table(media[bi], tab);
    const double tx = v.x[i], ty = v.y[i], tnx = v.nx[i], tny = v.ny[i];
    const int32_t ci = v.curve[i];
#pragma unroll 1
    for (int q = 0; q < kMvSources; ++q) {
        const int64_t j = j0 + q * kThreads;
        if (j >= jend) break;
        Block b;
        if (i == j) {
            b = diag_block(v.w[j], v.kappa[j], m);
        } else {
            b = pair_block(tx, ty, tnx, tny, v.x[j], v.y[j], v.nx[j], v.ny[j], v.w[j], m, ci == v.curve[j]);
        }
        const double2 xu = x[2 * j], xq = x[2 * j + 1];
        // row 2i: A00 xu + A01 xq ; row 2i+1: A10 xu + A11 xq
        acc[0] += b.v[0] * xu.x - b.v[1] * xu.y + b.v[2] * xq.x - b.v[3] * xq.y;
        acc[1] += b.v[0] * xu.y + b.v[1] * xu.x + b.v[2] * xq.y + b.v[3] * xq.x;
        acc[2] += b.v[4] * xu.x - b.v[5] * xu.y + b.v[6] * xq.x - b.v[7] * xq.y;
        acc[3] += b.v[4] * xu.y + b.v[5] * xu.x + b.v[6] * xq.y + b.v[7] * xq.x;
    }
    block_sum<4>(acc);
    if (threadIdx.x == 0) part[i * ntj + blockIdx.x % ntj] = make_double4(acc[0], acc[1], acc[2], acc[3]);
}

// y = A x, stage 2: sum the ntj partials of each target in a fixed order.
__global__ void __launch_bounds__(kThreads)
k_matvec_reduce(int64_t n, int64_t ntj, const double4* __restrict__ part, double2* __restrict__ y) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int64_t t = 0; t < ntj; ++t) {
        const double4 p = part[i * ntj + t];
        s.x += p.x; s.y += p.y; s.z += p.z; s.w += p.w;
    }
    y[2 * i] = make_double2(s.x, s.y);
    y[2 * i + 1] = make_double2(s.z, s.w);
}

// Far field: one workgroup per (observation angle, body); a body's far field
// sums over its own nodes with its own exterior wavenumber.
__global__ void __launch_bounds__(kThreads)
k_far_field(NodeView v, const int64_t* __restrict__ body_lo, const Media* __restrict__ media,
            const double2* __restrict__ phi, const double* __restrict__ angles, int64_t nang,
            double2* __restrict__ uinf) {
    const int64_t a = blockIdx.x;
    const int b = blockIdx.y;
    const Media m = media[b];
    double sa, ca;
    sincos(angles[a], &sa, &ca);
    double acc[2] = {0.0, 0.0};
    for (int64_t j = body_lo[b] + threadIdx.x; j < body_lo[b + 1]; j += kThreads) {
        const double2 u = phi[2 * j], q = phi[2 * j + 1];
        const double xn = ca * v.nx[j] + sa * v.ny[j];
        // density = -i k0 (xhat.n) u - eps0 q
        const double d_re = m.k0 * xn * u.y - m.eps0 * q.x;
        const double d_im = -m.k0 * xn * u.x - m.eps0 * q.y;
        double s, c;
        sincos(-m.k0 * (ca * v.x[j] + sa * v.y[j]), &s, &c);
        const double w = v.w[j];
        acc[0] += w * (d_re * c - d_im * s);
        acc[1] += w * (d_re * s + d_im * c);
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        // e^{i pi/4} / sqrt(8 pi k0)
        const double f = 1.0 / sqrt(8.0 * kPi * m.k0);
        const double cr = f * kSqrtHalf, ci = f * kSqrtHalf;
        uinf[b * nang + a] = make_double2(cr * acc[0] - ci * acc[1], cr * acc[1] + ci * acc[0]);
    }
}

inline unsigned blocks_for(int64_t n, int per) {
    return static_cast<unsigned>((n + per - 1) / per);
}

}  // namespace

hipError_t launch_geometry(const double* xyd, const int64_t* offsets, int ncurves, int64_t n,
                           double* soa, int32_t* curve, hipStream_t s) {
    hipLaunchKernelGGL(k_geometry, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, xyd,
                       offsets, ncurves, n, soa, curve);
    return hipGetLastError();
}

hipError_t launch_dense(const NodeView& v, int64_t n, const Media* m, const BesselTable* tab, double* A,
                        int64_t ld, hipStream_t s) {
    const int64_t ntj = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_dense, dim3(static_cast<unsigned>(n * ntj)), dim3(kThreads), 0, s, v, n,
                       ntj, m, A, ld, tab);
    return hipGetLastError();
}

hipError_t launch_rhs_plane_wave(const NodeView& v, int64_t n, const Media* m, double angle,
                                 double* rhs, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs_plane_wave, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, v, n,
                       m, std::cos(angle), std::sin(angle), reinterpret_cast<double2*>(rhs));
    return hipGetLastError();
}

hipError_t launch_rhs_incident(const NodeView& v, int64_t n, const Media* m, const double* uin, const double* dn_uin,
                               double* rhs, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs_incident, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, v, n, m,
                       reinterpret_cast<const double2*>(uin), reinterpret_cast<const double2*>(dn_uin),
                       reinterpret_cast<double2*>(rhs));
    return hipGetLastError();
}

hipError_t launch_matvec(const NodeView& v, int64_t n, int64_t max_body, const int64_t* body_lo,
                         const Media* m, const BesselTable* tab, const double* x, double* y, double* work,
                         hipStream_t s) {
    const int64_t ntj = (max_body + kThreads * kMvSources - 1) / (kThreads * kMvSources);
    double4* part = reinterpret_cast<double4*>(work);
    // at most 2^24 - 1 workgroups (2^32 - 1 work-items) per launch
    const int64_t chunk = std::max<int64_t>(1, (int64_t{0xFFFFFFFF} / kThreads) / ntj);
    for (int64_t i0 = 0; i0 < n; i0 += chunk) {
        const int64_t nt = std::min(chunk, n - i0);
        hipLaunchKernelGGL(k_matvec_partial, dim3(static_cast<unsigned>(nt * ntj)), dim3(kThreads), 0,
                           s, v, body_lo, ntj, i0, m, reinterpret_cast<const double2*>(x), part, tab);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_matvec_reduce, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, n,
                       ntj, part, reinterpret_cast<double2*>(y));
    return hipGetLastError();
}

int64_t matvec_work_doubles(int64_t n, int64_t max_body) {
    return 4 * n * ((max_body + kThreads * kMvSources - 1) / (kThreads * kMvSources));
}

// Fixed device buffer of the allocation-free product: the block partial sums
// of k_matvec_partial (every slot is written before k_matvec_reduce reads it,
// so nothing needs clearing).  In host code `scratch` names a host-side
// stand-in, not device memory: kernels receive the address that
// hipGetSymbolAddress gives for the current device, looked up once per device.
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, double*> g_scratch_ptr;
}  // namespace

hipError_t noalloc_scratch(double** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    double* ptr = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr.emplace(dev, ptr);
    *out = ptr;
    return hipSuccess;
}

hipError_t launch_far_field(const NodeView& v, int nbodies, const int64_t* body_lo, const Media* m,
                            const double* phi, const double* angles, int64_t nang, double* uinf,
                            hipStream_t s) {
    if (nang == 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_field, dim3(static_cast<unsigned>(nang), static_cast<unsigned>(nbodies)),
                       dim3(kThreads), 0, s, v, body_lo, m, reinterpret_cast<const double2*>(phi), angles,
                       nang, reinterpret_cast<double2*>(uinf));
    return hipGetLastError();
}

}  // namespace bm
