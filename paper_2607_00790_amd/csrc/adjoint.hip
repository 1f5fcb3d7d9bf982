// Shape derivative of far-field objectives by the adjoint method, and the
// Fourier-parametrised boundary it is taken for.
//
// For a solution A phi = b (Eq. (3)) and a far field u_inf = g^T phi, the
// derivative with respect to any geometric parameter p is
//   du_inf/dp = dL/dp,  L = g^T phi + lam^T (b - A phi),  A^T lam = g,
// with phi and lam held fixed.  L depends on the geometry through the node
// positions x_i, normals n_i, weights w_i and curvatures kappa_i (the last two
// only in the corrected diagonal), and those through the samples x, x', x''
// of the curve (Sec. II).  The kernels here form dL per node:
//   k_shape_pairs  sum over source nodes j of d(lam_i^T A_ij phi_j) for every
//                  target i, and over targets for every source, on 256 x 256
//                  pair tiles of one body (pairs of different bodies are zero);
//   k_shape_nodes  adds the diagonal, right-hand-side and far-field terms and
//                  applies the chain rule to the six curve samples.
//
// k_shape_pairs: lanes own targets; the 256 sources of the tile sit in LDS.
// Each wave walks a 64-source chunk in skewed order (lane l takes source
// (l + s) mod 64 at step s), so at every step the 64 lanes touch 64 different
// sources and add their source-side terms to per-source LDS accumulators
// (LDS FP64 atomic adds, free of bank conflicts); the four waves rotate over
// the four chunks between barriers, so a chunk's accumulators have one wave
// writing them at a time.
// Every pair's Bessel functions are evaluated once for both of its nodes.
// A workgroup's sums go to the node accumulators with one FP64 atomic add per
// node and component.
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "wsbm_adjoint.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;                 // targets and sources of a pair tile
constexpr int kSrcComp = 10;               // source-side components per node
constexpr int kTgtComp = 8;                // target-side components per node
// node accumulators: acc[c * n + i], c < kTgtComp target side, then source side
constexpr int kAccComp = kTgtComp + kSrcComp;

__device__ __forceinline__ int body_of(const NodeView& v, int64_t i) { return v.body ? v.body[i] : 0; }

__global__ void __launch_bounds__(kThreads) k_zero(double* __restrict__ p, int64_t count) {
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; e < count;
         e += static_cast<int64_t>(gridDim.x) * kThreads)
        p[e] = 0.0;
}

__global__ void __launch_bounds__(kThreads) k_fill(double* __restrict__ p, double v) { p[threadIdx.x] = v; }

// Far-field weights of every unknown: u_inf,b(angle) = sum over the body's
// unknowns of g_k phi_k, from the exterior representation D_k0[u] - S_k0[eps0 q]
// at large |x| (the same formula as the far-field kernel).
__global__ void __launch_bounds__(kThreads)
k_far_weights(NodeView v, int64_t n, const Media* __restrict__ media, double ca, double sa,
              double2* __restrict__ g) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= n) return;
    const Media m = media[body_of(v, j)];
    double s, c;
    sincos(-m.k0 * (ca * v.x[j] + sa * v.y[j]), &s, &c);
    // e^{i pi/4} / sqrt(8 pi k0) * exp(-i k0 xhat.x) * w
    const double f = v.w[j] * kSqrtHalf / sqrt(8.0 * kPi * m.k0);
    const double2 ph = make_double2(f * (c - s), f * (s + c));
    const double xn = ca * v.nx[j] + sa * v.ny[j];
    g[2 * j] = c_iscale(-m.k0 * xn, ph);       // -i k0 (xhat.n) ph
    g[2 * j + 1] = c_scale(-m.eps0, ph);
}

// 3 waves per SIMD: the compiler then keeps the pair arithmetic in 168 VGPRs
// with 23 spilled, which measured 9% faster than 2 waves in 194 VGPRs.
__global__ void __launch_bounds__(kThreads, 3)
k_shape_pairs(NodeView v, const int64_t* __restrict__ body_lo, const int64_t* __restrict__ tile_off,
              int nbodies, int64_t t0, const Media* __restrict__ media, const BesselTable* __restrict__ tab,
              const double2* __restrict__ lam, const double2* __restrict__ phi, int64_t n,
              double* __restrict__ acc) {
    __shared__ double s_x[kTile], s_y[kTile], s_nx[kTile], s_ny[kTile], s_w[kTile];
    __shared__ double2 s_u[kTile], s_q[kTile];
    __shared__ int32_t s_c[kTile];
    __shared__ double s_acc[kSrcComp][kTile];
    const int64_t t = t0 + blockIdx.x;
    int lo = 0, hi = nbodies;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= t) lo = mid; else hi = mid;
    }
    const int b = lo;
    const int64_t blo = body_lo[b], bhi = body_lo[b + 1];
    const int64_t nt = (bhi - blo + kTile - 1) / kTile;
    const int64_t local = t - tile_off[b];
    const int64_t ti = local / nt, tj = local % nt;
    const int tid = threadIdx.x;
    const int64_t i = blo + ti * kTile + tid;
    const int64_t j0 = blo + tj * kTile;
    {
        const int64_t j = j0 + tid;
        const bool ok = j < bhi;
        s_x[tid] = ok ? v.x[j] : 0.0;
        s_y[tid] = ok ? v.y[j] : 0.0;
        s_nx[tid] = ok ? v.nx[j] : 0.0;
        s_ny[tid] = ok ? v.ny[j] : 0.0;
        s_w[tid] = ok ? v.w[j] : 0.0;
        s_u[tid] = ok ? phi[2 * j] : make_double2(0.0, 0.0);
        s_q[tid] = ok ? phi[2 * j + 1] : make_double2(0.0, 0.0);
        s_c[tid] = ok ? v.curve[j] : -1;
#pragma unroll
        for (int q = 0; q < kSrcComp; ++q) s_acc[q][tid] = 0.0;
    }
    const bool t_ok = i < bhi;
    const double tx = t_ok ? v.x[i] : 0.0, ty = t_ok ? v.y[i] : 0.0;
    const double tnx = t_ok ? v.nx[i] : 0.0, tny = t_ok ? v.ny[i] : 0.0;
    const int32_t tc = t_ok ? v.curve[i] : -2;
    const double2 l0 = t_ok ? lam[2 * i] : make_double2(0.0, 0.0);
    const double2 l1 = t_ok ? lam[2 * i + 1] : make_double2(0.0, 0.0);
    Media m = media[b];
    m.tab = tab;   // the same table, through a kernel argument: known to be global memory
    __syncthreads();
    double2 g[kTgtComp / 2];
#pragma unroll
    for (int q = 0; q < kTgtComp / 2; ++q) g[q] = make_double2(0.0, 0.0);
    const int lane = tid & 63, wv = tid >> 6;
    for (int ph = 0; ph < kTile / 64; ++ph) {
        const int chunk = ((wv + ph) & 3) * 64;
        for (int s = 0; s < 64; ++s) {
            const int js = chunk + ((lane + s) & 63);
            const int64_t j = j0 + js;
            // a pair that does not exist (diagonal, outside the body) gets lam = 0
            // and a source point away from the target, so it adds exact zeros
            const bool ok = t_ok && j < bhi && j != i;
            const double2 zero = make_double2(0.0, 0.0);
            const double sx = ok ? s_x[js] : tx + 1.0;
            const PairAdjoint pa = pair_adjoint(tx, ty, tnx, tny, ok ? l0 : zero, ok ? l1 : zero, sx, s_y[js],
                                                s_nx[js], s_ny[js], s_w[js], s_u[js], s_q[js], m,
                                                s_c[js] == tc);
            g[0] = c_add(g[0], pa.g_rho[0]);
            g[1] = c_add(g[1], pa.g_rho[1]);
            g[2] = c_add(g[2], pa.g_ni[0]);
            g[3] = c_add(g[3], pa.g_ni[1]);
            // LDS atomics (ds_add_f64): well defined although the lanes that
            // touch a source change from step to step
            atomicAdd(&s_acc[0][js], pa.g_rho[0].x);
            atomicAdd(&s_acc[1][js], pa.g_rho[0].y);
            atomicAdd(&s_acc[2][js], pa.g_rho[1].x);
            atomicAdd(&s_acc[3][js], pa.g_rho[1].y);
            atomicAdd(&s_acc[4][js], pa.g_nj[0].x);
            atomicAdd(&s_acc[5][js], pa.g_nj[0].y);
            atomicAdd(&s_acc[6][js], pa.g_nj[1].x);
            atomicAdd(&s_acc[7][js], pa.g_nj[1].y);
            atomicAdd(&s_acc[8][js], pa.g_w.x);
            atomicAdd(&s_acc[9][js], pa.g_w.y);
        }
        __syncthreads();
    }
    if (t_ok) {
#pragma unroll
        for (int q = 0; q < kTgtComp / 2; ++q) {
            unsafeAtomicAdd(acc + (2 * q) * n + i, g[q].x);
            unsafeAtomicAdd(acc + (2 * q + 1) * n + i, g[q].y);
        }
    }
    const int64_t j = j0 + tid;
    if (j < bhi) {
#pragma unroll
        for (int q = 0; q < kSrcComp; ++q) unsafeAtomicAdd(acc + (kTgtComp + q) * n + j, s_acc[q][tid]);
    }
}

// Per node: dL = d(g^T phi) + d(lam^T b) - d(lam^T A phi), then
// grad[q * n + i] = Re(coef_b dL/ds_q) for the samples s = (x, y, x', y', x'', y'').
// coef_b = coef[b], or 2 conj(uinf[b]) when from_uinf (J = |u_inf|^2).
__global__ void __launch_bounds__(kThreads)
k_shape_nodes(NodeView v, const double* __restrict__ xyd, int64_t n, const Media* __restrict__ media,
              const double2* __restrict__ lam, const double2* __restrict__ phi, const double* __restrict__ acc,
              double cd, double sd, double ca, double sa, const double2* __restrict__ coef, int from_uinf,
              double* __restrict__ grad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int b = body_of(v, i);
    const Media m = media[b];
    double2 cf = coef[b];
    if (from_uinf) cf = make_double2(2.0 * cf.x, -2.0 * cf.y);
    double a[kAccComp];
#pragma unroll
    for (int c = 0; c < kAccComp; ++c) a[c] = acc[c * n + i];
    double g[6];
    node_adjoint(v.x[i], v.y[i], v.nx[i], v.ny[i], v.w[i], v.kappa[i], xyd[2 * n + i], xyd[3 * n + i],
                 xyd[4 * n + i], xyd[5 * n + i], m, lam[2 * i], lam[2 * i + 1], phi[2 * i], phi[2 * i + 1], a,
                 cd, sd, ca, sa, cf, g);
#pragma unroll
    for (int q = 0; q < 6; ++q) grad[q * n + i] = g[q];
}

// Samples of x(t) = c + R r(t) (cos t, sin t), r = 1 + sum_j (a_j cos jt + b_j sin jt),
// at t_i = 2 pi i / n: rows x, y, x', y', x'', y''.
__global__ void __launch_bounds__(kThreads)
k_fourier_curve(const double* __restrict__ coef, int M, double R, double cx, double cy, int64_t n,
                double* __restrict__ xyd) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const double t = 2.0 * kPi * static_cast<double>(i) / static_cast<double>(n);
    double r = 1.0, dr = 0.0, ddr = 0.0;
    for (int j = 1; j <= M; ++j) {
        double s, c;
        sincos(j * t, &s, &c);
        const double aj = coef[j - 1], bj = coef[M + j - 1];
        r += aj * c + bj * s;
        dr += j * (-aj * s + bj * c);
        ddr += -(j * j) * (aj * c + bj * s);
    }
    r *= R;
    dr *= R;
    ddr *= R;
    double s, c;
    sincos(t, &s, &c);
    xyd[i] = cx + r * c;
    xyd[n + i] = cy + r * s;
    xyd[2 * n + i] = dr * c - r * s;
    xyd[3 * n + i] = dr * s + r * c;
    xyd[4 * n + i] = ddr * c - 2.0 * dr * s - r * c;
    xyd[5 * n + i] = ddr * s + 2.0 * dr * c - r * s;
}

// out[m] = sum_i sum_q grad[q * n + i] d s_q(t_i) / d coef_m: the transposed
// Jacobian of k_fourier_curve.  One workgroup per coefficient.
__global__ void __launch_bounds__(kThreads)
k_fourier_chain(const double* __restrict__ grad, int64_t n, int M, double R, double* __restrict__ out) {
    __shared__ double red[kThreads / 64];
    const int mi = blockIdx.x;
    const int j = mi % M + 1;
    const bool is_b = mi >= M;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        const double t = 2.0 * kPi * static_cast<double>(i) / static_cast<double>(n);
        double sj, cj, s, c;
        sincos(j * t, &sj, &cj);
        sincos(t, &s, &c);
        // basis f = cos jt (a_j) or sin jt (b_j) and its first two derivatives
        const double f = is_b ? sj : cj;
        const double f1 = is_b ? j * cj : -j * sj;
        const double f2 = -(j * j) * f;
        acc += grad[i] * (f * c) + grad[n + i] * (f * s) + grad[2 * n + i] * (f1 * c - f * s) +
               grad[3 * n + i] * (f1 * s + f * c) + grad[4 * n + i] * (f2 * c - 2.0 * f1 * s - f * c) +
               grad[5 * n + i] * (f2 * s + 2.0 * f1 * c - f * s);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w];
        out[mi] = R * s;
    }
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_far_weights(const NodeView& v, int64_t n, const Media* media, double angle, double* g,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_far_weights, dim3(blocks_for(n)), dim3(kThreads), 0, s, v, n, media, std::cos(angle),
                       std::sin(angle), reinterpret_cast<double2*>(g));
    return hipGetLastError();
}

int64_t pair_tiles(int64_t nodes) {
    const int64_t t = (nodes + kTile - 1) / kTile;
    return t * t;
}

int64_t shape_work_doubles(int64_t n, int nbodies) {
    return kAccComp * n + 2 * nbodies + 8;
}

hipError_t launch_shape_derivative(const NodeView& v, const double* xyd, int64_t n, int nbodies,
                                   const int64_t* body_lo, const int64_t* tile_off, int64_t ntiles,
                                   const Media* media, const BesselTable* tab, const double* phi,
                                   const double* lam, double inc, double obs, const double* coef, double* grad,
                                   double* work, hipStream_t s) {
    double* acc = work;
    double* uinf = work + kAccComp * n;
    double* angle = uinf + 2 * nbodies;
    hipLaunchKernelGGL(k_zero, dim3(std::min<int64_t>(blocks_for(kAccComp * n), 4096)), dim3(kThreads), 0, s, acc,
                       kAccComp * n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!coef) {
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(1), 0, s, angle, obs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_far_field(v, nbodies, body_lo, media, phi, angle, 1, uinf, s)) != hipSuccess) return e;
    }
    // at most 2^24 - 1 workgroups per launch
    constexpr int64_t kMaxGroups = 0xFFFFFFFFll / kThreads;
    for (int64_t t0 = 0; t0 < ntiles; t0 += kMaxGroups) {
        const int64_t nt = std::min(kMaxGroups, ntiles - t0);
        hipLaunchKernelGGL(k_shape_pairs, dim3(static_cast<unsigned>(nt)), dim3(kThreads), 0, s, v, body_lo,
                           tile_off, nbodies, t0, media, tab, reinterpret_cast<const double2*>(lam),
                           reinterpret_cast<const double2*>(phi), n, acc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_shape_nodes, dim3(blocks_for(n)), dim3(kThreads), 0, s, v, xyd, n, media,
                       reinterpret_cast<const double2*>(lam), reinterpret_cast<const double2*>(phi), acc,
                       std::cos(inc), std::sin(inc), std::cos(obs), std::sin(obs),
                       reinterpret_cast<const double2*>(coef ? coef : uinf), coef ? 0 : 1, grad);
    return hipGetLastError();
}

hipError_t launch_fourier_curve(const double* coef, int M, double R, double cx, double cy, int64_t n, double* xyd,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_fourier_curve, dim3(blocks_for(n)), dim3(kThreads), 0, s, coef, M, R, cx, cy, n, xyd);
    return hipGetLastError();
}

hipError_t launch_fourier_chain(const double* grad, int64_t n, int M, double R, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_fourier_chain, dim3(2 * M), dim3(kThreads), 0, s, grad, n, M, R, out);
    return hipGetLastError();
}

}  // namespace bm
