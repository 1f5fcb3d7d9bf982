// Batched device kernels of the proxy-surface HSS build and solve.
//
//   k_proxy_points   the proxy circle points of every box of a level (centres
//                    and radii come from the host)
//   k_near_count     per box: active unknowns of other boxes inside its proxy
//   k_near_list      ... and their compacted slot lists
//   k_gen_jobs       one launch generates every WSBM block a level needs
//                    (near, proxy, diagonal and skeleton blocks of all boxes),
//                    one node pair per thread, masked 2x2 writes
//   k_cpqr_*         column-pivoted Householder QR of M_b^T for all boxes of a
//                    level, one launch per elimination step, with the relative
//                    rank rule |R_kk| > tol |R_00|
//   k_interp_wave    T_b = [I; (R11^-1 R12)^T] in pivoted order, column-oriented
//   k_interp         the same, row-oriented, for ranks beyond 256
//   k_sketch         Y = Omega X of the randomized ID on the matrix cores
//   k_gauss_jordan_* batched in-place inverse with partial row pivoting, the
//                    block held in registers (a row per lane up to 64, 4 x 4
//                    complex tiles per thread up to 128)
//   k_gemm           batched strided complex GEMM on the matrix cores
#include "hss_internal.hpp"

namespace bm {
namespace hss {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {   // a*b + c
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cconj_mul(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Loads and stores through pointers known to address global memory.  Pointers
// read from job descriptors are generic to the compiler, which then emits flat
// memory instructions; these casts let it use global ones.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double2 gload2(const double2* p) {
    const gdouble* q = (const gdouble*)(const double*)p;
    return make_double2(q[0], q[1]);
}
__device__ __forceinline__ void gstore2(double2* p, double2 v) {
    gdouble* q = (gdouble*)(double*)p;
    q[0] = v.x;
    q[1] = v.y;
}
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
    *(__attribute__((address_space(1))) T*)p = v;
}

// x from lane l (l wave-uniform).
__device__ __forceinline__ double readlane_d(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Maximum over the wave of an unsigned 64-bit key, by DPP row shifts and row
// broadcasts (no LDS traffic); the result is wave-uniform.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t key) {
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(key), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(key >> 32), CTRL, ROW_MASK, 0xF, false);
    const uint64_t o = (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
    return o > key ? o : key;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t key) {
    key = dpp_max_step<0x111, 0xF>(key);   // row_shr:1
    key = dpp_max_step<0x112, 0xF>(key);   // row_shr:2
    key = dpp_max_step<0x114, 0xF>(key);   // row_shr:4
    key = dpp_max_step<0x118, 0xF>(key);   // row_shr:8   -> lane 15 of each row: row maximum
    key = dpp_max_step<0x142, 0xA>(key);   // row_bcast:15 -> lanes 31, 63: two rows each
    key = dpp_max_step<0x143, 0xC>(key);   // row_bcast:31 -> lane 63: all four rows
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(key), 63);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(key >> 32), 63);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ double2 readlane2(double2 v, int l) {
    return make_double2(readlane_d(v.x, l), readlane_d(v.y, l));
}

// max(v, v from the lane DPP control CTRL selects), lanes without a source
// keeping v: one step of a wave maximum (VOP2 with a DPP source).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_fmax(float v) {
    const int o = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
    return fmaxf(v, __int_as_float(o));
}

// The lowest lane holding the wave's largest value of `mag` (wave-uniform);
// -1 if no lane holds a positive value.
__device__ __forceinline__ int wave_argmax_f32(float mag) {
    float m = dpp_fmax<0x111, 0xF>(mag);   // row_shr:1
    m = dpp_fmax<0x112, 0xF>(m);           // row_shr:2
    m = dpp_fmax<0x114, 0xF>(m);           // row_shr:4
    m = dpp_fmax<0x118, 0xF>(m);           // row_shr:8   -> lane 15 of each row
    m = dpp_fmax<0x142, 0xA>(m);           // row_bcast:15
    m = dpp_fmax<0x143, 0xC>(m);           // row_bcast:31 -> lane 63: the maximum
    const float mx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 63));
    if (!(mx > 0.0f)) return -1;
    const uint64_t hit = __builtin_amdgcn_ballot_w64(mag == mx);
    return static_cast<int>(__builtin_ctzll(hit));
}

// DPP move of a double (two 32-bit moves); rows outside ROW_MASK receive `old`
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov_d(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the wave, returned to every lane (wave-uniform): four DPP steps
// within each 16-lane row, two row broadcasts to lane 63, one lane read.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_mov_d<0xB1, 0xF>(x, x);   // quad_perm [1, 0, 3, 2]
    x += dpp_mov_d<0x4E, 0xF>(x, x);   // quad_perm [2, 3, 0, 1]
    {
        const double up = dpp_mov_d<0x104, 0xF>(x, x), dn = dpp_mov_d<0x114, 0xF>(x, x);   // row_shl/shr:4
        x += (threadIdx.x & 4) ? dn : up;
    }
    x += dpp_mov_d<0x128, 0xF>(x, x);  // row_ror:8 -> every lane holds its row's sum
    x += dpp_mov_d<0x142, 0xA>(x, 0.0);  // row_bcast:15 -> rows 1, 3 add rows 0, 2
    x += dpp_mov_d<0x143, 0xC>(x, 0.0);  // row_bcast:31 -> rows 2, 3 add rows 0 + 1
    return readlane_d(x, 63);
}

// Block-wide argmax of (value, index) for values >= 0 or a negative value
// for "none"; ties go to the lowest index.  The wave maximum is exact (the
// bit pattern of a non-negative double orders like the value), the lowest
// index among the lanes that hold it a second DPP maximum.
__device__ void block_argmax(double& v, int& idx, double* sv, int* si) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    {
        const uint64_t key = v >= 0.0 ? static_cast<uint64_t>(__double_as_longlong(v)) + 1 : 0;
        const uint64_t mk = wave_max_u64(key);
        // lowest index among the maxima: the largest complement
        const uint64_t ik = key == mk ? static_cast<uint64_t>(0x7FFFFFFF - idx) : 0;
        const uint64_t mi = wave_max_u64(ik);
        if (lane == 0) {
            sv[wid] = mk > 0 ? __longlong_as_double(static_cast<long long>(mk - 1)) : -1.0;
            si[wid] = 0x7FFFFFFF - static_cast<int>(mi);
        }
    }
    __syncthreads();
    const int nw = static_cast<int>(blockDim.x >> 6);
    double bv = sv[0];
    int bi = si[0];
    for (int w = 1; w < nw; ++w) {
        const double ov = sv[w];
        const int oi = si[w];
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    v = bv;
    idx = bi;
    __syncthreads();
}

__device__ double block_sum(double v, double* sv) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) sv[wid] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += sv[w];
    __syncthreads();
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Proxy circles: one workgroup per box; box b (centre box_c[3b], box_c[3b+1],
// proxy radius box_c[3b+2]) gets pcount[b] equispaced proxy points, written to
// the point table at nnodes + poff[b] + p, with radial normals, weights
// 2 pi R_p / P_b and the box's body.
__global__ void __launch_bounds__(kThreads)
k_proxy_points(const double* __restrict__ box_c, const int32_t* __restrict__ box_body,
               const int64_t* __restrict__ poff, const int32_t* __restrict__ pcount, int64_t nnodes,
               PointTable pt) {
    const int b = blockIdx.x;
    const double cx = box_c[3 * b], cy = box_c[3 * b + 1], rp = box_c[3 * b + 2];
    const int P = pcount[b];
    for (int p = threadIdx.x; p < P; p += kThreads) {
        double s, c;
        sincospi(2.0 * p / P, &s, &c);
        const int64_t q = nnodes + poff[b] + p;
        pt.x[q] = cx + rp * c;
        pt.y[q] = cy + rp * s;
        pt.nx[q] = c;
        pt.ny[q] = s;
        pt.w[q] = 2.0 * kPi * rp / P;
        pt.kappa[q] = 0.0;
        pt.curve[q] = -1;
        pt.body[q] = box_body[b];
    }
}

// ---------------------------------------------------------------------------
// Near sets.  Candidates are the active slots of the boxes of the level
// (slot_box[s] = owning box); box b scans only [scan_lo[b], scan_hi[b]), the
// slots of its own body.  A slot is near box b if it belongs to another box and
// its node lies strictly inside b's proxy circle.
__device__ __forceinline__ bool is_near(const PointTable& pt, const Slot& s, int owner, int b,
                                        const double* box_c) {
    if (owner == b) return false;
    const double dx = pt.x[s.pt] - box_c[3 * b], dy = pt.y[s.pt] - box_c[3 * b + 1];
    const double r = box_c[3 * b + 2];
    return dx * dx + dy * dy < r * r;
}

__device__ __forceinline__ int slot_unknowns(const Slot& s) {
    return (s.pos0 >= 0 ? 1 : 0) + (s.pos1 >= 0 ? 1 : 0);
}

// counts[2b] = near slots of box b, counts[2b+1] = near unknowns of box b.
__global__ void __launch_bounds__(kThreads)
k_near_count(PointTable pt, const Slot* __restrict__ slots, const int32_t* __restrict__ slot_box,
             const int64_t* __restrict__ scan_lo, const int64_t* __restrict__ scan_hi,
             const double* __restrict__ box_c, int64_t* __restrict__ counts) {
    __shared__ double red[kThreads / 64];
    const int b = blockIdx.x;
    double ns = 0, nu = 0;
    for (int64_t s = scan_lo[b] + threadIdx.x; s < scan_hi[b]; s += kThreads) {
        const Slot sl = slots[s];
        if (is_near(pt, sl, slot_box[s], b, box_c)) {
            ns += 1;
            nu += slot_unknowns(sl);
        }
    }
    ns = block_sum(ns, red);
    nu = block_sum(nu, red);
    if (threadIdx.x == 0) {
        counts[2 * b] = static_cast<int64_t>(ns);
        counts[2 * b + 1] = static_cast<int64_t>(nu);
    }
}

// Writes box b's near slots at out + slot_off[b], with unknown positions
// renumbered 0..(near unknowns - 1) in candidate order.
__global__ void __launch_bounds__(kThreads)
k_near_list(PointTable pt, const Slot* __restrict__ slots, const int32_t* __restrict__ slot_box,
            const int64_t* __restrict__ scan_lo, const int64_t* __restrict__ scan_hi,
            const double* __restrict__ box_c, const int64_t* __restrict__ slot_off,
            Slot* __restrict__ out) {
    __shared__ int scan_s[kThreads];
    __shared__ int scan_u[kThreads];
    __shared__ int base[2];
    const int b = blockIdx.x;
    const int64_t s_lo = scan_lo[b], s_hi = scan_hi[b];
    if (threadIdx.x == 0) { base[0] = 0; base[1] = 0; }
    __syncthreads();
    for (int64_t s0 = s_lo; s0 < s_hi; s0 += kThreads) {
        const int64_t s = s0 + threadIdx.x;
        Slot sl{0, -1, -1};
        bool nearb = false;
        if (s < s_hi) {
            sl = slots[s];
            nearb = is_near(pt, sl, slot_box[s], b, box_c);
        }
        const int fs = nearb ? 1 : 0;
        const int fu = nearb ? slot_unknowns(sl) : 0;
        scan_s[threadIdx.x] = fs;
        scan_u[threadIdx.x] = fu;
        __syncthreads();
        // inclusive Hillis-Steele scans
        for (int off = 1; off < kThreads; off <<= 1) {
            const int vs = threadIdx.x >= off ? scan_s[threadIdx.x - off] : 0;
            const int vu = threadIdx.x >= off ? scan_u[threadIdx.x - off] : 0;
            __syncthreads();
            scan_s[threadIdx.x] += vs;
            scan_u[threadIdx.x] += vu;
            __syncthreads();
        }
        if (nearb) {
            const int is = base[0] + scan_s[threadIdx.x] - fs;
            int pu = base[1] + scan_u[threadIdx.x] - fu;
            Slot o{sl.pt, -1, -1};
            if (sl.pos0 >= 0) o.pos0 = pu++;
            if (sl.pos1 >= 0) o.pos1 = pu++;
            out[slot_off[b] + is] = o;
        }
        __syncthreads();
        if (threadIdx.x == kThreads - 1) {
            base[0] += scan_s[kThreads - 1];
            base[1] += scan_u[kThreads - 1];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Entry generation for a batch of jobs: every WSBM block the HSS build needs
// (near, proxy, diagonal and skeleton blocks) and the public block and proxy
// entry points.  Job j covers nt x ns slot pairs in tiles of kThreads pairs;
// tile_off is the exclusive prefix sum of the tile counts.  One pair per
// thread, no loop (the Bessel coefficients stay scalar operands).
//
// Pair order: a wave takes 64 consecutive pairs with the source index running
// fastest, except for jobs stored transposed (rs == 1, cs != 1: the stacked
// matrix's A(near, U)^T and A(proxy, U)^T parts), where the target index runs
// fastest so that the wave's stores still land on consecutive positions.  The
// wave's first pair is split into (slow, fast) indices once per wave with an
// FP64 reciprocal; the lanes then offset the fast index.
//
// Media: a job with body >= 0 uses that body's media for every pair.  With
// body < 0 (the public entry points) each pair takes the body of its node
// points -- a proxy point (body < 0 in the point table) takes its partner's --
// and a pair of nodes in two different bodies is a zero block.
//
// R = double: FP64 arithmetic.  R = float: the FP32 formulas of
// wsbm_pair_f32.hpp (ftab the FP32 coefficient table), results widened to
// FP64 on store.
template <class R>
__global__ void __launch_bounds__(kThreads, kPairWavesPerSimd)
k_gen_jobs(const GenJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs,
           const Slot* __restrict__ slots, PointTable pt, const Media* __restrict__ media,
           double2* __restrict__ out, const BesselTable* __restrict__ tab, const float* __restrict__ ftab) {
    int lo = 0, hi = njobs;
    const int64_t tile = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    const GenJob jb = jobs[lo];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q0 = (tile - tile_off[lo]) * kThreads + 64 * wave;   // the wave's first pair
    if (q0 + lane >= static_cast<int64_t>(jb.nt) * jb.ns) return;
    const bool tfast = jb.rs == 1 && jb.cs != 1;
    const int32_t nf = tfast ? jb.nt : jb.ns;
    int64_t slow = static_cast<int64_t>(static_cast<double>(q0) * recip(static_cast<double>(nf)));
    int64_t rem = q0 - slow * nf;
    if (rem < 0) { --slow; rem += nf; } else if (rem >= nf) { ++slow; rem -= nf; }
    int32_t fast = static_cast<int32_t>(rem) + lane;
    if (nf >= 64) {
        if (fast >= nf) { fast -= nf; ++slow; }
    } else {
        slow += fast / nf;
        fast = fast % nf;
    }
    const int32_t t = tfast ? fast : static_cast<int32_t>(slow);
    const int32_t s = tfast ? static_cast<int32_t>(slow) : fast;
    const Slot ts = slots[jb.tslot + t];
    const Slot ss = slots[jb.sslot + s];
    const int32_t i = ts.pt, j = ss.pt;
    double2* o = out + jb.out;
    // one row of the 2x2 block (v: re/im of the u and q columns) to the selected columns
    auto put = [&](int32_t row, const double (&v)[4]) {
        if (ss.pos0 >= 0) o[row * jb.rs + ss.pos0 * jb.cs] = make_double2(v[0], v[1]);
        if (ss.pos1 >= 0) o[row * jb.rs + ss.pos1 * jb.cs] = make_double2(v[2], v[3]);
    };
    int body = jb.body;
    if (body < 0) {
        const int bi = pt.body[i], bj = pt.body[j];
        if (bi >= 0 && bj >= 0 && bi != bj) {
            if (ts.pos0 >= 0) put(ts.pos0, {0.0, 0.0, 0.0, 0.0});
            if (ts.pos1 >= 0) put(ts.pos1, {0.0, 0.0, 0.0, 0.0});
            return;
        }
        body = bi >= 0 ? bi : bj;
    }
    Media m = media[body];
    m.tab = tab;   // the table through a kernel argument: scalar loads of known global memory
    const int32_t ci = pt.curve[i], cj = pt.curve[j];
    const bool interior = ci == cj || ci < 0 || cj < 0;
    if constexpr (sizeof(R) == sizeof(double)) {
        if (i == j) {
            const Block b = diag_block(pt.w[j], pt.kappa[j], m);
            if (ts.pos0 >= 0) put(ts.pos0, {b.v[0], b.v[1], b.v[2], b.v[3]});
            if (ts.pos1 >= 0) put(ts.pos1, {b.v[4], b.v[5], b.v[6], b.v[7]});
            return;
        }
        // Rows are formed separately: row 2i needs only the interior kernels, and
        // when a skeleton keeps row 2i alone the exterior ones are never evaluated.
        const double sw = pt.w[j];
        const PairGeom g = pair_geom(pt.x[i], pt.y[i], pt.nx[i], pt.ny[i], pt.x[j], pt.y[j], pt.nx[j],
                                     pt.ny[j]);
        const Hankel01 h1 = pair_interior(g, m, interior);
        double v[4];
        if (ts.pos0 >= 0) {
            pair_row0(g, h1, sw, m, v);
            put(ts.pos0, v);
        }
        if (ts.pos1 >= 0) {
            pair_row1(g, interior_terms(h1, m), sw, m, v);
            put(ts.pos1, v);
        }
    } else {
        const f32::MediaF mf = f32::media_f(m);
        if (i == j) {
            const Block b = f32::diag_block(static_cast<float>(pt.w[j]), static_cast<float>(pt.kappa[j]), mf);
            if (ts.pos0 >= 0) put(ts.pos0, {b.v[0], b.v[1], b.v[2], b.v[3]});
            if (ts.pos1 >= 0) put(ts.pos1, {b.v[4], b.v[5], b.v[6], b.v[7]});
            return;
        }
        const float sw = static_cast<float>(pt.w[j]);
        const f32::PairGeomF g = f32::pair_geom(pt.x[i], pt.y[i], static_cast<float>(pt.nx[i]),
                                                static_cast<float>(pt.ny[i]), pt.x[j], pt.y[j],
                                                static_cast<float>(pt.nx[j]), static_cast<float>(pt.ny[j]));
        const f32::Hankel01F h1 = f32::pair_interior(g, mf, interior, tab, ftab);
        float vf[4];
        if (ts.pos0 >= 0) {
            f32::pair_row0(g, h1, sw, mf, vf);
            put(ts.pos0, {vf[0], vf[1], vf[2], vf[3]});
        }
        if (ts.pos1 >= 0) {
            f32::pair_row1(g, h1, sw, mf, tab, ftab, vf);
            put(ts.pos1, {vf[0], vf[1], vf[2], vf[3]});
        }
    }
}

template __global__ void k_gen_jobs<double>(const GenJob*, const int64_t*, int, const Slot*, PointTable,
                                            const Media*, double2*, const BesselTable*, const float*);
template __global__ void k_gen_jobs<float>(const GenJob*, const int64_t*, int, const Slot*, PointTable,
                                           const Media*, double2*, const BesselTable*, const float*);

// ---------------------------------------------------------------------------
// Level-batched CPQR by steps, for levels with few, large boxes: per
// elimination step k one launch of k_cpqr_pivot (one workgroup per box: pivot,
// column swap, Householder vector) and one of k_cpqr_update (many workgroups
// per box, one wave per trailing column).  State per box lives in global
// memory: column norms, the reference |R_00|, the Householder scale, rank, done.
__global__ void __launch_bounds__(kThreads)
k_cpqr_init(const CpqrJob* __restrict__ jobs) {
    const CpqrJob jb = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kThreads / 64;
    const int j = blockIdx.x * nw + wid;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        gst(&jb.st->ref, 0.0);
        gst(&jb.st->beta, 0.0);
        gst(&jb.st->rank, 0);
        gst(&jb.st->done, 0);
    }
    if (j >= jb.n) return;
    if (lane == 0) {
        gst(jb.perm + j, j);
        gst(jb.used + j, 0);
    }
    double s = 0;
    for (int r = lane; r < jb.m; r += 64) s += cabs2(gload2(jb.x + static_cast<int64_t>(j) * jb.m + r));
    s = wave_sum(s);
    if (lane == 0) gst(jb.nrm + j, s);
}

// One elimination step k of the level-batched CPQR, fused into one launch.
// Pivoting is logical: columns stay in place, perm[k] records the k-th pivot
// and used[] marks retired columns (the pivot of step k-1 is excluded
// explicitly, since its used[] entry is written during this launch).  Column
// norms are double-buffered (read nrm[k % 2], write nrm[(k+1) % 2]), so every
// workgroup of a box computes the same pivot from the same data.  Grid: (box,
// chunk of kThreads/64 columns), one wave per column.
__global__ void __launch_bounds__(kThreads)
k_cpqr_step(const CpqrJob* __restrict__ jobs, int k, double tol) {
    __shared__ double sv[kThreads / 64];
    __shared__ int si[kThreads / 64];
    const CpqrJob jb = jobs[blockIdx.y];
    CpqrState* st = jb.st;
    if (gld(&st->done)) return;
    const int n = jb.n, m = jb.m;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (k >= (n < m ? n : m)) {
        if (lead) { gst(&st->rank, k); gst(&st->done, 1); }
        return;
    }
    const double* __restrict__ nin = jb.nrm + (k & 1) * n;
    double* __restrict__ nout = jb.nrm + ((k + 1) & 1) * n;
    const int prev = k > 0 ? gld(jb.perm + k - 1) : -1;
    double bv = -1;
    int bi = n;
    for (int j = threadIdx.x; j < n; j += kThreads)
        if (!gld(jb.used + j) && j != prev && gld(nin + j) > bv) { bv = gld(nin + j); bi = j; }
    block_argmax(bv, bi, sv, si);
    const double ref = k == 0 ? sqrt(bv) : gld(&st->ref);
    if (!(sqrt(bv) > tol * ref) || ref == 0 || bi >= n) {
        if (lead) { gst(&st->rank, k); gst(&st->done, 1); }
        return;
    }
    const int p = bi;
    const double2* __restrict__ w = jb.x + static_cast<int64_t>(p) * m;   // rows >= k
    const double xn = sqrt(gld(nin + p));
    const double2 x0 = gload2(w + k);
    const double a0 = sqrt(cabs2(x0));
    const double2 ph = a0 > 0 ? make_double2(x0.x / a0, x0.y / a0) : make_double2(1.0, 0.0);
    const double2 alpha = make_double2(-ph.x * xn, -ph.y * xn);
    const double2 w0 = make_double2(x0.x - alpha.x, x0.y - alpha.y);   // first entry of w
    const double beta = xn > 0 ? 1.0 / (xn * (xn + a0)) : 0.0;
    if (lead) {
        gst(jb.perm + k, p);
        gstore2(jb.rdiag + k, alpha);
        if (prev >= 0) gst(jb.used + prev, 1);
        if (k == 0) gst(&st->ref, ref);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kThreads / 64;
    const int j = blockIdx.x * nw + wid;
    if (j >= n || j == p || j == prev || gld(jb.used + j)) return;
    double2* __restrict__ cj = jb.x + static_cast<int64_t>(j) * m;
    double gr = 0, gi = 0;
    for (int r = k + lane; r < m; r += 64) {
        const double2 wr = r == k ? w0 : gload2(w + r);
        const double2 t = cconj_mul(wr, gload2(cj + r));
        gr += t.x;
        gi += t.y;
    }
    gr = wave_sum(gr) * beta;
    gi = wave_sum(gi) * beta;
    double s = 0;
    for (int r = k + lane; r < m; r += 64) {
        const double2 wr = r == k ? w0 : gload2(w + r);
        double2 y = gload2(cj + r);
        y.x -= gr * wr.x - gi * wr.y;
        y.y -= gr * wr.y + gi * wr.x;
        gstore2(cj + r, y);
        if (r > k) s += cabs2(y);
    }
    s = wave_sum(s);
    if (lane == 0) gst(nout + j, s);
}

// The same elimination step for matrices of at most 64 R rows: the block
// stages the Householder column (rows k..m) in LDS once, and each wave keeps
// its trailing column in registers (R complex values per lane), so a column
// is read from memory once and written once per step, with all R loads of a
// lane in flight together.  Pivot choice, rank rule, logical pivoting and the
// double-buffered norms are those of k_cpqr_step.
template <int R>
__global__ void __launch_bounds__(kThreads)
k_cpqr_step_reg(const CpqrJob* __restrict__ jobs, int k, double tol) {
    __shared__ double sv[kThreads / 64];
    __shared__ int si[kThreads / 64];
    __shared__ double2 ws[64 * R];
    const CpqrJob jb = jobs[blockIdx.y];
    CpqrState* st = jb.st;
    if (gld(&st->done)) return;
    const int n = jb.n, m = jb.m;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (k >= (n < m ? n : m)) {
        if (lead) { gst(&st->rank, k); gst(&st->done, 1); }
        return;
    }
    const double* __restrict__ nin = jb.nrm + (k & 1) * n;
    double* __restrict__ nout = jb.nrm + ((k + 1) & 1) * n;
    const int prev = k > 0 ? gld(jb.perm + k - 1) : -1;
    double bv = -1;
    int bi = n;
    for (int j = threadIdx.x; j < n; j += kThreads)
        if (!gld(jb.used + j) && j != prev && gld(nin + j) > bv) { bv = gld(nin + j); bi = j; }
    block_argmax(bv, bi, sv, si);
    const double ref = k == 0 ? sqrt(bv) : gld(&st->ref);
    if (!(sqrt(bv) > tol * ref) || ref == 0 || bi >= n) {
        if (lead) { gst(&st->rank, k); gst(&st->done, 1); }
        return;
    }
    const int p = bi;
    const double2* __restrict__ w = jb.x + static_cast<int64_t>(p) * m;
    const double xn = sqrt(gld(nin + p));
    const double2 x0 = gload2(w + k);
    const double a0 = sqrt(cabs2(x0));
    const double2 ph = a0 > 0 ? make_double2(x0.x / a0, x0.y / a0) : make_double2(1.0, 0.0);
    const double2 alpha = make_double2(-ph.x * xn, -ph.y * xn);
    const double2 w0 = make_double2(x0.x - alpha.x, x0.y - alpha.y);
    const double beta = xn > 0 ? 1.0 / (xn * (xn + a0)) : 0.0;
    if (lead) {
        gst(jb.perm + k, p);
        gstore2(jb.rdiag + k, alpha);
        if (prev >= 0) gst(jb.used + prev, 1);
        if (k == 0) gst(&st->ref, ref);
    }
    const int mk = m - k;   // active rows, <= 64 R
    for (int r = threadIdx.x; r < mk; r += kThreads) ws[r] = gload2(w + k + r);
    if (threadIdx.x == 0) ws[0] = w0;   // after its own store of w[k] above
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kThreads / 64;
    // kCpqrCols consecutive columns per wave: the pivot search and the staging
    // of w above are paid once per kCpqrCols * 4 columns
    for (int jj = 0; jj < kCpqrCols; ++jj) {
        const int j = (blockIdx.x * nw + wid) * kCpqrCols + jj;
        if (j >= n) break;
        if (j == p || j == prev || gld(jb.used + j)) continue;
        double2* __restrict__ cj = jb.x + static_cast<int64_t>(j) * m + k;
        double2 c[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            c[t] = r < mk ? gload2(cj + r) : make_double2(0.0, 0.0);
        }
        double gr = 0, gi = 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            if (r < mk) {
                const double2 v = cconj_mul(ws[r], c[t]);
                gr += v.x;
                gi += v.y;
            }
        }
        gr = wave_sum(gr) * beta;
        gi = wave_sum(gi) * beta;
        double sn = 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int r = lane + 64 * t;
            if (r < mk) {
                const double2 wr = ws[r];
                double2 y = c[t];
                y.x -= gr * wr.x - gi * wr.y;
                y.y -= gr * wr.y + gi * wr.x;
                gstore2(cj + r, y);
                if (r > 0) sn += cabs2(y);
            }
        }
        sn = wave_sum(sn);
        if (lane == 0) gst(nout + j, sn);
    }
}

// Sum over the 16 lanes of each DPP row (every lane of the row gets the total):
// xor 1 and xor 2 by quad permutations, the other quad of the half-row by a
// shift of 4 in the direction that stays inside it, the other half-row by a
// rotation of 8.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    const double up = dpp_d<0x104>(v), dn = dpp_d<0x114>(v);   // row_shl:4, row_shr:4
    v += (threadIdx.x & 4) ? dn : up;
    v += dpp_d<0x128>(v);  // row_ror:8
    return v;
}

// The whole CPQR of one box in one workgroup of NT threads, for boxes of at
// most C NT / 16 columns and 16 R rows: the matrix stays in registers for all
// steps.  Lane (c, g) of a wave, c = lane / 16, g = lane % 16, holds rows
// g, g + 16, ..., g + 16 (R - 1) of the C columns C (4 w + c) .. + C - 1 (w
// the wave), so a column lives in one 16-lane DPP row and its dot products and
// norms need four DPP steps, and each lane reads the Householder vector (R
// values from LDS, once for the dot products and once for the update) for C
// columns at a time (for C = 5, in two chunks of at most three columns: the
// 160 x 160 box takes 200 of the 256 registers).  Per step: the pivot (largest
// remaining column norm, lowest index on ties: an exact maximum of the norm's
// bit pattern, per wave by DPP, then over the waves through LDS), then the
// lanes of the pivot column stage the Householder vector in LDS (zeros above
// row k; the lane of row k writes w0 = x_k - alpha and the scalars alpha and
// beta), then every lane applies it to its columns and recomputes their
// norms below row k.  Blocks of 16 rows entirely above row k are skipped.
// Rank rule |R_kk| > tol |R_00|, logical pivoting and the layout of the
// result (R in the columns perm[0..rank), diagonal in rdiag) are those of the
// step-wise kernels, so k_cpqr_finish and k_interp follow unchanged.  Grid:
// one workgroup per box.
template <int R, int C, int NT>
__global__ void __launch_bounds__(NT)
k_cpqr_fused(const CpqrJob* __restrict__ jobs, double tol) {
    constexpr int NW = NT / 64;
    constexpr int CB = C <= 4 ? C : (C + 1) / 2;
    __shared__ double2 ws[16 * R];
    __shared__ uint64_t wkey[NW];
    __shared__ int wcol[NW];
    __shared__ double sbeta;
    __shared__ double2 salpha;
    const CpqrJob jb = jobs[blockIdx.x];
    const int n = jb.n, m = jb.m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane & 15, c0 = C * (4 * wave + (lane >> 4));   // first of this lane's C columns
    double2 X[R][C];
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int r = g + 16 * t;
            X[t][c] = (c0 + c < n && r < m) ? gload2(jb.x + static_cast<int64_t>(c0 + c) * m + r)
                                            : make_double2(0.0, 0.0);
        }
    double nrm[C];
    uint32_t used = 0;   // bit c: column c0 + c pivoted (or past n)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double q = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) q = fma(X[t][c].x, X[t][c].x, fma(X[t][c].y, X[t][c].y, q));
        nrm[c] = row16_sum(q);
        if (c0 + c >= n) used |= 1u << c;
        else if (g == 0) gst(jb.used + c0 + c, 0);
    }
    const int kmax = n < m ? n : m;
    double ref = 0;
    int k = 0;
    for (; k < kmax; ++k) {
        // the pivot: per lane the best of its columns (as norm bits + 1, 0 for
        // none), per wave the lowest lane holding the maximum, then the waves
        uint64_t key = 0;
        int bj = 0;
#pragma unroll
        for (int c = C - 1; c >= 0; --c) {
            const uint64_t kc = (used >> c) & 1 ? 0 : static_cast<uint64_t>(__double_as_longlong(nrm[c])) + 1;
            if (kc >= key && kc > 0) {
                key = kc;
                bj = c0 + c;
            }
        }
        uint64_t mk = wave_max_u64(key);
        {
            const uint64_t hit = __builtin_amdgcn_ballot_w64(key == mk && mk > 0);
            const int l = hit ? static_cast<int>(__builtin_ctzll(hit)) : 0;
            const int wj = __builtin_amdgcn_readlane(bj, l);
            if (lane == 0) {
                wkey[wave] = mk;
                wcol[wave] = wj;
            }
        }
        __syncthreads();   // also: every read of ws of the previous step is done
        const uint64_t ek = lane < NW ? wkey[lane] : 0;
        const int ej = lane < NW ? wcol[lane] : 0;
        mk = wave_max_u64(ek);
        const uint64_t hit = __builtin_amdgcn_ballot_w64(ek == mk && mk > 0);
        const int p = hit ? __builtin_amdgcn_readlane(ej, static_cast<int>(__builtin_ctzll(hit))) : n;
        const double bv = mk > 0 ? __longlong_as_double(static_cast<long long>(mk - 1)) : 0.0;
        if (k == 0) ref = sqrt(bv);
        if (!(sqrt(bv) > tol * ref) || ref == 0 || p >= n) break;   // uniform
        const int kb = k >> 4;   // blocks of 16 rows below kb lie above row k
        if (c0 == p / C * C) {
            const int pc = p % C;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (c != pc) continue;   // uniform
                used |= 1u << c;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    if (t < kb) continue;   // uniform
                    const int r = g + 16 * t;
                    double2 v = r >= k && r < m ? X[t][c] : make_double2(0.0, 0.0);
                    if (r == k) {
                        const double xn = sqrt(bv);
                        const double a0 = sqrt(cabs2(v));
                        const double ia = a0 > 0 ? recip(a0) : 0.0;
                        const double2 ph = a0 > 0 ? make_double2(v.x * ia, v.y * ia) : make_double2(1.0, 0.0);
                        const double2 alpha = make_double2(-ph.x * xn, -ph.y * xn);
                        v = make_double2(v.x - alpha.x, v.y - alpha.y);
                        sbeta = xn > 0 ? recip(xn * (xn + a0)) : 0.0;
                        salpha = alpha;
                    }
                    ws[r] = v;
                }
            }
        }
        __syncthreads();
        const double beta = sbeta;
        if (threadIdx.x == 0) {
            gst(jb.perm + k, p);
            gstore2(jb.rdiag + k, salpha);
        }
        // the columns in chunks of CB (all at once for C <= 4; more chunks
        // read w more often but hold fewer projections)
#pragma unroll
        for (int cb = 0; cb < C; cb += CB) {
            double ar[CB], ai[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) ar[c] = ai[c] = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (t < kb) continue;   // uniform
                const double2 w = ws[g + 16 * t];
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    if (cb + c >= C) continue;
                    ar[c] = fma(w.x, X[t][cb + c].x, fma(w.y, X[t][cb + c].y, ar[c]));
                    ai[c] = fma(w.x, X[t][cb + c].y, fma(-w.y, X[t][cb + c].x, ai[c]));
                }
            }
            // the projections, in place: pivoted columns (and columns past n) stay as they are
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const bool u = cb + c >= C || ((used >> (cb + c)) & 1);
                ar[c] = u ? 0.0 : row16_sum(ar[c]) * beta;
                ai[c] = u ? 0.0 : row16_sum(ai[c]) * beta;
            }
            // w is read again below instead of being kept in R more registers
            // across the reductions (a compiler barrier only: no instruction)
            asm volatile("" ::: "memory");
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (t < kb) continue;   // uniform
                const double2 w = ws[g + 16 * t];
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    if (cb + c >= C) continue;
                    X[t][cb + c].x = fma(-ar[c], w.x, fma(ai[c], w.y, X[t][cb + c].x));
                    X[t][cb + c].y = fma(-ar[c], w.y, fma(-ai[c], w.x, X[t][cb + c].y));
                }
            }
            asm volatile("" ::: "memory");
        }
        // the norms of the rows below k, after the update (not during it, so
        // that the norms and the projections are never live together)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double q = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (t < kb) continue;   // uniform
                const double e = fma(X[t][c].x, X[t][c].x, X[t][c].y * X[t][c].y);
                q += g + 16 * t > k ? e : 0.0;
            }
            nrm[c] = row16_sum(q);
        }
    }
#pragma unroll
    for (int t = 0; t < R; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int r = g + 16 * t;
            if (c0 + c < n && r < m) gstore2(jb.x + static_cast<int64_t>(c0 + c) * m + r, X[t][c]);
        }
    if (threadIdx.x == 0) {
        gst(&jb.st->ref, ref);
        gst(&jb.st->rank, k);
        gst(&jb.st->done, 1);
    }
}

template __global__ void k_cpqr_fused<8, 4, kFusedThreads>(const CpqrJob*, double);
template __global__ void k_cpqr_fused<9, 4, kFusedThreads>(const CpqrJob*, double);
template __global__ void k_cpqr_fused<10, 4, kFusedThreads>(const CpqrJob*, double);
template __global__ void k_cpqr_fused<10, kFusedWideC, kFusedThreads>(const CpqrJob*, double);

template __global__ void k_cpqr_step_reg<4>(const CpqrJob*, int, double);
template __global__ void k_cpqr_step_reg<8>(const CpqrJob*, int, double);
template __global__ void k_cpqr_step_reg<16>(const CpqrJob*, int, double);
template __global__ void k_cpqr_step_reg<32>(const CpqrJob*, int, double);

// After the step-wise CPQR: mark the last pivot used and list the remaining
// columns after the pivots, perm[rank..n) in increasing order.  One workgroup
// per box.
__global__ void __launch_bounds__(kThreads)
k_cpqr_finish(const CpqrJob* __restrict__ jobs) {
    __shared__ int scan[kThreads];
    __shared__ int base;
    const CpqrJob jb = jobs[blockIdx.x];
    const int n = jb.n, r = gld(&jb.st->rank);
    if (threadIdx.x == 0) base = r;
    for (int i = threadIdx.x; i < r; i += kThreads) gst(jb.used + gld(jb.perm + i), 1);
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += kThreads) {
        const int j = j0 + threadIdx.x;
        const int f = (j < n && !gld(jb.used + j)) ? 1 : 0;
        scan[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < kThreads; off <<= 1) {
            const int v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) gst(jb.perm + base + scan[threadIdx.x] - 1, j);
        __syncthreads();
        if (threadIdx.x == kThreads - 1) base += scan[kThreads - 1];
        __syncthreads();
    }
}

// Ranks of the step-wise CPQR.
__global__ void k_cpqr_ranks(const CpqrJob* __restrict__ jobs, int nb, int32_t* __restrict__ ranks,
                             int32_t* __restrict__ active) {
    int cnt = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        ranks[b] = gld(&jobs[b].st->rank);
        cnt += gld(&jobs[b].st->done) ? 0 : 1;
    }
    cnt = static_cast<int>(wave_sum(static_cast<double>(cnt)));
    if (threadIdx.x == 0) *active = cnt;
}

// T_b (n x k, row-major) from the CPQR result: rows perm[0..k) are the
// identity, row perm[k + c] holds column c of Z = R11^-1 R12.  Back
// substitution by one wave per column: lane l owns the entries z_i with
// i = l (mod 64) and keeps them in the column's own row of T, so a lane only
// ever reads values it wrote itself; the partial dot products are combined by
// a butterfly sum, after which every lane knows the new z_i.  T must be zeroed
// beforehand.  Grid: (box, column chunk of kThreads/64 columns).
__global__ void __launch_bounds__(kThreads)
k_interp(const CpqrJob* __restrict__ jobs, const int32_t* __restrict__ ranks,
         const int64_t* __restrict__ t_off, double2* __restrict__ Tbuf) {
    const CpqrJob jb = jobs[blockIdx.y];
    const int n = jb.n, m = jb.m, k = ranks[blockIdx.y];
    double2* T = Tbuf + t_off[blockIdx.y];
    const double2* X = jb.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kThreads / 64;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += kThreads)
            gstore2(T + static_cast<int64_t>(gld(jb.perm + i)) * k + i, make_double2(1.0, 0.0));
    const int c = blockIdx.x * nw + wid;
    const bool logical = jb.used != nullptr;
    if (c >= n - k) return;
    // column of X holding pivot l: l after physical swaps, perm[l] with logical pivoting
    const int pc = gld(jb.perm + k + c);
    const double2* rc = X + static_cast<int64_t>(logical ? pc : k + c) * m;
    double2* z = T + static_cast<int64_t>(pc) * k;
    for (int i = k - 1; i >= 0; --i) {
        double sr = 0, si = 0;
        for (int l = i + 1 + ((lane - i - 1) & 63); l < k; l += 64) {   // l = lane (mod 64)
            const int64_t cl = logical ? gld(jb.perm + l) : l;
            const double2 t = cmul(gload2(X + cl * m + i), gload2(z + l));
            sr += t.x;
            si += t.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        const double2 ri = gload2(rc + i);
        const double2 num = make_double2(ri.x - sr, ri.y - si);
        const double2 d = gload2(jb.rdiag + i);
        const double dd = cabs2(d);
        if ((i & 63) == lane)
            gstore2(z + i, make_double2((num.x * d.x + num.y * d.y) / dd, (num.y * d.x - num.x * d.y) / dd));
    }
}

// ---------------------------------------------------------------------------
// T_b as k_interp, for ranks k <= 64 RPL: one wave per column c of
// Z = R11^-1 R12, lane j keeps rows j + 64 s (s < RPL) of the right-hand side
// R12[:, c] in registers and overwrites each with z once it is solved.  The
// substitution is column-oriented: for l = k-1 .. 0 the owner lane forms
// z_l = y_l / d_l, a lane broadcast hands it to the wave, and every row i < l
// subtracts R11[i][l] z_l.  Column l of R11 is one contiguous read of X,
// independent of the recurrence, so the unrolled loop keeps the reads of
// several columns in flight while the dependent chain per step is a complex
// product, the broadcast and one complex FMA.  Needs logical pivoting.
template <int RPL>
__global__ void __launch_bounds__(kThreads)
k_interp_wave(const CpqrJob* __restrict__ jobs, const int32_t* __restrict__ ranks,
              const int64_t* __restrict__ t_off, double2* __restrict__ Tbuf) {
    const CpqrJob jb = jobs[blockIdx.y];
    const int n = jb.n, m = jb.m, k = ranks[blockIdx.y];
    double2* T = Tbuf + t_off[blockIdx.y];
    const double2* X = jb.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kThreads / 64;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += kThreads)
            gstore2(T + static_cast<int64_t>(gld(jb.perm + i)) * k + i, make_double2(1.0, 0.0));
    const int c = blockIdx.x * nw + wid;
    if (c >= n - k) return;
    const int pc = gld(jb.perm + k + c);
    const double2 zero = make_double2(0.0, 0.0);
    double2 y[RPL], dinv[RPL];
    int pv[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int i = lane + 64 * s;
        const bool in = i < k;
        y[s] = in ? gload2(X + static_cast<int64_t>(pc) * m + i) : zero;
        const double2 d = in ? gload2(jb.rdiag + i) : make_double2(1.0, 0.0);
        const double id = 1.0 / cabs2(d);
        dinv[s] = make_double2(d.x * id, -d.y * id);
        pv[s] = in ? gld(jb.perm + i) : 0;
    }
    // The reads of U steps are issued before their recurrence (the compiler
    // does not unroll a loop around lane broadcasts by itself).
    constexpr int U = RPL == 4 ? 4 : 8;
#pragma unroll
    for (int s = RPL - 1; s >= 0; --s) {
        for (int j0 = min(63, k - 1 - 64 * s); j0 >= 0; j0 -= U) {   // wave-uniform
            double2 r[U][RPL];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 - u, l = 64 * s + j;
                const double2* xc = X + static_cast<int64_t>(__builtin_amdgcn_readlane(pv[s], j < 0 ? 0 : j)) * m;
#pragma unroll
                for (int t = 0; t <= s; ++t) {
                    const int i = lane + 64 * t;
                    r[u][t] = (j >= 0 && i < l) ? gload2(xc + i) : zero;   // rows i < l < k <= m only
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 - u;
                if (j < 0) break;
                const double2 z = cmul(y[s], dinv[s]);
                const double2 zl = make_double2(readlane_d(z.x, j), readlane_d(z.y, j));
                if (lane == j) y[s] = zl;
                const double2 nz = make_double2(-zl.x, -zl.y);
#pragma unroll
                for (int t = 0; t <= s; ++t) y[t] = cfma(r[u][t], nz, y[t]);   // r is 0 for rows >= l
            }
        }
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int i = lane + 64 * s;
        if (i < k) gstore2(T + static_cast<int64_t>(pc) * k + i, y[s]);
    }
}

template __global__ void k_interp_wave<1>(const CpqrJob*, const int32_t*, const int64_t*, double2*);
template __global__ void k_interp_wave<2>(const CpqrJob*, const int32_t*, const int64_t*, double2*);
template __global__ void k_interp_wave<4>(const CpqrJob*, const int32_t*, const int64_t*, double2*);

// ---------------------------------------------------------------------------
// Batched in-place inverse by Gauss-Jordan elimination with partial row
// pivoting, one workgroup of TG x TG threads per matrix (n <= 4 TG, row-major,
// leading dimension ld).  Thread (ty, tx) keeps the 4 x 4 complex tile of rows
// 4ty.., columns 4tx.. in registers for the whole elimination; a step moves
// one column (for the pivot search and the multipliers) and the pivot row
// through LDS, with two barriers.
//
// Pivoting is logical: rows stay in place, every wave finds the same pivot
// from the same column copy and keeps the same mask of used rows, and the
// permutation is applied on the way out.  With p_k the pivot row of step k the
// in-place result S satisfies  A^-1[k][p_j] = S[p_k][j].  The pivot is the
// unused row of largest |a_ik|^2, compared with the last 7 bits of its binary
// representation replaced by the row index, so that magnitudes within a
// relative 2^-45 count as ties and ties go to the lowest row.  A zero or
// non-finite pivot sets the job's status flag and leaves the block unspecified.
namespace {

template <int TG>
__device__ __forceinline__ void gauss_jordan_tiles(const InvJob& jb) {
    constexpr int NMAX = 4 * TG;
    constexpr int NWORD = (NMAX + 63) / 64;
    static_assert(NMAX <= 128, "row index must fit the 7 low key bits");
    __shared__ double2 colbuf[2][NMAX];
    __shared__ double2 urow[NMAX];
    __shared__ int perm[NMAX], pinv[NMAX];
    __shared__ double wmax[(TG * TG + 63) / 64];
    const int n = jb.n;
    const int64_t ld = jb.ld;
    const int tid = threadIdx.x, ty = tid / TG, tx = tid % TG, lane = tid & 63;
    const int r0 = 4 * ty, c0 = 4 * tx;
    double2 S[4][4];
    double m2 = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = r0 + r, j = c0 + c;
            S[r][c] = (i < n && j < n) ? gload2(jb.a + i * ld + j) : make_double2(0.0, 0.0);
            m2 = fmax(m2, cabs2(S[r][c]));
        }
    if (tx == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) colbuf[0][r0 + r] = S[r][0];
    }
    {
        const int q = wave_argmax_f32(static_cast<float>(m2));
        const double wm = q < 0 ? 0.0 : readlane_d(m2, q);
        if (lane == 0) wmax[tid >> 6] = wm;
    }
    __syncthreads();
    m2 = wmax[0];
    for (int w = 1; w < (TG * TG + 63) / 64; ++w) m2 = fmax(m2, wmax[w]);
    // pivots at or below 64 eps of the block's largest magnitude are singular
    const double tiny2 = (64.0 * 2.220446049250313e-16) * (64.0 * 2.220446049250313e-16) * m2;
    uint64_t used[NWORD];
#pragma unroll
    for (int q = 0; q < NWORD; ++q) used[q] = 0;
    for (int k = 0; k < n; ++k) {
        const double2* col = colbuf[k & 1];
        uint64_t key = 0;
        double2 cv[NWORD];
#pragma unroll
        for (int q = 0; q < NWORD; ++q) {
            const int i = lane + 64 * q;
            cv[q] = i < n ? col[i] : make_double2(0.0, 0.0);
            if (i < n && !((used[q] >> lane) & 1)) {
                const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(cabs2(cv[q])));
                const uint64_t kq = (bits & ~0x7Full) | static_cast<uint64_t>(0x7F - i);
                key = kq > key ? kq : key;
            }
        }
        key = wave_max_u64(key);
        const int p = 0x7F - static_cast<int>(key & 0x7F);
        // the pivot row, unscaled, to LDS first: its readers scale it, so the
        // reciprocal of the pivot is off the path to the barrier
        const int rp = p - r0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r == rp) {
#pragma unroll
                for (int c = 0; c < 4; ++c) urow[c0 + c] = S[r][c];
            }
        // pivot value from the lane that loaded it
        double2 pv = cv[0];
#pragma unroll
        for (int q = 1; q < NWORD; ++q)
            if ((p >> 6) == q) pv = cv[q];
        pv.x = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(pv.x), p & 63),
                                __builtin_amdgcn_readlane(__double2loint(pv.x), p & 63));
        pv.y = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(pv.y), p & 63),
                                __builtin_amdgcn_readlane(__double2loint(pv.y), p & 63));
        const double pd = cabs2(pv);
        if ((key >> 7) == 0 || !(pd > tiny2) || !(pd < INFINITY)) {
            if (tid == 0) gst(jb.status, 1);
            return;   // key and pd are the same in every wave: the whole workgroup leaves
        }
        used[p >> 6] |= 1ull << (p & 63);
        const double rpd = recip(pd);
        const double2 inv = make_double2(pv.x * rpd, -pv.y * rpd);
        if (tid == 0) {
            perm[k] = p;
            pinv[p] = k;
        }
        __syncthreads();
        // multipliers f (column k) and the scaled pivot row u; u[k] = 1/pivot
        double2 f[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f[q] = col[r0 + q];
            u[q] = (c0 + q == k) ? inv : cmul(urow[c0 + q], inv);
        }
        const int ck = k - c0, cn = k + 1 - c0;
        // update the tile column by column (column k becomes -f inv); the
        // owners of column k+1 publish it as soon as it is done, so that its
        // LDS write overlaps the rest of the update
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c == ck) {
#pragma unroll
                for (int r = 0; r < 4; ++r) S[r][c] = make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                S[r][c].x = fma(-f[r].x, u[c].x, fma(f[r].y, u[c].y, S[r][c].x));
                S[r][c].y = fma(-f[r].x, u[c].y, fma(-f[r].y, u[c].x, S[r][c].y));
            }
            if (c == cn) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r == rp) S[r][c] = u[c];
#pragma unroll
                for (int r = 0; r < 4; ++r) colbuf[(k + 1) & 1][r0 + r] = S[r][c];
            }
        }
        // row p becomes u
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r == rp) {
#pragma unroll
                for (int c = 0; c < 4; ++c) S[r][c] = u[c];
            }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = r0 + r;
        if (i >= n) continue;
        double2* out = jb.a + pinv[i] * ld;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c0 + c < n) gstore2(out + perm[c0 + c], S[r][c]);
    }
}

}  // namespace

namespace {

// Gauss-Jordan exchange steps for blocks of up to 64 x 64 with a row per lane:
// a workgroup of NW waves per block, wave w holding the columns
// [w NC, (w + 1) NC) of every row in registers (NC = 64 / NW).  Step j pivots
// on column j: the wave that owns it has chosen the pivot row p (the largest
// |a_ij| among rows not yet used) and published column j and p in LDS, double
// buffered, so one barrier per step suffices.  Each wave then reads its slice
// of row p from lane p (v_readlane, into scalar registers) and applies the
// exchange to its own columns:
//   row p:        a_pc <- a_pc / a_pj,    a_pj <- 1 / a_pj
//   other rows:   a_ic <- a_ic - a_ij a_pc / a_pj,    a_ij <- -a_ij / a_pj
// and the owner of column j + 1 picks the next pivot.  The pivot row's new
// values come from the same fused update with its own old values multiplied
// by zero (so they are rounded once, as a_pc / a_pj).  Rows are not swapped:
// the inverse is written out through the recorded pivot order.  A pivot with
// |a_pj| <= 64 eps max |a| (or none, or not finite) ends the block with
// status 1 after the barrier, every wave leaving together.
template <int NW>
__device__ void gauss_jordan_cols(const InvJob& jb) {
    constexpr int NC = 64 / NW;
    __shared__ double2 colv[2][64];   // column j before its step, by row
    __shared__ int pj[2];             // its pivot row (-1: singular)
    __shared__ int perm[64], pinv[64];
    __shared__ double wmax[NW];
    const int n = jb.n;
    const int64_t ld = jb.ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c0 = wave * NC;
    const bool rowok = lane < n;
    double2 a[NC];
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        a[c] = (rowok && c0 + c < n) ? gload2(jb.a + lane * ld + c0 + c) : make_double2(0.0, 0.0);
        m2 = fmax(m2, cabs2(a[c]));
    }
    {
        const int q = wave_argmax_f32(static_cast<float>(m2));
        const double wm = q < 0 ? 0.0 : readlane_d(m2, q);
        if (lane == 0) wmax[wave] = wm;
    }
    __syncthreads();
    m2 = wmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m2 = fmax(m2, wmax[w]);
    const double tiny2 = (64.0 * 2.220446049250313e-16) * (64.0 * 2.220446049250313e-16) * m2;
    const double rscale = m2 > 0.0 ? recip(m2) : 0.0;
    uint64_t used = 0;   // pivot rows so far (the same value in every thread)
    // the owner of column j chooses its pivot row and publishes column j
    auto choose = [&](const double2 v, const int j, const int b) {
        const bool cand = rowok && !((used >> lane) & 1);
        const float mag = cand ? static_cast<float>(cabs2(v) * rscale) : -1.0f;
        int p = wave_argmax_f32(mag);
        if (p >= 0) {
            const double pd = cabs2(readlane2(v, p));
            if (!(pd > tiny2) || !(pd < INFINITY)) p = -1;
        }
        colv[b][lane] = v;
        if (lane == 0) {
            pj[b] = p;
            if (p >= 0) {
                perm[j] = p;
                pinv[p] = j;
            }
        }
    };
    if (wave == 0) choose(a[0], 0, 0);
    __syncthreads();
    int b = 0;
    for (int j0 = 0; j0 < n; j0 += NC) {
        const int owner = j0 / NC;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int j = j0 + cc;
            if (j >= n) break;
            const int p = __builtin_amdgcn_readfirstlane(pj[b]);
            if (p < 0) {
                if (threadIdx.x == 0) gst(jb.status, 1);
                return;   // every wave read the same p after the barrier
            }
            const double2 f = colv[b][lane];
            const double2 pv = colv[b][p];
            const double rpd = recip(cabs2(pv));
            const double2 inv = make_double2(pv.x * rpd, -pv.y * rpd);
            const bool isp = lane == p;

            // g = a_ij / a_pj for the other rows; -1 / a_pj for row p, whose
            // old values are multiplied by s = 0
            const double2 g = isp ? make_double2(-inv.x, -inv.y) : cmul(f, inv);
            const double s = isp ? 0.0 : 1.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double2 r = readlane2(a[c], p);   // row p of this column
                a[c] = make_double2(fma(-g.x, r.x, fma(g.y, r.y, a[c].x * s)),
                                    fma(-g.x, r.y, fma(-g.y, r.x, a[c].y * s)));
            }
            if (wave == owner) a[cc] = make_double2(-g.x, -g.y);
            used |= 1ull << p;
            b ^= 1;
            if (j + 1 < n) {
                if (cc + 1 < NC) {
                    if (wave == owner) choose(a[cc + 1 < NC ? cc + 1 : 0], j + 1, b);
                } else if (wave == owner + 1) {
                    choose(a[0], j + 1, b);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (rowok && c0 + c < n) gstore2(jb.a + pinv[lane] * ld + perm[c0 + c], a[c]);
}

// One Gauss-Jordan exchange of gauss_jordan_cols on this lane's columns:
// pivot row p, f = this row's value in the pivot column, pv = the pivot; the
// column at register index ownc (-1: none here) becomes -g.
template <int NC>
__device__ __forceinline__ void gj_exchange(double2 (&a)[NC], const int p, const double2 f, const double2 pv,
                                            const int ownc, const int lane) {
    const double rpd = recip(cabs2(pv));
    const double2 inv = make_double2(pv.x * rpd, -pv.y * rpd);
    const bool isp = lane == p;
    const double2 g = isp ? make_double2(-inv.x, -inv.y) : cmul(f, inv);
    const double s = isp ? 0.0 : 1.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double2 r = readlane2(a[c], p);   // row p of this column
        a[c] = make_double2(fma(-g.x, r.x, fma(g.y, r.y, a[c].x * s)),
                            fma(-g.x, r.y, fma(-g.y, r.x, a[c].y * s)));
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c == ownc) a[c] = make_double2(-g.x, -g.y);
}

// The exchanges of gauss_jordan_cols two columns at a time: the wave that owns
// columns j and j + 1 chooses both pivots by itself (column j + 1's pivot from
// a copy of that column with step j applied) and publishes both columns and
// both pivot rows; every wave then applies the two exchanges in turn, and one
// barrier covers two elimination steps.  The copy is made by the same
// arithmetic as the update that follows.  NC = 64 / NW columns per wave
// (even, so that a pair never straddles two waves).
template <int NW>
__device__ void gauss_jordan_pairs(const InvJob& jb) {
    constexpr int NC = 64 / NW;
    static_assert(NC % 2 == 0, "pairs of columns per wave");
    __shared__ double2 colv[2][2][64];   // column j before step j, column j + 1 after it
    __shared__ int pj[2][2];             // their pivot rows (-1: singular; -2: no column j + 1)
    __shared__ int perm[64], pinv[64];
    __shared__ double wmax[NW];
    const int n = jb.n;
    const int64_t ld = jb.ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c0 = wave * NC;
    const bool rowok = lane < n;
    double2 a[NC];
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        a[c] = (rowok && c0 + c < n) ? gload2(jb.a + lane * ld + c0 + c) : make_double2(0.0, 0.0);
        m2 = fmax(m2, cabs2(a[c]));
    }
    {
        const int q = wave_argmax_f32(static_cast<float>(m2));
        const double wm = q < 0 ? 0.0 : readlane_d(m2, q);
        if (lane == 0) wmax[wave] = wm;
    }
    __syncthreads();
    m2 = wmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m2 = fmax(m2, wmax[w]);
    const double tiny2 = (64.0 * 2.220446049250313e-16) * (64.0 * 2.220446049250313e-16) * m2;
    const double rscale = m2 > 0.0 ? recip(m2) : 0.0;
    uint64_t used = 0;   // pivot rows so far (the same value in every thread)
    // the largest candidate of column v (rows below n not in `u`), or -1
    auto pivot_of = [&](const double2 v, const uint64_t u) {
        const bool cand = rowok && !((u >> lane) & 1);
        const float mag = cand ? static_cast<float>(cabs2(v) * rscale) : -1.0f;
        int p = wave_argmax_f32(mag);
        if (p >= 0) {
            const double pd = cabs2(readlane2(v, p));
            if (!(pd > tiny2) || !(pd < INFINITY)) p = -1;
        }
        return p;
    };
    // the owner of columns j, j + 1 (values va, vb in registers) chooses both
    // pivots and publishes them in buffer b
    auto choose2 = [&](const double2 va, const double2 vb, const int j, const int b) {
        const int pa = pivot_of(va, used);
        int pb = -2;
        double2 wb = vb;
        if (pa >= 0 && j + 1 < n) {
            double2 t[1] = {vb};
            gj_exchange<1>(t, pa, va, readlane2(va, pa), -1, lane);
            wb = t[0];
            pb = pivot_of(wb, used | (1ull << pa));
        }
        colv[b][0][lane] = va;
        colv[b][1][lane] = wb;
        if (lane == 0) {
            pj[b][0] = pa;
            pj[b][1] = pb;
            if (pa >= 0) {
                perm[j] = pa;
                pinv[pa] = j;
            }
            if (pb >= 0) {
                perm[j + 1] = pb;
                pinv[pb] = j + 1;
            }
        }
    };
    if (wave == 0) choose2(a[0], a[1], 0, 0);
    __syncthreads();
    int b = 0;
    for (int j0 = 0; j0 < n; j0 += NC) {
        const int owner = j0 / NC;
#pragma unroll
        for (int cc = 0; cc < NC; cc += 2) {
            const int j = j0 + cc;
            if (j >= n) break;
            const int pa = __builtin_amdgcn_readfirstlane(pj[b][0]);
            const int pb = __builtin_amdgcn_readfirstlane(pj[b][1]);
            if (pa < 0 || pb == -1) {
                if (threadIdx.x == 0) gst(jb.status, 1);
                return;   // every wave read the same pivots after the barrier
            }
            gj_exchange<NC>(a, pa, colv[b][0][lane], colv[b][0][pa], wave == owner ? cc : -1, lane);
            used |= 1ull << pa;
            if (pb >= 0) {
                gj_exchange<NC>(a, pb, colv[b][1][lane], colv[b][1][pb], wave == owner ? cc + 1 : -1, lane);
                used |= 1ull << pb;
            }
            b ^= 1;
            if (j + 2 < n) {
                if (cc + 2 < NC) {
                    if (wave == owner) choose2(a[cc + 2 < NC ? cc + 2 : 0], a[cc + 3 < NC ? cc + 3 : 1], j + 2, b);
                } else if (wave == owner + 1) {
                    choose2(a[0], a[1], j + 2, b);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (rowok && c0 + c < n) gstore2(jb.a + pinv[lane] * ld + perm[c0 + c], a[c]);
}

}  // namespace

template <int NW>
__global__ void __launch_bounds__(64 * NW) k_gauss_jordan_cols(const InvJob* __restrict__ jobs) {
    gauss_jordan_cols<NW>(jobs[blockIdx.x]);
}
template __global__ void k_gauss_jordan_cols<8>(const InvJob*);
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_gauss_jordan_pairs(const InvJob* __restrict__ jobs) {
    gauss_jordan_pairs<NW>(jobs[blockIdx.x]);
}
template __global__ void k_gauss_jordan_pairs<8>(const InvJob*);
__global__ void __launch_bounds__(1024) k_gauss_jordan_32(const InvJob* __restrict__ jobs) {
    gauss_jordan_tiles<32>(jobs[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Batched sketch Y = Omega X with a real Omega and complex X (randomized ID:
// the CPQR then runs on the l x n sketch instead of the m x n stacked matrix),
// on the FP64 matrix cores: X is read as a real m x 2n matrix (column 2j the
// real part of complex column j, 2j + 1 its imaginary part), so that Y is one
// real product.  Workgroup: 4 waves (2 x 2) on a 64 x 64 real tile of Y (64
// rows, 32 complex columns); each wave owns 32 x 32 as 2 x 2 blocks of
// 16 x 16, updated by v_mfma_f64_16x16x4f64 (operand layout at gemm_tile
// below).  K runs in stages of 16 rows of X through LDS, the next stage's
// loads in flight during the current stage's products.  With ksplit > 1 the K
// range is cut into ksplit slices of whole 16-row stages, one workgroup per
// (tile, slice), and slice s writes its partial tile to part + s * pstride
// (the levels with few tiles, which would otherwise leave most compute units
// idle); k_sum_partials adds the slices in a fixed order.
namespace {
typedef double v4d_s __attribute__((ext_vector_type(4)));
}  // namespace

__global__ void __launch_bounds__(kThreads)
k_sketch(const SketchJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs,
         const double* __restrict__ omega, int64_t ldo, int ksplit, int64_t pstride) {
    constexpr int TR = 64, TC = 32, KS = 16;   // tile rows, complex columns, K stage
    // k-fast in LDS with rows padded to KS + 1: the stage stores (16 lanes along
    // k) and the fragment reads (16 lanes along rows or columns) then fall on
    // distinct banks
    __shared__ double Os[TR][KS + 1];          // Omega tile by rows
    __shared__ double2 Xs[TC][KS + 1];         // X tile by columns
    int lo = 0, hi = njobs;
    const int64_t tile = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    const SketchJob jb = jobs[lo];
    const int64_t local_s = tile - tile_off[lo];
    const int slice = static_cast<int>(local_s % ksplit);
    const int64_t local = local_s / ksplit;
    const int kc = ((jb.m + ksplit - 1) / ksplit + KS - 1) / KS * KS;
    const int kb = slice * kc, ke = min(jb.m, kb + kc);   // rows [kb, ke) of X, empty for trailing slices
    const int tiles_c = (jb.n + TC - 1) / TC;
    const int r0 = static_cast<int>(local / tiles_c) * TR;
    const int c0 = static_cast<int>(local % tiles_c) * TC;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;   // the wave's rows and real columns in the tile
    const int fl = lane & 15, fk = lane >> 4;
    // stage loads: 16 consecutive threads read 16 consecutive k of one row of
    // Omega (4 rows each) or of one column of X (2 columns each)
    const int lk = tid & 15, lr = tid >> 4;
    double po[4];
    double2 px[2];
    auto load_stage = [&](int l0) {
        const int l = l0 + lk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + lr + 16 * q;
            po[q] = (r < jb.l && l < ke) ? omega[static_cast<int64_t>(r) * ldo + l] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = c0 + lr + 16 * q;
            px[q] = (j < jb.n && l < ke) ? gload2(jb.x + static_cast<int64_t>(j) * jb.m + l) : make_double2(0.0, 0.0);
        }
    };
    v4d_s acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4d_s{0.0, 0.0, 0.0, 0.0};
    if (kb < ke) load_stage(kb);
    for (int l0 = kb; l0 < ke; l0 += KS) {
        __syncthreads();   // the previous stage's fragment reads are done
#pragma unroll
        for (int q = 0; q < 4; ++q) Os[lr + 16 * q][lk] = po[q];
#pragma unroll
        for (int q = 0; q < 2; ++q) Xs[lr + 16 * q][lk] = px[q];
        __syncthreads();
        if (l0 + KS < ke) load_stage(l0 + KS);   // in flight during the products
        const double* xs = reinterpret_cast<const double*>(&Xs[0][0]);
#pragma unroll
        for (int kk = 0; kk < KS; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = Os[wr + 16 * x + fl][kk + fk];
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int rc = wc + 16 * y + fl;   // real column: complex column rc / 2, part rc % 2
                bv[y] = xs[((rc >> 1) * (KS + 1) + kk + fk) * 2 + (rc & 1)];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
        }
    }
    // result register q of lane l: row 4 q + l / 16 of the block, real column
    // l % 16 (complex column (l % 16) / 2, part l % 2)
    double* dst = reinterpret_cast<double*>(ksplit == 1 ? jb.y : jb.part + slice * pstride);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr + 16 * x + 4 * q + fk;
                const int rc = wc + 16 * y + fl;   // real column within the tile
                const int j = c0 + (rc >> 1);
                if (r < jb.l && j < jb.n)
                    gst(dst + 2 * (static_cast<int64_t>(j) * jb.l + r) + (rc & 1), acc[x][y][q]);
            }
}

__global__ void __launch_bounds__(kThreads)
k_sum_partials(const double2* __restrict__ part, int ns, int64_t stride, int64_t len, double2* __restrict__ y) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; e < len;
         e += static_cast<int64_t>(gridDim.x) * kThreads) {
        double2 v = gload2(part + e);
        for (int s = 1; s < ns; ++s) {
            const double2 w = gload2(part + s * stride + e);
            v.x += w.x;
            v.y += w.y;
        }
        gstore2(y + e, v);
    }
}

// ---------------------------------------------------------------------------
// Batched strided complex GEMM on the FP64 matrix cores: C = alpha A B + beta C
// with element (i, j) of X at X[i*rs + j*cs].  A workgroup of NW waves (1, or 4
// as 2 x 2) computes one TT x TT tile of C, TT = WT sqrt(NW); each wave owns a
// WT x WT part of it as (WT/16)^2 blocks of 16 x 16, updated by
// v_mfma_f64_16x16x4f64: per 4-deep step of K and block, four real products
// (re re, -im im into the real part; re im, im re into the imaginary part).
// K runs in chunks of kGemmK through LDS, real and imaginary parts in separate
// arrays, the next chunk's loads issued before the current chunk's products.
// Small tiles give the many small per-box products (and short, wide ones) enough
// waves; the 64 x 64 tiles halve the operand traffic of the large products.
//
// Operand layout of v_mfma_f64_16x16x4f64 (one double per lane; taken from a
// probe on the device that fed unit vectors through every lane pair): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l
// holds D[4 r + l / 16][l % 16].
namespace {
typedef double v4d __attribute__((ext_vector_type(4)));
// K chunk per LDS stage of each tile size
#ifndef BMHSS_GEMM_KC
#define BMHSS_GEMM_KC 16
#endif
constexpr int kGemmK16 = 8, kGemmK32 = 8, kGemmK64 = BMHSS_GEMM_KC;

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int WT, int NW, int kGemmK>
__device__ __forceinline__ void gemm_tile(const GemmJob* __restrict__ jobs, const int64_t* __restrict__ tile_off,
                                          int njobs) {
    constexpr int SQ = NW == 4 ? 2 : 1, TT = WT * SQ, BL = WT / 16, THREADS = 64 * NW;
    constexpr int LOADS = TT * kGemmK / THREADS;   // elements of each operand per thread and chunk
    static_assert(LOADS * THREADS == TT * kGemmK && THREADS % TT == 0, "tile shape");
    // k-major tiles with rows padded by two doubles: the chunk stores of an
    // operand whose k index is contiguous in memory (8 lanes along k, then the
    // next row or column) and the fragment reads (16 lanes along a row) then
    // fall on distinct banks
    __shared__ double Ar[kGemmK][TT + 2], Ai[kGemmK][TT + 2];   // A tile, k-major
    __shared__ double Br[kGemmK][TT + 2], Bi[kGemmK][TT + 2];   // B tile, k-major
    int lo = 0, hi = njobs;
    const int64_t tile = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    const GemmJob g = jobs[lo];
    const int64_t local = tile - tile_off[lo];
    const int tiles_n = (g.N + TT - 1) / TT;
    const int i0 = static_cast<int>(local / tiles_n) * TT;
    const int j0 = static_cast<int>(local % tiles_n) * TT;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w / SQ) * WT, wc = (w % SQ) * WT;   // the wave's part of the tile
    const int fl = lane & 15, fk = lane >> 4;           // fragment row/column and k index
    // chunk loads: consecutive threads along the contiguous index of each operand;
    // element q of a thread is (base index + q * step) of the tile
    const bool a_kfast = g.a_cs == 1, b_kfast = g.b_rs == 1;
    const int ia0 = a_kfast ? tid / kGemmK : tid % TT, ka0 = a_kfast ? tid % kGemmK : tid / TT;
    const int jb0 = b_kfast ? tid / kGemmK : tid % TT, kb0 = b_kfast ? tid % kGemmK : tid / TT;
    const int ia_step = a_kfast ? THREADS / kGemmK : 0, ka_step = a_kfast ? 0 : THREADS / TT;
    const int jb_step = b_kfast ? THREADS / kGemmK : 0, kb_step = b_kfast ? 0 : THREADS / TT;
    double2 pa[LOADS], pb[LOADS];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const int gi = i0 + ia0 + q * ia_step, gk = k0 + ka0 + q * ka_step;
            pa[q] = (gi < g.M && gk < g.K)
                        ? gload2(g.a + static_cast<int64_t>(gi) * g.a_rs + static_cast<int64_t>(gk) * g.a_cs)
                        : make_double2(0.0, 0.0);
            const int gj = j0 + jb0 + q * jb_step, gkb = k0 + kb0 + q * kb_step;
            pb[q] = (gj < g.N && gkb < g.K)
                        ? gload2(g.b + static_cast<int64_t>(gkb) * g.b_rs + static_cast<int64_t>(gj) * g.b_cs)
                        : make_double2(0.0, 0.0);
        }
    };
    v4d accr[BL][BL], acci[BL][BL];
#pragma unroll
    for (int x = 0; x < BL; ++x)
#pragma unroll
        for (int y = 0; y < BL; ++y) {
            accr[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
            acci[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
        }
    load_chunk(0);
    for (int k0 = 0; k0 < g.K; k0 += kGemmK) {
        __syncthreads();   // the previous chunk's fragment reads are done
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            Ar[ka0 + q * ka_step][ia0 + q * ia_step] = pa[q].x;
            Ai[ka0 + q * ka_step][ia0 + q * ia_step] = pa[q].y;
            Br[kb0 + q * kb_step][jb0 + q * jb_step] = pb[q].x;
            Bi[kb0 + q * kb_step][jb0 + q * jb_step] = pb[q].y;
        }
        __syncthreads();
        if (k0 + kGemmK < g.K) load_chunk(k0 + kGemmK);   // in flight during the products
#pragma unroll
        for (int kk = 0; kk < kGemmK; kk += 4) {
            double ar[BL], ai[BL], nai[BL], br[BL], bi[BL];
#pragma unroll
            for (int x = 0; x < BL; ++x) {
                ar[x] = Ar[kk + fk][wr + 16 * x + fl];
                ai[x] = Ai[kk + fk][wr + 16 * x + fl];
                nai[x] = -ai[x];
                br[x] = Br[kk + fk][wc + 16 * x + fl];
                bi[x] = Bi[kk + fk][wc + 16 * x + fl];
            }
#pragma unroll
            for (int x = 0; x < BL; ++x)
#pragma unroll
                for (int y = 0; y < BL; ++y) {
                    accr[x][y] = mfma16(ar[x], br[y], accr[x][y]);
                    accr[x][y] = mfma16(nai[x], bi[y], accr[x][y]);
                    acci[x][y] = mfma16(ar[x], bi[y], acci[x][y]);
                    acci[x][y] = mfma16(ai[x], br[y], acci[x][y]);
                }
        }
    }
    const bool has_beta = g.beta.x != 0.0 || g.beta.y != 0.0;
#pragma unroll
    for (int x = 0; x < BL; ++x)
#pragma unroll
        for (int y = 0; y < BL; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wr + 16 * x + 4 * r + fk, gj = j0 + wc + 16 * y + fl;
                if (gi >= g.M || gj >= g.N) continue;
                double2* cp = g.c + static_cast<int64_t>(gi) * g.c_rs + static_cast<int64_t>(gj) * g.c_cs;
                double2 v = cmul(g.alpha, make_double2(accr[x][y][r], acci[x][y][r]));
                if (has_beta) v = cfma(g.beta, gload2(cp), v);
                gstore2(cp, v);
            }
}
}  // namespace

__global__ void __launch_bounds__(64)
k_gemm_t16(const GemmJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs) {
    gemm_tile<16, 1, kGemmK16>(jobs, tile_off, njobs);
}
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
k_gemm(const GemmJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs) {
    gemm_tile<32, 1, kGemmK32>(jobs, tile_off, njobs);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_gemm_t64(const GemmJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs) {
    gemm_tile<32, 4, kGemmK64>(jobs, tile_off, njobs);
}

// ---------------------------------------------------------------------------
// Gauss-Jordan of one block of n <= 64 by panels of eight columns, the block
// held in LDS.  Wave 0 loads a panel (a row per lane) and runs its eight
// elimination steps on those eight columns alone, with the pivot rule and
// exchange arithmetic of gauss_jordan_cols; the panel then holds W = M E_P
// (M the product of the eight exchanges, E_P the unit columns of the pivot
// rows p_0..p_7), since an exchange fixes every unit vector but its own
// pivot's.  Every other column follows from one rank-8 product,
//   a_new = (a with rows p_k zeroed) + W a[P, :],
// which the eight waves compute on the FP64 matrix cores, a 16-row block of
// two 16-column blocks each (four real products per 4-deep step, the operand
// layout of gemm_tile).  Wave 0 copies the rows p_k, before the product, into
// a buffer of their own, so that the waves need not wait for each other
// between reading them and overwriting the block; the panel's own columns
// are not overwritten.  The eight steps are straight-line code (no branch
// depends on the data): each step updates the next column first, so that the
// next pivot search can overlap the update of the other columns.  Pivoting
// is logical and the result is stored permuted, as in the other kernels; a
// tiny or missing pivot ends the block with status 1 after the barrier,
// leaving the matrix unwritten.
namespace {
constexpr int kGjbLd = 65;   // complex values per LDS row of the block (one of padding)

// The lowest lane holding the wave's largest positive `mag`, or -1 (as
// wave_argmax_f32, without a branch)
__device__ __forceinline__ int wave_argmax_f32_nb(float mag) {
    float m = dpp_fmax<0x111, 0xF>(mag);
    m = dpp_fmax<0x112, 0xF>(m);
    m = dpp_fmax<0x114, 0xF>(m);
    m = dpp_fmax<0x118, 0xF>(m);
    m = dpp_fmax<0x142, 0xA>(m);
    m = dpp_fmax<0x143, 0xC>(m);
    const float mx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 63));
    const uint64_t hit = __builtin_amdgcn_ballot_w64(mag == mx);
    return mx > 0.0f && hit ? static_cast<int>(__builtin_ctzll(hit)) : -1;
}

// PANEL = false: the inverse is stored in place; true: it goes to pt
// (row-major, row stride n) and the block itself becomes the identity (the
// panel inverse's diagonal block, see k_gauss_jordan_blk_panel).
template <bool PANEL>
__device__ __forceinline__ void gauss_jordan_blocked(const InvJob& jb, double2* __restrict__ pt) {
    extern __shared__ double2 gjb_lds[];
    double2* A = gjb_lds;                        // 64 x kGjbLd
    double2* Rb = gjb_lds + 64 * kGjbLd;         // the panel's pivot rows, 8 x 64
    __shared__ int perm[64], pinv[64];
    __shared__ uint64_t pmask_s;
    __shared__ int bad;
    __shared__ double wmax[8];
    const int n = jb.n;
    const int64_t ld = jb.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double m2 = 0.0;
    for (int idx = tid; idx < 64 * 64; idx += 512) {
        const int i = idx >> 6, j = idx & 63;
        const double2 v = (i < n && j < n) ? gload2(jb.a + i * ld + j) : make_double2(0.0, 0.0);
        A[i * kGjbLd + j] = v;
        m2 = fmax(m2, cabs2(v));
    }
    {
        const int q = wave_argmax_f32(static_cast<float>(m2));
        const double wm = q < 0 ? 0.0 : readlane_d(m2, q);
        if (lane == 0) wmax[wave] = wm;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    m2 = wmax[0];
#pragma unroll
    for (int w = 1; w < 8; ++w) m2 = fmax(m2, wmax[w]);
    const double tiny2 = (64.0 * 2.220446049250313e-16) * (64.0 * 2.220446049250313e-16) * m2;
    const double rscale = m2 > 0.0 ? recip(m2) : 0.0;
    const bool rowok = lane < n;
    uint64_t used = 0;   // pivot rows so far (kept by wave 0)
    const int rb = wave & 3, cb0 = 2 * (wave >> 2);   // this wave's output blocks
    const int fl = lane & 15, fk = lane >> 4;
    for (int p0 = 0; p0 < n; p0 += 8) {
        const int np = n - p0 < 8 ? n - p0 : 8;
        if (wave == 0) {
            double2 c[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) c[t] = A[lane * kGjbLd + p0 + t];
            int pk[8];
            bool fail = false;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const bool act = t < np;   // uniform
                const bool cand = rowok && !((used >> lane) & 1);
                const float mag = cand ? static_cast<float>(cabs2(c[t]) * rscale) : -1.0f;
                const int q = wave_argmax_f32_nb(mag);
                const double2 pq = readlane2(c[t], q < 0 ? 0 : q);
                const double pd = cabs2(pq);
                const bool ok = q >= 0 && pd > tiny2 && pd < INFINITY;
                fail = fail || (act && !ok);
                const bool go = act && ok;   // uniform
                const int p = go ? q : 0;
                const double2 pv = go ? pq : make_double2(1.0, 0.0);
                const double rpd = recip(cabs2(pv));
                const double2 inv = make_double2(pv.x * rpd, -pv.y * rpd);
                const bool isp = go && lane == p;
                const double2 g = isp ? make_double2(-inv.x, -inv.y) : (go ? cmul(c[t], inv) : make_double2(0.0, 0.0));
                const double sc = isp ? 0.0 : 1.0;
                // the next column first, then the others; column t becomes -g
#pragma unroll
                for (int k = 1; k < 8; ++k) {
                    const int u = (t + k) & 7;
                    const double2 r = readlane2(c[u], p);
                    c[u] = make_double2(fma(-g.x, r.x, fma(g.y, r.y, c[u].x * sc)),
                                        fma(-g.x, r.y, fma(-g.y, r.x, c[u].y * sc)));
                }
                if (go) c[t] = make_double2(-g.x, -g.y);   // uniform select
                used |= go ? (1ull << p) : 0ull;
                pk[t] = go ? p : -1;
            }
            // the pivot rows' current values (before this panel's product) into
            // their buffer, and W back into the block.  All eight rows are read
            // before anything is written, so that the reads need not wait for
            // the writes; in the panel's columns they are then the values before
            // the steps, which only enter products that the panel does not keep.
            double2 rbv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int q = pk[t] < 0 ? 0 : pk[t];
                rbv[t] = pk[t] < 0 ? make_double2(0.0, 0.0) : A[q * kGjbLd + lane];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) A[lane * kGjbLd + p0 + t] = c[t];
            uint64_t pm = 0;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                Rb[t * 64 + lane] = rbv[t];
                pm |= pk[t] < 0 ? 0ull : (1ull << pk[t]);
            }
            if (lane == 0) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (pk[t] >= 0) {
                        perm[p0 + t] = pk[t];
                        pinv[pk[t]] = p0 + t;
                    }
                pmask_s = pm;
                if (fail) bad = 1;
            }
        }
        __syncthreads();
        if (bad) {
            if (tid == 0) gst(jb.status, 1);
            return;   // every wave read the flag after the barrier
        }
        // the rank-np product: W (the panel's columns) times the pivot rows
        const uint64_t pmask = pmask_s;
        double war[2], wai[2];   // W[16 rb + fl][4 s + fk]
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double2 w = A[(16 * rb + fl) * kGjbLd + p0 + 4 * s + fk];
            war[s] = w.x;
            wai[s] = w.y;
        }
        double br[2][2], bi[2][2];   // [block][s]: row p_{4s+fk}, column 16 cb + fl
        v4d accr[2], acci[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int cb = cb0 + x;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double2 r = Rb[(4 * s + fk) * 64 + 16 * cb + fl];
                br[x][s] = r.x;
                bi[x][s] = r.y;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + 4 * r + fk;
                const double2 cv = A[row * kGjbLd + 16 * cb + fl];
                const bool z = (pmask >> row) & 1;
                accr[x][r] = z ? 0.0 : cv.x;
                acci[x][r] = z ? 0.0 : cv.y;
            }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                accr[x] = mfma16(war[s], br[x][s], accr[x]);
                accr[x] = mfma16(-wai[s], bi[x][s], accr[x]);
                acci[x] = mfma16(war[s], bi[x][s], acci[x]);
                acci[x] = mfma16(wai[s], br[x][s], acci[x]);
            }
            const int col = 16 * (cb0 + x) + fl;
            if (col < p0 || col >= p0 + 8) {   // the panel keeps W
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    A[(16 * rb + 4 * r + fk) * kGjbLd + col] = make_double2(accr[x][r], acci[x][r]);
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < 64 * 64; idx += 512) {
        const int i = idx >> 6, j = idx & 63;
        if (i >= n || j >= n) continue;
        if constexpr (PANEL) {
            gstore2(pt + pinv[i] * n + perm[j], A[i * kGjbLd + j]);
            gstore2(jb.a + i * ld + j, make_double2(i == j ? 1.0 : 0.0, 0.0));
        } else {
            gstore2(jb.a + static_cast<int64_t>(pinv[i]) * ld + perm[j], A[i * kGjbLd + j]);
        }
    }
}
}  // namespace

__global__ void __launch_bounds__(512) k_gauss_jordan_blk(const InvJob* __restrict__ jobs) {
    gauss_jordan_blocked<false>(jobs[blockIdx.x], nullptr);
}

namespace {
// One 64 x 64 tile (rows i0.., columns j0..) of the previous panel's trailing
// update in the panel inverse: rows outside that panel (po, pb) get
// A -= Lp_i Rp_j, its own rows A = Rp (Lp: K x pb row-major with zeros in the
// panel's rows, Rp: pb x K row-major).  Eight waves, each 16 rows by two
// 16-column blocks, the operands read straight from memory (L2) in the
// MFMA layout of gemm_tile, four real products per 4-deep step.
__device__ __forceinline__ void panel_rest_tile(double2* __restrict__ A, int64_t ld, int64_t K, int64_t po, int pb,
                                                const double2* __restrict__ Lp, const double2* __restrict__ Rp,
                                                int64_t i0, int64_t j0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fl = lane & 15, fk = lane >> 4;
    const int64_t r0 = i0 + 16 * (wave & 3), c0 = j0 + 32 * (wave >> 2);
    v4d accr[2], acci[2];
#pragma unroll
    for (int y = 0; y < 2; ++y) accr[y] = acci[y] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t lrow = r0 + fl;
    for (int kc = 0; kc < pb; kc += 16) {
        double2 lv[4], rv[2][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kc + 4 * s + fk;
            lv[s] = (lrow < K && k < pb) ? gload2(Lp + lrow * pb + k) : make_double2(0.0, 0.0);
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int64_t col = c0 + 16 * y + fl;
                rv[y][s] = (col < K && k < pb) ? gload2(Rp + static_cast<int64_t>(k) * K + col) : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                accr[y] = mfma16(lv[s].x, rv[y][s].x, accr[y]);
                accr[y] = mfma16(-lv[s].y, rv[y][s].y, accr[y]);
                acci[y] = mfma16(lv[s].x, rv[y][s].y, acci[y]);
                acci[y] = mfma16(lv[s].y, rv[y][s].x, acci[y]);
            }
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        const int64_t col = c0 + 16 * y + fl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + 4 * r + fk;
            if (row >= K || col >= K) continue;
            double2* a = A + row * ld + col;
            if (row >= po && row < po + pb) {
                gstore2(a, gload2(Rp + (row - po) * K + col));
            } else {
                const double2 v = gload2(a);
                gstore2(a, make_double2(v.x - accr[y][r], v.y - acci[y][r]));
            }
        }
    }
}
}  // namespace

// One panel step of the panel inverse in one launch (panels of 64 columns):
//  - workgroup 0 inverts the diagonal block A[o:o+b, o:o+b] (the blocked
//    Gauss-Jordan, b >= 48), writing the inverse to Pt (b x b) and the
//    identity into the block;
//  - the next ncopy workgroups move the rest of the panel's column block to L
//    (K x b, its rows o..o+b zero) and zero it in A (what k_panel_prep does);
//  - the remaining workgroups, if the previous panel (po >= 0, width pb, its
//    Lp and Rp) is given, apply its trailing update to every column panel but
//    this one, a 64 x 64 tile each (npan panels in all).
// The three touch disjoint parts of A: the block; this panel's columns
// outside it; the other panels' columns.
__global__ void __launch_bounds__(512)
k_gauss_jordan_blk_panel(InvJob diag, double2* __restrict__ A, int64_t ld, int64_t K, int64_t o, int b,
                         double2* __restrict__ L, double2* __restrict__ Pt, int ncopy, int64_t po, int pb,
                         const double2* __restrict__ Lp, const double2* __restrict__ Rp, int npan) {
    if (blockIdx.x == 0) {
        gauss_jordan_blocked<true>(diag, Pt);
        return;
    }
    if (static_cast<int>(blockIdx.x) <= ncopy) {
        const int64_t total = K * b;
        const int64_t stride = static_cast<int64_t>(ncopy) * 512;
        for (int64_t e = static_cast<int64_t>(blockIdx.x - 1) * 512 + threadIdx.x; e < total; e += stride) {
            const int64_t i = e / b;
            const int c = static_cast<int>(e - i * b);
            if (i >= o && i < o + b) {
                gstore2(L + i * b + c, make_double2(0.0, 0.0));
            } else {
                double2* a = A + i * ld + o + c;
                gstore2(L + i * b + c, gload2(a));
                gstore2(a, make_double2(0.0, 0.0));
            }
        }
        return;
    }
    if (po < 0) return;
    const int t = static_cast<int>(blockIdx.x) - 1 - ncopy;   // tile of the previous panel's update
    const int cur = static_cast<int>(o / 64);
    const int I = t / (npan - 1), Jx = t % (npan - 1);
    const int J = Jx < cur ? Jx : Jx + 1;
    panel_rest_tile(A, ld, K, po, pb, Lp, Rp, static_cast<int64_t>(I) * 64, static_cast<int64_t>(J) * 64);
}

// Batched strided complex products with few columns (N <= kGemvMaxN, the
// solves): C = alpha A B + beta C.  With A's rows contiguous (a_cs == 1) one
// wave computes one row of C: its lanes stride along the row and the partial
// sums meet in a butterfly; with A's columns contiguous (a_rs == 1) one thread
// computes one row, so that the lanes read consecutive elements of a column.
// A tile is kGemvRows rows of one job.
__global__ void __launch_bounds__(kThreads)
k_gemv(const GemmJob* __restrict__ jobs, const int64_t* __restrict__ tile_off, int njobs) {
    int lo = 0, hi = njobs;
    const int64_t tile = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    const GemmJob g = jobs[lo];
    const int64_t local = tile - tile_off[lo];
    double2 acc[kGemvMaxN];
#pragma unroll
    for (int j = 0; j < kGemvMaxN; ++j) acc[j] = make_double2(0.0, 0.0);
    int64_t i;
    bool owner;
    if (g.a_cs == 1) {
        const int lane = threadIdx.x & 63;
        i = local * kGemvRows + (threadIdx.x >> 6);
        if (i >= g.M) return;   // the whole wave: no workgroup barrier follows
        const double2* a = g.a + i * g.a_rs;
        for (int k = lane; k < g.K; k += 64) {
            const double2 av = gload2(a + k);
#pragma unroll
            for (int j = 0; j < kGemvMaxN; ++j)
                if (j < g.N) acc[j] = cfma(av, gload2(g.b + k * g.b_rs + j * g.b_cs), acc[j]);
        }
#pragma unroll
        for (int j = 0; j < kGemvMaxN; ++j) {
            acc[j].x = wave_sum(acc[j].x);
            acc[j].y = wave_sum(acc[j].y);
        }
        owner = lane == 0;
    } else {
        i = local * kThreads + threadIdx.x;
        if (i >= g.M) return;
        for (int k = 0; k < g.K; ++k) {
            const double2 av = gload2(g.a + i + k * g.a_cs);
#pragma unroll
            for (int j = 0; j < kGemvMaxN; ++j)
                if (j < g.N) acc[j] = cfma(av, gload2(g.b + k * g.b_rs + j * g.b_cs), acc[j]);
        }
        owner = true;
    }
    if (!owner) return;
#pragma unroll
    for (int j = 0; j < kGemvMaxN; ++j) {
        if (j >= g.N) break;
        double2* cp = g.c + i * g.c_rs + j * g.c_cs;
        double2 r = cmul(g.alpha, acc[j]);
        if (g.beta.x != 0.0 || g.beta.y != 0.0) r = cfma(g.beta, gload2(cp), r);
        gstore2(cp, r);
    }
}

// One panel of the block Gauss-Jordan inverse of a large matrix (K x K,
// leading dimension ld), after its diagonal block A_pp (rows and columns
// [o, o + b)) has been inverted in place: L = A[:, p] with its rows p cleared,
// Pt = A_pp (the inverse), then A[:, p] = 0 off the diagonal block and A_pp = I,
// so that R = Pt A[p, :] holds Pt in its columns p.  L: K x b, Pt: b x b,
// row-major.  Grid-stride over the K x b elements of the panel.
__global__ void __launch_bounds__(kThreads)
k_panel_prep(double2* __restrict__ A, int64_t ld, int64_t K, int64_t o, int b, double2* __restrict__ L,
             double2* __restrict__ Pt) {
    const int64_t total = K * b;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int64_t i = e / b;
        const int c = static_cast<int>(e - i * b);
        double2* a = A + i * ld + o + c;
        const double2 v = gload2(a);
        const bool in_p = i >= o && i < o + b;
        if (in_p) {
            const int r = static_cast<int>(i - o);
            gstore2(Pt + r * b + c, v);
            gstore2(L + i * b + c, make_double2(0.0, 0.0));
            gstore2(a, make_double2(r == c ? 1.0 : 0.0, 0.0));
        } else {
            gstore2(L + i * b + c, v);
            gstore2(a, make_double2(0.0, 0.0));
        }
    }
}

// Strided complex block copy: dst(i, j) = src(i, j) for i < rows, j < cols.
__global__ void __launch_bounds__(kThreads)
k_copy_blocks(const CopyJob* __restrict__ jobs) {
    const CopyJob c = jobs[blockIdx.y];
    const int64_t total = static_cast<int64_t>(c.rows) * c.cols;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int i = static_cast<int>(e / c.cols), j = static_cast<int>(e % c.cols);
        gstore2(c.dst + i * c.dst_rs + j * c.dst_cs, gload2(c.src + i * c.src_rs + j * c.src_cs));
    }
}

}  // namespace hss
}  // namespace bm
