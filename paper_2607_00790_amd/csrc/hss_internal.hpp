// Data structures shared by the HSS kernels and their host driver.
#pragma once

#include "internal.hpp"
#include "wsbm_pair_f32.hpp"

namespace bm {
namespace hss {

constexpr int kThreads = 256;

// Point table of a level: the N boundary nodes followed by the proxy points of
// every box (curve = -1 marks a proxy point); body = the node's body, or the
// body of the box a proxy point belongs to.
struct PointTable {
    double* x;
    double* y;
    double* nx;
    double* ny;
    double* w;
    double* kappa;
    int32_t* curve;
    int32_t* body;
};

// A point with up to two unknowns (u at pos0, q at pos1; -1 when absent).
// Positions index the rows or columns of the block being generated.
struct Slot {
    int32_t pt;
    int32_t pos0;
    int32_t pos1;
};

// Generate A(targets, sources) for slot lists [tslot, tslot + nt) x
// [sslot, sslot + ns); entry (row position r, column position c) goes to
// out[off + r*rs + c*cs] (complex elements).  body >= 0: every point of the
// job belongs to that body; body < 0: each pair takes the body of its node
// points (zero block across bodies).
struct GenJob {
    int64_t tslot;
    int64_t sslot;
    int64_t out;
    int64_t rs;
    int64_t cs;
    int32_t nt;
    int32_t ns;
    int32_t body;   // the body of every point of the job (its media), or -1: per pair
};

struct CpqrState {
    double ref;    // |R_00|
    double beta;   // scale of the current Householder reflector
    int32_t rank;
    int32_t done;
};

// Column-pivoted QR of an m x n column-major complex matrix x (columns are the
// candidate unknowns of a box).  nrm and st are used by the step-wise kernels.
// The step kernels pivot logically and need nrm (2n doubles, double-buffered),
// used (n flags) and st; k_interp also accepts physically pivoted columns
// (used == nullptr).
struct CpqrJob {
    double2* x;
    int32_t* perm;
    double2* rdiag;
    double* nrm;
    int32_t* used;
    CpqrState* st;
    int32_t n;
    int32_t m;
};

struct InvJob {
    double2* a;       // n x n, row-major with leading dimension ld, inverted in place
    int32_t* status;  // set to 1 on a zero pivot (caller zeroes it)
    int64_t ld;
    int32_t n;
};

// C = alpha A B + beta C, element (i, j) of X at X[i*rs + j*cs].
struct GemmJob {
    const double2* a;
    const double2* b;
    double2* c;
    int64_t a_rs, a_cs, b_rs, b_cs, c_rs, c_cs;
    double2 alpha, beta;
    int32_t M, N, K;
};

// Y = Omega X for one box: X (m x n, column j at x + j*m), Omega the leading
// l x m block of a real matrix (row-major, leading dimension ldo), Y (l x n,
// column j at y + j*l).
struct SketchJob {
    const double2* x;
    double2* y;
    double2* part;   // split-K: partial product s of this job at part + s * (partial stride)
    int32_t m, n, l;
};

struct CopyJob {
    const double2* src;
    double2* dst;
    int64_t src_rs, src_cs, dst_rs, dst_cs;
    int32_t rows, cols;
};

__global__ void k_proxy_points(const double* box_c, const int32_t* box_body, const int64_t* poff,
                               const int32_t* pcount, int64_t nnodes, PointTable pt);
// near sets: box b scans the candidate slots [scan_lo[b], scan_hi[b]) (its body's)
__global__ void k_near_count(PointTable pt, const Slot* slots, const int32_t* slot_box,
                             const int64_t* scan_lo, const int64_t* scan_hi, const double* box_c,
                             int64_t* counts);
__global__ void k_near_list(PointTable pt, const Slot* slots, const int32_t* slot_box,
                            const int64_t* scan_lo, const int64_t* scan_hi, const double* box_c,
                            const int64_t* slot_off, Slot* out);
// R = double: FP64 entries; R = float: FP32 arithmetic (ftab: the FP32
// coefficient table), widened to FP64 on store
template <class R>
__global__ void k_gen_jobs(const GenJob* jobs, const int64_t* tile_off, int njobs,
                           const Slot* slots, PointTable pt, const Media* media, double2* out,
                           const BesselTable* tab, const float* ftab);
__global__ void k_interp(const CpqrJob* jobs, const int32_t* ranks, const int64_t* t_off,
                         double2* Tbuf);
// the same for ranks k <= 64 RPL (RPL = 1, 2, 4), logically pivoted jobs only
template <int RPL>
__global__ void k_interp_wave(const CpqrJob* jobs, const int32_t* ranks, const int64_t* t_off,
                              double2* Tbuf);
// in-place inverse of n x n blocks: n <= 64, a row per lane, blockDim 64 NW
// (NW = 8); n <= 128, 4 x 4 register tiles, blockDim 1024
template <int NW>
__global__ void k_gauss_jordan_cols(const InvJob* jobs);
// the same, two elimination steps per barrier
template <int NW>
__global__ void k_gauss_jordan_pairs(const InvJob* jobs);
// the same inverse by panels of eight columns, the block in LDS (dynamic
// shared memory: kGjbLdsBytes), the rank-8 updates on the matrix cores
__global__ void k_gauss_jordan_blk(const InvJob* jobs);
// the panel inverse's step: the diagonal block's inverse into Pt (workgroup 0),
// the panel preparation of k_panel_prep (ncopy workgroups) and the previous
// panel's trailing update (64 x 64 tiles, (npan - 1) npan of them)
__global__ void k_gauss_jordan_blk_panel(InvJob diag, double2* A, int64_t ld, int64_t K, int64_t o, int b,
                                         double2* L, double2* Pt, int ncopy, int64_t po, int pb,
                                         const double2* Lp, const double2* Rp, int npan);
constexpr int kGjbLdsBytes = (64 * 65 + 8 * 64) * 16;
__global__ void k_gauss_jordan_32(const InvJob* jobs);
__global__ void k_cpqr_init(const CpqrJob* jobs);
__global__ void k_cpqr_step(const CpqrJob* jobs, int k, double tol);
// the same step with the trailing columns in registers, for at most 64 R rows;
// each wave takes kCpqrCols consecutive columns (grid: n / (4 kCpqrCols) per
// box).  One column per wave is fastest: at 4 the N = 16384 benchmark build
// took 30 ms instead of 25 (fewer waves in flight per step).
constexpr int kCpqrCols = 1;
template <int R>
__global__ void k_cpqr_step_reg(const CpqrJob* jobs, int k, double tol);
// whole-box CPQR in registers, rows g + 16 t (t < R) of C columns per lane,
// NT threads: n <= kFusedCols columns (C = 4) or kFusedWideCols (C = 5, rows
// up to 160 only: all 256 registers), m <= 16 R rows
constexpr int kFusedThreads = 512;
constexpr int kFusedCols = 4 * kFusedThreads / 16;
constexpr int kFusedWideC = 5;
constexpr int kFusedWideCols = kFusedWideC * kFusedThreads / 16;
template <int R, int C, int NT>
__global__ void k_cpqr_fused(const CpqrJob* jobs, double tol);
__global__ void k_cpqr_finish(const CpqrJob* jobs);
__global__ void k_cpqr_ranks(const CpqrJob* jobs, int nb, int32_t* ranks, int32_t* active);

// batched strided complex GEMM on the FP64 matrix cores, one tile of C per
// workgroup: 16 x 16 (k_gemm_t16, one wave), 32 x 32 (k_gemm, one wave) or
// 64 x 64 (k_gemm_t64, four waves)
__global__ void k_gemm_t16(const GemmJob* jobs, const int64_t* tile_off, int njobs);
__global__ void k_gemm(const GemmJob* jobs, const int64_t* tile_off, int njobs);
__global__ void k_gemm_t64(const GemmJob* jobs, const int64_t* tile_off, int njobs);
// products with at most kGemvMaxN columns whose A has unit row or column stride;
// a tile is kGemvRows rows (wave per row when a_cs == 1) or kThreads rows
constexpr int kGemvMaxN = 4;
constexpr int kGemvRows = kThreads / 64;
__global__ void k_gemv(const GemmJob* jobs, const int64_t* tile_off, int njobs);
// 64 x 64 tiles of Y per workgroup (kThreads threads), the sum over the rows
// of X split into ksplit slices (ksplit > 1: partial products, summed by
// k_sum_partials)
__global__ void k_sketch(const SketchJob* jobs, const int64_t* tile_off, int njobs,
                         const double* omega, int64_t ldo, int ksplit, int64_t pstride);
// y[e] = sum over s < ns of part[s * stride + e], e < len
__global__ void k_sum_partials(const double2* part, int ns, int64_t stride, int64_t len, double2* y);
__global__ void k_copy_blocks(const CopyJob* jobs);
// the panel step of the block Gauss-Jordan inverse (after the diagonal block's
// inverse): L = A[:, p] without rows p, Pt = A_pp, A[:, p] = [0; I; 0]
__global__ void k_panel_prep(double2* A, int64_t ld, int64_t K, int64_t o, int b, double2* L, double2* Pt);

}  // namespace hss
}  // namespace bm
