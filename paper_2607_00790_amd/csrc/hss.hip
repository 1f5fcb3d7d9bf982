// Host driver of the proxy-surface HSS build and solve (C-ABI bm_hss_*).
//
// Tree (paper Sec. III, Fig. 2): a perfect binary tree of contiguous node
// ranges; level l has 2^l boxes, box b covers nodes [b N / 2^l, (b+1) N / 2^l).
// Per compressed level, leaves first:
//   1. box centres/radii (host) and proxy circles        (k_proxy_points)
//   2. near sets: other boxes' active unknowns inside the proxy circle
//                                                        (k_near_count/list)
//   3. M_b = [A(U_b, near) | A(near, U_b)^T | A(U_b, proxy) | A(proxy, U_b)^T]
//      for every box in ONE generation launch            (k_gen_jobs)
//   4. ID of the rows of M_b: CPQR of M_b^T, skeleton J_b, interpolation T_b
//                                                        (k_cpqr_*, k_interp)
//   5. D_b: leaf A(U_b, U_b); above, [[Dhat_a, A(J_a,J_b)], [A(J_b,J_a), Dhat_b]]
//   6. Martinsson-Rokhlin factors Dhat, E, F^T, G        (k_gauss_jordan, k_gemm)
// The reduced system above the last compressed level is inverted densely.
// The host only does index bookkeeping (slot lists, offsets); it reads back the
// near counts and the ranks once per level to size the next buffers.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <vector>

#include <unordered_map>

#include <rocblas/rocblas.h>

#include "hss_internal.hpp"
#include "hss_plan.hpp"
#include "tuned_params.h"

using namespace bm;
using namespace bm::hss;

namespace {

// The factors of one iteration of the build (the boxes compressed together:
// one level of every body's tree that is still compressing), and the offsets
// the solve needs to move between iterations.
struct LevelFactor {
    int nb = 0;
    std::vector<int64_t> n, k;       // unknowns and ranks per box
    std::vector<int64_t> uoff, koff; // prefix sums of n and k
    std::vector<int64_t> nkoff, nnoff;
    int64_t nu = 0, nk = 0;
    std::vector<int64_t> in_off;     // input of the box: in the right-hand side (first
                                     // iteration) or in the previous iteration's F^T output
    std::vector<int64_t> xt_off;     // where the box's skeleton solution is found: in the
    std::vector<int8_t> xt_root;     // next iteration's output (0) or the root solutions (1)
    double2* E = nullptr;   // per box n x k
    double2* Ft = nullptr;  // per box k x n
    double2* G = nullptr;   // per box n x n
};

// The root of one body: its reduced system, inverted densely.
struct RootJob {
    int body;
    int64_t K, r_off, x_off;   // size; inverse at Rinv + r_off; solution at xroot + x_off
    int stage;                 // iteration whose F^T output feeds it (-1: the right-hand side)
    int64_t in_off;            // offset of its input in that vector
    int64_t slot_off;          // its slots in the root slot list
    int32_t nslots;
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Progress lines on stderr during long builds, when the environment variable
// BMHSS_VERBOSE is set to a non-zero value.
bool verbose() {
    static const bool v = [] {
        const char* e = std::getenv("BMHSS_VERBOSE");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return v;
}

template <class... A>
void progress(const char* fmt, A... a) {
    if (!verbose()) return;
    std::fprintf(stderr, fmt, a...);
    std::fflush(stderr);
}

// Pinned host staging chunks are expensive to allocate, so they are kept in
// a process-wide cache and reused by later phases and builds.
struct PinnedCache {
    std::mutex mu;
    std::vector<std::pair<char*, size_t>> free_list;
    char* get(size_t bytes, size_t* cap) {
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < free_list.size(); ++i) {
                if (free_list[i].second >= bytes) {
                    char* p = free_list[i].first;
                    *cap = free_list[i].second;
                    free_list.erase(free_list.begin() + static_cast<std::ptrdiff_t>(i));
                    return p;
                }
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        *cap = bytes;
        return static_cast<char*>(p);
    }
    void put(char* p, size_t cap) {
        std::lock_guard<std::mutex> lk(mu);
        free_list.emplace_back(p, cap);
    }
};
PinnedCache& pinned_cache() {
    static PinnedCache* c = new PinnedCache;   // never destroyed: pinned memory lives until exit
    return *c;
}

// One device-to-host read through a pinned buffer of the cache: a pageable
// destination makes HIP stage the copy and block on it.  read() enqueues the
// copy on s (straight into dst if no pinned buffer is to be had); after the
// caller has synchronised s, finish() moves the bytes to dst.  The buffer goes
// back to the cache on destruction, after s has drained if a copy may still
// be writing it (an error between read() and finish()).
struct PinnedRead {
    hipStream_t s;
    char* p = nullptr;
    size_t cap = 0, bytes = 0;
    void* dst = nullptr;
    bool pending = false;
    explicit PinnedRead(hipStream_t st) : s(st) {}
    PinnedRead(const PinnedRead&) = delete;
    PinnedRead& operator=(const PinnedRead&) = delete;
    hipError_t read(void* d, const void* src, size_t n) {
        dst = d;
        bytes = n;
        p = pinned_cache().get(std::max<size_t>(n, 1), &cap);
        if (!p) return hipMemcpyAsync(d, src, n, hipMemcpyDeviceToHost, s);
        pending = true;
        return hipMemcpyAsync(p, src, n, hipMemcpyDeviceToHost, s);
    }
    void finish() {
        if (p && pending && bytes) std::memcpy(dst, p, bytes);
        pending = false;
    }
    ~PinnedRead() {
        if (!p) return;
        if (pending) (void)hipStreamSynchronize(s);
        pinned_cache().put(p, cap);
    }
};

// Device temporaries, staged descriptor uploads and recorded stream commands
// of one phase of the build or solve.  upload() copies a host array into a
// staging chunk whose device address is known at once; stream work is recorded
// with rec(); flush() issues one host-to-device copy per chunk and then replays
// the recorded commands in order, so a phase costs a handful of copies however
// many small descriptor arrays it uses.  Everything is released after the
// stream has been synchronised.
struct Scratch {
    hipStream_t s;
    std::vector<void*> dev;
    struct Chunk {
        char* d;      // device
        char* h;      // pinned host
        size_t cap, used, flushed;
    };
    std::vector<Chunk> chunks;
    std::vector<std::function<hipError_t()>> cmds;
    bool pending = false;   // copies issued from host staging not yet known complete
    static constexpr size_t kChunk = size_t{1} << 20;

    explicit Scratch(hipStream_t st) : s(st) {}
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    ~Scratch() { release(); }
    template <class T>
    hipError_t alloc(T** p, size_t count) {
        *p = nullptr;
        void* q = nullptr;
        hipError_t e = dev_alloc(&q, std::max<size_t>(count, 1) * sizeof(T), s);
        *p = static_cast<T*>(q);
        if (e == hipSuccess) dev.push_back(q);
        return e;
    }
    template <class T>
    hipError_t upload(T** p, const std::vector<T>& v) {
        const size_t bytes = std::max<size_t>((v.size() * sizeof(T) + 15) / 16 * 16, 16);
        Chunk* c = nullptr;
        for (Chunk& q : chunks)
            if (q.cap - q.used >= bytes) { c = &q; break; }
        if (!c) {
            size_t cap = 0;
            char* hp = pinned_cache().get(std::max(kChunk, bytes), &cap);
            if (!hp) return hipErrorOutOfMemory;
            char* d = nullptr;
            hipError_t e = alloc(&d, cap);
            if (e != hipSuccess) {
                pinned_cache().put(hp, cap);
                return e;
            }
            chunks.push_back(Chunk{d, hp, cap, 0, 0});
            c = &chunks.back();
        }
        if (!v.empty()) std::memcpy(c->h + c->used, v.data(), v.size() * sizeof(T));
        *p = reinterpret_cast<T*>(c->d + c->used);
        c->used += bytes;
        return hipSuccess;
    }
    void rec(std::function<hipError_t()> f) { cmds.push_back(std::move(f)); }
    std::vector<hipEvent_t> events;   // events the recorded commands use, destroyed on release
    bool uses_blas = false;   // a recorded command calls rocBLAS
    bool allow_blas = true;   // false: every product stays in the tile kernel (graph capture)
    // the host-to-device copies of the uploads so far
    hipError_t flush_uploads() {
        for (Chunk& c : chunks) {
            if (c.used > c.flushed) {
                hipError_t e = hipMemcpyAsync(c.d + c.flushed, c.h + c.flushed, c.used - c.flushed,
                                              hipMemcpyHostToDevice, s);
                if (e != hipSuccess) return e;
                c.flushed = c.used;
                pending = true;
            }
        }
        return hipSuccess;
    }
    hipError_t flush() {
        const hipError_t e = flush_uploads();
        if (e != hipSuccess) return e;
        return run_recorded();
    }
    // the recorded commands, in order
    hipError_t run_recorded() {
        for (auto& f : cmds) {
            hipError_t e = f();
            if (e != hipSuccess) {
                cmds.clear();
                return e;
            }
        }
        cmds.clear();
        return hipSuccess;
    }
    // After a stream synchronisation: staging may be reused.
    void synced() { pending = false; }
    // Frees are stream-ordered; the pinned chunks go back to the cache only when
    // no copy from them can still be pending.
    void release() {
        cmds.clear();
        if (pending) (void)hipStreamSynchronize(s);
        pending = false;
        for (void* p : dev) dev_free(p, s);
        dev.clear();
        for (Chunk& c : chunks) pinned_cache().put(c.h, c.cap);
        chunks.clear();
        for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
        events.clear();
    }
};

// A 1D launch may not exceed 2^32 - 1 work-items (2^24 - 1 workgroups of
// kThreads): job lists whose tiles exceed that are launched in groups.
constexpr int64_t kMaxBlocks = int64_t{0xFFFFFFFF} / kThreads;

template <class Job, class Tiles, class Launch>
hipError_t launch_in_groups(const std::vector<Job>& jobs, Tiles tiles, Launch launch) {
    size_t a = 0;
    while (a < jobs.size()) {
        size_t b = a;
        int64_t t = 0;
        while (b < jobs.size() && (b == a || t + tiles(jobs[b]) <= kMaxBlocks)) t += tiles(jobs[b++]);
        if (t > kMaxBlocks) return hipErrorInvalidValue;   // one job alone is too large
        const hipError_t e = launch(std::vector<Job>(jobs.begin() + a, jobs.begin() + b));
        if (e != hipSuccess) return e;
        a = b;
    }
    return hipSuccess;
}

// Per-launch HIP-event timing of the batched GEMM, Gauss-Jordan, sketch and
// entry-generation kernels during a build with opts.kernel_timing set: the
// launchers record an event pair around each launch into the collector of the
// calling build.
struct KernelTimes {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> gemm, inv, sketch, gen;
    double gemm_flops = 0, inv_flops = 0, sketch_flops = 0, gen_pairs = 0;
    ~KernelTimes() {
        for (auto* v : {&gemm, &inv, &sketch, &gen})
            for (auto& pr : *v) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
    }
    static double seconds(const std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
        double t = 0;
        for (auto& pr : v) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) t += ms * 1e-3;
        }
        return t;
    }
};
thread_local KernelTimes* g_ktimes = nullptr;

// an event pair around one launch when the calling build times its kernels
bool timed_pair(std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    if (hipEventCreate(a) != hipSuccess) return false;
    if (hipEventCreate(b) != hipSuccess) {
        (void)hipEventDestroy(*a);
        *a = nullptr;
        return false;
    }
    v.emplace_back(*a, *b);
    return true;
}

hipError_t launch_gen_group(Scratch& sc, const std::vector<GenJob>& jobs, const Slot* slots,
                            const PointTable& pt, const Media* media, const BesselTable* tab, double2* out,
                            const float* ftab);

// `media` is the device media array, `tab` the device coefficient table every
// Media points to (passed to the kernel as an argument of its own).  ftab
// non-null: the jobs are generated in FP32 arithmetic from that FP32 table.
hipError_t launch_gen(Scratch& sc, const std::vector<GenJob>& jobs, const Slot* slots,
                      const PointTable& pt, const Media* media, const BesselTable* tab, double2* out,
                      const float* ftab = nullptr) {
    return launch_in_groups(
        jobs, [](const GenJob& j) { return ceil_div(static_cast<int64_t>(j.nt) * j.ns, kThreads); },
        [&](const std::vector<GenJob>& g) { return launch_gen_group(sc, g, slots, pt, media, tab, out, ftab); });
}

hipError_t launch_gen_group(Scratch& sc, const std::vector<GenJob>& jobs, const Slot* slots,
                            const PointTable& pt, const Media* media, const BesselTable* tab, double2* out,
                            const float* ftab) {
    if (jobs.empty()) return hipSuccess;
    std::vector<int64_t> toff(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j)
        toff[j + 1] = toff[j] + ceil_div(static_cast<int64_t>(jobs[j].nt) * jobs[j].ns, kThreads);
    if (toff.back() == 0) return hipSuccess;
    GenJob* dj;
    int64_t* dt;
    hipError_t e = sc.upload(&dj, jobs);
    if (e == hipSuccess) e = sc.upload(&dt, toff);
    if (e != hipSuccess) return e;
    const unsigned grid = static_cast<unsigned>(toff.back());
    const int nj = static_cast<int>(jobs.size());
    const PointTable ptc = pt;
    hipStream_t st = sc.s;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (g_ktimes && !ftab && timed_pair(g_ktimes->gen, &ea, &eb))
        for (const GenJob& j : jobs) g_ktimes->gen_pairs += static_cast<double>(j.nt) * j.ns;
    sc.rec([=]() {
        if (ea) (void)hipEventRecord(ea, st);
        if (ftab)
            hipLaunchKernelGGL(k_gen_jobs<float>, dim3(grid), dim3(kThreads), 0, st, dj, dt, nj, slots, ptc, media, out,
                               tab, ftab);
        else
            hipLaunchKernelGGL(k_gen_jobs<double>, dim3(grid), dim3(kThreads), 0, st, dj, dt, nj, slots, ptc, media,
                               out, tab, ftab);
        if (eb) (void)hipEventRecord(eb, st);
        return hipGetLastError();
    });
    return hipSuccess;
}

hipError_t launch_gemm_group(Scratch& sc, const std::vector<GemmJob>& jobs);
int gemm_tile_for(const std::vector<GemmJob>& jobs);

hipError_t launch_gemv_group(Scratch& sc, const std::vector<GemmJob>& jobs);
int64_t gemv_tiles(const GemmJob& j);

// rocBLAS handle of the current device, for the large products.
hipError_t blas_handle(rocblas_handle* out) {
    static std::mutex mu;
    static std::unordered_map<int, rocblas_handle> handles;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = handles.find(dev);
    if (it == handles.end()) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return hipErrorInitializationError;
        it = handles.emplace(dev, h).first;
    }
    *out = it->second;
    return hipSuccess;
}

// How the dense root of a one-body problem with at most kRootPanelsMax
// unknowns is inverted: by panels of inv_base() columns (block Gauss-Jordan,
// the default) or by the Schur recursion used for the batched blocks.  BMHSS_ROOT_PANELS=0 selects the
// recursion (for comparison).
constexpr int64_t kRootPanelsMax = 4096;
// largest matrix bm_dense_inverse accepts
constexpr int64_t kDenseInverseMax = 16384;
// bm_interp_decomp: matrices per call (a grid dimension) and rows / columns
constexpr int32_t kInterpDecompMaxBatch = 65535;
constexpr int32_t kInterpDecompMaxDim = 4096;
bool root_panels() {
    static const bool v = [] {
        const char* e = std::getenv("BMHSS_ROOT_PANELS");
        return !(e && std::atoi(e) == 0);
    }();
    return v;
}

// Test hook: with BMHSS_TEST_SINGULAR_ROOT=1 in the environment when a build
// starts, the first row of its (first) dense root is zeroed before the root is
// inverted, so that the build must end with BM_ESINGULAR.
bool singular_root_hook() {
    const char* e = std::getenv("BMHSS_TEST_SINGULAR_ROOT");
    return e && std::atoi(e) == 1;
}

// Tuned parameters (tuned_params.h), overridable through the environment for
// the tuner itself: BMHSS_TUNE_INV_BASE (32, 64 or 128) and
// BMHSS_TUNE_BLAS_FLOPS.
int inv_base() {
    static const int v = [] {
        const char* e = std::getenv("BMHSS_TUNE_INV_BASE");
        const int b = e ? std::atoi(e) : tuned::kInvBase;
        return (b == 32 || b == 64 || b == 128) ? b : tuned::kInvBase;
    }();
    return v;
}

// Gauss-Jordan for blocks up to 64: batches whose largest block has at least
// kGjBlockedMin rows run by panels of eight with the rank-8 updates on the
// matrix cores, smaller ones two elimination steps per barrier (the default,
// BMHSS_TUNE_GJ_PAIRS=1), or one step per barrier for every size
// (BMHSS_TUNE_GJ_PAIRS=0); BMHSS_TUNE_GJ_PAIRS=2 takes the two-step kernel
// for every size.
constexpr int kGjBlockedMin = 48;
int gj_pairs() {
    static const int v = [] {
        const char* e = std::getenv("BMHSS_TUNE_GJ_PAIRS");
        const int q = e ? std::atoi(e) : 1;
        return (q >= 0 && q <= 2) ? q : 1;
    }();
    return v;
}

// LDS requested by each panel step of the panel inverse.  The blocked
// Gauss-Jordan needs 74 KB, which admits two of the launch's workgroups per
// CU: a copy or trailing-update workgroup then shares the inverting
// workgroup's SIMDs and stretches its serial chain (65-67 against 52-54 us
// per panel step on the N = 16384 star's root).  96 KB (more than half of a
// CU's 160 KB) keeps every CU to one workgroup of the launch; the others run
// in more rounds, still within the inversion.  BMHSS_TUNE_PANEL_LDS_KB=0
// requests only the 74 KB, 81..160 another size.
size_t panel_lds_bytes() {
    static const size_t v = [] {
        const char* e = std::getenv("BMHSS_TUNE_PANEL_LDS_KB");
        const int q = e ? std::atoi(e) : 96;
        if (q == 0) return static_cast<size_t>(kGjbLdsBytes);
        return static_cast<size_t>((q >= 81 && q <= 160) ? q : 96) * 1024;
    }();
    return v;
}

// Whole-box CPQR for boxes of 129..160 unknowns (five columns per lane);
// BMHSS_TUNE_CPQR_WIDE=0 leaves them to the step-wise kernels.
bool fused_wide() {
    static const bool v = [] {
        const char* e = std::getenv("BMHSS_TUNE_CPQR_WIDE");
        return !(e && std::atoi(e) == 0);
    }();
    return v;
}

// A product worth a library call: the batched tile kernel runs one 32 x 32
// tile per workgroup without matrix cores, which is fine for the many small
// per-box products but slow for the few large ones (the root inverse's Schur
// recursion, large boxes), where rocBLAS's ZGEMM is used instead.
double blas_flops() {
    static const double v = [] {
        const char* e = std::getenv("BMHSS_TUNE_BLAS_FLOPS");
        const double f = e ? std::atof(e) : tuned::kBlasFlops;
        return f > 0 ? f : tuned::kBlasFlops;
    }();
    return v;
}

bool blas_layout(int64_t rs, int64_t cs, int64_t rows, int64_t cols, rocblas_operation* op, int64_t* ld) {
    // column-major X (rs == 1, ld = cs) or column-major X^T (cs == 1, ld = rs)
    if (rs == 1 && cs >= std::max<int64_t>(rows, 1)) { *op = rocblas_operation_none; *ld = cs; return true; }
    if (cs == 1 && rs >= std::max<int64_t>(cols, 1)) { *op = rocblas_operation_transpose; *ld = rs; return true; }
    return false;
}

// C = alpha A B + beta C through rocBLAS (column-major).  A row-major C is
// computed as C^T = B^T A^T.  Returns false if a stride pattern does not map.
bool blas_job(const GemmJob& g, rocblas_operation* oa, rocblas_operation* ob, int64_t* lda, int64_t* ldb,
              int64_t* ldc, bool* swap) {
    if (g.c_rs == 1 && g.c_cs >= std::max(g.M, 1)) {
        *swap = false;
        *ldc = g.c_cs;
        return blas_layout(g.a_rs, g.a_cs, g.M, g.K, oa, lda) && blas_layout(g.b_rs, g.b_cs, g.K, g.N, ob, ldb);
    }
    if (g.c_cs == 1 && g.c_rs >= std::max(g.N, 1)) {
        // C^T (N x M) = B^T (N x K) A^T (K x M): B^T has strides (b_cs, b_rs), A^T (a_cs, a_rs)
        *swap = true;
        *ldc = g.c_rs;
        return blas_layout(g.b_cs, g.b_rs, g.N, g.K, oa, lda) && blas_layout(g.a_cs, g.a_rs, g.K, g.M, ob, ldb);
    }
    return false;
}

hipError_t launch_gemm(Scratch& sc, const std::vector<GemmJob>& jobs) {
    std::vector<GemmJob> small;
    for (const GemmJob& g : jobs) {
        rocblas_operation oa, ob;
        int64_t lda, ldb, ldc;
        bool swap;
        const double flops = 8.0 * g.M * g.N * g.K;
        if (!sc.allow_blas || flops < blas_flops() || g.M == 0 || g.N == 0 || g.K == 0 || !blas_job(g, &oa, &ob, &lda, &ldb, &ldc, &swap)) {
            small.push_back(g);
            continue;
        }
        rocblas_handle h;
        const hipError_t e = blas_handle(&h);
        if (e != hipSuccess) return e;
        sc.uses_blas = true;
        hipStream_t st = sc.s;
        const GemmJob gj = g;
        sc.rec([=]() {
            if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorLaunchFailure;
            const rocblas_double_complex al(gj.alpha.x, gj.alpha.y), be(gj.beta.x, gj.beta.y);
            const auto* A = reinterpret_cast<const rocblas_double_complex*>(swap ? gj.b : gj.a);
            const auto* B = reinterpret_cast<const rocblas_double_complex*>(swap ? gj.a : gj.b);
            auto* C = reinterpret_cast<rocblas_double_complex*>(gj.c);
            const int64_t m = swap ? gj.N : gj.M, n = swap ? gj.M : gj.N;
            const rocblas_status r = rocblas_zgemm_64(h, oa, ob, m, n, gj.K, &al, A, lda, B, ldb, &be, C, ldc);
            return r == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
        });
    }
    // products with few columns (the solves) go to the matrix-vector kernel
    std::vector<GemmJob> tiled, narrow;
    for (const GemmJob& g : small)
        (g.N <= kGemvMaxN && (g.a_cs == 1 || g.a_rs == 1) ? narrow : tiled).push_back(g);
    hipError_t e = launch_in_groups(
        narrow, gemv_tiles, [&](const std::vector<GemmJob>& g) { return launch_gemv_group(sc, g); });
    if (e != hipSuccess) return e;
    return launch_in_groups(
        tiled, [](const GemmJob& j) { return ceil_div(j.M, 16) * ceil_div(j.N, 16); },
        [&](const std::vector<GemmJob>& g) { return launch_gemm_group(sc, g); });
}

// The tile of the matrix-core GEMM for a launch: 64 x 64 (four waves) when the
// products are large enough to keep the device busy with them (the operands
// are then read half as often), else 32 x 32, else 16 x 16 when even 32 x 32
// tiles would leave most compute units idle (short, wide products such as a
// 64-row panel times the whole root).
int gemm_tile_for(const std::vector<GemmJob>& jobs) {
    int64_t t32 = 0, t64 = 0;
    int mn = INT32_MAX;
    for (const GemmJob& g : jobs) {
        t32 += ceil_div(g.M, 32) * ceil_div(g.N, 32);
        t64 += ceil_div(g.M, 64) * ceil_div(g.N, 64);
        mn = std::min(mn, std::min(g.M, g.N));
    }
    if (mn >= 64 && t64 >= 512) return 64;
    if (t32 >= 512) return 32;
    return 16;
}

int64_t gemv_tiles(const GemmJob& j) {
    return j.a_cs == 1 ? ceil_div(j.M, kGemvRows) : ceil_div(j.M, kThreads);
}

hipError_t launch_gemv_group(Scratch& sc, const std::vector<GemmJob>& jobs) {
    if (jobs.empty()) return hipSuccess;
    std::vector<int64_t> toff(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j) toff[j + 1] = toff[j] + gemv_tiles(jobs[j]);
    if (toff.back() == 0) return hipSuccess;
    GemmJob* dj;
    int64_t* dt;
    hipError_t e = sc.upload(&dj, jobs);
    if (e == hipSuccess) e = sc.upload(&dt, toff);
    if (e != hipSuccess) return e;
    const unsigned grid = static_cast<unsigned>(toff.back());
    const int nj = static_cast<int>(jobs.size());
    hipStream_t st = sc.s;
    sc.rec([=]() {
        hipLaunchKernelGGL(k_gemv, dim3(grid), dim3(kThreads), 0, st, dj, dt, nj);
        return hipGetLastError();
    });
    return hipSuccess;
}

hipError_t launch_gemm_group(Scratch& sc, const std::vector<GemmJob>& jobs) {
    if (jobs.empty()) return hipSuccess;
    const int tt = gemm_tile_for(jobs);
    std::vector<int64_t> toff(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j)
        toff[j + 1] = toff[j] + ceil_div(jobs[j].M, tt) * ceil_div(jobs[j].N, tt);
    if (toff.back() == 0) return hipSuccess;
    GemmJob* dj;
    int64_t* dt;
    hipError_t e = sc.upload(&dj, jobs);
    if (e == hipSuccess) e = sc.upload(&dt, toff);
    if (e != hipSuccess) return e;
    const unsigned grid = static_cast<unsigned>(toff.back());
    const int nj = static_cast<int>(jobs.size());
    hipStream_t st = sc.s;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (g_ktimes && timed_pair(g_ktimes->gemm, &ea, &eb))
        for (const GemmJob& g : jobs) g_ktimes->gemm_flops += 8.0 * g.M * g.N * g.K;
    sc.rec([=]() {
        if (ea) (void)hipEventRecord(ea, st);
        if (tt == 64)
            hipLaunchKernelGGL(k_gemm_t64, dim3(grid), dim3(256), 0, st, dj, dt, nj);
        else if (tt == 32)
            hipLaunchKernelGGL(k_gemm, dim3(grid), dim3(64), 0, st, dj, dt, nj);
        else
            hipLaunchKernelGGL(k_gemm_t16, dim3(grid), dim3(64), 0, st, dj, dt, nj);
        if (eb) (void)hipEventRecord(eb, st);
        return hipGetLastError();
    });
    return hipSuccess;
}

hipError_t launch_copy(Scratch& sc, const std::vector<CopyJob>& jobs) {
    if (jobs.empty()) return hipSuccess;
    CopyJob* dj;
    hipError_t e = sc.upload(&dj, jobs);
    if (e != hipSuccess) return e;
    const unsigned nj = static_cast<unsigned>(jobs.size());
    hipStream_t st = sc.s;
    sc.rec([=]() {
        hipLaunchKernelGGL(k_copy_blocks, dim3(64, nj), dim3(kThreads), 0, st, dj);
        return hipGetLastError();
    });
    return hipSuccess;
}

// The sketching matrix: one real Gaussian matrix per device (fixed seed),
// regenerated larger when a level needs more rows or columns.  Replaced
// buffers are kept, since queued work may still read them.
struct OmegaCache {
    struct Entry { int dev; double* p; int64_t rows, cols; };
    std::mutex mu;
    std::vector<Entry> bufs;
};
OmegaCache& omega_cache() {
    static OmegaCache* c = new OmegaCache;
    return *c;
}

hipError_t omega_device(int64_t rows, int64_t cols, const double** out, int64_t* ld) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    OmegaCache& oc = omega_cache();
    std::lock_guard<std::mutex> lk(oc.mu);
    for (auto it = oc.bufs.rbegin(); it != oc.bufs.rend(); ++it)
        if (it->dev == dev && it->rows >= rows && it->cols >= cols) {
            *out = it->p;
            *ld = it->cols;
            return hipSuccess;
        }
    const int64_t R = std::max<int64_t>(rows, 512), C = std::max<int64_t>(cols, 2048);
    std::vector<double> hbuf(static_cast<size_t>(R * C));
    std::mt19937_64 gen(0x5eedULL + static_cast<uint64_t>(R) * 7919 + static_cast<uint64_t>(C));
    std::normal_distribution<double> nd(0.0, 1.0);
    for (double& v : hbuf) v = nd(gen);
    double* d = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&d), hbuf.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d, hbuf.data(), hbuf.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return e;
    }
    oc.bufs.push_back(OmegaCache::Entry{dev, d, R, C});
    *out = d;
    *ld = C;
    return hipSuccess;
}

hipError_t launch_sketch_group(Scratch& sc, const std::vector<SketchJob>& jobs, const double* omega,
                               int64_t ldo);

hipError_t launch_sketch(Scratch& sc, const std::vector<SketchJob>& jobs, const double* omega, int64_t ldo) {
    return launch_in_groups(
        jobs, [](const SketchJob& j) { return ceil_div(j.l, 64) * ceil_div(j.n, 32); },
        [&](const std::vector<SketchJob>& g) { return launch_sketch_group(sc, g, omega, ldo); });
}

// Workgroups a sketch launch should reach before its K range is split: four
// per compute unit, so that the waves of one unit hide each other's latency.
constexpr int64_t kSketchMinBlocks = 1024;

// The jobs of one group are consecutive in Y (the caller lays Y out in job
// order), so one partial buffer of the group's Y extent serves every slice.
hipError_t launch_sketch_group(Scratch& sc, const std::vector<SketchJob>& jobs_in, const double* omega,
                               int64_t ldo) {
    if (jobs_in.empty()) return hipSuccess;
    std::vector<SketchJob> jobs = jobs_in;
    int64_t tiles = 0, mmax = 0;
    double2* ylo = nullptr;
    double2* yhi = nullptr;
    for (const SketchJob& j : jobs) {
        tiles += ceil_div(j.l, 64) * ceil_div(j.n, 32);
        mmax = std::max<int64_t>(mmax, j.m);
        double2* y1 = j.y + static_cast<int64_t>(j.l) * j.n;
        if (ylo == nullptr || j.y < ylo) ylo = j.y;
        if (yhi == nullptr || y1 > yhi) yhi = y1;
    }
    if (tiles == 0) return hipSuccess;
    // split K while the tiles alone give fewer than kSketchMinBlocks workgroups,
    // keeping at least 64 rows of X per slice
    const int ks = static_cast<int>(std::max<int64_t>(
        1, std::min<int64_t>({kSketchMinBlocks / tiles, ceil_div(mmax, 64), 8})));
    const int64_t pstride = yhi - ylo;
    double2* part = nullptr;
    hipError_t e = hipSuccess;
    if (ks > 1) {
        if ((e = sc.alloc(&part, static_cast<size_t>(ks) * pstride)) != hipSuccess) return e;
        for (SketchJob& j : jobs) j.part = part + (j.y - ylo);
    }
    std::vector<int64_t> toff(jobs.size() + 1, 0);
    for (size_t j = 0; j < jobs.size(); ++j)
        toff[j + 1] = toff[j] + ceil_div(jobs[j].l, 64) * ceil_div(jobs[j].n, 32) * ks;
    SketchJob* dj;
    int64_t* dt;
    e = sc.upload(&dj, jobs);
    if (e == hipSuccess) e = sc.upload(&dt, toff);
    if (e != hipSuccess) return e;
    const unsigned grid = static_cast<unsigned>(toff.back());
    const int nj = static_cast<int>(jobs.size());
    hipStream_t st = sc.s;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (g_ktimes && timed_pair(g_ktimes->sketch, &ea, &eb))
        for (const SketchJob& j : jobs) g_ktimes->sketch_flops += 4.0 * j.l * j.m * j.n;
    sc.rec([=]() {
        if (ea) (void)hipEventRecord(ea, st);
        hipLaunchKernelGGL(k_sketch, dim3(grid), dim3(kThreads), 0, st, dj, dt, nj, omega, ldo, ks, pstride);
        if (ks > 1) {
            const unsigned g2 = static_cast<unsigned>(std::min<int64_t>(ceil_div(pstride, kThreads), 4096));
            hipLaunchKernelGGL(k_sum_partials, dim3(g2), dim3(kThreads), 0, st, part, ks, pstride, pstride, ylo);
        }
        if (eb) (void)hipEventRecord(eb, st);
        return hipGetLastError();
    });
    return hipSuccess;
}

GemmJob gemm(const double2* a, int64_t a_rs, int64_t a_cs, const double2* b, int64_t b_rs,
             int64_t b_cs, double2* c, int64_t c_rs, int64_t c_cs, int64_t M, int64_t N, int64_t K,
             double2 alpha = make_double2(1.0, 0.0), double2 beta = make_double2(0.0, 0.0)) {
    GemmJob g;
    g.a = a; g.b = b; g.c = c;
    g.a_rs = a_rs; g.a_cs = a_cs; g.b_rs = b_rs; g.b_cs = b_cs; g.c_rs = c_rs; g.c_cs = c_cs;
    g.alpha = alpha; g.beta = beta;
    g.M = static_cast<int32_t>(M); g.N = static_cast<int32_t>(N); g.K = static_cast<int32_t>(K);
    return g;
}

// Inversion of a batch of matrices.  Blocks with n <= inv_base() are inverted by
// pivoted Gauss-Jordan, one workgroup each, in a single launch.  Larger
// matrices are split 2 x 2, [[A, B], [C, D]], and inverted through the Schur
// complement S = D - C A^-1 B:
//   X = A^-1 B,  Yt = C A^-1,  B <- -X S^-1,  C <- -S^-1 Yt,  A <- A^-1 - X C,
// with A^-1 and S^-1 found recursively (batched over the whole batch at each
// recursion stage).  Pivoting is within the Gauss-Jordan blocks only.
hipError_t launch_inverse(Scratch& sc, const std::vector<InvJob>& jobs) {
    std::vector<InvJob> base, split;
    int nbase = 0;
    for (const InvJob& j : jobs) {
        if (j.n == 0) continue;
        if (j.n <= inv_base()) {
            base.push_back(j);
            nbase = std::max(nbase, j.n);
        } else {
            split.push_back(j);
        }
    }
    hipError_t e = hipSuccess;
    if (!base.empty()) {
        InvJob* dj;
        if ((e = sc.upload(&dj, base)) != hipSuccess) return e;
        const unsigned nj = static_cast<unsigned>(base.size());
        hipStream_t st = sc.s;
        hipEvent_t ea = nullptr, eb = nullptr;
        if (g_ktimes && timed_pair(g_ktimes->inv, &ea, &eb))
            for (const InvJob& j : base) g_ktimes->inv_flops += 8.0 * j.n * j.n * j.n;
        sc.rec([=]() {
            if (ea) (void)hipEventRecord(ea, st);
            if (nbase <= 64 && nbase >= kGjBlockedMin && gj_pairs() == 1)
                hipLaunchKernelGGL(k_gauss_jordan_blk, dim3(nj), dim3(512), kGjbLdsBytes, st, dj);
            else if (nbase <= 64 && gj_pairs())
                hipLaunchKernelGGL(k_gauss_jordan_pairs<8>, dim3(nj), dim3(512), 0, st, dj);
            else if (nbase <= 64)
                hipLaunchKernelGGL(k_gauss_jordan_cols<8>, dim3(nj), dim3(512), 0, st, dj);
            else
                hipLaunchKernelGGL(k_gauss_jordan_32, dim3(nj), dim3(1024), 0, st, dj);
            if (eb) (void)hipEventRecord(eb, st);
            return hipGetLastError();
        });
    }
    if (split.empty()) return e;
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0), zero = make_double2(0.0, 0.0);
    std::vector<InvJob> Aj, Sj;
    std::vector<int64_t> xoff(split.size() + 1, 0);
    for (size_t q = 0; q < split.size(); ++q) {
        const InvJob& j = split[q];
        const int n1 = j.n / 2, n2 = j.n - n1;
        Aj.push_back(InvJob{j.a, j.status, j.ld, n1});
        Sj.push_back(InvJob{j.a + n1 * j.ld + n1, j.status, j.ld, n2});
        xoff[q + 1] = xoff[q] + static_cast<int64_t>(n1) * n2;
    }
    if ((e = launch_inverse(sc, Aj)) != hipSuccess) return e;
    double2 *X, *Yt;
    if ((e = sc.alloc(&X, xoff.back())) != hipSuccess) return e;
    if ((e = sc.alloc(&Yt, xoff.back())) != hipSuccess) return e;
    std::vector<GemmJob> g1, g2, g3, g4;
    for (size_t q = 0; q < split.size(); ++q) {
        const InvJob& j = split[q];
        const int64_t n1 = j.n / 2, n2 = j.n - n1, ld = j.ld;
        double2 *A = j.a, *B = j.a + n1, *C = j.a + n1 * ld, *D = j.a + n1 * ld + n1;
        double2 *x = X + xoff[q], *yt = Yt + xoff[q];
        g1.push_back(gemm(A, ld, 1, B, ld, 1, x, n2, 1, n1, n2, n1));            // X = A^-1 B
        g1.push_back(gemm(C, ld, 1, A, ld, 1, yt, n1, 1, n2, n1, n1));           // Yt = C A^-1
        g2.push_back(gemm(C, ld, 1, x, n2, 1, D, ld, 1, n2, n2, n1, mone, one)); // S = D - C X
        g3.push_back(gemm(x, n2, 1, D, ld, 1, B, ld, 1, n1, n2, n2, mone, zero)); // B = -X S^-1
        g3.push_back(gemm(D, ld, 1, yt, n1, 1, C, ld, 1, n2, n1, n2, mone, zero)); // C = -S^-1 Yt
        g4.push_back(gemm(x, n2, 1, C, ld, 1, A, ld, 1, n1, n1, n2, mone, one));  // A = A^-1 - X C
    }
    if ((e = launch_gemm(sc, g1)) != hipSuccess) return e;
    if ((e = launch_gemm(sc, g2)) != hipSuccess) return e;
    if ((e = launch_inverse(sc, Sj)) != hipSuccess) return e;
    if ((e = launch_gemm(sc, g3)) != hipSuccess) return e;
    return launch_gemm(sc, g4);
}

// A second stream per device for the look-ahead of the panel inverse
// (non-blocking, default priority, kept for the life of the process).
hipError_t lookahead_stream(hipStream_t* out) {
    static std::mutex mu;
    static std::unordered_map<int, hipStream_t> streams;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it == streams.end()) {
        hipStream_t st = nullptr;
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
        it = streams.emplace(dev, st).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Inversion of one large matrix (the dense root of a one-body problem) by
// block Gauss-Jordan elimination over panels of b = inv_base() columns.  Per
// panel p the diagonal block is inverted in place by the pivoted Gauss-Jordan
// kernel, and with P = A_pp^-1 the rest of the matrix follows from one
// product of rank b:
//   A_pc <- P A_pc,   A_ic <- A_ic - A_ip P A_pc,   A_ip <- -A_ip P   (i, c != p).
// As in the Schur recursion, rows are pivoted within the diagonal blocks only
// (the same elimination, in another order).  Per panel: the diagonal block's
// inverse; k_panel_prep (L = A[:, p] without rows p, Pt = P, A[:, p] =
// [0; I; 0]); R = Pt A[p, :] (which holds P in its columns p); then
// A[i, :] -= L_i R above and below the panel and A[p, :] = I R, products on
// the matrix cores.
// With 64-column panels and the blocked Gauss-Jordan (the default), all of it
// runs on the caller's stream: each panel's one launch inverts its diagonal
// block, moves its column block to L and applies the previous panel's update
// to every column panel but its own; the R product and the next block
// column's update follow, so the next inverse never waits for the rest.
// Otherwise the update is split across two streams (look-ahead): the caller's
// stream updates only the next panel's block column, so the next diagonal
// inverse can start at once, and a second stream updates every other column
// meanwhile; the next panel's R waits for it (it reads the whole row block).
// In both, L and R alternate between two buffers: a buffer is written again
// only after the update that read it is known complete.
hipError_t launch_inverse_panels(Scratch& sc, const InvJob& j) {
    const int64_t K = j.n, ld = j.ld, b0 = std::min<int64_t>(inv_base(), K);
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0), zero = make_double2(0.0, 0.0);
    double2 *L[2], *Pt, *R[2], *eye;
    hipError_t e = hipSuccess;
    for (int q = 0; q < 2; ++q) {
        if ((e = sc.alloc(&L[q], K * b0)) != hipSuccess) return e;
        if ((e = sc.alloc(&R[q], b0 * K)) != hipSuccess) return e;
    }
    if ((e = sc.alloc(&Pt, b0 * b0)) != hipSuccess) return e;
    {
        std::vector<double2> id(static_cast<size_t>(b0 * b0), zero);
        for (int64_t q = 0; q < b0; ++q) id[q * b0 + q] = one;
        if ((e = sc.upload(&eye, id)) != hipSuccess) return e;
    }
    hipStream_t sa = sc.s, sb = nullptr;
    // every product of the panels stays in the library's matrix-core kernel
    struct Restore {
        Scratch& sc;
        bool blas;
        hipStream_t s;
        ~Restore() {
            sc.allow_blas = blas;
            sc.s = s;
        }
    } restore{sc, sc.allow_blas, sc.s};
    sc.allow_blas = false;
    // the update jobs of panel (o, b) for the columns [c0, c1): rows above and
    // below the panel, and the panel's own rows (= R)
    auto update_jobs = [&](std::vector<GemmJob>& jobs, int64_t o, int64_t b, const double2* Lp, const double2* Rp,
                           int64_t c0, int64_t c1) {
        if (c1 <= c0) return;
        const int64_t nc = c1 - c0;
        if (o > 0) jobs.push_back(gemm(Lp, b, 1, Rp + c0, K, 1, j.a + c0, ld, 1, o, nc, b, mone, one));
        if (o + b < K)
            jobs.push_back(gemm(Lp + (o + b) * b, b, 1, Rp + c0, K, 1, j.a + (o + b) * ld + c0, ld, 1, K - o - b, nc,
                                b, mone, one));
        jobs.push_back(gemm(eye, b0, 1, Rp + c0, K, 1, j.a + o * ld + c0, ld, 1, b, nc, b, one, zero));
    };
    if (b0 == 64 && gj_pairs() == 1) {
        // One stream, no events: each panel's launch (k_gauss_jordan_blk_panel)
        // inverts its diagonal block, moves its column block to L and applies
        // the previous panel's trailing update to every other column panel; the
        // R product and the next block column's update follow.  A last panel
        // narrower than the blocked kernel takes the separate launches.
        const int npan = static_cast<int>(ceil_div(K, 64));
        int64_t po = -1;   // the previous panel, whose trailing update is pending
        int pb = 0;
        int buf = 0;
        for (int64_t o = 0; o < K; o += b0, buf ^= 1) {
            const int64_t b = std::min(b0, K - o);
            double2* App = j.a + o * ld + o;
            const InvJob diag{App, j.status, ld, static_cast<int32_t>(b)};
            const double2* Lq = L[buf ^ 1];
            const double2* Rq = R[buf ^ 1];
            if (b >= kGjBlockedMin) {
                double2* a = j.a;
                double2* Lc = L[buf];
                const int ncopy = static_cast<int>(std::min<int64_t>(ceil_div(K * b, 512), 2048));
                const int ntile = po >= 0 ? npan * (npan - 1) : 0;
                const unsigned grid = 1 + static_cast<unsigned>(ncopy + ntile);
                const int bb = static_cast<int>(b);
                const int64_t pq = po;
                const int pw = pb;
                const size_t lds = panel_lds_bytes();
                // timed with the matrix-core products: its work is the trailing
                // update's 8 K^2 pb flops and the inverse's 8 b^3
                hipEvent_t ea = nullptr, eb = nullptr;
                if (g_ktimes && timed_pair(g_ktimes->gemm, &ea, &eb))
                    g_ktimes->gemm_flops += 8.0 * b * b * b + (po >= 0 ? 8.0 * K * K * pb : 0.0);
                sc.rec([=]() {
                    if (ea) (void)hipEventRecord(ea, sa);
                    hipLaunchKernelGGL(k_gauss_jordan_blk_panel, dim3(grid), dim3(512), lds, sa, diag, a, ld,
                                       K, o, bb, Lc, Pt, ncopy, pq, pw, Lq, Rq, npan);
                    if (eb) (void)hipEventRecord(eb, sa);
                    return hipGetLastError();
                });
            } else {
                if (po >= 0) {
                    std::vector<GemmJob> rest;
                    update_jobs(rest, po, pb, Lq, Rq, 0, o);
                    update_jobs(rest, po, pb, Lq, Rq, o + b, K);
                    if ((e = launch_gemm(sc, rest)) != hipSuccess) return e;
                }
                if ((e = launch_inverse(sc, {diag})) != hipSuccess) return e;
                double2* a = j.a;
                double2* Lc = L[buf];
                const unsigned grid = static_cast<unsigned>(std::min<int64_t>(ceil_div(K * b, kThreads), 2048));
                const int bb = static_cast<int>(b);
                sc.rec([=]() {
                    hipLaunchKernelGGL(k_panel_prep, dim3(grid), dim3(kThreads), 0, sa, a, ld, K, o, bb, Lc, Pt);
                    return hipGetLastError();
                });
            }
            if ((e = launch_gemm(sc, {gemm(Pt, b, 1, j.a + o * ld, ld, 1, R[buf], K, 1, b, K, b)})) != hipSuccess)
                return e;
            const int64_t on = o + b, bn = std::min(b0, K - on);   // the next panel
            std::vector<GemmJob> upd;
            update_jobs(upd, o, b, L[buf], R[buf], bn <= 0 ? 0 : on, bn <= 0 ? K : on + bn);
            if ((e = launch_gemm(sc, upd)) != hipSuccess) return e;
            if (bn <= 0) break;
            po = o;
            pb = static_cast<int>(b);
        }
        return hipSuccess;
    }
    if ((e = lookahead_stream(&sb)) != hipSuccess) return e;
    hipEvent_t upd_done = nullptr;   // the second stream's update of the previous panel
    int buf = 0;
    for (int64_t o = 0; o < K; o += b0, buf ^= 1) {
        const int64_t b = std::min(b0, K - o);
        double2* App = j.a + o * ld + o;
        const InvJob diag{App, j.status, ld, static_cast<int32_t>(b)};
        if (b >= kGjBlockedMin && b <= 64 && gj_pairs() == 1) {
            // the diagonal block's inverse and the panel preparation in one launch
            double2* a = j.a;
            double2* Lp = L[buf];
            const unsigned grid = 1 + static_cast<unsigned>(std::min<int64_t>(ceil_div(K * b, 512), 2048));
            const int bb = static_cast<int>(b);
            const size_t lds = panel_lds_bytes();
            hipEvent_t ea = nullptr, eb = nullptr;
            if (g_ktimes && timed_pair(g_ktimes->inv, &ea, &eb)) g_ktimes->inv_flops += 8.0 * b * b * b;
            sc.rec([=]() {
                if (ea) (void)hipEventRecord(ea, sa);
                hipLaunchKernelGGL(k_gauss_jordan_blk_panel, dim3(grid), dim3(512), lds, sa, diag, a, ld, K,
                                   o, bb, Lp, Pt, static_cast<int>(grid - 1), int64_t{-1}, 0,
                                   static_cast<const double2*>(nullptr), static_cast<const double2*>(nullptr), 1);
                if (eb) (void)hipEventRecord(eb, sa);
                return hipGetLastError();
            });
        } else {
            if ((e = launch_inverse(sc, {diag})) != hipSuccess) return e;
            double2* a = j.a;
            double2* Lp = L[buf];
            const unsigned grid = static_cast<unsigned>(std::min<int64_t>(ceil_div(K * b, kThreads), 2048));
            const int bb = static_cast<int>(b);
            sc.rec([=]() {
                hipLaunchKernelGGL(k_panel_prep, dim3(grid), dim3(kThreads), 0, sa, a, ld, K, o, bb, Lp, Pt);
                return hipGetLastError();
            });
        }
        if (upd_done) {
            hipEvent_t ev = upd_done;
            sc.rec([=]() { return hipStreamWaitEvent(sa, ev, 0); });
        }
        if ((e = launch_gemm(sc, {gemm(Pt, b, 1, j.a + o * ld, ld, 1, R[buf], K, 1, b, K, b)})) != hipSuccess) return e;
        const int64_t on = o + b, bn = std::min(b0, K - on);   // the next panel
        if (bn <= 0) {
            std::vector<GemmJob> upd;
            update_jobs(upd, o, b, L[buf], R[buf], 0, K);
            if ((e = launch_gemm(sc, upd)) != hipSuccess) return e;
            break;
        }
        std::vector<GemmJob> next, rest;
        update_jobs(next, o, b, L[buf], R[buf], on, on + bn);
        if ((e = launch_gemm(sc, next)) != hipSuccess) return e;
        hipEvent_t ready = nullptr, done = nullptr;
        if ((e = hipEventCreateWithFlags(&ready, hipEventDisableTiming)) != hipSuccess) return e;
        sc.events.push_back(ready);
        if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) return e;
        sc.events.push_back(done);
        sc.rec([=]() {
            hipError_t r = hipEventRecord(ready, sa);
            if (r == hipSuccess) r = hipStreamWaitEvent(sb, ready, 0);
            return r;
        });
        update_jobs(rest, o, b, L[buf], R[buf], 0, on);
        update_jobs(rest, o, b, L[buf], R[buf], on + bn, K);
        sc.s = sb;   // these products go to the second stream
        e = launch_gemm(sc, rest);
        sc.s = sa;
        if (e != hipSuccess) return e;
        sc.rec([=]() { return hipEventRecord(done, sb); });
        upd_done = done;
    }
    return hipSuccess;
}

// Column-pivoted QR of every box of a level, step-wise over many workgroups
// per box; ranks[] is copied back (the caller synchronises).
// The host does not know when every box has found its rank; it checks (one
// round trip) first after `first_check` steps -- a guess from the previous
// level's ranks -- and then every 16 steps.  Steps launched after a box is done
// return at once.
hipError_t run_cpqr(Scratch& sc, std::vector<CpqrJob>& cj, CpqrJob** dcj_out, int32_t* dranks,
                    double tol, std::vector<int32_t>& ranks, hipEvent_t ev0, hipEvent_t ev1,
                    int64_t* launches, int first_check, bool* fused_out,
                    const std::function<hipError_t()>& before_wait) {
    const int nb = static_cast<int>(cj.size());
    int nmax = 0, kmax = 0;
    for (const CpqrJob& j : cj) {
        nmax = std::max(nmax, j.n);
        kmax = std::max(kmax, std::min(j.n, j.m));
    }
    hipError_t e = hipSuccess;
    double* nrm;
    int32_t* used;
    CpqrState* st;
    int64_t tot = 0;
    for (const CpqrJob& j : cj) tot += j.n;
    if ((e = sc.alloc(&nrm, 2 * tot)) != hipSuccess) return e;
    if ((e = sc.alloc(&used, tot)) != hipSuccess) return e;
    if ((e = sc.alloc(&st, nb)) != hipSuccess) return e;
    int64_t off = 0;
    for (int b = 0; b < nb; ++b) {
        cj[b].nrm = nrm + 2 * off;
        cj[b].used = used + off;
        cj[b].st = st + b;
        off += cj[b].n;
    }
    if ((e = sc.upload(dcj_out, cj)) != hipSuccess) return e;
    CpqrJob* dcj = *dcj_out;
    int32_t* active;
    if ((e = sc.alloc(&active, 1)) != hipSuccess) return e;
    if ((e = sc.flush()) != hipSuccess) return e;
    int mmax = 0;
    for (const CpqrJob& j : cj) mmax = std::max(mmax, j.m);
    // every box small enough for one workgroup's registers: the whole CPQR in one launch
    const int RS = mmax <= 128 ? 8 : mmax <= 144 ? 9 : mmax <= 160 ? 10 : 0;   // rows per lane / 16
    const bool wide = nmax > kFusedCols && nmax <= kFusedWideCols && RS > 0 && fused_wide();
    *fused_out = (nmax <= kFusedCols && RS > 0) || wide;
    if (*fused_out) {
        if ((e = hipEventRecord(ev0, sc.s)) != hipSuccess) return e;
        if (wide) {
            hipLaunchKernelGGL((k_cpqr_fused<10, kFusedWideC, kFusedThreads>), dim3(nb), dim3(kFusedThreads), 0, sc.s,
                               dcj, tol);
        } else {
            switch (RS) {
                case 8: hipLaunchKernelGGL((k_cpqr_fused<8, 4, kFusedThreads>), dim3(nb), dim3(kFusedThreads), 0,
                                           sc.s, dcj, tol); break;
                case 9: hipLaunchKernelGGL((k_cpqr_fused<9, 4, kFusedThreads>), dim3(nb), dim3(kFusedThreads), 0,
                                           sc.s, dcj, tol); break;
                default: hipLaunchKernelGGL((k_cpqr_fused<10, 4, kFusedThreads>), dim3(nb), dim3(kFusedThreads), 0,
                                            sc.s, dcj, tol); break;
            }
        }
        if ((e = hipEventRecord(ev1, sc.s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_cpqr_finish, dim3(nb), dim3(kThreads), 0, sc.s, dcj);
        hipLaunchKernelGGL(k_cpqr_ranks, dim3(1), dim3(64), 0, sc.s, dcj, nb, dranks, active);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = before_wait()) != hipSuccess) return e;
        return hipMemcpyAsync(ranks.data(), dranks, nb * sizeof(int32_t), hipMemcpyDeviceToHost, sc.s);
    }
    const unsigned chunks = static_cast<unsigned>(ceil_div(std::max(nmax, 1), kThreads / 64));
    hipLaunchKernelGGL(k_cpqr_init, dim3(chunks, nb), dim3(kThreads), 0, sc.s, dcj);
    if ((e = hipEventRecord(ev0, sc.s)) != hipSuccess) return e;
    // register-resident columns when every box has at most 64 R rows
    const int R = mmax <= 256 ? 4 : mmax <= 512 ? 8 : mmax <= 1024 ? 16 : mmax <= 2048 ? 32 : 0;
    const unsigned rchunks = static_cast<unsigned>(ceil_div(std::max(nmax, 1), (kThreads / 64) * kCpqrCols));
    for (int k = 0; k <= kmax; ++k) {
        const dim3 grid(R ? rchunks : chunks, nb);
        switch (R) {
            case 4: hipLaunchKernelGGL(k_cpqr_step_reg<4>, grid, dim3(kThreads), 0, sc.s, dcj, k, tol); break;
            case 8: hipLaunchKernelGGL(k_cpqr_step_reg<8>, grid, dim3(kThreads), 0, sc.s, dcj, k, tol); break;
            case 16: hipLaunchKernelGGL(k_cpqr_step_reg<16>, grid, dim3(kThreads), 0, sc.s, dcj, k, tol); break;
            case 32: hipLaunchKernelGGL(k_cpqr_step_reg<32>, grid, dim3(kThreads), 0, sc.s, dcj, k, tol); break;
            default: hipLaunchKernelGGL(k_cpqr_step, grid, dim3(kThreads), 0, sc.s, dcj, k, tol); break;
        }
        ++*launches;
        if (k == 0 && (e = before_wait()) != hipSuccess) return e;
        if (k >= first_check && (k - first_check) % 16 == 0 && k < kmax) {
            int32_t h_active = 1;
            hipLaunchKernelGGL(k_cpqr_ranks, dim3(1), dim3(64), 0, sc.s, dcj, nb, dranks, active);
            e = hipMemcpyAsync(&h_active, active, sizeof(int32_t), hipMemcpyDeviceToHost, sc.s);
            if (e == hipSuccess) e = hipStreamSynchronize(sc.s);
            if (e != hipSuccess) return e;
            sc.synced();
            if (h_active == 0) break;
        }
    }
    if ((e = hipEventRecord(ev1, sc.s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cpqr_finish, dim3(nb), dim3(kThreads), 0, sc.s, dcj);
    hipLaunchKernelGGL(k_cpqr_ranks, dim3(1), dim3(64), 0, sc.s, dcj, nb, dranks, active);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipMemcpyAsync(ranks.data(), dranks, nb * sizeof(int32_t), hipMemcpyDeviceToHost, sc.s);
    return e;
}

// Slots of an unknown list (global unknown ids): one slot per node in order of
// first appearance, with the positions of its u / q unknowns in the list.  The
// node -> slot map is a flat array kept across calls (entries reset after use),
// so a call costs O(list length) with no allocation.
void make_slots(const std::vector<int32_t>& U, std::vector<Slot>& out) {
    thread_local std::vector<int32_t> slot_of;   // node -> slot index, -1 when unseen
    int32_t top = -1;
    for (int32_t u : U) top = std::max(top, u >> 1);
    if (static_cast<int64_t>(slot_of.size()) <= top) slot_of.resize(static_cast<size_t>(top) + 1, -1);
    const size_t first = out.size();
    for (size_t p = 0; p < U.size(); ++p) {
        const int32_t node = U[p] >> 1;
        const int comp = U[p] & 1;
        int32_t si = slot_of[node];
        if (si < 0) {
            out.push_back(Slot{node, -1, -1});
            si = static_cast<int32_t>(out.size() - 1);
            slot_of[node] = si;
        }
        if (comp == 0) out[si].pos0 = static_cast<int32_t>(p);
        else out[si].pos1 = static_cast<int32_t>(p);
    }
    for (size_t q = first; q < out.size(); ++q) slot_of[out[q].pt] = -1;
}

int count_unknowns(const Slot* s, size_t n) {
    int c = 0;
    for (size_t i = 0; i < n; ++i) c += (s[i].pos0 >= 0) + (s[i].pos1 >= 0);
    return c;
}

}  // namespace

// Library streams (non-blocking, default priority) are costly to create and
// destroy (hundreds of microseconds each on this runtime), so they are kept in
// a per-device pool: the build's second stream and the capture stream of each
// recorded solve come from it and go back to it.
hipError_t aux_stream_get(hipStream_t* out);
void aux_stream_put(hipStream_t st);

struct bm_hss {
    const bm_problem* p = nullptr;
    hipStream_t stream = nullptr;   // build stream: the factors' memory is tied to it
    bm_hss_opts opts{};
    int64_t N = 0;
    int levels = 0;
    std::vector<LevelFactor> lv;   // compressed iterations, leaves first
    std::vector<RootJob> roots;    // one per body
    int64_t Ktot = 0;              // total size of the roots
    int32_t guard_stops = 0;       // bodies the ID work guard stopped
    double2* Rinv = nullptr;       // the roots' inverses, packed
    bm_hss_stats_t stats{};
    std::vector<bm_hss_level_t> level_info;   // per compressed level, leaves first
    // captured solves (bm_hss_solve_graph), one per (nrhs, transpose)
    struct SolvePlan {
        int64_t nrhs = 0;
        bool trans = false;
        std::unique_ptr<Scratch> sc;      // device buffers and job descriptors of the graph
        double* bin = nullptr;            // the graph's input and output, 2N x nrhs complex
        double* xout = nullptr;
        hipStream_t cap = nullptr;        // capture stream
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t done = nullptr;        // recorded after every launch of the graph
        ~SolvePlan() {
            if (done) {
                (void)hipEventSynchronize(done);
                (void)hipEventDestroy(done);
            }
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (sc) {
                if (cap) (void)hipStreamSynchronize(cap);
                sc->release();
                sc.reset();
            }
            if (cap) aux_stream_put(cap);
        }
    };
    mutable std::mutex plan_mu;
    mutable std::vector<std::unique_ptr<SolvePlan>> plans;
};

namespace {

// Persistent buffers come from the caching allocator on the build stream and
// go back to it on that stream.
template <class T>
hipError_t palloc(T** p, int64_t count, hipStream_t s) {
    void* q = nullptr;
    hipError_t e = dev_alloc(&q, static_cast<size_t>(std::max<int64_t>(count, 1)) * sizeof(T), s);
    *p = static_cast<T*>(q);
    return e;
}

void free_factor(LevelFactor& f, hipStream_t s) {
    dev_free(f.E, s);
    dev_free(f.Ft, s);
    dev_free(f.G, s);
    f.E = f.Ft = f.G = nullptr;
}

struct EventTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipError_t start(Scratch& sc, hipEvent_t& a) {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) {
            hipStream_t st = sc.s;
            hipEvent_t ea = a;
            sc.rec([=]() { return hipEventRecord(ea, st); });
        }
        return e;
    }
    hipError_t stop(Scratch& sc, hipEvent_t a) {
        hipEvent_t b;
        hipError_t e = hipEventCreate(&b);
        if (e == hipSuccess) {
            hipStream_t st = sc.s;
            sc.rec([=]() { return hipEventRecord(b, st); });
            ev.emplace_back(a, b);
        }
        return e;
    }
    double seconds() {
        double t = 0;
        for (auto& pr : ev) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) t += ms * 1e-3;
        }
        return t;
    }
    ~EventTimer() {
        for (auto& pr : ev) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    }
};

// Second stream of a build: the factorisation of level l runs on it while
// the compression of level l+1 proceeds on the caller's stream (the ID of a
// level needs only the skeletons of the level below, not its factors).  The
// streams are non-blocking, default priority, and kept per device for reuse.
struct AuxStreams {
    std::mutex mu;
    std::vector<std::pair<int, hipStream_t>> free_list;
    hipError_t get(hipStream_t* out) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < free_list.size(); ++i)
                if (free_list[i].first == dev) {
                    *out = free_list[i].second;
                    free_list.erase(free_list.begin() + static_cast<std::ptrdiff_t>(i));
                    return hipSuccess;
                }
        }
        return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
    }
    void put(hipStream_t st) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        std::lock_guard<std::mutex> lk(mu);
        free_list.emplace_back(dev, st);
    }
};
AuxStreams& aux_streams() {
    static AuxStreams* a = new AuxStreams;
    return *a;
}
}  // namespace

hipError_t aux_stream_get(hipStream_t* out) { return aux_streams().get(out); }
void aux_stream_put(hipStream_t st) { aux_streams().put(st); }

namespace {

// Buffers of a level whose factorisation may still be running on the second
// stream: the compression scratch (T, slot lists, read by the factorisation)
// and the factorisation's own temporaries.  Released once `done` has fired.
struct PendingLevel {
    std::unique_ptr<Scratch> cmp, fac;
    hipEvent_t ready = nullptr, done = nullptr;
    bool flushed = true;   // false while fac's recorded commands wait to be issued
};

struct Pipeline {
    hipStream_t s, s2 = nullptr;
    std::vector<PendingLevel> pending;
    explicit Pipeline(hipStream_t st) : s(st) {}
    // release the levels whose factorisation has completed (all of them if wait)
    void reap(bool wait) {
        for (size_t i = 0; i < pending.size();) {
            PendingLevel& pl = pending[i];
            if (!pl.flushed) { ++i; continue; }   // its done event is not even recorded yet
            bool fin = true;
            if (pl.done) {
                const hipError_t q = wait ? hipEventSynchronize(pl.done) : hipEventQuery(pl.done);
                fin = (q == hipSuccess) || (wait && q != hipErrorNotReady);
            }
            if (!fin) { ++i; continue; }
            if (pl.cmp) { pl.cmp->pending = false; pl.cmp->release(); }
            if (pl.fac) { pl.fac->pending = false; pl.fac->release(); }
            if (pl.ready) (void)hipEventDestroy(pl.ready);
            if (pl.done) (void)hipEventDestroy(pl.done);
            pending.erase(pending.begin() + static_cast<std::ptrdiff_t>(i));
        }
    }
    ~Pipeline() {
        if (s2) (void)hipStreamSynchronize(s2);
        (void)hipStreamSynchronize(s);
        reap(true);
        if (s2) aux_streams().put(s2);
    }
};

// One body's state during the forest build.
struct BodyState {
    int64_t nlo = 0, nn = 0;   // node range [nlo, nlo + nn)
    int L = 0;                 // depth of its tree: the leaves are level L
    int level = 0;             // level of its current boxes
    bool active = true;        // still compressing (no root yet)
    std::vector<std::vector<int32_t>> U;   // active unknowns (global ids) per current box
    std::vector<int64_t> split_slots;      // per current box above the leaves: slots of the first child
    int iter_prev = -1;        // last iteration that compressed this body's boxes
    double last_ratio = 0;     // skeleton unknowns / unknowns over its boxes at that iteration
    int kept_prev = -1;        // index of its first box among that iteration's boxes
    std::vector<std::vector<double>> box_c;   // per level: centre x, y and proxy radius per box
    std::vector<std::vector<int32_t>> box_p;  // per level: proxy points per box
};

hipError_t record_solve(const bm_hss* h, Scratch& sc, const double* b, double* x, int64_t nrhs, bool trans);

// The captured solve of bm_hss_solve_graph for (nrhs, trans): record the
// solve on a capture stream, upload its job descriptors once, and capture its
// launches into a graph, appended to h->plans (the caller holds plan_mu, or
// is the build).  Needs the factors' addresses only, not their values.  On
// failure *where names the step.
hipError_t make_solve_plan(const bm_hss* h, int64_t nrhs, bool trans, bm_hss::SolvePlan** out, const char** where) {
    *out = nullptr;
    auto q = std::make_unique<bm_hss::SolvePlan>();
    q->nrhs = nrhs;
    q->trans = trans;
    *where = "bm_hss_solve_graph: stream";
    hipError_t e = aux_stream_get(&q->cap);
    if (e != hipSuccess) return e;
    q->sc = std::make_unique<Scratch>(q->cap);
    Scratch& sc = *q->sc;
    sc.allow_blas = false;   // library calls are not captured; the tile kernel runs every product
    double2 *bi = nullptr, *xo = nullptr;
    e = sc.alloc(&bi, static_cast<size_t>(2 * h->N * nrhs));
    if (e == hipSuccess) e = sc.alloc(&xo, static_cast<size_t>(2 * h->N * nrhs));
    q->bin = reinterpret_cast<double*>(bi);
    q->xout = reinterpret_cast<double*>(xo);
    *where = "bm_hss_solve_graph: record";
    if (e == hipSuccess) e = record_solve(h, sc, q->bin, q->xout, nrhs, q->trans);
    if (e != hipSuccess) return e;
    if (sc.uses_blas) return hipErrorNotSupported;   // cannot happen: allow_blas is off
    *where = "bm_hss_solve_graph: upload";
    e = sc.flush_uploads();
    if (e == hipSuccess) e = hipStreamSynchronize(q->cap);
    sc.synced();
    if (e != hipSuccess) return e;
    *where = "bm_hss_solve_graph: capture";
    e = hipStreamBeginCapture(q->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t er = sc.run_recorded();
    e = hipStreamEndCapture(q->cap, &q->graph);
    if (er != hipSuccess) return er;
    if (e != hipSuccess) return e;
    *where = "bm_hss_solve_graph: instantiate";
    if ((e = hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&q->done, hipEventDisableTiming)) != hipSuccess) return e;
    h->plans.push_back(std::move(q));
    *out = h->plans.back().get();
    return hipSuccess;
}

int build_impl(bm_hss* h, hipStream_t s) {
    const bm_problem* p = h->p;
    const bm_geom* g = p->g;
    const int64_t N = g->n;
    const int P = static_cast<int>(h->opts.proxy_points);
    const double tol = h->opts.id_tol;
    const int nbodies = p->nbodies;
    EventTimer t_gen, t_cmp, t_fac;
    const auto t_build0 = std::chrono::steady_clock::now();

    // bodies and their trees
    std::vector<BodyState> bodies(nbodies);
    int64_t leaf_boxes = 0;
    int Lmax = 0;
    for (int q = 0; q < nbodies; ++q) {
        BodyState& B = bodies[q];
        B.nlo = p->body_lo[q];
        B.nn = p->body_lo[q + 1] - p->body_lo[q];
        while ((B.nn >> (B.L + 1)) >= h->opts.leaf && B.L < 30) ++B.L;
        B.level = B.L;
        Lmax = std::max(Lmax, B.L);
        const int64_t nb = int64_t{1} << B.L;
        leaf_boxes += nb;
        B.U.resize(nb);
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t lo = B.nlo + ((b * B.nn) >> B.L), hi = B.nlo + (((b + 1) * B.nn) >> B.L);
            for (int64_t i = lo; i < hi; ++i) {
                B.U[b].push_back(static_cast<int32_t>(2 * i));
                B.U[b].push_back(static_cast<int32_t>(2 * i + 1));
            }
        }
    }
    h->levels = Lmax;

    // box centres (node means), proxy radii (proxy_ratio x the largest node
    // distance) and proxy counts of one level of one body, from the nodes
    // (kept on the host by the geometry).  Each level costs a pass over the
    // body's nodes, so a level is computed when the build first needs it: the
    // leaves now, every other level while the GPU runs the previous level's
    // ID (or all of them now when the proxy counts depend on the radii, which
    // the point table's size needs).
    std::vector<double> hxy_copy;
    const double* hx = g->host_xy.data();
    if (static_cast<int64_t>(g->host_xy.size()) != 2 * N) {
        hxy_copy.resize(2 * static_cast<size_t>(N));
        BM_HIP(hipMemcpyAsync(hxy_copy.data(), g->soa, 2 * N * sizeof(double), hipMemcpyDeviceToHost, s));
        BM_HIP(hipStreamSynchronize(s));
        hx = hxy_copy.data();
    }
    const double* hy = hx + N;
    auto level_geometry = [&](int q, int l) {
        BodyState& B = bodies[q];
        if (l < 1 || l > B.L || !B.box_c[l].empty()) return;
        const double kmax = std::max(p->media[q].k0, p->media[q].k1);
        const int64_t nb = int64_t{1} << l;
        B.box_c[l].resize(3 * nb);
        B.box_p[l].resize(nb);
        level_box_geometry(hx, hy, B.nlo, B.nn, l, h->opts.proxy_ratio, P, h->opts.proxy_adapt != 0, kmax,
                           B.box_c[l].data(), B.box_p[l].data());
    };
    std::vector<int64_t> proxies_at(Lmax + 1, 0);   // proxy points of iteration t (upper bound)
    for (int q = 0; q < nbodies; ++q) {
        BodyState& B = bodies[q];
        B.box_c.resize(B.L + 1);
        B.box_p.resize(B.L + 1);
        for (int l = 1; l <= B.L; ++l) {
            const int64_t nb = int64_t{1} << l;
            if (h->opts.proxy_adapt || l == B.L) {
                level_geometry(q, l);
                for (int64_t b = 0; b < nb; ++b) proxies_at[B.L - l] += B.box_p[l][b];
            } else {
                proxies_at[B.L - l] += nb * std::min<int64_t>(P, int64_t{1} << 20);
            }
        }
    }
    int64_t max_proxies = 0;
    for (int64_t v : proxies_at) max_proxies = std::max(max_proxies, v);

    // point table: nodes, then the proxy points of the boxes of the current iteration
    const int64_t npts = N + max_proxies;
    PointTable pt{};
    double* ptd = nullptr;
    Scratch persist(s);   // point table: freed (stream-ordered) when the build returns
    BM_HIP(persist.alloc(&ptd, 6 * npts));
    int32_t* ptc = nullptr;
    BM_HIP(persist.alloc(&ptc, 2 * npts));
    pt.x = ptd; pt.y = ptd + npts; pt.nx = ptd + 2 * npts; pt.ny = ptd + 3 * npts;
    pt.w = ptd + 4 * npts; pt.kappa = ptd + 5 * npts; pt.curve = ptc; pt.body = ptc + npts;
    for (int r = 0; r < 6; ++r)
        BM_HIP(hipMemcpyAsync(ptd + r * npts, g->soa + r * N, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    BM_HIP(hipMemcpyAsync(ptc, g->curve, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (p->d_body)
        BM_HIP(hipMemcpyAsync(pt.body, p->d_body, N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    else
        BM_HIP(hipMemsetAsync(pt.body, 0, N * sizeof(int32_t), s));
    // declared after the point table: on every return it first drains both
    // streams, so the table outlives the factorisation kernels that read it
    Pipeline pl(s);
    BM_HIP(aux_streams().get(&pl.s2));
    const hipStream_t s2 = pl.s2;
    // a level's factorisation recorded but not yet issued (at most one)
    Scratch* deferred_fac = nullptr;
    const std::function<hipError_t()> flush_deferred = [&]() -> hipError_t {
        if (!deferred_fac) return hipSuccess;
        Scratch* f = deferred_fac;
        deferred_fac = nullptr;
        for (PendingLevel& q : pl.pending)
            if (q.fac.get() == f) q.flushed = true;
        return f->flush();
    };

    std::vector<double2*> dhat;             // per iteration: Dhat of every kept box (k x k, packed)
    std::vector<std::vector<int64_t>> dhat_off;
    std::vector<int32_t*> status_bufs;
    std::vector<int64_t> status_cnt;    // entries of each status buffer
    int64_t status_tot = 0;
    int32_t* status_host = nullptr;     // pinned copy of every status
    size_t status_cap = 0;
    auto cleanup = [&]() {
        for (auto q : status_bufs) dev_free(q, s2);
        status_bufs.clear();
        for (auto q : dhat) dev_free(q, s2);
        dhat.clear();
        if (status_host) {
            (void)hipStreamSynchronize(s2);   // no copy into it may be pending
            pinned_cache().put(reinterpret_cast<char*>(status_host), status_cap);
            status_host = nullptr;
        }
    };
    int64_t entries = 0, pairs = 0, max_rank = 0, cpqr_launches = 0, cpqr_fused_launches = 0;
    double cpqr_bytes = 0, cpqr_fused_bytes = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> cpqr_events;
    std::vector<bool> cpqr_fused;   // per entry of cpqr_events: the whole-box kernel ran
    struct EventPairs {   // destroyed on every return
        std::vector<std::pair<hipEvent_t, hipEvent_t>>& v;
        ~EventPairs() {
            for (auto& pr : v) {
                if (pr.first) (void)hipEventDestroy(pr.first);
                if (pr.second) (void)hipEventDestroy(pr.second);
            }
        }
    } cpqr_events_guard{cpqr_events};

    // roots
    std::vector<RootJob> roots;
    std::vector<Slot> root_slots;
    std::vector<CopyJob> root_copies;   // Dhat blocks on the roots' diagonals
    std::vector<int64_t> root_copy_dst; // their offsets in the packed root inverses
    int64_t Ktot = 0, Rtot = 0;
    auto make_root = [&](int q) {
        BodyState& B = bodies[q];
        RootJob r{};
        r.body = q;
        std::vector<int32_t> Ur;
        for (auto& u : B.U) Ur.insert(Ur.end(), u.begin(), u.end());
        r.K = static_cast<int64_t>(Ur.size());
        r.r_off = Rtot;
        r.x_off = Ktot;
        Rtot += r.K * r.K;
        Ktot += r.K;
        r.stage = B.iter_prev;
        r.slot_off = static_cast<int64_t>(root_slots.size());
        make_slots(Ur, root_slots);
        r.nslots = static_cast<int32_t>(root_slots.size() - r.slot_off);
        if (B.iter_prev >= 0) {
            // the root is made of the skeletons of the boxes compressed last: two
            // children per current box, U(box) = J(child 0) then J(child 1)
            LevelFactor& F = h->lv[B.iter_prev];
            r.in_off = F.koff[B.kept_prev];
            int64_t off = 0;
            for (size_t c = 0; c < 2 * B.U.size(); ++c) {
                const int kb = B.kept_prev + static_cast<int>(c);
                const int64_t kc = F.k[kb];
                // source Dhat, destination offset in the root's inverse (pointer added later)
                root_copies.push_back(CopyJob{dhat[B.iter_prev] + dhat_off[B.iter_prev][kb], nullptr, kc, 1, r.K,
                                              1, static_cast<int32_t>(kc), static_cast<int32_t>(kc)});
                root_copy_dst.push_back(r.r_off + off * r.K + off);
                // the box's skeleton solution comes from the root
                F.xt_root[kb] = 1;
                F.xt_off[kb] = r.x_off + off;
                off += kc;
            }
        } else {
            r.in_off = 2 * B.nlo;
        }
        roots.push_back(r);
        B.active = false;
    };

    int iter = 0;
    for (;; ++iter) {
        // bodies that reached their top level become roots, and so do bodies
        // whose last compression kept more than max_rank_ratio of their unknowns
        // (ranks grow with the box size in wavelengths; above that the ID of the
        // next, larger boxes would cost far more than it saves)
        const double max_ratio = h->opts.max_rank_ratio;
        for (int q = 0; q < nbodies; ++q)
            if (bodies[q].active &&
                (bodies[q].level == 0 || (max_ratio > 0 && bodies[q].last_ratio > max_ratio))) {
                if (bodies[q].level > 0)
                    progress("bmhss build: body %d stops compressing at level %d (kept %.2f of its unknowns)\n", q,
                             bodies[q].level, bodies[q].last_ratio);
                make_root(q);
            }
        // ---- the boxes of this iteration: every active body at its current level
        struct Box { int body, local; int64_t lo, hi; };
        std::vector<Box> boxes;
        std::vector<int> bfirst(nbodies, -1);
        for (int q = 0; q < nbodies; ++q) {
            BodyState& B = bodies[q];
            if (!B.active) continue;
            bfirst[q] = static_cast<int>(boxes.size());
            const int64_t nb = int64_t{1} << B.level;
            for (int64_t b = 0; b < nb; ++b)
                boxes.push_back(Box{q, static_cast<int>(b), B.nlo + ((b * B.nn) >> B.level),
                                    B.nlo + (((b + 1) * B.nn) >> B.level)});
        }
        const int nbox = static_cast<int>(boxes.size());
        if (nbox == 0) break;
        auto scp = std::make_unique<Scratch>(s);   // compression scratch of this iteration
        Scratch& sc = *scp;
        std::vector<int32_t> box_body(nbox), pcount(nbox);
        std::vector<int64_t> poff(nbox + 1, 0);
        std::vector<double> hbox_c(3 * static_cast<size_t>(nbox));
        for (int q = 0; q < nbodies; ++q)
            if (bodies[q].active) level_geometry(q, bodies[q].level);
        for (int b = 0; b < nbox; ++b) {
            const BodyState& B = bodies[boxes[b].body];
            box_body[b] = boxes[b].body;
            pcount[b] = B.box_p[B.level][boxes[b].local];
            poff[b + 1] = poff[b] + pcount[b];
            for (int r = 0; r < 3; ++r) hbox_c[3 * b + r] = B.box_c[B.level][3 * boxes[b].local + r];
        }
        int64_t* dpoff;
        int32_t *dbody, *dpcount;
        double* box_c;
        hipError_t e = sc.upload(&dbody, box_body);
        if (e == hipSuccess) e = sc.upload(&dpcount, pcount);
        if (e == hipSuccess) e = sc.upload(&dpoff, std::vector<int64_t>(poff.begin(), poff.end() - 1));
        if (e == hipSuccess) e = sc.upload(&box_c, hbox_c);
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: level setup"); }
        sc.rec([=]() {
            hipLaunchKernelGGL(k_proxy_points, dim3(nbox), dim3(kThreads), 0, s, box_c, dbody, dpoff, dpcount, N, pt);
            return hipGetLastError();
        });
        // ---- active slots; each box scans the slots of its own body
        std::vector<Slot> act;
        std::vector<int64_t> soff(nbox + 1, 0), n(nbox), scan_lo(nbox), scan_hi(nbox);
        std::vector<int32_t> sbox;
        for (int b = 0; b < nbox; ++b) {
            make_slots(bodies[boxes[b].body].U[boxes[b].local], act);
            soff[b + 1] = static_cast<int64_t>(act.size());
            n[b] = static_cast<int64_t>(bodies[boxes[b].body].U[boxes[b].local].size());
            for (int64_t q = soff[b]; q < soff[b + 1]; ++q) sbox.push_back(b);
        }
        for (int b = 0; b < nbox; ++b) {
            const int q = boxes[b].body;
            const int first = bfirst[q], last = first + (1 << bodies[q].level);
            scan_lo[b] = soff[first];
            scan_hi[b] = soff[last];
        }
        const int64_t nact = soff[nbox];
        int64_t *dcounts, *dscan_lo, *dscan_hi;
        Slot* dact;
        int32_t* dsbox;
        e = sc.upload(&dact, act);
        if (e == hipSuccess) e = sc.upload(&dsbox, sbox);
        if (e == hipSuccess) e = sc.upload(&dscan_lo, scan_lo);
        if (e == hipSuccess) e = sc.upload(&dscan_hi, scan_hi);
        if (e == hipSuccess) e = sc.alloc(&dcounts, 2 * nbox);
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: slots"); }
        sc.rec([=]() {
            hipLaunchKernelGGL(k_near_count, dim3(nbox), dim3(kThreads), 0, s, pt, dact, dsbox, dscan_lo, dscan_hi,
                               box_c, dcounts);
            return hipGetLastError();
        });
        std::vector<int64_t> counts(2 * nbox);
        e = sc.flush();
        {
            PinnedRead rd(s);
            if (e == hipSuccess) e = rd.read(counts.data(), dcounts, counts.size() * sizeof(int64_t));
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) rd.finish();
        }
        sc.synced();
        pl.reap(false);
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: near counts"); }
        // ---- a body with a box that has no far unknowns stops: its current boxes form its root;
        // so does a body whose IDs at this level would exceed the work guard (hss_plan.hpp)
        {
            std::vector<int64_t> total_u(nbodies, 0), id_entries(nbodies, 0);
            std::vector<char> stop(nbodies, 0), guard(nbodies, 0);
            for (int b = 0; b < nbox; ++b) total_u[boxes[b].body] += n[b];
            for (int b = 0; b < nbox; ++b) {
                const int q = boxes[b].body;
                if (total_u[q] - n[b] - counts[2 * b + 1] <= 0) stop[q] = 1;
                const int64_t rows = 2 * counts[2 * b + 1] + 4 * static_cast<int64_t>(pcount[b]);
                if (id_box_over_budget(rows, n[b])) guard[q] = 1;
                id_entries[q] += rows * n[b];
            }
            for (int q = 0; q < nbodies; ++q) {
                if (!bodies[q].active || bfirst[q] < 0) continue;
                if (!stop[q] && (guard[q] || id_level_over_budget(id_entries[q]))) {
                    progress("bmhss build: body %d stops compressing at level %d: its IDs would hold %lld "
                             "entries (limits %lld per box, %lld per level)\n", q, bodies[q].level,
                             static_cast<long long>(id_entries[q]), static_cast<long long>(kMaxIdEntries),
                             static_cast<long long>(kMaxLevelIdEntries));
                    stop[q] = 1;
                    ++h->guard_stops;
                }
                if (stop[q]) make_root(q);
            }
        }
        // ---- kept boxes: those of bodies that still compress
        std::vector<int> kept;            // kept index -> box index
        std::vector<int> kfirst(nbodies, -1);
        for (int b = 0; b < nbox; ++b) {
            const int q = boxes[b].body;
            if (!bodies[q].active) continue;
            if (boxes[b].local == 0) kfirst[q] = static_cast<int>(kept.size());
            kept.push_back(b);
        }
        const int nk = static_cast<int>(kept.size());
        if (nk == 0) { sc.release(); break; }

        // ---- slot buffer: [active | near (every box) | proxy (every box)]
        std::vector<int64_t> nsoff(nbox + 1, 0), nearu(nbox);
        for (int b = 0; b < nbox; ++b) {
            nsoff[b + 1] = nsoff[b] + counts[2 * b];
            nearu[b] = counts[2 * b + 1];
        }
        const int64_t near_base = nact, prox_base = nact + nsoff[nbox];
        const int64_t nslots_all = prox_base + poff[nbox];
        Slot* dslots;
        if ((e = sc.alloc(&dslots, nslots_all)) != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: slot buffer"); }
        sc.rec([=]() { return hipMemcpyAsync(dslots, dact, nact * sizeof(Slot), hipMemcpyDeviceToDevice, s); });
        std::vector<Slot> prox(static_cast<size_t>(poff[nbox]));
        for (int b = 0; b < nbox; ++b)
            for (int q = 0; q < pcount[b]; ++q)
                prox[poff[b] + q] = Slot{static_cast<int32_t>(N + poff[b] + q), 2 * q, 2 * q + 1};
        Slot* dprox;
        e = sc.upload(&dprox, prox);
        {
            const size_t pbytes = prox.size() * sizeof(Slot);
            sc.rec([=]() { return hipMemcpyAsync(dslots + prox_base, dprox, pbytes, hipMemcpyDeviceToDevice, s); });
        }
        int64_t* dnsoff;
        if (e == hipSuccess) e = sc.upload(&dnsoff, std::vector<int64_t>(nsoff.begin(), nsoff.end() - 1));
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: slot upload"); }
        sc.rec([=]() {
            hipLaunchKernelGGL(k_near_list, dim3(nbox), dim3(kThreads), 0, s, pt, dact, dsbox, dscan_lo, dscan_hi,
                               box_c, dnsoff, dslots + near_base);
            return hipGetLastError();
        });

        // ---- per kept box: sizes
        std::vector<int64_t> kn(nk), km(nk), mo(nk + 1, 0);
        for (int c = 0; c < nk; ++c) {
            const int b = kept[c];
            kn[c] = n[b];
            km[c] = 2 * nearu[b] + 4 * static_cast<int64_t>(pcount[b]);
            mo[c + 1] = mo[c] + kn[c] * km[c];
        }
        // ---- M_b for every kept box in one generation launch
        double2* M;
        if ((e = sc.alloc(&M, mo[nk])) != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: M"); }
        std::vector<GenJob> jobs, pjobs;   // near blocks; proxy blocks (FP32 with opts.proxy_fp32)
        std::vector<GenJob>& proxy_jobs = h->opts.proxy_fp32 ? pjobs : jobs;
        for (int c = 0; c < nk; ++c) {
            const int b = kept[c];
            const int32_t body = boxes[b].body;
            const int32_t na = static_cast<int32_t>(soff[b + 1] - soff[b]);
            const int32_t nn = static_cast<int32_t>(nsoff[b + 1] - nsoff[b]);
            const int64_t base = mo[c], m = km[c];
            jobs.push_back(GenJob{soff[b], near_base + nsoff[b], base, m, 1, na, nn, body});
            jobs.push_back(GenJob{near_base + nsoff[b], soff[b], base + nearu[b], 1, m, nn, na, body});
            const int32_t pb = pcount[b];
            proxy_jobs.push_back(GenJob{soff[b], prox_base + poff[b], base + 2 * nearu[b], m, 1, na, pb, body});
            proxy_jobs.push_back(GenJob{prox_base + poff[b], soff[b], base + 2 * nearu[b] + 2 * pb, 1, m, pb, na, body});
            entries += kn[c] * m;
            pairs += 2 * static_cast<int64_t>(na) * (nn + pb);
        }
        hipEvent_t ev;
        if ((e = t_gen.start(sc, ev)) == hipSuccess) e = launch_gen(sc, jobs, dslots, pt, p->d_media, p->media[0].tab, M);
        if (e == hipSuccess && !pjobs.empty())
            e = launch_gen(sc, pjobs, dslots, pt, p->d_media, p->media[0].tab, M, p->d_ftab);
        if (e == hipSuccess) e = t_gen.stop(sc, ev);
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: generate M"); }

        // ---- optional sketch: Y_b = Omega M_b^T with min(rows, unknowns + p)
        // rows; the CPQR and the interpolation matrix then come from Y_b
        // (randomized ID).  The p extra rows keep Omega well conditioned on the
        // column space of M_b^T even when a box is close to full rank.
        std::vector<int64_t> idm(km), yo(nk + 1, 0);
        double2* Y_sk = nullptr;
        if (h->opts.sketch) {
            int64_t lmax = 0, mmax = 0;
            for (int c = 0; c < nk; ++c) {
                idm[c] = std::min(km[c], kn[c] + h->opts.sketch);
                yo[c + 1] = yo[c] + idm[c] * kn[c];
                lmax = std::max(lmax, idm[c]);
                mmax = std::max(mmax, km[c]);
            }
            if (yo[nk] < mo[nk]) {
                const double* omega = nullptr;
                int64_t ldo = 0;
                e = omega_device(lmax, mmax, &omega, &ldo);
                if (e == hipSuccess) e = sc.alloc(&Y_sk, yo[nk]);
                std::vector<SketchJob> sj(nk);
                for (int c = 0; c < nk; ++c)
                    sj[c] = SketchJob{M + mo[c], Y_sk + yo[c], nullptr, static_cast<int32_t>(km[c]),
                                      static_cast<int32_t>(kn[c]), static_cast<int32_t>(idm[c])};
                if (e == hipSuccess && (e = t_cmp.start(sc, ev)) == hipSuccess) {
                    e = launch_sketch(sc, sj, omega, ldo);
                    if (e == hipSuccess) e = t_cmp.stop(sc, ev);
                }
                if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: sketch"); }
            } else {
                idm = km;
                Y_sk = nullptr;
            }
        }

        // ---- ID: CPQR of M_b^T (or of its sketch)
        std::vector<int64_t> uoff(nk + 1, 0);
        for (int c = 0; c < nk; ++c) uoff[c + 1] = uoff[c] + kn[c];
        int32_t *dperm, *dranks;
        double2* drdiag;
        e = sc.alloc(&dperm, uoff[nk]);
        if (e == hipSuccess) e = sc.alloc(&drdiag, uoff[nk]);
        if (e == hipSuccess) e = sc.alloc(&dranks, nk);
        std::vector<CpqrJob> cj(nk);
        for (int c = 0; c < nk; ++c)
            cj[c] = CpqrJob{Y_sk ? Y_sk + yo[c] : M + mo[c], dperm + uoff[c], drdiag + uoff[c], nullptr,
                            nullptr, nullptr, static_cast<int32_t>(kn[c]),
                            static_cast<int32_t>(Y_sk ? idm[c] : km[c])};
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: cpqr setup"); }
        if ((e = t_cmp.start(sc, ev)) != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "event"); }
        {
            int64_t mu = 0, mr = 0;
            for (int c = 0; c < nk; ++c) { mu = std::max(mu, kn[c]); mr = std::max(mr, km[c]); }
            progress("bmhss build: iteration %d: ID of %d boxes, <= %lld unknowns x %lld rows, %.4f s\n",
                     static_cast<int>(h->level_info.size()), nk, static_cast<long long>(mu),
                     static_cast<long long>(mr),
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
        }
        CpqrJob* dcj = nullptr;
        std::vector<int32_t> ranks(nk), perm(uoff[nk]);
        hipEvent_t c0 = nullptr, c1 = nullptr;
        e = hipEventCreate(&c0);
        if (e == hipSuccess) e = hipEventCreate(&c1);
        if (e == hipSuccess) {
            cpqr_events.emplace_back(c0, c1);
            // first rank check: a little above the previous level's largest rank
            // (ranks grow slowly from level to level), or half the unknowns
            int64_t guess = 0;
            for (int c = 0; c < nk; ++c) guess = std::max(guess, kn[c] / 2);
            if (!h->level_info.empty()) guess = h->level_info.back().max_rank + h->level_info.back().max_rank / 4 + 8;
            bool fused = false;
            // while the GPU runs the ID: issue the deferred factorisation, and
            // compute the next level's box geometry
            const std::function<hipError_t()> before_wait = [&]() -> hipError_t {
                const hipError_t fe = flush_deferred();
                for (int q = 0; q < nbodies; ++q)
                    if (bodies[q].active) level_geometry(q, bodies[q].level - 1);
                return fe;
            };
            e = run_cpqr(sc, cj, &dcj, dranks, tol, ranks, c0, c1, &cpqr_launches, static_cast<int>(guess), &fused,
                         before_wait);
            cpqr_fused.push_back(fused);
        }
        {
            PinnedRead rd(s);
            if (e == hipSuccess) e = rd.read(perm.data(), dperm, perm.size() * sizeof(int32_t));
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) rd.finish();
        }
        sc.synced();
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: cpqr"); }
        {
            bm_hss_level_t li{};
            li.boxes = nk;
            li.min_rank = INT32_MAX;
            for (int c = 0; c < nk; ++c) {
                li.max_unknowns = std::max<int32_t>(li.max_unknowns, static_cast<int32_t>(kn[c]));
                li.max_rows = std::max<int32_t>(li.max_rows, static_cast<int32_t>(km[c]));
                li.id_rows = std::max<int32_t>(li.id_rows, static_cast<int32_t>(Y_sk ? idm[c] : km[c]));
                li.min_rank = std::min<int32_t>(li.min_rank, ranks[c]);
                li.max_rank = std::max<int32_t>(li.max_rank, ranks[c]);
            }
            h->level_info.push_back(li);
            progress("bmhss build: iteration %d: %d boxes, <= %d unknowns, <= %d rows, ranks %d..%d, %.4f s\n",
                     static_cast<int>(h->level_info.size()) - 1, li.boxes, li.max_unknowns, li.max_rows,
                     li.min_rank, li.max_rank,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
            // algorithmic bytes of the executed CPQR steps: at step k the trailing
            // columns (n - k - 1 of them, rows k..m) are read and written once, the
            // Householder column (rows k..m) and the n norms are read, and the
            // trailing norms written; the step that finds the rank reads the norms
            // (the whole-box kernel reads and writes each matrix once, and writes
            // the pivots and the diagonal of R)
            for (int c = 0; c < nk; ++c) {
                const double rows = static_cast<double>(Y_sk ? idm[c] : km[c]), cols = static_cast<double>(kn[c]);
                if (cpqr_fused.back()) {
                    cpqr_fused_bytes += 32.0 * rows * cols + 20.0 * ranks[c];
                    continue;
                }
                for (int64_t kk = 0; kk < ranks[c]; ++kk) {
                    const double r = rows - kk, cc = cols - kk - 1;
                    cpqr_bytes += 32.0 * r * cc + 16.0 * r + 8.0 * cols + 8.0 * cc;
                }
                cpqr_bytes += 8.0 * cols;
            }
            if (cpqr_fused.back()) ++cpqr_fused_launches;
        }
        std::vector<int64_t> k(nk), koff(nk + 1, 0), nkoff(nk + 1, 0), nnoff(nk + 1, 0), kkoff(nk + 1, 0);
        for (int c = 0; c < nk; ++c) {
            k[c] = ranks[c];
            max_rank = std::max(max_rank, k[c]);
            koff[c + 1] = koff[c] + k[c];
            nkoff[c + 1] = nkoff[c] + kn[c] * k[c];
            nnoff[c + 1] = nnoff[c] + kn[c] * kn[c];
            kkoff[c + 1] = kkoff[c] + k[c] * k[c];
        }
        double2* T;
        e = sc.alloc(&T, nkoff[nk]);
        {
            const size_t tbytes = std::max<int64_t>(nkoff[nk], 1) * sizeof(double2);
            sc.rec([=]() { return hipMemsetAsync(T, 0, tbytes, s); });
        }
        int64_t* dtoff;
        if (e == hipSuccess) e = sc.upload(&dtoff, std::vector<int64_t>(nkoff.begin(), nkoff.end() - 1));
        if (e != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: T"); }
        int64_t cmax = 1, kmax = 0;
        for (int c = 0; c < nk; ++c) {
            cmax = std::max(cmax, kn[c] - k[c]);
            kmax = std::max(kmax, k[c]);
        }
        {
            // rows per lane of the column-oriented substitution; the row-oriented
            // kernel takes ranks beyond 256
            const int rpl = kmax <= 64 ? 1 : kmax <= 128 ? 2 : kmax <= 256 ? 4 : 0;
            const unsigned cx = static_cast<unsigned>(ceil_div(cmax, kThreads / 64));
            sc.rec([=]() {
                const dim3 g(cx, nk), b(kThreads);
                switch (rpl) {
                    case 1: hipLaunchKernelGGL(k_interp_wave<1>, g, b, 0, s, dcj, dranks, dtoff, T); break;
                    case 2: hipLaunchKernelGGL(k_interp_wave<2>, g, b, 0, s, dcj, dranks, dtoff, T); break;
                    case 4: hipLaunchKernelGGL(k_interp_wave<4>, g, b, 0, s, dcj, dranks, dtoff, T); break;
                    default: hipLaunchKernelGGL(k_interp, g, b, 0, s, dcj, dranks, dtoff, T); break;
                }
                return hipGetLastError();
            });
        }
        if ((e = t_cmp.stop(sc, ev)) != hipSuccess) { sc.release(); cleanup(); return hip_fail(e, "event"); }

        // ---- the factors of this iteration, and how the solve moves between stages
        LevelFactor f;
        f.nb = nk; f.n = kn; f.k = k; f.uoff = uoff; f.koff = koff; f.nkoff = nkoff; f.nnoff = nnoff;
        f.nu = uoff[nk]; f.nk = koff[nk];
        f.in_off.resize(nk);
        f.xt_off.assign(nk, 0);
        f.xt_root.assign(nk, -1);   // set when the parent iteration or the root is known
        for (int c = 0; c < nk; ++c) {
            const int b = kept[c];
            const BodyState& B = bodies[boxes[b].body];
            if (B.iter_prev < 0) {
                f.in_off[c] = 2 * boxes[b].lo;   // leaves read the right-hand side
            } else {
                // the children are consecutive boxes of the previous iteration
                const LevelFactor& Fp = h->lv[B.iter_prev];
                const int child0 = B.kept_prev + 2 * boxes[b].local;
                f.in_off[c] = Fp.koff[child0];
            }
        }
        // the previous iteration's boxes of continuing bodies take their skeleton
        // solution from their parent here: U(parent) = J(child 0) then J(child 1)
        for (int c = 0; c < nk; ++c) {
            const int b = kept[c];
            const BodyState& B = bodies[boxes[b].body];
            if (B.iter_prev < 0) continue;
            LevelFactor& Fp = h->lv[B.iter_prev];
            const int child0 = B.kept_prev + 2 * boxes[b].local;
            Fp.xt_root[child0] = 0;
            Fp.xt_off[child0] = uoff[c];
            Fp.xt_root[child0 + 1] = 0;
            Fp.xt_off[child0 + 1] = uoff[c] + Fp.k[child0];
        }

        // ---- hand over to the second stream: everything below reads T, the
        // slot lists and the point table, and runs concurrently with the next
        // iteration's compression on the caller's stream
        hipEvent_t ready = nullptr, done = nullptr;
        e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (ready) (void)hipEventDestroy(ready);
            sc.release(); cleanup(); return hip_fail(e, "bm_hss_build: events");
        }
        sc.rec([=]() { return hipEventRecord(ready, s); });
        e = sc.flush();
        pl.pending.emplace_back();
        pl.pending.back().cmp = std::move(scp);
        pl.pending.back().ready = ready;
        pl.pending.back().done = done;
        pl.pending.back().fac = std::make_unique<Scratch>(s2);
        Scratch& fs = *pl.pending.back().fac;
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "bm_hss_build: compression"); }
        fs.rec([=]() { return hipStreamWaitEvent(s2, ready, 0); });

        // ---- diagonal blocks D_b (become G_b in place)
        e = palloc(&f.G, nnoff[nk], s2);
        if (e == hipSuccess) e = palloc(&f.E, nkoff[nk], s2);
        if (e == hipSuccess) e = palloc(&f.Ft, nkoff[nk], s2);
        if (e != hipSuccess) { free_factor(f, s2); cleanup(); return hip_fail(e, "bm_hss_build: factors"); }
        h->lv.push_back(f);   // owned by h from here on
        LevelFactor& F = h->lv.back();
        jobs.clear();
        std::vector<CopyJob> copies;
        for (int c = 0; c < nk; ++c) {
            const int b = kept[c];
            const BodyState& B = bodies[boxes[b].body];
            const int32_t body = boxes[b].body;
            const int32_t na = static_cast<int32_t>(soff[b + 1] - soff[b]);
            if (B.iter_prev < 0) {
                jobs.push_back(GenJob{soff[b], soff[b], nnoff[c], kn[c], 1, na, na, body});
                entries += kn[c] * kn[c];
                pairs += static_cast<int64_t>(na) * na;
            } else {
                const int64_t sa = B.split_slots[boxes[b].local];
                const int32_t n1 = static_cast<int32_t>(sa), n2 = na - n1;
                jobs.push_back(GenJob{soff[b], soff[b] + sa, nnoff[c], kn[c], 1, n1, n2, body});
                jobs.push_back(GenJob{soff[b] + sa, soff[b], nnoff[c], kn[c], 1, n2, n1, body});
                const LevelFactor& Fp = h->lv[B.iter_prev];
                const int child0 = B.kept_prev + 2 * boxes[b].local;
                const int64_t ka = Fp.k[child0], kb = Fp.k[child0 + 1];
                entries += 2 * ka * kb;
                pairs += 2 * static_cast<int64_t>(n1) * n2;
                const double2* Dp = dhat[B.iter_prev];
                copies.push_back(CopyJob{Dp + dhat_off[B.iter_prev][child0], F.G + nnoff[c], ka, 1, kn[c], 1,
                                         static_cast<int32_t>(ka), static_cast<int32_t>(ka)});
                copies.push_back(CopyJob{Dp + dhat_off[B.iter_prev][child0 + 1], F.G + nnoff[c] + ka * kn[c] + ka, kb, 1,
                                         kn[c], 1, static_cast<int32_t>(kb), static_cast<int32_t>(kb)});
            }
        }
        if ((e = t_gen.start(fs, ev)) == hipSuccess) e = launch_gen(fs, jobs, dslots, pt, p->d_media, p->media[0].tab, F.G);
        if (e == hipSuccess) e = t_gen.stop(fs, ev);
        if (e == hipSuccess) e = launch_copy(fs, copies);
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "bm_hss_build: D blocks"); }

        // ---- Martinsson-Rokhlin factors
        double2 *Y, *Wt, *S = nullptr;
        e = fs.alloc(&Y, nkoff[nk]);
        if (e == hipSuccess) e = fs.alloc(&Wt, nkoff[nk]);
        if (e == hipSuccess) e = palloc(&S, kkoff[nk], s2);
        if (e == hipSuccess) {
            dhat.push_back(S);   // kept until the roots are built
            dhat_off.emplace_back(kkoff.begin(), kkoff.end() - 1);
        }
        int32_t* st = nullptr;
        if (e == hipSuccess) e = palloc(&st, 2 * nk, s2);
        if (e == hipSuccess) {
            status_bufs.push_back(st);
            fs.rec([=]() { return hipMemsetAsync(st, 0, 2 * nk * sizeof(int32_t), s2); });
        }
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "bm_hss_build: factor buffers"); }
        if ((e = t_fac.start(fs, ev)) != hipSuccess) { cleanup(); return hip_fail(e, "event"); }
        std::vector<InvJob> inv(nk);
        for (int c = 0; c < nk; ++c) inv[c] = InvJob{F.G + nnoff[c], st + c, kn[c], static_cast<int32_t>(kn[c])};
        e = launch_inverse(fs, inv);
        std::vector<GemmJob> g1, g2, g3, g4;
        const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
        for (int c = 0; c < nk; ++c) {
            const int64_t nn = kn[c], kk = k[c];
            const double2* Di = F.G + nnoff[c];
            const double2* Tb = T + nkoff[c];
            // Y = D^-1 T (n x k); Wt = T^T D^-1 (k x n)
            g1.push_back(gemm(Di, nn, 1, Tb, kk, 1, Y + nkoff[c], kk, 1, nn, kk, nn));
            g1.push_back(gemm(Tb, 1, kk, Di, nn, 1, Wt + nkoff[c], nn, 1, kk, nn, nn));
        }
        if (e == hipSuccess) e = launch_gemm(fs, g1);
        for (int c = 0; c < nk; ++c) {
            const int64_t nn = kn[c], kk = k[c];
            // S = Wt T (k x k)
            g2.push_back(gemm(Wt + nkoff[c], nn, 1, T + nkoff[c], kk, 1, S + kkoff[c], kk, 1, kk, kk, nn));
        }
        if (e == hipSuccess) e = launch_gemm(fs, g2);
        std::vector<InvJob> inv2(nk);
        for (int c = 0; c < nk; ++c) inv2[c] = InvJob{S + kkoff[c], st + nk + c, k[c], static_cast<int32_t>(k[c])};
        if (e == hipSuccess) e = launch_inverse(fs, inv2);
        for (int c = 0; c < nk; ++c) {
            const int64_t nn = kn[c], kk = k[c];
            // E = Y Dhat (n x k); Ft = Dhat Wt (k x n)
            g3.push_back(gemm(Y + nkoff[c], kk, 1, S + kkoff[c], kk, 1, F.E + nkoff[c], kk, 1, nn, kk, kk));
            g3.push_back(gemm(S + kkoff[c], kk, 1, Wt + nkoff[c], nn, 1, F.Ft + nkoff[c], nn, 1, kk, nn, kk));
        }
        if (e == hipSuccess) e = launch_gemm(fs, g3);
        for (int c = 0; c < nk; ++c) {
            const int64_t nn = kn[c], kk = k[c];
            // G = D^-1 - E Wt (in place)
            g4.push_back(gemm(F.E + nkoff[c], kk, 1, Wt + nkoff[c], nn, 1, F.G + nnoff[c], nn, 1, nn, nn, kk, mone, one));
        }
        if (e == hipSuccess) e = launch_gemm(fs, g4);
        if (e == hipSuccess) e = t_fac.stop(fs, ev);
        if (e == hipSuccess) {
            fs.rec([=]() { return hipEventRecord(done, s2); });
            // the launches of this level's factorisation are issued later, while the
            // GPU compresses the next level (run_cpqr calls flush_deferred before it
            // waits), so that the host's launch work overlaps that compression
            e = flush_deferred();
            pl.pending.back().flushed = false;
            deferred_fac = &fs;
        }
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "bm_hss_build: factor"); }

        // ---- next level of every continuing body: U(parent) = J(first child) then J(second child)
        for (int q = 0; q < nbodies; ++q) {
            BodyState& B = bodies[q];
            if (!B.active || kfirst[q] < 0) continue;
            const int nbq = 1 << B.level;
            std::vector<std::vector<int32_t>> J(nbq);
            int64_t kept = 0, had = 0;
            for (int lb = 0; lb < nbq; ++lb) {
                const int c = kfirst[q] + lb;
                kept += k[c];
                had += static_cast<int64_t>(B.U[lb].size());
                J[lb].resize(k[c]);
                for (int64_t i = 0; i < k[c]; ++i) J[lb][i] = B.U[lb][perm[uoff[c] + i]];
            }
            B.U.assign(nbq / 2, {});
            B.split_slots.assign(nbq / 2, 0);
            for (int pq = 0; pq < nbq / 2; ++pq) {
                B.U[pq] = J[2 * pq];
                std::vector<Slot> tmp;
                make_slots(J[2 * pq], tmp);
                B.split_slots[pq] = static_cast<int64_t>(tmp.size());
                B.U[pq].insert(B.U[pq].end(), J[2 * pq + 1].begin(), J[2 * pq + 1].end());
            }
            B.iter_prev = iter;
            B.kept_prev = kfirst[q];
            B.last_ratio = had > 0 ? static_cast<double>(kept) / static_cast<double>(had) : 0.0;
            B.level -= 1;
        }
    }
    const int compressed = static_cast<int>(h->lv.size());

    // ---- roots: every body's reduced system, generated and inverted in one batch
    // on the second stream after the last compression (and after the last
    // level's factorisation, whose Dhat blocks the roots take)
    {
        const hipError_t ed = flush_deferred();
        if (ed != hipSuccess) { cleanup(); return hip_fail(ed, "bm_hss_build: factor"); }
        hipEvent_t rready = nullptr;
        BM_HIP(hipEventCreateWithFlags(&rready, hipEventDisableTiming));
        const hipError_t er = hipEventRecord(rready, s);
        if (er != hipSuccess) { (void)hipEventDestroy(rready); cleanup(); return hip_fail(er, "bm_hss_build: root"); }
        Scratch sc(s2);
        sc.rec([=]() { return hipStreamWaitEvent(s2, rready, 0); });
        h->roots = roots;
        h->Ktot = Ktot;
        progress("bmhss build: %d roots, %lld unknowns in total, %.4f s\n", static_cast<int>(roots.size()),
                 static_cast<long long>(Ktot),
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
        Slot* drs;
        hipError_t e = sc.upload(&drs, root_slots);
        if (e == hipSuccess) e = palloc(&h->Rinv, Rtot, s2);
        if (e != hipSuccess) { sc.release(); (void)hipEventDestroy(rready); cleanup(); return hip_fail(e, "bm_hss_build: root"); }
        std::vector<GenJob> jobs;
        for (const RootJob& r : roots) {
            jobs.push_back(GenJob{r.slot_off, r.slot_off, r.r_off, r.K, 1, r.nslots, r.nslots, r.body});
            entries += r.K * r.K;
            pairs += static_cast<int64_t>(r.nslots) * r.nslots;
        }
        hipEvent_t ev;
        if ((e = t_gen.start(sc, ev)) == hipSuccess) e = launch_gen(sc, jobs, drs, pt, p->d_media, p->media[0].tab, h->Rinv);
        if (e == hipSuccess) e = t_gen.stop(sc, ev);
        // diagonal blocks of a root are the Dhat of the boxes it is made of
        for (size_t c = 0; c < root_copies.size(); ++c) root_copies[c].dst = h->Rinv + root_copy_dst[c];
        if (e == hipSuccess) e = launch_copy(sc, root_copies);
        int32_t* st = nullptr;
        if (e == hipSuccess) e = palloc(&st, static_cast<int64_t>(roots.size()), s2);
        if (e == hipSuccess) {
            status_bufs.push_back(st);
            const size_t nr = roots.size();
            sc.rec([=]() { return hipMemsetAsync(st, 0, nr * sizeof(int32_t), s2); });
        }
        if (e == hipSuccess && singular_root_hook()) {
            double2* r0 = h->Rinv + roots[0].r_off;
            const size_t bytes = static_cast<size_t>(roots[0].K) * sizeof(double2);
            sc.rec([=]() { return hipMemsetAsync(r0, 0, bytes, s2); });
        }
        if (e == hipSuccess && (e = t_fac.start(sc, ev)) == hipSuccess) {
            std::vector<InvJob> inv;
            for (size_t q = 0; q < roots.size(); ++q)
                inv.push_back(InvJob{h->Rinv + roots[q].r_off, st + q, roots[q].K, static_cast<int32_t>(roots[q].K)});
            // one root of moderate size: panels (a serial chain of short launches
            // either way, panels make it shorter); several roots (a forest): the
            // recursion, batched over the roots; very large roots: the
            // recursion, whose large square products run near the FP64 peak
            // where the panels' rank-b updates would stream the whole matrix
            // through memory once per panel
            if (inv.size() == 1 && inv[0].n > inv_base() && inv[0].n <= kRootPanelsMax && root_panels())
                e = launch_inverse_panels(sc, inv[0]);
            else
                e = launch_inverse(sc, inv);
            if (e == hipSuccess) e = t_fac.stop(sc, ev);
        }
        if (e == hipSuccess) e = sc.flush();
        progress("bmhss build: root inversion enqueued, %.4f s\n",
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
        // every inversion's status, copied behind the root on the second stream
        // into pinned memory, so that one wait covers them all
        for (size_t q = 0; q < status_bufs.size(); ++q) {
            const int64_t cnt = (q + 1 == status_bufs.size()) ? static_cast<int64_t>(roots.size()) : 2 * h->lv[q].nb;
            status_cnt.push_back(cnt);
            status_tot += cnt;
        }
        if (e == hipSuccess) {
            status_host = reinterpret_cast<int32_t*>(
                pinned_cache().get(static_cast<size_t>(std::max<int64_t>(status_tot, 1)) * sizeof(int32_t), &status_cap));
            if (!status_host) e = hipErrorOutOfMemory;
        }
        for (size_t q = 0, o = 0; q < status_bufs.size() && e == hipSuccess; o += status_cnt[q], ++q)
            e = hipMemcpyAsync(status_host + o, status_bufs[q], status_cnt[q] * sizeof(int32_t), hipMemcpyDeviceToHost, s2);
        // while the GPU inverts the root: capture the one-right-hand-side solve
        // for bm_hss_solve_graph (host work; a failure only leaves it to the
        // first call)
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(h->plan_mu);
            bm_hss::SolvePlan* plan = nullptr;
            const char* where = nullptr;
            if (make_solve_plan(h, 1, false, &plan, &where) != hipSuccess) {
                (void)hipGetLastError();
                h->plans.clear();
            }
            progress("bmhss build: solve graph recorded, %.4f s\n",
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s2);
        progress("bmhss build: root inverted, %.4f s\n",
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
        sc.synced();
        sc.release();
        (void)hipEventDestroy(rready);
        pl.reap(true);
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "bm_hss_build: root factor"); }
    }
    // every compressed box must know where its skeleton solution comes from
    for (const LevelFactor& f : h->lv)
        for (int8_t r : f.xt_root)
            if (r < 0) { cleanup(); return fail(BM_ESTATE, "bm_hss_build: internal error (unlinked box)"); }
    // ---- statuses of every inversion (copied before the last wait)
    for (int64_t i = 0; i < status_tot; ++i)
        if (status_host[i]) { cleanup(); return fail(BM_ESINGULAR, "bm_hss_build: singular block in the HSS factorisation"); }
    cleanup();
    progress("bmhss build: done, %.4f s\n",
             std::chrono::duration<double>(std::chrono::steady_clock::now() - t_build0).count());
    h->stats.levels = Lmax;
    h->stats.compressed_levels = compressed;
    h->stats.root_size = static_cast<int32_t>(std::min<int64_t>(Ktot, INT32_MAX));
    h->stats.guard_stops = h->guard_stops;
    h->stats.max_rank = max_rank;
    h->stats.entries = entries;
    h->stats.pairs = pairs;
    h->stats.seconds_generate = t_gen.seconds();
    h->stats.seconds_compress = t_cmp.seconds();
    h->stats.seconds_factor = t_fac.seconds();
    h->stats.cpqr_launches = cpqr_launches;
    h->stats.cpqr_bytes = cpqr_bytes;
    double tcq = 0, tcf = 0;
    for (size_t q = 0; q < cpqr_events.size(); ++q) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, cpqr_events[q].first, cpqr_events[q].second) == hipSuccess)
            (q < cpqr_fused.size() && cpqr_fused[q] ? tcf : tcq) += ms * 1e-3;
    }
    h->stats.seconds_cpqr = tcq;
    h->stats.cpqr_fused_launches = cpqr_fused_launches;
    h->stats.cpqr_fused_bytes = cpqr_fused_bytes;
    h->stats.seconds_cpqr_fused = tcf;
    return BM_OK;
}

// The solution operator x = M b of the factorisation (M ~ A^-1):
//   upward    v_l = F_l^T v_{l-1}            (v_{-1} = b, per box: its input slice)
//   roots     xr = Rinv v_stage
//   downward  y_l = G_l v_{l-1} + E_l y_{l+1} (y_{l+1} of the parent, or xr)
//   x = y_0 (or xr for a body that was never compressed).
// trans = true applies M^T (plain transpose, no conjugation), reusing the same
// factors with every edge of that data flow reversed:
//   y_0 = c;  for l = 0, 1, ..: v_{l-1} = G_l^T y_l  and  y_{l+1} (or xr) = E_l^T y_l
//   v_stage = Rinv^T xr;  for l = .., 1, 0: v_{l-1} += F_l v_l;  result v_{-1}.
// Every slice of a y or v vector is written by exactly one box (a parent's
// unknowns are its children's skeletons; an iteration's output feeds either
// the next iteration or a root), so the first write of each slice overwrites.
hipError_t record_solve(const bm_hss* h, Scratch& sc, const double* b, double* x, int64_t nrhs, bool trans) {
    const int nl = static_cast<int>(h->lv.size());
    const int64_t N2 = 2 * h->N;
    std::vector<double2*> bt(nl), xl(nl);
    hipError_t e = hipSuccess;
    for (int li = 0; li < nl && e == hipSuccess; ++li) {
        e = sc.alloc(&bt[li], h->lv[li].nk * nrhs);
        if (e == hipSuccess) e = sc.alloc(&xl[li], h->lv[li].nu * nrhs);
    }
    double2* xroot;
    if (e == hipSuccess) e = sc.alloc(&xroot, h->Ktot * nrhs);
    if (e != hipSuccess) return e;
    const double2* bin = reinterpret_cast<const double2*>(b);
    if (trans) {
        double2* z = reinterpret_cast<double2*>(x);
        // output of iteration li's transposed G / F^T products: the result, or
        // the adjoint of the previous iteration's F^T output
        auto stage_out = [&](int li, double2** ptr, int64_t* ld) {
            if (li < 0) { *ptr = z; *ld = N2; }
            else { *ptr = bt[li]; *ld = h->lv[li].nk; }
        };
        // y_0 = c per body: into the first iteration's output, or the root of
        // a body that was never compressed
        {
            std::vector<CopyJob> cp;
            const bm_problem* p = h->p;
            for (const RootJob& r : h->roots) {
                const int64_t lo = p->body_lo[r.body], nn2 = 2 * (p->body_lo[r.body + 1] - lo);
                double2* dst;
                int64_t ld;
                if (r.stage < 0) {
                    dst = xroot + r.x_off;
                    ld = h->Ktot;
                } else {
                    const LevelFactor& f0 = h->lv[0];
                    int64_t off = -1;
                    for (int q = 0; q < f0.nb; ++q)
                        if (f0.in_off[q] == 2 * lo) { off = f0.uoff[q]; break; }
                    if (off < 0) { e = hipErrorInvalidValue; break; }
                    dst = xl[0] + off;
                    ld = f0.nu;
                }
                cp.push_back(CopyJob{bin + 2 * lo, dst, 1, N2, 1, ld, static_cast<int32_t>(nn2),
                                     static_cast<int32_t>(nrhs)});
            }
            if (e == hipSuccess) e = launch_copy(sc, cp);
        }
        // reversed downward sweep: G^T into the stage below, E^T into the parent
        for (int li = 0; li < nl && e == hipSuccess; ++li) {
            const LevelFactor& f = h->lv[li];
            double2* out;
            int64_t ldout;
            stage_out(li - 1, &out, &ldout);
            std::vector<GemmJob> gj;
            for (int q = 0; q < f.nb; ++q) {
                double2* xt = f.xt_root[q] ? xroot : xl[li + 1];
                const int64_t ldxt = f.xt_root[q] ? h->Ktot : h->lv[li + 1].nu;
                const double2* y = xl[li] + f.uoff[q];
                gj.push_back(gemm(f.G + f.nnoff[q], 1, f.n[q], y, 1, f.nu, out + f.in_off[q], 1, ldout,
                                  f.n[q], nrhs, f.n[q]));
                gj.push_back(gemm(f.E + f.nkoff[q], 1, f.k[q], y, 1, f.nu, xt + f.xt_off[q], 1, ldxt,
                                  f.k[q], nrhs, f.n[q]));
            }
            e = launch_gemm(sc, gj);
        }
        // roots: v_stage = Rinv^T xr
        if (e == hipSuccess) {
            std::vector<GemmJob> gj;
            for (const RootJob& r : h->roots) {
                double2* out;
                int64_t ldout;
                stage_out(r.stage, &out, &ldout);
                gj.push_back(gemm(h->Rinv + r.r_off, 1, r.K, xroot + r.x_off, 1, h->Ktot, out + r.in_off, 1, ldout,
                                  r.K, nrhs, r.K));
            }
            e = launch_gemm(sc, gj);
        }
        // reversed upward sweep: v_{l-1} += (F^T)^T v_l, top iteration first
        for (int li = nl - 1; li >= 0 && e == hipSuccess; --li) {
            const LevelFactor& f = h->lv[li];
            double2* out;
            int64_t ldout;
            stage_out(li - 1, &out, &ldout);
            std::vector<GemmJob> gj;
            for (int q = 0; q < f.nb; ++q)
                gj.push_back(gemm(f.Ft + f.nkoff[q], 1, f.n[q], bt[li] + f.koff[q], 1, f.nk, out + f.in_off[q], 1,
                                  ldout, f.n[q], nrhs, f.k[q], make_double2(1.0, 0.0), make_double2(1.0, 0.0)));
            e = launch_gemm(sc, gj);
        }
    } else {
        // input of iteration li: the right-hand side, or the previous iteration's F^T output
        auto stage_in = [&](int li, const double2** ptr, int64_t* ld) {
            if (li < 0) { *ptr = bin; *ld = N2; }
            else { *ptr = bt[li]; *ld = h->lv[li].nk; }
        };
        // upward: bt = F^T in
        for (int li = 0; li < nl && e == hipSuccess; ++li) {
            const LevelFactor& f = h->lv[li];
            const double2* in;
            int64_t ldin;
            stage_in(li - 1, &in, &ldin);
            std::vector<GemmJob> gj;
            for (int q = 0; q < f.nb; ++q)
                gj.push_back(gemm(f.Ft + f.nkoff[q], f.n[q], 1, in + f.in_off[q], 1, ldin, bt[li] + f.koff[q], 1, f.nk,
                                  f.k[q], nrhs, f.n[q]));
            e = launch_gemm(sc, gj);
        }
        // roots: xroot = Rinv in, one product per body
        {
            std::vector<GemmJob> gj;
            for (const RootJob& r : h->roots) {
                const double2* in;
                int64_t ldin;
                stage_in(r.stage, &in, &ldin);
                gj.push_back(gemm(h->Rinv + r.r_off, r.K, 1, in + r.in_off, 1, ldin, xroot + r.x_off, 1, h->Ktot,
                                  r.K, nrhs, r.K));
            }
            if (e == hipSuccess) e = launch_gemm(sc, gj);
        }
        // downward: x = G in + E xt, xt from the parent iteration or the body's root
        for (int li = nl - 1; li >= 0 && e == hipSuccess; --li) {
            const LevelFactor& f = h->lv[li];
            const double2* in;
            int64_t ldin;
            stage_in(li - 1, &in, &ldin);
            std::vector<GemmJob> g1, g2;
            for (int q = 0; q < f.nb; ++q) {
                const double2* xt = f.xt_root[q] ? xroot : xl[li + 1];
                const int64_t ldxt = f.xt_root[q] ? h->Ktot : h->lv[li + 1].nu;
                g1.push_back(gemm(f.G + f.nnoff[q], f.n[q], 1, in + f.in_off[q], 1, ldin, xl[li] + f.uoff[q], 1, f.nu,
                                  f.n[q], nrhs, f.n[q]));
                g2.push_back(gemm(f.E + f.nkoff[q], f.k[q], 1, xt + f.xt_off[q], 1, ldxt, xl[li] + f.uoff[q], 1, f.nu,
                                  f.n[q], nrhs, f.k[q], make_double2(1.0, 0.0), make_double2(1.0, 0.0)));
            }
            e = launch_gemm(sc, g1);
            if (e == hipSuccess) e = launch_gemm(sc, g2);
        }
        // the solution of every body in global unknown order: from the first
        // iteration's output (its leaf boxes are contiguous and in node order), or
        // from its root when the body was never compressed
        if (e == hipSuccess) {
            std::vector<CopyJob> cp;
            const bm_problem* p = h->p;
            for (const RootJob& r : h->roots) {
                const int64_t lo = p->body_lo[r.body], nn2 = 2 * (p->body_lo[r.body + 1] - lo);
                const double2* src;
                int64_t ld;
                if (r.stage < 0) {
                    src = xroot + r.x_off;
                    ld = h->Ktot;
                } else {
                    // the body's first leaf box: the first box of its in iteration 0 with in_off 2*lo
                    const LevelFactor& f0 = h->lv[0];
                    int64_t off = -1;
                    for (int q = 0; q < f0.nb; ++q)
                        if (f0.in_off[q] == 2 * lo) { off = f0.uoff[q]; break; }
                    if (off < 0) { e = hipErrorInvalidValue; break; }
                    src = xl[0] + off;
                    ld = f0.nu;
                }
                cp.push_back(CopyJob{src, reinterpret_cast<double2*>(x) + 2 * lo, 1, ld, 1, N2,
                                     static_cast<int32_t>(nn2), static_cast<int32_t>(nrhs)});
            }
            if (e == hipSuccess) e = launch_copy(sc, cp);
        }
    }
    return e;
}

int solve_impl(const bm_hss* h, const double* b, double* x, int64_t nrhs, hipStream_t s, bool trans) {
    Scratch sc(s);
    hipError_t e = record_solve(h, sc, b, x, nrhs, trans);
    if (e == hipSuccess) e = sc.flush();
    // the job descriptors are staged from host memory: finish before releasing them
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    sc.synced();
    sc.release();
    if (e != hipSuccess) return hip_fail(e, trans ? "bm_hss_solve_transpose" : "bm_hss_solve");
    return BM_OK;
}

}  // namespace

extern "C" {

int bm_hss_build(const bm_problem* p, const bm_hss_opts* opts, hipStream_t stream, bm_hss** out) {
    clear_error();
    if (!out) return fail(BM_EINVAL, "bm_hss_build: out is null");
    *out = nullptr;
    if (!p || !opts) return fail(BM_EINVAL, "bm_hss_build: null argument");
    if (opts->leaf < 4 || !(opts->proxy_ratio > 1.0) || opts->proxy_points < 8 ||
        !(opts->id_tol > 0.0 && opts->id_tol < 1.0) || !std::isfinite(opts->proxy_ratio) ||
        opts->sketch < -1 || opts->sketch > (int64_t{1} << 20) ||
        !(opts->max_rank_ratio == -1.0 || (opts->max_rank_ratio >= 0.0 && opts->max_rank_ratio <= 1.0)) ||
        opts->kernel_timing < 0 || opts->kernel_timing > 1 || opts->proxy_fp32 < 0 || opts->proxy_fp32 > 1)
        return fail(BM_EINVAL, "bm_hss_build: need leaf >= 4, proxy_ratio > 1, proxy_points >= 8, "
                               "0 < id_tol < 1, sketch -1 or 0..2^20, max_rank_ratio -1 or in [0, 1], "
                               "kernel_timing 0 or 1, proxy_fp32 0 or 1");
    if (p->g->n > (int64_t{1} << 30)) return fail(BM_EINVAL, "bm_hss_build: N too large");
    const auto t0 = std::chrono::steady_clock::now();
    bm_hss* h = new (std::nothrow) bm_hss;
    if (!h) return fail(BM_ENOMEM, "bm_hss_build: host allocation");
    h->p = p;
    h->stream = stream;
    h->opts = *opts;
    if (h->opts.sketch == -1) h->opts.sketch = tuned::kSketchRows;
    if (h->opts.max_rank_ratio == -1.0) h->opts.max_rank_ratio = tuned::kStopRankRatio;
    h->N = p->g->n;
    int rc;
    {
        KernelTimes kt;
        struct Guard {
            ~Guard() { g_ktimes = nullptr; }
        } guard;
        g_ktimes = opts->kernel_timing ? &kt : nullptr;
        try {
            rc = build_impl(h, stream);
        } catch (const std::bad_alloc&) {
            rc = fail(BM_ENOMEM, "bm_hss_build: host allocation");
        }
        // build_impl returns after the whole build has completed
        if (rc == BM_OK && opts->kernel_timing) {
            h->stats.gemm_launches = static_cast<int64_t>(kt.gemm.size());
            h->stats.gemm_flops = kt.gemm_flops;
            h->stats.seconds_gemm = KernelTimes::seconds(kt.gemm);
            h->stats.inv_launches = static_cast<int64_t>(kt.inv.size());
            h->stats.inv_flops = kt.inv_flops;
            h->stats.seconds_inv = KernelTimes::seconds(kt.inv);
            h->stats.sketch_launches = static_cast<int64_t>(kt.sketch.size());
            h->stats.sketch_flops = kt.sketch_flops;
            h->stats.seconds_sketch = KernelTimes::seconds(kt.sketch);
            h->stats.gen_launches = static_cast<int64_t>(kt.gen.size());
            h->stats.gen_pairs = kt.gen_pairs;
            h->stats.seconds_gen = KernelTimes::seconds(kt.gen);
        }
    }
    if (rc != BM_OK) {
        (void)hipStreamSynchronize(stream);
        bm_hss_destroy(h);
        return rc;
    }
    h->stats.seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return BM_OK;
}

int bm_dense_inverse(double* a, int64_t n, int64_t ld, hipStream_t stream) {
    clear_error();
    if (!a) return fail(BM_EINVAL, "bm_dense_inverse: a is null");
    if (n < 1 || n > kDenseInverseMax || ld < n || ld > (int64_t{1} << 30))
        return fail(BM_EINVAL, "bm_dense_inverse: need 1 <= n <= 16384 and n <= ld <= 2^30");
    int32_t hs = 0;
    hipError_t e = hipSuccess;
    {
        Scratch sc(stream);
        int32_t* st = nullptr;
        e = sc.alloc(&st, 1);
        if (e == hipSuccess) {
            sc.rec([=]() { return hipMemsetAsync(st, 0, sizeof(int32_t), stream); });
            const InvJob j{reinterpret_cast<double2*>(a), st, ld, static_cast<int32_t>(n)};
            e = (n > inv_base() && n <= kRootPanelsMax && root_panels()) ? launch_inverse_panels(sc, j)
                                                                         : launch_inverse(sc, {j});
        }
        if (e == hipSuccess) e = sc.flush();
        if (e == hipSuccess) e = hipMemcpyAsync(&hs, st, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) sc.synced();
    }
    if (e != hipSuccess) return hip_fail(e, "bm_dense_inverse");
    if (hs) return fail(BM_ESINGULAR, "bm_dense_inverse: singular or tiny pivot");
    return BM_OK;
}

int bm_sketch(const double* omega, int64_t ldo, const double* x, int64_t m, int64_t n, int64_t l, double* y,
              hipStream_t stream) {
    clear_error();
    if (!omega || !x || !y) return fail(BM_EINVAL, "bm_sketch: null argument");
    if (m < 1 || n < 1 || l < 1 || m > (int64_t{1} << 30) || n > (int64_t{1} << 30) || l > (int64_t{1} << 30) ||
        ldo < m || l * n > (int64_t{1} << 34))
        return fail(BM_EINVAL, "bm_sketch: need 1 <= m, n, l <= 2^30, m <= ldo and l n <= 2^34");
    hipError_t e = hipSuccess;
    {
        Scratch sc(stream);
        SketchJob j{};
        j.x = reinterpret_cast<const double2*>(x);
        j.y = reinterpret_cast<double2*>(y);
        j.m = static_cast<int32_t>(m);
        j.n = static_cast<int32_t>(n);
        j.l = static_cast<int32_t>(l);
        e = launch_sketch(sc, {j}, omega, ldo);
        if (e == hipSuccess) e = sc.flush();
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) sc.synced();
    }
    if (e != hipSuccess) return hip_fail(e, "bm_sketch");
    return BM_OK;
}

int bm_interp_decomp(int32_t nb, const int32_t* m, const int32_t* n, double* x, double tol, int32_t* ranks,
                     int32_t* perm, double* T, hipStream_t stream) {
    clear_error();
    if (!m || !n || !x || !ranks || !perm || !T) return fail(BM_EINVAL, "bm_interp_decomp: null argument");
    if (nb < 1 || nb > kInterpDecompMaxBatch || !(tol >= 0.0 && tol < 1.0))
        return fail(BM_EINVAL, "bm_interp_decomp: need 1 <= nb <= 65535 and 0 <= tol < 1");
    for (int32_t b = 0; b < nb; ++b)
        if (m[b] < 1 || n[b] < 1 || m[b] > kInterpDecompMaxDim || n[b] > kInterpDecompMaxDim)
            return fail(BM_EINVAL, "bm_interp_decomp: need 1 <= m, n <= 4096 for every matrix");
    std::vector<CpqrJob> cj(nb);
    std::vector<int64_t> toff(nb);
    int64_t xo = 0, po = 0, to = 0, nmax = 1;
    hipError_t e = hipSuccess;
    std::vector<int32_t> rk(nb);
    {
        Scratch sc(stream);
        double2* rdiag = nullptr;
        int32_t* dranks = nullptr;
        for (int32_t b = 0; b < nb; ++b) po += n[b];
        e = sc.alloc(&rdiag, po);
        if (e == hipSuccess) e = sc.alloc(&dranks, nb);
        po = 0;
        for (int32_t b = 0; b < nb; ++b) {
            cj[b] = CpqrJob{reinterpret_cast<double2*>(x) + xo, perm + po, rdiag + po, nullptr, nullptr, nullptr,
                            n[b], m[b]};
            toff[b] = to;
            xo += static_cast<int64_t>(m[b]) * n[b];
            po += n[b];
            to += static_cast<int64_t>(n[b]) * n[b];
            nmax = std::max<int64_t>(nmax, n[b]);
        }
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&ev0);
        if (e == hipSuccess) e = hipEventCreate(&ev1);
        if (ev0) sc.events.push_back(ev0);
        if (ev1) sc.events.push_back(ev1);
        CpqrJob* dcj = nullptr;
        int64_t launches = 0;
        bool fused = false;
        if (e == hipSuccess)
            e = run_cpqr(sc, cj, &dcj, dranks, tol, rk, ev0, ev1, &launches, static_cast<int>(nmax / 2), &fused,
                         []() { return hipSuccess; });
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) sc.synced();
        // T = [I; (R11^-1 R12)^T] in pivoted order, each in its n x n slot
        int64_t* dtoff = nullptr;
        if (e == hipSuccess) e = sc.upload(&dtoff, toff);
        if (e == hipSuccess) e = sc.flush();
        if (e == hipSuccess) e = hipMemsetAsync(T, 0, static_cast<size_t>(to) * sizeof(double2), stream);
        int64_t cmax = 1, kmax = 0;
        for (int32_t b = 0; b < nb; ++b) {
            cmax = std::max<int64_t>(cmax, n[b] - rk[b]);
            kmax = std::max<int64_t>(kmax, rk[b]);
        }
        if (e == hipSuccess) {
            const int rpl = kmax <= 64 ? 1 : kmax <= 128 ? 2 : kmax <= 256 ? 4 : 0;
            const dim3 g(static_cast<unsigned>(ceil_div(cmax, kThreads / 64)), static_cast<unsigned>(nb)), bl(kThreads);
            double2* Td = reinterpret_cast<double2*>(T);
            switch (rpl) {
                case 1: hipLaunchKernelGGL(k_interp_wave<1>, g, bl, 0, stream, dcj, dranks, dtoff, Td); break;
                case 2: hipLaunchKernelGGL(k_interp_wave<2>, g, bl, 0, stream, dcj, dranks, dtoff, Td); break;
                case 4: hipLaunchKernelGGL(k_interp_wave<4>, g, bl, 0, stream, dcj, dranks, dtoff, Td); break;
                default: hipLaunchKernelGGL(k_interp, g, bl, 0, stream, dcj, dranks, dtoff, Td); break;
            }
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) sc.synced();
    }
    if (e != hipSuccess) return hip_fail(e, "bm_interp_decomp");
    std::copy(rk.begin(), rk.end(), ranks);
    return BM_OK;
}

int bm_hss_solve(const bm_hss* h, const double* b, double* x, int64_t nrhs, hipStream_t s) {
    clear_error();
    if (!h || !b || !x) return fail(BM_EINVAL, "bm_hss_solve: null argument");
    if (nrhs < 1 || nrhs > (int64_t{1} << 20)) return fail(BM_EINVAL, "bm_hss_solve: nrhs out of range");
    return solve_impl(h, b, x, nrhs, s, false);
}

int bm_hss_solve_transpose(const bm_hss* h, const double* b, double* x, int64_t nrhs, hipStream_t s) {
    clear_error();
    if (!h || !b || !x) return fail(BM_EINVAL, "bm_hss_solve_transpose: null argument");
    if (nrhs < 1 || nrhs > (int64_t{1} << 20))
        return fail(BM_EINVAL, "bm_hss_solve_transpose: nrhs out of range");
    return solve_impl(h, b, x, nrhs, s, true);
}

int bm_hss_solve_graph(const bm_hss* h, const double* b, double* x, int64_t nrhs, int transpose, hipStream_t s) {
    clear_error();
    if (!h || !b || !x) return fail(BM_EINVAL, "bm_hss_solve_graph: null argument");
    if (nrhs < 1 || nrhs > (int64_t{1} << 20)) return fail(BM_EINVAL, "bm_hss_solve_graph: nrhs out of range");
    if (transpose != 0 && transpose != 1) return fail(BM_EINVAL, "bm_hss_solve_graph: transpose must be 0 or 1");
    std::lock_guard<std::mutex> lk(h->plan_mu);
    bm_hss::SolvePlan* plan = nullptr;
    for (auto& q : h->plans)
        if (q->nrhs == nrhs && q->trans == (transpose != 0)) plan = q.get();
    const size_t bytes = static_cast<size_t>(2 * h->N * nrhs) * sizeof(double2);
    if (!plan) {
        const char* where = nullptr;
        const hipError_t e = make_solve_plan(h, nrhs, transpose != 0, &plan, &where);
        if (e != hipSuccess) return hip_fail(e, where);
    }
    BM_HIP(hipMemcpyAsync(plan->bin, b, bytes, hipMemcpyDeviceToDevice, s));
    BM_HIP(hipGraphLaunch(plan->exec, s));
    BM_HIP(hipMemcpyAsync(x, plan->xout, bytes, hipMemcpyDeviceToDevice, s));
    BM_HIP(hipEventRecord(plan->done, s));
    return BM_OK;
}

int bm_hss_stats(const bm_hss* h, bm_hss_stats_t* out) {
    clear_error();
    if (!h || !out) return fail(BM_EINVAL, "bm_hss_stats: null argument");
    *out = h->stats;
    out->sketch = h->opts.sketch;
    out->max_rank_ratio = h->opts.max_rank_ratio;
    return BM_OK;
}

int bm_hss_level(const bm_hss* h, int level, bm_hss_level_t* out) {
    clear_error();
    if (!h || !out) return fail(BM_EINVAL, "bm_hss_level: null argument");
    if (level < 0 || level >= static_cast<int>(h->level_info.size()))
        return fail(BM_EINVAL, "bm_hss_level: level out of range");
    *out = h->level_info[level];
    return BM_OK;
}

int bm_hss_destroy(bm_hss* h) {
    if (!h) return BM_OK;
    h->plans.clear();   // waits for their last launches
    // nothing else can still use the factors: the build and the eager solves
    // return after completion and the graph-replayed solves were waited for
    // above, so the blocks go back to the allocator reusable on any stream (the
    // next build allocates its factors on its second stream)
    for (auto& f : h->lv) {
        dev_free_idle(f.E);
        dev_free_idle(f.Ft);
        dev_free_idle(f.G);
    }
    dev_free_idle(h->Rinv);
    delete h;
    return BM_OK;
}

}  // extern "C"
