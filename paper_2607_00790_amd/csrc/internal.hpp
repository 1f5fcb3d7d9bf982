// Library-internal declarations shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bmhss.h"
#include "wsbm_pair.hpp"

// Device node data of a discretised boundary: six FP64 rows of length n
// (x, y, nx, ny, w, kappa) and the index of the closed curve of each node.
struct bm_geom {
    int64_t n = 0;
    int ncurves = 0;
    double* soa = nullptr;    // device, 6 * n
    int32_t* curve = nullptr; // device, n
    int device = 0;
    std::vector<int64_t> curve_lo;   // host: first node of each curve (ncurves + 1)
    double* xyd = nullptr;    // device, 6 * n: the samples x, y, x', y', x'', y'' as given
    std::vector<double> host_xy;   // host, 2 * n: the node coordinates x then y (the HSS tree's box geometry)
};

// A problem: one geometry split into independent bodies (consecutive runs of
// curves), each with its own media.  Pairs in different bodies give zero
// blocks, so the system is block diagonal over the bodies.
struct bm_problem {
    const bm_geom* g = nullptr;
    int nbodies = 1;
    std::vector<bm::Media> media;        // host, per body
    std::vector<int64_t> body_lo;        // host, first node of each body (nbodies + 1)
    bm::Media* d_media = nullptr;        // device copy of media
    int32_t* d_body = nullptr;           // device, body of each node (nullptr: one body)
    int64_t* d_body_lo = nullptr;        // device copy of body_lo
    std::vector<int64_t> tile_off;       // host: first 256 x 256 pair tile of each body (nbodies + 1)
    int64_t* d_tile_off = nullptr;       // device copy of tile_off
    int32_t* d_body_all = nullptr;       // device, body of each node (zeros for one body)
    const float* d_ftab = nullptr;       // device FP32 copy of the coefficient table
};

namespace bm {

// thread-local error reporting
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
void clear_error();

#define BM_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::bm::hip_fail(e_, #call);        \
    } while (0)

// Node fields as separate row pointers.
struct NodeView {
    const double* x;
    const double* y;
    const double* nx;
    const double* ny;
    const double* w;
    const double* kappa;
    const int32_t* curve;
    const int32_t* body;   // body of each node; nullptr when the problem has one body
};

inline NodeView view(const bm_geom* g, const int32_t* body = nullptr) {
    const int64_t n = g->n;
    return NodeView{g->soa, g->soa + n, g->soa + 2 * n, g->soa + 3 * n,
                    g->soa + 4 * n, g->soa + 5 * n, g->curve, body};
}

inline NodeView view(const bm_problem* p) { return view(p->g, p->d_body); }

// Caching device allocator (devmem.hip): blocks are reused only on the stream
// they were released on.
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
// release a block that no queued or running work uses any more
void dev_free_idle(void* p);

// Kernel launchers (assemble.hip)
hipError_t launch_geometry(const double* xyd, const int64_t* offsets, int ncurves, int64_t n,
                           double* soa, int32_t* curve, hipStream_t s);
// `media` is the device array of per-body media (NodeView::body selects).
// `tab` is the device coefficient table (the one every Media points to), passed
// to the kernels as an argument of its own.
hipError_t launch_dense(const NodeView& v, int64_t n, const Media* media, const BesselTable* tab, double* A,
                        int64_t ld, hipStream_t s);
hipError_t launch_rhs_plane_wave(const NodeView& v, int64_t n, const Media* media, double angle,
                                 double* rhs, hipStream_t s);
// rhs (2N complex) from u_in and du_in/dn at the nodes (N complex each)
hipError_t launch_rhs_incident(const NodeView& v, int64_t n, const Media* media, const double* uin,
                               const double* dn_uin, double* rhs, hipStream_t s);

// Public block and proxy entry points through the HSS entry generator
// (gen_api.hip).  body_all: device body of every node (zeros for one body);
// ftab: the device FP32 coefficient table; prec 0 = FP64, 1 = FP32 arithmetic.
hipError_t launch_block(const NodeView& v, const int32_t* body_all, const Media* media, const BesselTable* tab,
                        const float* ftab, const int64_t* rows, int64_t nr, const int64_t* cols, int64_t nc,
                        int prec, double* out, int64_t ld, hipStream_t s);
hipError_t launch_proxy(const NodeView& v, int64_t n_nodes, const Media* media, const BesselTable* tab,
                        const float* ftab, const int64_t* nodes, int64_t n, const double* pts, int64_t P, int dir,
                        int prec, double* out, int64_t ld, hipStream_t s);
// matrix-free product over the bodies' diagonal blocks (max_body = largest body
// in nodes, body_lo = device node offsets of the bodies); `work` is a device
// buffer of matvec_work_doubles(n, max_body) doubles
hipError_t launch_matvec(const NodeView& v, int64_t n, int64_t max_body, const int64_t* body_lo,
                         const Media* media, const BesselTable* tab, const double* x, double* y, double* work,
                         hipStream_t s);
int64_t matvec_work_doubles(int64_t n, int64_t max_body);
// Size of the fixed device buffer of bm_matvec_noalloc, in doubles (16 MiB):
// enough for one body of up to 32768 nodes.
constexpr int64_t kNoAllocScratchDoubles = int64_t{1} << 21;
// Address of that buffer on the current device (looked up once per device).
hipError_t noalloc_scratch(double** out);
// far field of every body: uinf[b * nang + a]; body_lo = first node of each body
hipError_t launch_far_field(const NodeView& v, int nbodies, const int64_t* body_lo, const Media* media,
                            const double* phi, const double* angles, int64_t nang, double* uinf,
                            hipStream_t s);

// Adjoint kernels (adjoint.hip).
// far-field weights g (2N complex): u_inf,b(angle) = sum over body b's unknowns of g_k phi_k
hipError_t launch_far_weights(const NodeView& v, int64_t n, const Media* media, double angle, double* g,
                              hipStream_t s);
// pair tiles of a body of `nodes` nodes in the shape-derivative kernel
int64_t pair_tiles(int64_t nodes);
// device work buffer of the shape derivative, in doubles
int64_t shape_work_doubles(int64_t n, int nbodies);
// grad (6 x n) = Re(coef_b dL/d samples), L = g^T phi + lam^T (b - A phi) per body;
// coef null: coef_b = 2 conj(u_inf,b(obs)) (J = |u_inf|^2)
hipError_t launch_shape_derivative(const NodeView& v, const double* xyd, int64_t n, int nbodies,
                                   const int64_t* body_lo, const int64_t* tile_off, int64_t ntiles,
                                   const Media* media, const BesselTable* tab, const double* phi,
                                   const double* lam, double inc, double obs, const double* coef, double* grad,
                                   double* work, hipStream_t s);
hipError_t launch_fourier_curve(const double* coef, int M, double R, double cx, double cy, int64_t n, double* xyd,
                                hipStream_t s);
hipError_t launch_fourier_chain(const double* grad, int64_t n, int M, double R, double* out, hipStream_t s);

}  // namespace bm
