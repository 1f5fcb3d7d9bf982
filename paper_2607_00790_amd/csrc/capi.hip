// C-ABI entry points declared in include/bmhss.h: argument validation, handle
// management and error reporting.  All arithmetic runs in the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <string>
#include <vector>

#include "internal.hpp"
#include "wsbm_pair_f32.hpp"

namespace bm {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP;
}

void clear_error() { g_last_error.clear(); }

namespace {

// The coefficient table, copied once to every device the library runs on.
std::mutex g_table_mu;
std::unordered_map<int, BesselTable*> g_tables;

hipError_t device_table(const BesselTable** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_tables.find(dev);
    if (it != g_tables.end()) {
        *out = it->second;
        return hipSuccess;
    }
    BesselTable* d = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&d), sizeof(BesselTable));
    if (e == hipSuccess) e = hipMemcpy(d, &bm_bessel_coef::kTable, sizeof(BesselTable), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return e;
    }
    g_tables[dev] = d;
    *out = d;
    return hipSuccess;
}

// The FP32 copy of the table (entry for entry, rounded to nearest), for the
// FP32 entry path; one per device.
std::unordered_map<int, float*> g_ftables;

hipError_t device_table_f32(const float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_ftables.find(dev);
    if (it != g_ftables.end()) {
        *out = it->second;
        return hipSuccess;
    }
    std::vector<float> h(f32::kTableEntries);
    const double* src = reinterpret_cast<const double*>(&bm_bessel_coef::kTable);
    for (int q = 0; q < f32::kTableEntries; ++q) h[q] = static_cast<float>(src[q]);
    float* d = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&d), h.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return e;
    }
    g_ftables[dev] = d;
    *out = d;
    return hipSuccess;
}

bool finite_media(const bm_media* m) {
    return std::isfinite(m->k0) && std::isfinite(m->k1) && std::isfinite(m->eps0) &&
           std::isfinite(m->eps1) && m->k0 > 0 && m->k1 > 0 && m->eps0 > 0 && m->eps1 > 0;
}

// A 1D launch may not exceed 2^32 - 1 work-items: with 256-thread workgroups
// that is 2^24 - 1 workgroups.
constexpr int64_t kMaxGrid = 0xFFFFFFFFll / 256;

}  // namespace
}  // namespace bm

using namespace bm;

extern "C" {

const char* bm_last_error(void) { return g_last_error.c_str(); }

int bm_geom_create(int ncurves, const int64_t* n_per_curve, const double* xyd, int on_device,
                   hipStream_t stream, bm_geom** out) {
    clear_error();
    if (!out) return fail(BM_EINVAL, "bm_geom_create: out is null");
    *out = nullptr;
    if (ncurves <= 0 || !n_per_curve || !xyd)
        return fail(BM_EINVAL, "bm_geom_create: need ncurves > 0 and non-null arrays");
    std::vector<int64_t> offsets(ncurves + 1, 0);
    for (int c = 0; c < ncurves; ++c) {
        if (n_per_curve[c] < 8)
            return fail(BM_EINVAL, "bm_geom_create: every curve needs at least 8 nodes");
        offsets[c + 1] = offsets[c] + n_per_curve[c];
    }
    const int64_t n = offsets[ncurves];
    if (n > (int64_t{1} << 31))
        return fail(BM_EINVAL, "bm_geom_create: more than 2^31 nodes");
    // host copy for validation
    std::vector<double> h(6 * static_cast<size_t>(n));
    if (on_device) {
        BM_HIP(hipMemcpyAsync(h.data(), xyd, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                              stream));
        BM_HIP(hipStreamSynchronize(stream));
    } else {
        std::memcpy(h.data(), xyd, h.size() * sizeof(double));
    }
    for (double v : h)
        if (!std::isfinite(v)) return fail(BM_EINVAL, "bm_geom_create: non-finite coordinates");
    for (int c = 0; c < ncurves; ++c) {
        // signed area (shoelace on the trapezoidal rule) must be positive: ccw
        double area = 0;
        for (int64_t j = offsets[c]; j < offsets[c + 1]; ++j) {
            const double s2 = h[2 * n + j] * h[2 * n + j] + h[3 * n + j] * h[3 * n + j];
            if (!(s2 > 0)) return fail(BM_EINVAL, "bm_geom_create: zero speed |x'(t)|");
            area += h[j] * h[3 * n + j] - h[n + j] * h[2 * n + j];
        }
        if (!(area > 0))
            return fail(BM_EINVAL, "bm_geom_create: curve " + std::to_string(c) +
                                       " is not counter-clockwise");
    }
    bm_geom* g = new (std::nothrow) bm_geom;
    if (!g) return fail(BM_ENOMEM, "bm_geom_create: host allocation");
    g->n = n;
    g->ncurves = ncurves;
    g->curve_lo = offsets;
    g->host_xy.assign(h.begin(), h.begin() + 2 * n);   // the nodes are the samples themselves
    (void)hipGetDevice(&g->device);
    double* d_xyd = nullptr;
    int64_t* d_off = nullptr;
    hipError_t e = hipMalloc(&g->soa, 6 * n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&g->curve, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_xyd, 6 * n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_off, (ncurves + 1) * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_xyd, h.data(), 6 * n * sizeof(double), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, offsets.data(), (ncurves + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_geometry(d_xyd, d_off, ncurves, n, g->soa, g->curve, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    g->xyd = d_xyd;   // kept: the shape derivative's chain rule needs the samples
    (void)hipFree(d_off);
    if (e != hipSuccess) {
        bm_geom_destroy(g);
        return hip_fail(e, "bm_geom_create");
    }
    *out = g;
    return BM_OK;
}

int bm_geom_destroy(bm_geom* g) {
    if (!g) return BM_OK;
    (void)hipFree(g->soa);
    (void)hipFree(g->curve);
    (void)hipFree(g->xyd);
    delete g;
    return BM_OK;
}

int64_t bm_geom_size(const bm_geom* g) { return g ? g->n : -1; }

int bm_geom_nodes(const bm_geom* g, double* soa, hipStream_t stream) {
    clear_error();
    if (!g || !soa) return fail(BM_EINVAL, "bm_geom_nodes: null argument");
    BM_HIP(hipMemcpyAsync(soa, g->soa, 6 * g->n * sizeof(double), hipMemcpyDeviceToDevice,
                          stream));
    return BM_OK;
}

int bm_problem_create_bodies(const bm_geom* g, int nbodies, const int32_t* body_of_curve,
                             const bm_media* media, bm_problem** out) {
    clear_error();
    if (!out) return fail(BM_EINVAL, "bm_problem_create: out is null");
    *out = nullptr;
    if (!g || !media || (nbodies > 1 && !body_of_curve))
        return fail(BM_EINVAL, "bm_problem_create: null argument");
    if (nbodies < 1) return fail(BM_EINVAL, "bm_problem_create: need nbodies >= 1");
    for (int b = 0; b < nbodies; ++b)
        if (!finite_media(media + b))
            return fail(BM_EINVAL, "bm_problem_create: wavenumbers and permittivities must be finite and > 0");
    if (nbodies > g->ncurves)
        return fail(BM_EINVAL, "bm_problem_create: more bodies than curves");
    // bodies are consecutive runs of curves: body_of_curve = 0, .., 0, 1, .., nbodies - 1
    std::vector<int64_t> lo(nbodies + 1, 0);
    if (body_of_curve) {
        if (body_of_curve[0] != 0 || body_of_curve[g->ncurves - 1] != nbodies - 1)
            return fail(BM_EINVAL, "bm_problem_create: body_of_curve must run from 0 to nbodies - 1");
        for (int c = 1; c < g->ncurves; ++c) {
            const int32_t d = body_of_curve[c] - body_of_curve[c - 1];
            if (d != 0 && d != 1)
                return fail(BM_EINVAL, "bm_problem_create: body_of_curve must be non-decreasing in steps of 1");
            if (d == 1) lo[body_of_curve[c]] = g->curve_lo[c];
        }
    }
    lo[nbodies] = g->n;
    std::vector<int64_t> tiles(nbodies + 1, 0);
    for (int b = 0; b < nbodies; ++b) tiles[b + 1] = tiles[b] + pair_tiles(lo[b + 1] - lo[b]);
    const BesselTable* tab = nullptr;
    BM_HIP(device_table(&tab));
    const float* ftab = nullptr;
    BM_HIP(device_table_f32(&ftab));
    bm_problem* p = new (std::nothrow) bm_problem;
    if (!p) return fail(BM_ENOMEM, "bm_problem_create: host allocation");
    p->g = g;
    p->nbodies = nbodies;
    p->d_ftab = ftab;
    p->body_lo = lo;
    p->tile_off = tiles;
    for (int b = 0; b < nbodies; ++b)
        p->media.push_back(make_media(media[b].k0, media[b].k1, media[b].eps0, media[b].eps1, tab));
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->d_media), nbodies * sizeof(Media));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_media, p->media.data(), nbodies * sizeof(Media), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_body_lo), (nbodies + 1) * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_body_lo, lo.data(), (nbodies + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_tile_off), (nbodies + 1) * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_tile_off, tiles.data(), (nbodies + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        std::vector<int32_t> nb(static_cast<size_t>(g->n));
        for (int b = 0; b < nbodies; ++b)
            for (int64_t i = lo[b]; i < lo[b + 1]; ++i) nb[i] = b;
        e = hipMalloc(reinterpret_cast<void**>(&p->d_body_all), g->n * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemcpy(p->d_body_all, nb.data(), g->n * sizeof(int32_t), hipMemcpyHostToDevice);
        // kernels that test for one body read a null body array
        if (e == hipSuccess && nbodies > 1) p->d_body = p->d_body_all;
    }
    if (e != hipSuccess) {
        bm_problem_destroy(p);
        return hip_fail(e, "bm_problem_create");
    }
    *out = p;
    return BM_OK;
}

int bm_problem_create(const bm_geom* g, const bm_media* media, bm_problem** out) {
    return bm_problem_create_bodies(g, 1, nullptr, media, out);
}

int bm_problem_destroy(bm_problem* p) {
    if (!p) return BM_OK;
    (void)hipFree(p->d_media);
    (void)hipFree(p->d_body_all);   // p->d_body is null or the same array
    (void)hipFree(p->d_body_lo);
    (void)hipFree(p->d_tile_off);
    delete p;
    return BM_OK;
}

int bm_rhs_plane_wave(const bm_problem* p, double angle, double* rhs, hipStream_t stream) {
    clear_error();
    if (!p || !rhs) return fail(BM_EINVAL, "bm_rhs_plane_wave: null argument");
    if (!std::isfinite(angle)) return fail(BM_EINVAL, "bm_rhs_plane_wave: non-finite angle");
    BM_HIP(launch_rhs_plane_wave(view(p), p->g->n, p->d_media, angle, rhs, stream));
    return BM_OK;
}

int bm_rhs_incident(const bm_problem* p, const double* uin, const double* dn_uin, double* rhs,
                    hipStream_t stream) {
    clear_error();
    if (!p || !uin || !dn_uin || !rhs) return fail(BM_EINVAL, "bm_rhs_incident: null argument");
    if (rhs == uin || rhs == dn_uin) return fail(BM_EINVAL, "bm_rhs_incident: rhs must not alias the inputs");
    BM_HIP(launch_rhs_incident(view(p), p->g->n, p->d_media, uin, dn_uin, rhs, stream));
    return BM_OK;
}

int bm_assemble_dense(const bm_problem* p, double* A, int64_t ld, hipStream_t stream) {
    clear_error();
    if (!p || !A) return fail(BM_EINVAL, "bm_assemble_dense: null argument");
    const int64_t n = p->g->n;
    if (ld < 2 * n) return fail(BM_EINVAL, "bm_assemble_dense: ld < 2N");
    if (n * ((n + 255) / 256) > kMaxGrid) return fail(BM_EINVAL, "bm_assemble_dense: N too large");
    BM_HIP(launch_dense(view(p), n, p->d_media, p->media[0].tab, A, ld, stream));
    return BM_OK;
}

int bm_assemble_block(const bm_problem* p, const int64_t* rows, int64_t nr, const int64_t* cols,
                      int64_t nc, double* out, int64_t ld, int prec, hipStream_t stream) {
    clear_error();
    if (!p) return fail(BM_EINVAL, "bm_assemble_block: null problem");
    if (nr < 0 || nc < 0) return fail(BM_EINVAL, "bm_assemble_block: negative size");
    if (prec != 0 && prec != 1) return fail(BM_EINVAL, "bm_assemble_block: prec must be 0 (FP64) or 1 (FP32)");
    if (nr == 0 || nc == 0) return BM_OK;
    if (!rows || !cols || !out) return fail(BM_EINVAL, "bm_assemble_block: null array");
    if (ld < 2 * nc) return fail(BM_EINVAL, "bm_assemble_block: ld < 2 nc");
    if (nr >= (int64_t{1} << 30) || nc >= (int64_t{1} << 30) || (nr * nc + 255) / 256 > kMaxGrid)
        return fail(BM_EINVAL, "bm_assemble_block: too large");
    BM_HIP(launch_block(view(p), p->d_body_all, p->d_media, p->media[0].tab, p->d_ftab, rows, nr, cols, nc, prec,
                        out, ld, stream));
    return BM_OK;
}

int bm_assemble_proxy(const bm_problem* p, const int64_t* nodes, int64_t n, const double* pts,
                      int64_t P, int dir, double* out, int64_t ld, int prec, hipStream_t stream) {
    clear_error();
    if (!p) return fail(BM_EINVAL, "bm_assemble_proxy: null problem");
    if (n < 0 || P < 0) return fail(BM_EINVAL, "bm_assemble_proxy: negative size");
    if (dir != 0 && dir != 1) return fail(BM_EINVAL, "bm_assemble_proxy: dir must be 0 or 1");
    if (prec != 0 && prec != 1) return fail(BM_EINVAL, "bm_assemble_proxy: prec must be 0 (FP64) or 1 (FP32)");
    if (n == 0 || P == 0) return BM_OK;
    if (!nodes || !pts || !out) return fail(BM_EINVAL, "bm_assemble_proxy: null array");
    const int64_t ncol = dir == 0 ? P : n;
    if (ld < 2 * ncol) return fail(BM_EINVAL, "bm_assemble_proxy: ld too small");
    if (n >= (int64_t{1} << 30) || P >= (int64_t{1} << 30) || p->g->n + P >= (int64_t{1} << 31) ||
        (n * P + 255) / 256 > kMaxGrid)
        return fail(BM_EINVAL, "bm_assemble_proxy: too large");
    BM_HIP(launch_proxy(view(p), p->g->n, p->d_media, p->media[0].tab, p->d_ftab, nodes, n, pts, P, dir, prec, out,
                        ld, stream));
    return BM_OK;
}

int bm_matvec(const bm_problem* p, const double* x, double* y, hipStream_t stream) {
    clear_error();
    if (!p || !x || !y) return fail(BM_EINVAL, "bm_matvec: null argument");
    if (x == y) return fail(BM_EINVAL, "bm_matvec: x and y must not alias");
    int64_t max_body = 0;
    for (int b = 0; b < p->nbodies; ++b) max_body = std::max(max_body, p->body_lo[b + 1] - p->body_lo[b]);
    const int64_t n = p->g->n;
    if ((max_body + 255) / 256 > kMaxGrid) return fail(BM_EINVAL, "bm_matvec: body too large");
    void* work = nullptr;
    BM_HIP(dev_alloc(&work, matvec_work_doubles(n, max_body) * sizeof(double), stream));
    const hipError_t e = launch_matvec(view(p), n, max_body, p->d_body_lo, p->d_media, p->media[0].tab, x, y,
                                       static_cast<double*>(work), stream);
    dev_free(work, stream);
    if (e != hipSuccess) return hip_fail(e, "bm_matvec");
    return BM_OK;
}

int bm_matvec_noalloc(const bm_problem* p, const double* x, double* y, hipStream_t stream) {
    clear_error();
    if (!p || !x || !y) return fail(BM_EINVAL, "bm_matvec_noalloc: null argument");
    if (x == y) return fail(BM_EINVAL, "bm_matvec_noalloc: x and y must not alias");
    int64_t max_body = 0;
    for (int b = 0; b < p->nbodies; ++b) max_body = std::max(max_body, p->body_lo[b + 1] - p->body_lo[b]);
    const int64_t n = p->g->n;
    const int64_t need = matvec_work_doubles(n, max_body);
    if (need > kNoAllocScratchDoubles)
        return fail(BM_EINVAL, "bm_matvec_noalloc: needs " + std::to_string(need) +
                                   " doubles of partial sums, above its fixed buffer of " +
                                   std::to_string(kNoAllocScratchDoubles) + " (use bm_matvec)");
    double* work = nullptr;
    BM_HIP(noalloc_scratch(&work));
    BM_HIP(launch_matvec(view(p), n, max_body, p->d_body_lo, p->d_media, p->media[0].tab, x, y, work, stream));
    return BM_OK;
}

int bm_far_field(const bm_problem* p, const double* phi, const double* angles, int64_t nang,
                 double* uinf, hipStream_t stream) {
    clear_error();
    if (!p || nang < 0) return fail(BM_EINVAL, "bm_far_field: bad argument");
    if (nang == 0) return BM_OK;
    if (!phi || !angles || !uinf) return fail(BM_EINVAL, "bm_far_field: null array");
    if (nang > (int64_t{1} << 31)) return fail(BM_EINVAL, "bm_far_field: too many angles");
    BM_HIP(launch_far_field(view(p), p->nbodies, p->d_body_lo, p->d_media, phi, angles, nang, uinf, stream));
    return BM_OK;
}

int bm_far_field_weights(const bm_problem* p, double angle, double* g, hipStream_t stream) {
    clear_error();
    if (!p || !g) return fail(BM_EINVAL, "bm_far_field_weights: null argument");
    if (!std::isfinite(angle)) return fail(BM_EINVAL, "bm_far_field_weights: non-finite angle");
    BM_HIP(launch_far_weights(view(p), p->g->n, p->d_media, angle, g, stream));
    return BM_OK;
}

int bm_shape_derivative(const bm_problem* p, const double* phi, const double* lam, double inc_angle,
                        double obs_angle, const double* coef, double* grad, hipStream_t stream) {
    clear_error();
    if (!p || !phi || !lam || !grad) return fail(BM_EINVAL, "bm_shape_derivative: null argument");
    if (!std::isfinite(inc_angle) || !std::isfinite(obs_angle))
        return fail(BM_EINVAL, "bm_shape_derivative: non-finite angle");
    const int64_t n = p->g->n;
    const int64_t ntiles = p->tile_off[p->nbodies];
    void* work = nullptr;
    BM_HIP(dev_alloc(&work, shape_work_doubles(n, p->nbodies) * sizeof(double), stream));
    const hipError_t e = launch_shape_derivative(view(p), p->g->xyd, n, p->nbodies, p->d_body_lo, p->d_tile_off,
                                                 ntiles, p->d_media, p->media[0].tab, phi, lam, inc_angle,
                                                 obs_angle, coef, grad,
                                                 static_cast<double*>(work), stream);
    dev_free(work, stream);
    if (e != hipSuccess) return hip_fail(e, "bm_shape_derivative");
    return BM_OK;
}

int bm_fourier_curve(const double* coef, int nmodes, double radius, double cx, double cy, int64_t n,
                     double* xyd, hipStream_t stream) {
    clear_error();
    if (!xyd || (nmodes > 0 && !coef)) return fail(BM_EINVAL, "bm_fourier_curve: null argument");
    if (nmodes < 0 || n < 1 || n > (int64_t{1} << 31) || !(radius > 0) || !std::isfinite(radius) ||
        !std::isfinite(cx) || !std::isfinite(cy))
        return fail(BM_EINVAL, "bm_fourier_curve: need nmodes >= 0, 1 <= n <= 2^31, finite radius > 0");
    BM_HIP(launch_fourier_curve(coef, nmodes, radius, cx, cy, n, xyd, stream));
    return BM_OK;
}

int bm_fourier_chain(const double* grad, int64_t n, int nmodes, double radius, double* out, hipStream_t stream) {
    clear_error();
    if (!grad || !out) return fail(BM_EINVAL, "bm_fourier_chain: null argument");
    if (nmodes < 1 || nmodes > (1 << 20) || n < 1 || n > (int64_t{1} << 31) || !(radius > 0) ||
        !std::isfinite(radius))
        return fail(BM_EINVAL, "bm_fourier_chain: need 1 <= nmodes <= 2^20, 1 <= n <= 2^31, finite radius > 0");
    BM_HIP(launch_fourier_chain(grad, n, nmodes, radius, out, stream));
    return BM_OK;
}

}  // extern "C"
