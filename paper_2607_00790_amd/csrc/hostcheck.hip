// Host-compiled instances of the device math (bessel.hpp, wsbm_pair.hpp) for
// CPU unit tests.  This library is loaded only by the test suite, to check the
// kernels' arithmetic without a GPU; the product library never calls it.
#include <cmath>
#include <cstdint>
#include <vector>

#include "hss_plan.hpp"
#include "wsbm_adjoint.hpp"
#include "wsbm_pair_f32.hpp"

extern "C" {

// The ID work guard's decisions (hss_plan.hpp): bit 0 = a box of rows x
// unknowns is over the per-box budget, bit 1 = a level total of `total`
// entries is over the per-body budget.
int bmh_id_guard(int64_t rows, int64_t unknowns, int64_t total) {
    return (bm::hss::id_box_over_budget(rows, unknowns) ? 1 : 0) | (bm::hss::id_level_over_budget(total) ? 2 : 0);
}

// The boxes of one level of a body's tree (hss_plan.hpp): centre, proxy
// radius (box_c, 3 per box) and proxy points (box_p) of its 2^l boxes.
void bmh_level_box_geometry(const double* x, const double* y, int64_t nlo, int64_t nn, int l, double proxy_ratio,
                            int64_t P, int adapt, double kmax, double* box_c, int32_t* box_p) {
    bm::hss::level_box_geometry(x, y, nlo, nn, l, proxy_ratio, P, adapt != 0, kmax, box_c, box_p);
}

// Blocks A(rows, cols) in FP32 arithmetic, as the FP32 entry path forms them
// (coefficients rounded to FP32 entry by entry); arguments as
// bmh_system_blocks, one curve per node given by `curve`.
int bmh_system_blocks_f32(const double* soa, const int32_t* curve, int64_t N, const int64_t* rows, int64_t nr,
                          const int64_t* cols, int64_t nc, const double* media, double* out) {
    const bm::Media m = bm::make_media(media[0], media[1], media[2], media[3], &bm_bessel_coef::kTable);
    const bm::f32::MediaF mf = bm::f32::media_f(m);
    std::vector<float> ft(bm::f32::kTableEntries);
    const double* src = reinterpret_cast<const double*>(&bm_bessel_coef::kTable);
    for (int q = 0; q < bm::f32::kTableEntries; ++q) ft[q] = static_cast<float>(src[q]);
    const double *x = soa, *y = soa + N, *nx = soa + 2 * N, *ny = soa + 3 * N, *w = soa + 4 * N,
                 *kap = soa + 5 * N;
    const int64_t ld = 2 * nc;
    for (int64_t a = 0; a < nr; ++a) {
        for (int64_t b = 0; b < nc; ++b) {
            const int64_t i = rows[a], j = cols[b];
            bm::Block blk;
            if (i == j) {
                blk = bm::f32::diag_block(static_cast<float>(w[j]), static_cast<float>(kap[j]), mf);
            } else {
                const bm::f32::PairGeomF g = bm::f32::pair_geom(
                    x[i], y[i], static_cast<float>(nx[i]), static_cast<float>(ny[i]), x[j], y[j],
                    static_cast<float>(nx[j]), static_cast<float>(ny[j]));
                const bm::f32::Hankel01F h1 =
                    bm::f32::pair_interior(g, mf, curve[i] == curve[j], &bm_bessel_coef::kTable, ft.data());
                float r0[4], r1[4];
                bm::f32::pair_row0(g, h1, static_cast<float>(w[j]), mf, r0);
                bm::f32::pair_row1(g, h1, static_cast<float>(w[j]), mf, &bm_bessel_coef::kTable, ft.data(), r1);
                for (int q = 0; q < 4; ++q) {
                    blk.v[q] = r0[q];
                    blk.v[4 + q] = r1[q];
                }
            }
            double* o0 = out + 2 * ((2 * a) * ld + 2 * b);
            double* o1 = out + 2 * ((2 * a + 1) * ld + 2 * b);
            for (int q = 0; q < 4; ++q) {
                o0[q] = blk.v[q];
                o1[q] = blk.v[4 + q];
            }
        }
    }
    return 0;
}

// out[4*q + {0,1,2,3}] = J0, Y0, J1, Y1 + 2/(pi z) at z[q].
int bmh_bessel01(const double* z, int64_t n, double* out) {
    for (int64_t q = 0; q < n; ++q)
        bm::bessel01(z[q], 1.0 / z[q], &bm_bessel_coef::kTable, out[4 * q], out[4 * q + 1],
                     out[4 * q + 2], out[4 * q + 3]);
    return 0;
}

// out[2*q + {0,1}] = sin, cos of x[q] by the kernels' Cody-Waite routine.
int bmh_sincos(const double* x, int64_t n, double* out) {
    for (int64_t q = 0; q < n; ++q) bm::sincos_cw(x[q], &bm_bessel_coef::kTable, out[2 * q], out[2 * q + 1]);
    return 0;
}

// Blocks A(rows, cols) exactly as the dense/block kernels form them.
// soa: 6 x N (x, y, nx, ny, w, kappa); media: k0, k1, eps0, eps1;
// out: 2nr x 2nc complex row-major.
int bmh_system_blocks(const double* soa, const int32_t* curve, int64_t N, const int64_t* rows,
                      int64_t nr, const int64_t* cols, int64_t nc, const double* media,
                      double* out) {
    const bm::Media m = bm::make_media(media[0], media[1], media[2], media[3], &bm_bessel_coef::kTable);
    const double *x = soa, *y = soa + N, *nx = soa + 2 * N, *ny = soa + 3 * N, *w = soa + 4 * N,
                 *kap = soa + 5 * N;
    const int64_t ld = 2 * nc;
    for (int64_t a = 0; a < nr; ++a) {
        for (int64_t b = 0; b < nc; ++b) {
            const int64_t i = rows[a], j = cols[b];
            const bm::Block blk = (i == j)
                ? bm::diag_block(w[j], kap[j], m)
                : bm::pair_block(x[i], y[i], nx[i], ny[i], x[j], y[j], nx[j], ny[j], w[j], m,
                                 curve[i] == curve[j]);
            double* r0 = out + 2 * ((2 * a) * ld + 2 * b);
            double* r1 = r0 + 2 * ld;
            for (int q = 0; q < 4; ++q) {
                r0[q] = blk.v[q];
                r1[q] = blk.v[4 + q];
            }
        }
    }
    return 0;
}

// Pair derivatives of lam_i^T A_ij phi_j as the shape-derivative kernel forms
// them.  Per pair q: in[16*q ..]: tx, ty, tnx, tny, l0 (re, im), l1 (re, im),
// sx, sy, snx, sny, sw, interior (0/1), unused x2; phi[4*q ..] = u (re, im),
// q (re, im); out[14*q ..] = re/im of d/drho (x, y), d/dn_i (x, y), d/dn_j (x, y), d/dw_j.
int bmh_pair_adjoint(const double* in, const double* phi, int64_t n, const double* media, double* out) {
    const bm::Media m = bm::make_media(media[0], media[1], media[2], media[3], &bm_bessel_coef::kTable);
    for (int64_t q = 0; q < n; ++q) {
        const double* a = in + 16 * q;
        const double* f = phi + 4 * q;
        const bm::PairAdjoint pa = bm::pair_adjoint(a[0], a[1], a[2], a[3], make_double2(a[4], a[5]),
                                                    make_double2(a[6], a[7]), a[8], a[9], a[10], a[11], a[12],
                                                    make_double2(f[0], f[1]), make_double2(f[2], f[3]), m,
                                                    a[13] != 0.0);
        const double2 v[7] = {pa.g_rho[0], pa.g_rho[1], pa.g_ni[0], pa.g_ni[1], pa.g_nj[0], pa.g_nj[1], pa.g_w};
        for (int c = 0; c < 7; ++c) {
            out[14 * q + 2 * c] = v[c].x;
            out[14 * q + 2 * c + 1] = v[c].y;
        }
    }
    return 0;
}

// Derivatives of lam_i^T A_ii phi_i with respect to w and kappa.  in[8*q ..]:
// w, kappa, l0 (re, im), l1 (re, im), unused x2; phi as above;
// out[4*q ..] = d/dw (re, im), d/dkappa (re, im).
int bmh_diag_adjoint(const double* in, const double* phi, int64_t n, const double* media, double* out) {
    const bm::Media m = bm::make_media(media[0], media[1], media[2], media[3], &bm_bessel_coef::kTable);
    for (int64_t q = 0; q < n; ++q) {
        const double* a = in + 8 * q;
        const double* f = phi + 4 * q;
        double2 gw, gk;
        bm::diag_adjoint(a[0], a[1], m, make_double2(a[2], a[3]), make_double2(a[4], a[5]),
                         make_double2(f[0], f[1]), make_double2(f[2], f[3]), gw, gk);
        out[4 * q] = gw.x;
        out[4 * q + 1] = gw.y;
        out[4 * q + 2] = gk.x;
        out[4 * q + 3] = gk.y;
    }
    return 0;
}

// The whole shape derivative of one body on the host, with the kernels' pair
// and node arithmetic: soa 6 x N (x, y, nx, ny, w, kappa), xyd 6 x N samples,
// curve ids, lam and phi 2N complex (interleaved), coef complex, inc/obs
// angles; grad 6 x N.
int bmh_shape_derivative(const double* soa, const double* xyd, const int32_t* curve, int64_t N,
                         const double* media, const double* lam, const double* phi, double inc, double obs,
                         const double* coef, double* grad) {
    const bm::Media m = bm::make_media(media[0], media[1], media[2], media[3], &bm_bessel_coef::kTable);
    const double *x = soa, *y = soa + N, *nx = soa + 2 * N, *ny = soa + 3 * N, *w = soa + 4 * N,
                 *kap = soa + 5 * N;
    auto c2 = [](const double* p, int64_t k) { return make_double2(p[2 * k], p[2 * k + 1]); };
    std::vector<double> acc(18 * N, 0.0);
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            if (i == j) continue;
            const bm::PairAdjoint pa = bm::pair_adjoint(x[i], y[i], nx[i], ny[i], c2(lam, 2 * i), c2(lam, 2 * i + 1),
                                                        x[j], y[j], nx[j], ny[j], w[j], c2(phi, 2 * j),
                                                        c2(phi, 2 * j + 1), m, curve[i] == curve[j]);
            const double2 t[4] = {pa.g_rho[0], pa.g_rho[1], pa.g_ni[0], pa.g_ni[1]};
            const double2 u[5] = {pa.g_rho[0], pa.g_rho[1], pa.g_nj[0], pa.g_nj[1], pa.g_w};
            for (int c = 0; c < 4; ++c) {
                acc[18 * i + 2 * c] += t[c].x;
                acc[18 * i + 2 * c + 1] += t[c].y;
            }
            for (int c = 0; c < 5; ++c) {
                acc[18 * j + 8 + 2 * c] += u[c].x;
                acc[18 * j + 8 + 2 * c + 1] += u[c].y;
            }
        }
    }
    for (int64_t i = 0; i < N; ++i) {
        double g[6];
        bm::node_adjoint(x[i], y[i], nx[i], ny[i], w[i], kap[i], xyd[2 * N + i], xyd[3 * N + i], xyd[4 * N + i],
                         xyd[5 * N + i], m, c2(lam, 2 * i), c2(lam, 2 * i + 1), c2(phi, 2 * i), c2(phi, 2 * i + 1),
                         acc.data() + 18 * i, std::cos(inc), std::sin(inc), std::cos(obs), std::sin(obs),
                         make_double2(coef[0], coef[1]), g);
        for (int q = 0; q < 6; ++q) grad[q * N + i] = g[q];
    }
    return 0;
}

}  // extern "C"
