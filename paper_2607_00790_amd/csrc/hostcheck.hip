// Host-compiled instances of the device math (bessel.hpp, wsbm_pair.hpp) for
// CPU unit tests.  This library is loaded only by the test suite, to check the
// kernels' arithmetic without a GPU; the product library never calls it.
#include <cstdint>

#include "wsbm_pair.hpp"

extern "C" {

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

}  // extern "C"
