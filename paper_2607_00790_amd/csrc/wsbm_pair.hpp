// One 2x2 block of the weakly singular Burton-Miller (WSBM) Nystrom matrix:
// target node i (position x_i, outward normal n_i) against source j (x_j, n_j,
// quadrature weight w_j), paper Eq. (3) and its block form Eq. (5).
//
// With G_k(x, y) = (i/4) H0^(1)(k|x - y|), rho = x_i - x_j, r = |rho|,
// a = rho.n_i, b = rho.n_j, c = n_i.n_j, z = k r, the weighted kernels are
//   S_k  = (i/4) H0(z) w_j                       single layer
//   D_k  = (ik/4) H1(z) (b/r) w_j                dG/dn_y
//   D*_k = -(ik/4) H1(z) (a/r) w_j               dG/dn_x
//   N_k  = (ik/4) [H1(z) c/r - k H2(z) a b/r^2] w_j   d2G/dn_x dn_y
// and the block is
//   [ D_k1                  , -eps1 S_k1                          ]
//   [ D_k0 + alpha (N_k0 - N_k1), -eps0 S_k0 - alpha (eps0 D*_k0 - eps1 D*_k1) ]
// with alpha = i/k0.  The difference N_k0 - N_k1 is formed from the regular
// parts H1r = H1 + 2i/(pi z) and H2r = H2 + 4i/(pi z^2) + i/pi, so the
// k-independent 1/r^2 singularities of the two hypersingular kernels cancel
// analytically instead of numerically:
//   N_k = Nr_k + c/(2 pi r^2) - a b/(pi r^4),
//   Nr_k = (i/4) [k H1r c/r - k^2 H2r a b/r^2] - k^2 a b/(4 pi r^2),
//   H2r = 2 H1r/z - H0 + i/pi.
// Pairs on different closed curves carry no interior (k1) operators.
//
// The diagonal block (i == j) uses the one-point corrected entries
//   S_k[i,i]  = -(w/2pi) (L_k - i pi/2),  L_k = ln(k w/4pi) + gamma
//   D_k[i,i]  = D*_k[i,i] = -kappa w/(4 pi)
//   (N_k0 - N_k1)[i,i] = -(w/4pi) [k0^2 (L_k0 - 1/2 - i pi/2) - k1^2 (L_k1 - 1/2 - i pi/2)]
// plus the identity terms +1/2, -1/2 and -alpha (eps0 + eps1)/2 of Eq. (3).
#pragma once

#include "bessel.hpp"

namespace bm {

// Minimum waves per SIMD requested for the kernels that evaluate pair blocks
// (launch bound): the pair arithmetic fits in ~62 VGPRs without spills, and
// the extra waves hide the store and scalar-load latency of the
// compute-then-store pattern.
constexpr int kPairWavesPerSimd = 6;

struct Media {
    double k0, k1, eps0, eps1;
    double ik0, ik1;              // 1/k0, 1/k1
    const BesselTable* tab;       // Bessel / sine-cosine coefficients (device memory in kernels)
};

inline Media make_media(double k0, double k1, double eps0, double eps1, const BesselTable* tab) {
    return Media{k0, k1, eps0, eps1, 1.0 / k0, 1.0 / k1, tab};
}

// Output: blk[0..7] = re/im of A(2i,2j), A(2i,2j+1), A(2i+1,2j), A(2i+1,2j+1).
struct Block {
    double v[8];
};

// Per-wavenumber pieces of the kernels (divided by w_j).
struct KernelParts {
    double s_re, s_im;     // S_k
    double d_re, d_im;     // D_k
    double ds_re, ds_im;   // D*_k
    double nr_re, nr_im;   // Nr_k (regular part of N_k)
};

__host__ __device__ __forceinline__ KernelParts kernel_parts(double k, double ik, double r, double ir,
                                                            double ar, double br, double cr, double abr2,
                                                            const BesselTable* __restrict__ tab) {
    const double z = k * r;
    const double iz = ir * ik;                      // 1/z
    double j0, y0, j1, y1r;
    bessel01(z, iz, tab, j0, y0, j1, y1r);
    const double y1 = y1r - kTwoOverPi * iz;        // Y1
    KernelParts p;
    p.s_re = -0.25 * y0;
    p.s_im = 0.25 * j0;
    const double k4 = 0.25 * k;
    p.d_re = -k4 * br * y1;
    p.d_im = k4 * br * j1;
    p.ds_re = k4 * ar * y1;
    p.ds_im = -k4 * ar * j1;
    // X = k (c/r) H1r - k^2 (ab/r^2) H2r,  H2r = 2 H1r/z - H0 + i/pi
    const double kk = k * k;
    const double h2r_re = 2.0 * j1 * iz - j0;
    const double h2r_im = 2.0 * y1r * iz - y0 + (1.0 / kPi);
    const double x_re = k * cr * j1 - kk * abr2 * h2r_re;
    const double x_im = k * cr * y1r - kk * abr2 * h2r_im;
    p.nr_re = -0.25 * x_im - kk * abr2 * (0.25 / kPi);
    p.nr_im = 0.25 * x_re;
    return p;
}

// Geometry of one off-diagonal pair (the points must not coincide).
struct PairGeom {
    double r, ir, ar, br, cr, abr2;
};

__host__ __device__ __forceinline__ PairGeom pair_geom(double tx, double ty, double tnx, double tny,
                                                       double sx, double sy, double snx, double sny) {
    const double rx = tx - sx, ry = ty - sy;
    const double r2 = rx * rx + ry * ry;
    PairGeom g;
    g.ir = rsqrt_pos(r2);
    g.r = r2 * g.ir;
    const double a = rx * tnx + ry * tny;
    const double b = rx * snx + ry * sny;
    const double c = tnx * snx + tny * sny;
    g.ar = a * g.ir;
    g.br = b * g.ir;
    g.cr = c * g.ir;
    g.abr2 = g.ar * g.br;
    return g;
}

// Interior-medium (k1) parts of a pair; all zero for pairs on different curves.
__host__ __device__ __forceinline__ KernelParts pair_interior(const PairGeom& g, const Media& m,
                                                              bool interior) {
    if (interior) return kernel_parts(m.k1, m.ik1, g.r, g.ir, g.ar, g.br, g.cr, g.abr2, m.tab);
    return KernelParts{0, 0, 0, 0, 0, 0, 0, 0};
}

// Row 2i of the block: re/im of A(2i,2j) = D_k1 w_j and A(2i,2j+1) = -eps1 S_k1 w_j.
__host__ __device__ __forceinline__ void pair_row0(const KernelParts& p1, double sw, const Media& m,
                                                   double (&o)[4]) {
    o[0] = sw * p1.d_re;
    o[1] = sw * p1.d_im;
    o[2] = -sw * m.eps1 * p1.s_re;
    o[3] = -sw * m.eps1 * p1.s_im;
}

// Row 2i+1: A(2i+1,2j) = D_k0 + alpha (N_k0 - N_k1), A(2i+1,2j+1) = -eps0 S_k0 - alpha (eps0 D*_k0 - eps1 D*_k1).
__host__ __device__ __forceinline__ void pair_row1(const PairGeom& g, const KernelParts& p1, double sw,
                                                   const Media& m, bool interior, double (&o)[4]) {
    const KernelParts p0 = kernel_parts(m.k0, m.ik0, g.r, g.ir, g.ar, g.br, g.cr, g.abr2, m.tab);
    double nd_re, nd_im;
    if (interior) {
        nd_re = p0.nr_re - p1.nr_re;
        nd_im = p0.nr_im - p1.nr_im;
    } else {
        // N_k0 alone: add back the k-independent singular parts
        nd_re = p0.nr_re + (0.5 / kPi) * g.cr * g.ir - (1.0 / kPi) * g.abr2 * g.ir * g.ir;
        nd_im = p0.nr_im;
    }
    const double ik0 = m.ik0;   // alpha = i/k0: alpha (x + i y) = (-y + i x)/k0
    o[0] = sw * (p0.d_re - nd_im * ik0);
    o[1] = sw * (p0.d_im + nd_re * ik0);
    const double t_re = m.eps0 * p0.ds_re - m.eps1 * p1.ds_re;
    const double t_im = m.eps0 * p0.ds_im - m.eps1 * p1.ds_im;
    o[2] = sw * (-m.eps0 * p0.s_re + t_im * ik0);
    o[3] = sw * (-m.eps0 * p0.s_im - t_re * ik0);
}

// Whole off-diagonal block (the points must not coincide).
__host__ __device__ __forceinline__ Block pair_block(double tx, double ty, double tnx, double tny,
                                                     double sx, double sy, double snx, double sny,
                                                     double sw, const Media& m, bool interior) {
    const PairGeom g = pair_geom(tx, ty, tnx, tny, sx, sy, snx, sny);
    const KernelParts p1 = pair_interior(g, m, interior);
    double r0[4], r1[4];
    pair_row0(p1, sw, m, r0);
    pair_row1(g, p1, sw, m, interior, r1);
    Block o;
    for (int q = 0; q < 4; ++q) {
        o.v[q] = r0[q];
        o.v[4 + q] = r1[q];
    }
    return o;
}

// Diagonal block A_ii with the one-point correction and identity terms.
__host__ __device__ __forceinline__ Block diag_block(double w, double kappa, const Media& m) {
    const double inv4pi = 0.25 / kPi;
    const double L0 = log(m.k0 * w * inv4pi) + kEulerGamma;
    const double L1 = log(m.k1 * w * inv4pi) + kEulerGamma;
    // S_k = -(w/2pi) L_k + i w/4
    const double s0_re = -(0.5 / kPi) * w * L0, s1_re = -(0.5 / kPi) * w * L1;
    const double s_im = 0.25 * w;
    const double dd = -kappa * w * inv4pi;
    // N_k0 - N_k1 = -(w/4pi) [k0^2 (L0 - 1/2) - k1^2 (L1 - 1/2)] + i (w/8)(k0^2 - k1^2)
    const double kk0 = m.k0 * m.k0, kk1 = m.k1 * m.k1;
    const double nd_re = -w * inv4pi * (kk0 * (L0 - 0.5) - kk1 * (L1 - 0.5));
    const double nd_im = 0.125 * w * (kk0 - kk1);
    const double ik0 = m.ik0;
    Block o;
    o.v[0] = dd + 0.5;
    o.v[1] = 0.0;
    o.v[2] = -m.eps1 * s1_re;
    o.v[3] = -m.eps1 * s_im;
    o.v[4] = dd - 0.5 - nd_im * ik0;
    o.v[5] = nd_re * ik0;
    // -eps0 S0 - alpha (eps0 - eps1) dd - alpha (eps0 + eps1)/2
    const double t = (m.eps0 - m.eps1) * dd + 0.5 * (m.eps0 + m.eps1);
    o.v[6] = -m.eps0 * s0_re;
    o.v[7] = -m.eps0 * s_im - t * ik0;
    return o;
}

}  // namespace bm
