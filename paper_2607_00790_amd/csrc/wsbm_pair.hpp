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
    double q10, q10k1, e1q10;     // k1/k0, k1^2/k0, eps1 k1/k0
    const BesselTable* tab;       // Bessel / sine-cosine coefficients (device memory in kernels)
};

inline Media make_media(double k0, double k1, double eps0, double eps1, const BesselTable* tab) {
    return Media{k0, k1, eps0, eps1, 1.0 / k0, 1.0 / k1, k1 / k0, k1 * k1 / k0, eps1 * k1 / k0, tab};
}

// Output: blk[0..7] = re/im of A(2i,2j), A(2i,2j+1), A(2i+1,2j), A(2i+1,2j+1).
struct Block {
    double v[8];
};

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

// J0, Y0, J1, Y1 and Y1r = Y1 + 2/(pi z) of one wavenumber at z = k r.
struct Hankel01 {
    double j0, y0, j1, y1, y1r;
};

__host__ __device__ __forceinline__ Hankel01 hankel01(double k, double ik, const PairGeom& g,
                                                     const BesselTable* __restrict__ tab) {
    const double iz = g.ir * ik;
    Hankel01 h;
    bessel01(k * g.r, iz, tab, h.j0, h.y0, h.j1, h.y1r);
    h.y1 = fma(-kTwoOverPi, iz, h.y1r);
    return h;
}

// Interior-medium (k1) functions of a pair.  For a pair on different curves
// the interior operators vanish: J0 = Y0 = J1 = Y1 = 0, and Y1r keeps only the
// removed pole 2/(pi z1), so that the k0 - k1 combination of pole-free parts in
// pair_row1 reduces to the k0 term with its pole.
__host__ __device__ __forceinline__ Hankel01 pair_interior(const PairGeom& g, const Media& m,
                                                          bool interior) {
    if (interior) return hankel01(m.k1, m.ik1, g, m.tab);
    return Hankel01{0.0, 0.0, 0.0, 0.0, kTwoOverPi * (g.ir * m.ik1)};
}

// The block in terms of the Hankel functions.  With alpha = i/k0 the
// hypersingular difference alpha (N_k0 - N_k1) reduces (the i/pi parts of H2r
// and the k^2 ab/(4 pi r^2) terms cancel) to
//   -(1/4) [ e (H1r(z0) - (k1/k0) H1r(z1)) + (ab/r^2) (k0 H0(z0) - (k1^2/k0) H0(z1)) ],
// e = (c - 2 ab/r^2)/r, and alpha (eps0 D*_k0 - eps1 D*_k1) to
//   (a/(4r)) (eps0 H1(z0) - eps1 (k1/k0) H1(z1)).
// Each output is then a short combination of the eight Bessel values.

// Row 2i of the block: re/im of A(2i,2j) = D_k1 w_j and A(2i,2j+1) = -eps1 S_k1 w_j.
__host__ __device__ __forceinline__ void pair_row0(const PairGeom& g, const Hankel01& h1, double sw,
                                                   const Media& m, double (&o)[4]) {
    const double sw4 = 0.25 * sw;
    const double d = (sw4 * g.br) * m.k1;     // D_k1 = i (k1/4) H1(z1) b/r
    o[0] = -d * h1.y1;
    o[1] = d * h1.j1;
    const double s = sw4 * m.eps1;            // -eps1 S_k1 = -i (eps1/4) H0(z1)
    o[2] = s * h1.y0;
    o[3] = -s * h1.j0;
}

// What row 2i+1 needs of the interior functions: (k1/k0) J1(z1), (k1/k0) Y1r(z1),
// (k1^2/k0) J0(z1), (k1^2/k0) Y0(z1).  (k1/k0) Y1(z1) follows from the second,
// since (k1/k0) 2/(pi z1) = 2/(pi z0): four values stay live across the
// exterior Bessel evaluation instead of five.
struct InteriorTerms {
    double j1, y1r, j0, y0;
};

__host__ __device__ __forceinline__ InteriorTerms interior_terms(const Hankel01& h1, const Media& m) {
    return InteriorTerms{m.q10 * h1.j1, m.q10 * h1.y1r, m.q10k1 * h1.j0, m.q10k1 * h1.y0};
}

// Row 2i+1: A(2i+1,2j) = D_k0 + alpha (N_k0 - N_k1), A(2i+1,2j+1) = -eps0 S_k0 - alpha (eps0 D*_k0 - eps1 D*_k1).
__host__ __device__ __forceinline__ void pair_row1(const PairGeom& g, const InteriorTerms& it, double sw,
                                                   const Media& m, double (&o)[4]) {
    const double iz0 = g.ir * m.ik0;
    double j0, y0, j1, y1r;
    bessel01(m.k0 * g.r, iz0, m.tab, j0, y0, j1, y1r);
    const double y1 = fma(-kTwoOverPi, iz0, y1r);
    const double sw4 = 0.25 * sw;
    const double e = fma(-2.0 * g.abr2, g.ir, g.cr);
    // pole-free J1 and Y1 differences, and the H0 combination
    const double dj1 = j1 - it.j1;
    const double dy1 = y1r - it.y1r;
    const double cj0 = fma(m.k0, j0, -it.j0);
    const double cy0 = fma(m.k0, y0, -it.y0);
    const double kb = m.k0 * g.br;
    double t = fma(-g.abr2, cj0, fma(-e, dj1, -kb * y1));
    o[0] = sw4 * t;
    t = fma(-g.abr2, cy0, fma(-e, dy1, kb * j1));
    o[1] = sw4 * t;
    // eps0 J1(z0) - eps1 (k1/k0) J1(z1) and the same of Y1
    const double fj = fma(m.eps0, j1, -m.eps1 * it.j1);
    const double fy = fma(m.eps0, y1, -m.eps1 * fma(-kTwoOverPi, iz0, it.y1r));
    t = fma(-g.ar, fj, m.eps0 * y0);
    o[2] = sw4 * t;
    t = fma(-g.ar, fy, -m.eps0 * j0);
    o[3] = sw4 * t;
}

// Whole off-diagonal block (the points must not coincide).
__host__ __device__ __forceinline__ Block pair_block(double tx, double ty, double tnx, double tny,
                                                     double sx, double sy, double snx, double sny,
                                                     double sw, const Media& m, bool interior) {
    const PairGeom g = pair_geom(tx, ty, tnx, tny, sx, sy, snx, sny);
    const Hankel01 h1 = pair_interior(g, m, interior);
    double r0[4], r1[4];
    pair_row0(g, h1, sw, m, r0);
    pair_row1(g, interior_terms(h1, m), sw, m, r1);
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
