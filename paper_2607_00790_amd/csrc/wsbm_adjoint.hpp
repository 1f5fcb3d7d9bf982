// Derivatives of one pair's contribution lam_i^T A_ij phi_j to the bilinear
// form lam^T A phi of the WSBM matrix (Eq. (3)/(5)) with respect to the
// geometry of the two nodes: the building block of the shape derivative
// (adjoint method) of any objective of the solution.
//
// Notation as in wsbm_pair.hpp: rho = x_i - x_j, r = |rho|, a = rho.n_i,
// b = rho.n_j, c = n_i.n_j, z = k r.  With lam_i = (l0, l1) (rows 2i, 2i+1)
// and phi_j = (u, q), the pair term divided by the weight is
//   F/w_j = l0 (D_k1 u - eps1 S_k1 q)
//         + l1 (D_k0 u + alpha ND u - eps0 S_k0 q - alpha (eps0 D*_k0 - eps1 D*_k1) q)
// = sum over k of  cS S_k + cD D_k + cDs D*_k  plus  cN ND,  alpha = i/k0.
// Its partial derivatives with respect to (r, a, b, c), per wavenumber
// (H_n = H_n^(1)(z), derivatives dH0 = -H1, d(H1/r)/dr = -k H2/r):
//   S_k  = (i/4) H0                    dS/dr  = -(ik/4) H1
//   D_k  = (ik/4) H1 b/r               dD/dr  = -(ik^2/4) H2 b/r,  dD/db  = (ik/4) H1/r
//   D*_k = -(ik/4) H1 a/r              dD*/dr =  (ik^2/4) H2 a/r,  dD*/da = -(ik/4) H1/r
// The hypersingular difference uses the regular parts of wsbm_pair.hpp,
// N_k = M_k + c/(2 pi r^2) - a b/(pi r^4) with
//   M_k = -k^2 ab/(4 pi r^2) + (ik/4) [H1r c/r - k H2r ab/r^2],
// whose derivatives need one more regular part, H3r = H3 + 16i/(pi z^3) +
// 2i/(pi z) = 4 H2r/z - H1r:
//   dM/dr = k^2 ab/(2 pi r^3) - k^2 c/(4 pi r) + (ik^2/4) [-c H2r/r + k ab H3r/r^2]
//   dM/da = -(k^2 b/r^2) [1/(4 pi) + (i/4) H2r]      (dM/db: a and b swapped)
//   dM/dc = (ik/4) H1r/r
// so ND = M_k0 - M_k1 inside one curve keeps no 1/r^3 cancellation; across
// curves ND = N_k0 = M_k0 plus the k-independent singular part.
// The chain rule to the node data: dr = rho/r . drho, da = n_i . drho + rho . dn_i,
// db = n_j . drho + rho . dn_j, dc = n_j . dn_i + n_i . dn_j, and rho = x_i - x_j.
#pragma once

#include "wsbm_pair.hpp"

namespace bm {

__host__ __device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 c_scale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// i * s * a
__host__ __device__ __forceinline__ double2 c_iscale(double s, double2 a) { return make_double2(-s * a.y, s * a.x); }
// acc += a * b
__host__ __device__ __forceinline__ void c_fma(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// Coefficients of one wavenumber's operators in F/w_j.
struct AdjCoef {
    double2 cs, cd, cds, cm;
};

// Partial derivatives of F/w_j: value and d/dr, d/da, d/db, d/dc.
struct AdjSums {
    double2 v, fr, fa, fb, fc;
};

// Adds the terms of wavenumber k (S, D, D* and M parts) to s.
__host__ __device__ __forceinline__ void adj_wavenumber(double k, double ik, const PairGeom& g,
                                                        const AdjCoef& cf, const BesselTable* __restrict__ tab,
                                                        AdjSums& s) {
    const double z = k * g.r;
    const double iz = g.ir * ik;
    double j0, y0, j1, y1r;
    bessel01(z, iz, tab, j0, y0, j1, y1r);
    const double y1 = y1r - kTwoOverPi * iz;
    const double2 h0 = make_double2(j0, y0);
    const double2 h1 = make_double2(j1, y1);
    const double2 h1r = make_double2(j1, y1r);
    const double2 h2 = make_double2(2.0 * j1 * iz - j0, 2.0 * y1 * iz - y0);
    const double2 h2r = make_double2(2.0 * j1 * iz - j0, 2.0 * y1r * iz - y0 + 1.0 / kPi);
    const double2 h3r = make_double2(4.0 * h2r.x * iz - j1, 4.0 * h2r.y * iz - y1r);
    const double k4 = 0.25 * k, kk = k * k, kk4 = 0.25 * kk;
    // S, D, D*: with Akr = cD b/r - cDs a/r,
    //   value  cS (i/4) H0 + (ik/4) H1 Akr
    //   d/dr  -(ik/4) cS H1 - (ik^2/4) H2 Akr
    const double2 akr = c_sub(c_scale(g.br, cf.cd), c_scale(g.ar, cf.cds));
    c_fma(s.v, c_iscale(0.25, cf.cs), h0);
    c_fma(s.v, c_iscale(k4, h1), akr);
    c_fma(s.fr, c_iscale(-k4, cf.cs), h1);
    c_fma(s.fr, c_iscale(-kk4, h2), akr);
    const double2 h1ir = c_iscale(k4 * g.ir, h1);     // (ik/4) H1 / r
    c_fma(s.fb, cf.cd, h1ir);
    c_fma(s.fa, c_scale(-1.0, cf.cds), h1ir);
    // M_k with coefficient cm
    const double inv4pi = 0.25 / kPi;
    // value: -k^2 abr2/(4 pi) + (ik/4)(H1r cr - k H2r abr2)
    const double2 mv = make_double2(-kk * g.abr2 * inv4pi - k4 * (h1r.y * g.cr - k * h2r.y * g.abr2),
                                    k4 * (h1r.x * g.cr - k * h2r.x * g.abr2));
    // d/dr: k^2 abr2 ir/(2 pi) - k^2 cr/(4 pi) + (ik^2/4)(-cr H2r + k abr2 H3r)
    const double2 t3 = make_double2(-g.cr * h2r.x + k * g.abr2 * h3r.x, -g.cr * h2r.y + k * g.abr2 * h3r.y);
    const double2 mr = make_double2(kk * (g.abr2 * g.ir * (0.5 / kPi) - g.cr * inv4pi) - kk4 * t3.y, kk4 * t3.x);
    // d/da, d/db: -k^2 (b/r or a/r)(1/r) [1/(4 pi) + (i/4) H2r]
    const double2 bracket = make_double2(inv4pi - 0.25 * h2r.y, 0.25 * h2r.x);
    const double2 ma = c_scale(-kk * g.br * g.ir, bracket);
    const double2 mb = c_scale(-kk * g.ar * g.ir, bracket);
    const double2 mc = c_iscale(k4 * g.ir, h1r);
    c_fma(s.v, cf.cm, mv);
    c_fma(s.fr, cf.cm, mr);
    c_fma(s.fa, cf.cm, ma);
    c_fma(s.fb, cf.cm, mb);
    c_fma(s.fc, cf.cm, mc);
}

// k-independent singular part of N_k: c/(2 pi r^2) - ab/(pi r^4), with coefficient cn.
__host__ __device__ __forceinline__ void adj_singular(const PairGeom& g, double2 cn, AdjSums& s) {
    const double ir2 = g.ir * g.ir, ir3 = ir2 * g.ir;
    const double ipi = 1.0 / kPi;
    c_fma(s.v, cn, make_double2(g.cr * g.ir * (0.5 * ipi) - g.abr2 * ir2 * ipi, 0.0));
    c_fma(s.fr, cn, make_double2(-g.cr * ir2 * ipi + 4.0 * g.abr2 * ir3 * ipi, 0.0));
    c_fma(s.fa, cn, make_double2(-g.br * ir3 * ipi, 0.0));
    c_fma(s.fb, cn, make_double2(-g.ar * ir3 * ipi, 0.0));
    c_fma(s.fc, cn, make_double2(0.5 * ipi * ir2, 0.0));
}

// Derivatives of lam_i^T A_ij phi_j (i != j) with respect to rho = x_i - x_j
// (so d/dx_i = +g_rho, d/dx_j = -g_rho), n_i, n_j and w_j.
struct PairAdjoint {
    double2 g_rho[2], g_ni[2], g_nj[2], g_w;
};

__host__ __device__ __forceinline__ PairAdjoint pair_adjoint(double tx, double ty, double tnx, double tny,
                                                             double2 l0, double2 l1, double sx, double sy,
                                                             double snx, double sny, double sw, double2 u,
                                                             double2 q, const Media& m, bool interior) {
    const PairGeom g = pair_geom(tx, ty, tnx, tny, sx, sy, snx, sny);
    const double2 P = c_mul(l1, u), Q = c_mul(l1, q);
    const double2 cn = c_iscale(m.ik0, P);                      // alpha l1 u
    AdjSums s;
    s.v = s.fr = s.fa = s.fb = s.fc = make_double2(0.0, 0.0);
    // exterior: -eps0 S_k0 q l1 + D_k0 u l1 - alpha eps0 D*_k0 q l1 + alpha M_k0 u l1
    adj_wavenumber(m.k0, m.ik0, g,
                   AdjCoef{c_scale(-m.eps0, Q), P, c_iscale(-m.ik0 * m.eps0, Q), cn}, m.tab, s);
    if (interior) {
        const double2 R0 = c_mul(l0, u), R1 = c_mul(l0, q);
        // interior: D_k1 u l0 - eps1 S_k1 q l0 + alpha eps1 D*_k1 q l1 - alpha M_k1 u l1
        adj_wavenumber(m.k1, m.ik1, g,
                       AdjCoef{c_scale(-m.eps1, R1), R0, c_iscale(m.ik0 * m.eps1, Q), c_scale(-1.0, cn)},
                       m.tab, s);
    } else {
        adj_singular(g, cn, s);
    }
    const double rx = tx - sx, ry = ty - sy;
    PairAdjoint o;
    // d/drho = w (Fr rho/r + Fa n_i + Fb n_j)
    const double2 frr = c_scale(g.ir * sw, s.fr);
    const double2 fa = c_scale(sw, s.fa), fb = c_scale(sw, s.fb), fc = c_scale(sw, s.fc);
    o.g_rho[0] = make_double2(frr.x * rx + fa.x * tnx + fb.x * snx, frr.y * rx + fa.y * tnx + fb.y * snx);
    o.g_rho[1] = make_double2(frr.x * ry + fa.x * tny + fb.x * sny, frr.y * ry + fa.y * tny + fb.y * sny);
    // d/dn_i = w (Fa rho + Fc n_j),  d/dn_j = w (Fb rho + Fc n_i)
    o.g_ni[0] = make_double2(fa.x * rx + fc.x * snx, fa.y * rx + fc.y * snx);
    o.g_ni[1] = make_double2(fa.x * ry + fc.x * sny, fa.y * ry + fc.y * sny);
    o.g_nj[0] = make_double2(fb.x * rx + fc.x * tnx, fb.y * rx + fc.y * tnx);
    o.g_nj[1] = make_double2(fb.x * ry + fc.x * tny, fb.y * ry + fc.y * tny);
    o.g_w = s.v;
    return o;
}

// Derivatives of lam_i^T A_ii phi_i with respect to w_i and kappa_i (the
// one-point corrected diagonal of wsbm_pair.hpp, identity terms constant):
//   d/dw  D_k[i,i] = -kappa/(4 pi),   d/dkappa D_k[i,i] = -w/(4 pi)
//   d/dw  S_k[i,i] = -(L_k + 1)/(2 pi) + i/4
//   d/dw  ND[i,i]  = -(1/4pi) [k0^2 (L_k0 + 1/2) - k1^2 (L_k1 + 1/2)] + i (k0^2 - k1^2)/8
__host__ __device__ __forceinline__ void diag_adjoint(double w, double kappa, const Media& m, double2 l0, double2 l1,
                                                      double2 u, double2 q, double2& gw, double2& gk) {
    const double inv4pi = 0.25 / kPi;
    const double L0 = log(m.k0 * w * inv4pi) + kEulerGamma;
    const double L1 = log(m.k1 * w * inv4pi) + kEulerGamma;
    const double kk0 = m.k0 * m.k0, kk1 = m.k1 * m.k1;
    const double2 s0w = make_double2(-(L0 + 1.0) * (0.5 / kPi), 0.25);
    const double2 s1w = make_double2(-(L1 + 1.0) * (0.5 / kPi), 0.25);
    const double2 ndw = make_double2(-inv4pi * (kk0 * (L0 + 0.5) - kk1 * (L1 + 0.5)), 0.125 * (kk0 - kk1));
    const double ddw = -kappa * inv4pi, ddk = -w * inv4pi;
    // entry derivatives (alpha = i/k0):
    //   v0 = dd + 1/2, v1 = -eps1 S1, v2 = dd - 1/2 + alpha ND,
    //   v3 = -eps0 S0 - alpha (eps0 - eps1) dd - alpha (eps0 + eps1)/2
    const double2 v0w = make_double2(ddw, 0.0);
    const double2 v1w = c_scale(-m.eps1, s1w);
    const double2 v2w = c_add(make_double2(ddw, 0.0), c_iscale(m.ik0, ndw));
    const double2 v3w = c_add(c_scale(-m.eps0, s0w), make_double2(0.0, -m.ik0 * (m.eps0 - m.eps1) * ddw));
    const double2 R0 = c_mul(l0, u), R1 = c_mul(l0, q), P = c_mul(l1, u), Q = c_mul(l1, q);
    gw = make_double2(0.0, 0.0);
    c_fma(gw, v0w, R0);
    c_fma(gw, v1w, R1);
    c_fma(gw, v2w, P);
    c_fma(gw, v3w, Q);
    // kappa enters v0, v2 with coefficient 1 and v3 with -alpha (eps0 - eps1)
    gk = c_scale(ddk, c_add(R0, P));
    c_fma(gk, make_double2(0.0, -m.ik0 * (m.eps0 - m.eps1) * ddk), Q);
}

// One node's derivative of L = g^T phi + lam^T (b - A phi), weighted by coef
// and reduced to the six curve samples (x, y, x', y', x'', y'').
//   acc[0..7]  sum over sources j of d(lam_i^T A_ij phi_j)/d(rho, n_i) (re/im of
//              d/drho_x, d/drho_y, d/dn_x, d/dn_y) with the node as target i;
//   acc[8..17] sum over targets of d/drho (x, y), d/dn_j (x, y), d/dw_j with the
//              node as source j (d/dx_j = -d/drho).
// The right-hand side b_{2i+1} = -exp(i k0 d.x)(1 - d.n) (d = (cd, sd)) adds
// d/dx = i k0 d b_{2i+1} lam_{2i+1} and d/dn = exp(i k0 d.x) d lam_{2i+1}; the far
// field G = c0 exp(-i k0 xhat.x) w (-i k0 (xhat.n) u - eps0 q) (xhat = (ca, sa),
// c0 = e^{i pi/4}/sqrt(8 pi k0)) adds d/dx = -i k0 xhat G, d/dn = c0 exp(..) w
// (-i k0 u) xhat and d/dw = G/w.  The chain rule to the samples, with s = |x'|,
// tangent t = x'/s, n = (y', -x')/s, w = h s, kappa = (x' y'' - y' x'')/s^3:
//   d/dx' = -((dL/dn . t)/s) n + h (dL/dw) t + (dL/dkappa) dkappa/dx',
//   dkappa/dx' = (y'', -x'')/s^3 - 3 kappa x'/s^2,  dkappa/dx'' = (-y', x')/s^3.
// g[q] = Re(coef dL/ds_q).
__host__ __device__ __forceinline__ void node_adjoint(double x, double y, double nx, double ny, double w,
                                                      double kap, double dx, double dy, double ddx, double ddy,
                                                      const Media& m, double2 l0, double2 l1, double2 u, double2 q,
                                                      const double* acc, double cd, double sd, double ca,
                                                      double sa, double2 cf, double* g) {
    auto a2 = [&](int c) { return make_double2(acc[c], acc[c + 1]); };
    const double2 ax = c_sub(a2(0), a2(8)), ay = c_sub(a2(2), a2(10));
    const double2 anx = c_add(a2(4), a2(12)), any = c_add(a2(6), a2(14));
    double2 aw, ak;
    diag_adjoint(w, kap, m, l0, l1, u, q, aw, ak);
    aw = c_add(aw, a2(16));
    double si, ci;
    sincos(m.k0 * (cd * x + sd * y), &si, &ci);
    const double2 ein = make_double2(ci, si);
    const double2 b1 = c_scale(-(1.0 - (cd * nx + sd * ny)), ein);
    const double2 lb = c_iscale(m.k0, c_mul(l1, b1));      // lam_{2i+1} i k0 b_{2i+1}
    const double2 le = c_mul(l1, ein);
    double so, co;
    sincos(-m.k0 * (ca * x + sa * y), &so, &co);
    const double f = kSqrtHalf / sqrt(8.0 * kPi * m.k0);
    const double2 ce = make_double2(f * (co - so), f * (so + co));   // c0 exp(-i k0 xhat.x)
    const double2 dens = c_sub(c_iscale(-m.k0 * (ca * nx + sa * ny), u), c_scale(m.eps0, q));
    const double2 gw = c_mul(ce, dens);                    // G / w
    const double2 gfx = c_iscale(-m.k0 * w, gw);           // -i k0 G
    const double2 gfn = c_mul(c_scale(w, ce), c_iscale(-m.k0, u));
    auto re = [&](double2 z) { return cf.x * z.x - cf.y * z.y; };
    const double GX = re(c_sub(c_add(c_scale(ca, gfx), c_scale(cd, lb)), ax));
    const double GY = re(c_sub(c_add(c_scale(sa, gfx), c_scale(sd, lb)), ay));
    const double GNX = re(c_sub(c_add(c_scale(ca, gfn), c_scale(cd, le)), anx));
    const double GNY = re(c_sub(c_add(c_scale(sa, gfn), c_scale(sd, le)), any));
    const double GW = re(c_sub(gw, aw));
    const double GK = -re(ak);
    const double s = sqrt(dx * dx + dy * dy), is = 1.0 / s;
    const double tx = dx * is, ty = dy * is;
    const double h = w * is;
    const double gnt = (GNX * tx + GNY * ty) * is;
    const double is3 = is * is * is;
    const double kx = ddy * is3 - 3.0 * kap * dx * is * is;
    const double ky = -ddx * is3 - 3.0 * kap * dy * is * is;
    g[0] = GX;
    g[1] = GY;
    g[2] = -gnt * nx + GW * h * tx + GK * kx;
    g[3] = -gnt * ny + GW * h * ty + GK * ky;
    g[4] = -GK * dy * is3;
    g[5] = GK * dx * is3;
}

}  // namespace bm
