// FP32 evaluation of the off-diagonal WSBM pair block and of the diagonal
// block (paper Eq. (3)/(5)): the formulas of wsbm_pair.hpp and bessel.hpp,
// term for term, in single precision.  Used where entries only select
// skeletons (the proxy blocks of the proxy-surface compression, Sec. I and
// III), never for near-field, skeleton or factor blocks.
//
// What stays in FP64: the distance r = |x_i - x_j| (coordinate differences,
// square root) and the phase z = k r with its Cody-Waite reduction for large
// arguments.  An FP32 r would carry a relative error of ~6e-8, i.e. a phase
// error of 6e-8 z in the oscillating Hankel functions (6e-6 at z = 100),
// above the FP32 rounding of everything else.  The rest -- the Bessel
// polynomials, the logarithm, 1/r, the block algebra -- is FP32, with the
// coefficients read from an FP32 copy of the FP64 table (same layout, entry
// for entry).
#pragma once

#include <cstddef>

#include "wsbm_pair.hpp"

namespace bm {
namespace f32 {

// Offsets of the coefficient arrays in the table, in entries (the FP32 copy
// keeps the FP64 table's order).
namespace off {
#define BM_TABLE_OFF(F) constexpr int F = static_cast<int>(offsetof(BesselTable, F) / sizeof(double))
BM_TABLE_OFF(A_J0);
BM_TABLE_OFF(A_J1);
BM_TABLE_OFF(A_R0);
BM_TABLE_OFF(A_R1);
BM_TABLE_OFF(C_P0);
BM_TABLE_OFF(C_Q0);
BM_TABLE_OFF(C_P1);
BM_TABLE_OFF(C_Q1);
BM_TABLE_OFF(D_P0);
BM_TABLE_OFF(D_Q0);
BM_TABLE_OFF(D_P1);
BM_TABLE_OFF(D_Q1);
BM_TABLE_OFF(E_P0);
BM_TABLE_OFF(E_Q0);
BM_TABLE_OFF(E_P1);
BM_TABLE_OFF(E_Q1);
BM_TABLE_OFF(T_SIN);
BM_TABLE_OFF(T_COS);
BM_TABLE_OFF(B_TAB);
#undef BM_TABLE_OFF
}  // namespace off

// Entries of the FP32 table (one float per FP64 coefficient).
constexpr int kTableEntries = static_cast<int>(sizeof(BesselTable) / sizeof(double));

// a * b + c with c wave-uniform: one v_fma_f32 with c as a scalar operand.
__host__ __device__ __forceinline__ float fma_uniform(float a, float b, float c) {
#if defined(__HIP_DEVICE_COMPILE__)
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
#else
    return fmaf(a, b, c);
#endif
}

template <int N>
__host__ __device__ __forceinline__ float horner(const float* __restrict__ c, float x) {
    float acc = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fma_uniform(acc, x, c[k]);
    return acc;
}

__host__ __device__ __forceinline__ float rsqrt_pos(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);   // one Newton step
#else
    return 1.0f / sqrtf(x);
#endif
}

// sin x and cos x: the quadrant k and the reduced argument from the FP64
// Cody-Waite split of pi/2 (tab64->T_CW), the polynomials in FP32.
__host__ __device__ __forceinline__ void sincos_cw(double x, const BesselTable* __restrict__ tab64,
                                                   const float* __restrict__ t, float& s, float& c) {
    const double k = rint(x * kTwoOverPi);
    double rd = fma(-k, tab64->T_CW[0], x);
    rd = fma(-k, tab64->T_CW[1], rd);
    rd = fma(-k, tab64->T_CW[2], rd);
    const float r = static_cast<float>(rd);
    const float w = r * r;
    const float sr = fmaf(r * w, horner<bm_bessel_coef::NT>(t + off::T_SIN, w), r);
    const float cr = fmaf(w * w, horner<bm_bessel_coef::NT>(t + off::T_COS, w), fmaf(-0.5f, w, 1.0f));
    const int q = static_cast<int>(k) & 3;
    const float ss = (q & 1) ? cr : sr;
    const float cc = (q & 1) ? sr : cr;
    s = (q & 2) ? -ss : ss;
    c = ((q + 1) & 2) ? -cc : cc;
}

// J0, Y0, J1 and Y1r = Y1 + 2/(pi z) at z > 0 (zd: z in FP64, iz = 1/z):
// bm::bessel01 in FP32, the large-argument phase reduced from zd.
__host__ __device__ __forceinline__ void bessel01(double zd, float iz, const BesselTable* __restrict__ tab64,
                                                  const float* __restrict__ t, float& j0, float& y0, float& j1,
                                                  float& y1r) {
    using namespace bm_bessel_coef;
    const float z = static_cast<float>(zd);
    constexpr float kTwoOverPiF = static_cast<float>(kTwoOverPi);
    if (z < static_cast<float>(ZA)) {
        const float w = z * z;
        j0 = horner<NA>(t + off::A_J0, w);
        j1 = z * horner<NA>(t + off::A_J1, w);
        const float lg = kTwoOverPiF * logf(0.5f * z);
        y0 = fmaf(lg, j0, horner<NA>(t + off::A_R0, w));
        y1r = fmaf(lg, j1, z * horner<NA>(t + off::A_R1, w));
    } else if (z < static_cast<float>(ZC)) {
        int i = static_cast<int>((z - static_cast<float>(ZA)) * static_cast<float>(1.0 / HB));
        i = i < NB - 1 ? i : NB - 1;
        const float s = z - static_cast<float>(ZA + (i + 0.5) * HB);
        const float* c = t + off::B_TAB + i * 4 * DB;
        j0 = horner<DB>(c, s);
        y0 = horner<DB>(c + DB, s);
        j1 = horner<DB>(c + 2 * DB, s);
        y1r = horner<DB>(c + 3 * DB, s);
    } else {
        float p0, q0, p1, q1;
        if (z >= static_cast<float>(ZE)) {
            const float u = (static_cast<float>(ZE) * iz) * (static_cast<float>(ZE) * iz);
            p0 = horner<NE>(t + off::E_P0, u);
            q0 = horner<NE>(t + off::E_Q0, u);
            p1 = horner<NE>(t + off::E_P1, u);
            q1 = horner<NE>(t + off::E_Q1, u);
        } else if (z >= static_cast<float>(ZD)) {
            const float u = (static_cast<float>(ZD) * iz) * (static_cast<float>(ZD) * iz);
            p0 = horner<ND>(t + off::D_P0, u);
            q0 = horner<ND>(t + off::D_Q0, u);
            p1 = horner<ND>(t + off::D_P1, u);
            q1 = horner<ND>(t + off::D_Q1, u);
        } else {
            const float u = (static_cast<float>(ZC) * iz) * (static_cast<float>(ZC) * iz);
            p0 = horner<NC>(t + off::C_P0, u);
            q0 = horner<NC>(t + off::C_Q0, u);
            p1 = horner<NC>(t + off::C_P1, u);
            q1 = horner<NC>(t + off::C_Q1, u);
        }
        q0 *= iz;
        q1 *= iz;
        float sz, cz;
        sincos_cw(zd, tab64, t, sz, cz);
        const float amp = static_cast<float>(kSqrtTwoOverPi * kSqrtHalf) * rsqrt_pos(z);
        const float cr = (cz + sz) * amp;
        const float ci = (sz - cz) * amp;
        j0 = fmaf(p0, cr, -q0 * ci);
        y0 = fmaf(p0, ci, q0 * cr);
        j1 = fmaf(p1, ci, q1 * cr);
        y1r = fmaf(q1, ci, fmaf(-p1, cr, kTwoOverPiF * iz));
    }
}

// The media constants the block needs, in FP32.
struct MediaF {
    float k0, k1, eps0, eps1, ik0, ik1, q10, q10k1;
    double k0d, k1d;   // the wavenumbers in FP64, for the phases z = k r
};

__host__ __device__ __forceinline__ MediaF media_f(const Media& m) {
    return MediaF{static_cast<float>(m.k0),  static_cast<float>(m.k1),  static_cast<float>(m.eps0),
                  static_cast<float>(m.eps1), static_cast<float>(m.ik0), static_cast<float>(m.ik1),
                  static_cast<float>(m.q10), static_cast<float>(m.q10k1), m.k0, m.k1};
}

struct PairGeomF {
    double rd;   // r in FP64
    float ir, ar, br, cr, abr2;
};

__host__ __device__ __forceinline__ PairGeomF pair_geom(double tx, double ty, float tnx, float tny, double sx,
                                                        double sy, float snx, float sny) {
    const double rxd = tx - sx, ryd = ty - sy;
    const double r2 = rxd * rxd + ryd * ryd;
    PairGeomF g;
    g.rd = r2 * bm::rsqrt_pos(r2);
    const float rx = static_cast<float>(rxd), ry = static_cast<float>(ryd);
    g.ir = 1.0f / static_cast<float>(g.rd);
    g.ar = (rx * tnx + ry * tny) * g.ir;
    g.br = (rx * snx + ry * sny) * g.ir;
    g.cr = (tnx * snx + tny * sny) * g.ir;
    g.abr2 = g.ar * g.br;
    return g;
}

struct Hankel01F {
    float j0, y0, j1, y1, y1r;
};

// Interior (k1) functions; on different curves only the removed pole of Y1r
// remains (as in bm::pair_interior).
__host__ __device__ __forceinline__ Hankel01F pair_interior(const PairGeomF& g, const MediaF& m, bool interior,
                                                           const BesselTable* __restrict__ tab64,
                                                           const float* __restrict__ t) {
    const float iz = g.ir * m.ik1;
    if (!interior) return Hankel01F{0.0f, 0.0f, 0.0f, 0.0f, static_cast<float>(kTwoOverPi) * iz};
    Hankel01F h;
    bessel01(m.k1d * g.rd, iz, tab64, t, h.j0, h.y0, h.j1, h.y1r);
    h.y1 = fmaf(-static_cast<float>(kTwoOverPi), iz, h.y1r);
    return h;
}

// Row 2i: D_k1 w_j and -eps1 S_k1 w_j (re, im of each), as bm::pair_row0.
__host__ __device__ __forceinline__ void pair_row0(const PairGeomF& g, const Hankel01F& h1, float sw,
                                                   const MediaF& m, float (&o)[4]) {
    const float sw4 = 0.25f * sw;
    const float d = (sw4 * g.br) * m.k1;
    o[0] = -d * h1.y1;
    o[1] = d * h1.j1;
    const float s = sw4 * m.eps1;
    o[2] = s * h1.y0;
    o[3] = -s * h1.j0;
}

// Row 2i+1 (as bm::pair_row1 with bm::interior_terms folded in).
__host__ __device__ __forceinline__ void pair_row1(const PairGeomF& g, const Hankel01F& h1, float sw,
                                                   const MediaF& m, const BesselTable* __restrict__ tab64,
                                                   const float* __restrict__ t, float (&o)[4]) {
    const float it_j1 = m.q10 * h1.j1, it_y1r = m.q10 * h1.y1r;
    const float it_j0 = m.q10k1 * h1.j0, it_y0 = m.q10k1 * h1.y0;
    const float iz0 = g.ir * m.ik0;
    float j0, y0, j1, y1r;
    bessel01(m.k0d * g.rd, iz0, tab64, t, j0, y0, j1, y1r);
    constexpr float kTwoOverPiF = static_cast<float>(kTwoOverPi);
    const float y1 = fmaf(-kTwoOverPiF, iz0, y1r);
    const float sw4 = 0.25f * sw;
    const float e = fmaf(-2.0f * g.abr2, g.ir, g.cr);
    const float dj1 = j1 - it_j1;
    const float dy1 = y1r - it_y1r;
    const float cj0 = fmaf(m.k0, j0, -it_j0);
    const float cy0 = fmaf(m.k0, y0, -it_y0);
    const float kb = m.k0 * g.br;
    o[0] = sw4 * fmaf(-g.abr2, cj0, fmaf(-e, dj1, -kb * y1));
    o[1] = sw4 * fmaf(-g.abr2, cy0, fmaf(-e, dy1, kb * j1));
    const float fj = fmaf(m.eps0, j1, -m.eps1 * it_j1);
    const float fy = fmaf(m.eps0, y1, -m.eps1 * fmaf(-kTwoOverPiF, iz0, it_y1r));
    o[2] = sw4 * fmaf(-g.ar, fj, m.eps0 * y0);
    o[3] = sw4 * fmaf(-g.ar, fy, -m.eps0 * j0);
}

// Diagonal block (one-point corrected entries and identity terms, as
// bm::diag_block) in FP32.
__host__ __device__ __forceinline__ Block diag_block(float w, float kappa, const MediaF& m) {
    constexpr float inv4pi = static_cast<float>(0.25 / kPi);
    const float L0 = logf(m.k0 * w * inv4pi) + static_cast<float>(kEulerGamma);
    const float L1 = logf(m.k1 * w * inv4pi) + static_cast<float>(kEulerGamma);
    const float s0_re = -static_cast<float>(0.5 / kPi) * w * L0, s1_re = -static_cast<float>(0.5 / kPi) * w * L1;
    const float s_im = 0.25f * w;
    const float dd = -kappa * w * inv4pi;
    const float kk0 = m.k0 * m.k0, kk1 = m.k1 * m.k1;
    const float nd_re = -w * inv4pi * (kk0 * (L0 - 0.5f) - kk1 * (L1 - 0.5f));
    const float nd_im = 0.125f * w * (kk0 - kk1);
    Block o;
    o.v[0] = dd + 0.5f;
    o.v[1] = 0.0;
    o.v[2] = -m.eps1 * s1_re;
    o.v[3] = -m.eps1 * s_im;
    o.v[4] = dd - 0.5f - nd_im * m.ik0;
    o.v[5] = nd_re * m.ik0;
    const float tt = (m.eps0 - m.eps1) * dd + 0.5f * (m.eps0 + m.eps1);
    o.v[6] = -m.eps0 * s0_re;
    o.v[7] = -m.eps0 * s_im - tt * m.ik0;
    return o;
}

}  // namespace f32
}  // namespace bm
