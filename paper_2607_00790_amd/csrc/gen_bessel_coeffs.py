#!/usr/bin/env python3
"""Generate the coefficient tables of the library's FP64 Bessel functions.

Writes ``bessel_coeffs.h`` next to this file.  The approximations are derived
here from the mathematics, with mpmath (40 digits) as the source of truth:

Region A, 0 < z < ZA (ascending series, A&S 9.1.10/9.1.11 structure).
    J0(z)  = PA_J0(w)                          w = z^2
    J1(z)  = z PA_J1(w)
    Y0(z)  = (2/pi) ln(z/2) J0(z) + PA_R0(w)
    Y1r(z) := Y1(z) + 2/(pi z) = (2/pi) ln(z/2) J1(z) + z PA_R1(w)
  The four functions of w are entire; each is replaced by its least-squares
  polynomial on Chebyshev points of [0, ZA^2] (near-minimax).

Region B, ZA <= z < ZC (piecewise local polynomials).
  [ZA, ZC) is cut into intervals of width HB; on each, J0, Y0, J1 and Y1r are
  least-squares polynomials in s = z - centre.

Regions C (ZC <= z < ZD), D (ZD <= z < ZE) and E (z >= ZE): Hankel's
large-argument form (A&S 9.2.5-9.2.10 structure).
    H_n(z) = sqrt(2/(pi z)) (P_n(z) + i Q_n(z)) exp(i (z - (2n+1) pi/4)),  n = 0, 1
  P_n and z Q_n are smooth in u = (Z0/z)^2 on [0, 1] (Z0 = ZC, ZD or ZE) and
  are replaced by their least-squares polynomials in u; the degree falls with
  Z0, and most node pairs of a scatterer at the frequencies of interest fall
  in region E.

Sine and cosine for the large-argument region (Cody and Waite's argument
reduction): x = k pi/2 + r with pi/2 split into three doubles C1 + C2 + C3,
C1 and C2 carrying 33 significant bits so that k C1 and k C2 are exact for
|k| < 2^20; then on |r| <= pi/4
    sin r = r + r w PS(w),   cos r = 1 - w/2 + w^2 PC(w),   w = r^2,
with PS, PC least-squares polynomials in w.

The script reports the worst relative error of H0 and H1 (complex, relative to
|H|) of a float64 Horner evaluation over 0 < z <= 1e4.
"""
from __future__ import annotations

import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 40

ZA = 4.0
ZC = 8.0
HB = 0.5
DEG_A = 16
DEG_B = 11
DEG_C = 11
ZD = 16.0
DEG_D = 6
ZE = 32.0
DEG_E = 4
DEG_TRIG = 5


def _j(n, z):
    return mp.besselj(n, z)


def _y(n, z):
    return mp.bessely(n, z)


def fa(which, w):
    z = mp.sqrt(w) if w > 0 else mp.mpf(0)
    if w == 0:
        g = mp.euler
        return {"J0": mp.mpf(1), "J1": mp.mpf(1) / 2,
                "R0": 2 / mp.pi * (g), "R1": (2 * g - 1) / (2 * mp.pi)}[which]
    lg = 2 / mp.pi * mp.log(z / 2)
    if which == "J0":
        return _j(0, z)
    if which == "J1":
        return _j(1, z) / z
    if which == "R0":
        return _y(0, z) - lg * _j(0, z)
    if which == "R1":
        return (_y(1, z) + 2 / (mp.pi * z) - lg * _j(1, z)) / z
    raise KeyError(which)


def fb(which, z):
    if which == "J0":
        return _j(0, z)
    if which == "Y0":
        return _y(0, z)
    if which == "J1":
        return _j(1, z)
    if which == "Y1r":
        return _y(1, z) + 2 / (mp.pi * z)
    raise KeyError(which)


def fc(which, u, z0=ZC):
    z = z0 / mp.sqrt(u)
    n = 0 if which in ("P0", "Q0") else 1
    h = _j(n, z) + 1j * _y(n, z)
    v = h * mp.exp(-1j * (z - (2 * n + 1) * mp.pi / 4)) * mp.sqrt(mp.pi * z / 2)
    return v.real if which[0] == "P" else v.imag * z


def lsq_poly(f, a, b, deg, npts=None):
    """Least-squares polynomial (monomial coefficients in x - a0) on Chebyshev points."""
    npts = npts or 3 * deg + 30
    xs = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / npts) for k in range(npts)]
    ys = [f(x) for x in xs]
    # scaled variable for conditioning, then expand back to the unscaled monomials
    c, h = (a + b) / 2, (b - a) / 2
    V = mp.matrix([[((x - c) / h) ** k for k in range(deg + 1)] for x in xs])
    coef = mp.lu_solve(V.T * V, V.T * mp.matrix(ys))
    return [coef[k] for k in range(deg + 1)], c, h


def to_monomial(coef_scaled, c, h, shift):
    """Coefficients of p((x - c)/h) as a polynomial in (x - shift)."""
    deg = len(coef_scaled) - 1
    # p(x) = sum a_k ((x - shift + shift - c)/h)^k
    d = (mp.mpf(shift) - c) / h
    out = [mp.mpf(0)] * (deg + 1)
    for k, a in enumerate(coef_scaled):
        # ((t + d*h)/h)^k with t = x - shift = sum_j C(k,j) t^j d^(k-j) / h^j
        for j in range(k + 1):
            out[j] += a * mp.binomial(k, j) * d ** (k - j) / h ** j
    return out


def build():
    tables = {}
    for name in ("J0", "J1", "R0", "R1"):
        cs, c, h = lsq_poly(lambda w, n=name: fa(n, w), mp.mpf(0), mp.mpf(ZA) ** 2, DEG_A)
        tables["A_" + name] = to_monomial(cs, c, h, 0)
    nint = int(round((ZC - ZA) / HB))
    btab = []
    for i in range(nint):
        lo = mp.mpf(ZA) + i * mp.mpf(HB)
        hi = lo + mp.mpf(HB)
        row = []
        for name in ("J0", "Y0", "J1", "Y1r"):
            cs, c, h = lsq_poly(lambda z, n=name: fb(n, z), lo, hi, DEG_B)
            row.append(to_monomial(cs, c, h, c))
        btab.append(row)
    tables["B"] = btab
    for name in ("P0", "Q0", "P1", "Q1"):
        eps = mp.mpf("1e-40")
        cs, c, h = lsq_poly(lambda u, n=name: fc(n, u if u > eps else eps), mp.mpf(0), mp.mpf(1), DEG_C)
        tables["C_" + name] = to_monomial(cs, c, h, 0)
        cs, c, h = lsq_poly(lambda u, n=name: fc(n, u if u > eps else eps, ZD), mp.mpf(0), mp.mpf(1), DEG_D)
        tables["D_" + name] = to_monomial(cs, c, h, 0)
        cs, c, h = lsq_poly(lambda u, n=name: fc(n, u if u > eps else eps, ZE), mp.mpf(0), mp.mpf(1), DEG_E)
        tables["E_" + name] = to_monomial(cs, c, h, 0)
    # sine / cosine on |r| <= pi/4, as polynomials in w = r^2
    wmax = (mp.pi / 4) ** 2
    tiny = mp.mpf("1e-30")

    def fsin(w):
        w = w if w > tiny else tiny
        r = mp.sqrt(w)
        return (mp.sin(r) / r - 1) / w

    def fcos(w):
        w = w if w > tiny else tiny
        r = mp.sqrt(w)
        return (mp.cos(r) - 1 + w / 2) / (w * w)

    cs, c, h = lsq_poly(fsin, mp.mpf(0), wmax, DEG_TRIG)
    tables["T_SIN"] = to_monomial(cs, c, h, 0)
    cs, c, h = lsq_poly(fcos, mp.mpf(0), wmax, DEG_TRIG)
    tables["T_COS"] = to_monomial(cs, c, h, 0)
    # Cody-Waite split of pi/2: C1, C2 with 33 significant bits, C3 the rest
    half_pi = mp.pi / 2

    def round_bits(x, bits):
        e = mp.floor(mp.log(abs(x), 2))
        q = mp.mpf(2) ** (e - bits + 1)
        return mp.nint(x / q) * q

    c1 = round_bits(half_pi, 33)
    c2 = round_bits(half_pi - c1, 33)
    c3 = mp.mpf(float(half_pi - c1 - c2))
    tables["T_CW"] = [c1, c2, c3]
    return tables


# ----------------------------------------------------------------------------
# float64 model of the device evaluation (used only to report the error here)

def _horner(c, x):
    acc = np.zeros_like(x) + float(c[-1])
    for a in reversed(c[:-1]):
        acc = acc * x + float(a)
    return acc


def model_sincos(t, x):
    """float64 model of the Cody-Waite sine/cosine used by the kernels."""
    c1, c2, c3 = (float(v) for v in t["T_CW"])
    k = np.rint(x * (2 / np.pi))
    r = ((x - k * c1) - k * c2) - k * c3
    w = r * r
    sr = r + r * w * _horner(t["T_SIN"], w)
    cr = (1.0 - 0.5 * w) + w * w * _horner(t["T_COS"], w)
    q = k.astype(np.int64) & 3
    s = np.select([q == 0, q == 1, q == 2, q == 3], [sr, cr, -sr, -cr])
    c = np.select([q == 0, q == 1, q == 2, q == 3], [cr, -sr, -cr, sr])
    return s, c


def eval_f64(t, z):
    z = np.asarray(z, dtype=np.float64)
    out = np.empty((2,) + z.shape, dtype=np.complex128)
    A = z < ZA
    E = z >= ZE
    D = (z >= ZD) & ~E
    C = (z >= ZC) & (z < ZD)
    B = ~A & (z < ZC)
    if A.any():
        za = z[A]
        w = za * za
        j0 = _horner(t["A_J0"], w)
        j1 = za * _horner(t["A_J1"], w)
        lg = (2 / np.pi) * np.log(0.5 * za)
        y0 = lg * j0 + _horner(t["A_R0"], w)
        y1 = lg * j1 + za * _horner(t["A_R1"], w) - 2 / (np.pi * za)
        out[0, A], out[1, A] = j0 + 1j * y0, j1 + 1j * y1
    if B.any():
        zb = z[B]
        idx = np.minimum(((zb - ZA) / HB).astype(int), len(t["B"]) - 1)
        res = np.empty((4, zb.size))
        for q in range(zb.size):
            row = t["B"][idx[q]]
            s = zb[q] - (ZA + (idx[q] + 0.5) * HB)
            res[:, q] = [_horner(row[f], np.array(s)) for f in range(4)]
        out[0, B] = res[0] + 1j * res[1]
        out[1, B] = res[2] + 1j * (res[3] - 2 / (np.pi * zb))
    if C.any():
        zc = z[C]
        u = (ZC / zc) ** 2
        amp = np.sqrt(2 / (np.pi * zc))
        # exp(i (z - pi/4)) = (cos z + sin z + i (sin z - cos z)) / sqrt 2
        sz, cz = model_sincos(t, zc)
        ph = ((cz + sz) + 1j * (sz - cz)) * np.sqrt(0.5)
        out[0, C] = amp * (_horner(t["C_P0"], u) + 1j * _horner(t["C_Q0"], u) / zc) * ph
        out[1, C] = amp * (_horner(t["C_P1"], u) + 1j * _horner(t["C_Q1"], u) / zc) * ph * (-1j)
    if D.any():
        zd = z[D]
        u = (ZD / zd) ** 2
        amp = np.sqrt(2 / (np.pi * zd))
        sz, cz = model_sincos(t, zd)
        ph = ((cz + sz) + 1j * (sz - cz)) * np.sqrt(0.5)
        out[0, D] = amp * (_horner(t["D_P0"], u) + 1j * _horner(t["D_Q0"], u) / zd) * ph
        out[1, D] = amp * (_horner(t["D_P1"], u) + 1j * _horner(t["D_Q1"], u) / zd) * ph * (-1j)
    if E.any():
        ze = z[E]
        u = (ZE / ze) ** 2
        amp = np.sqrt(2 / (np.pi * ze))
        sz, cz = model_sincos(t, ze)
        ph = ((cz + sz) + 1j * (sz - cz)) * np.sqrt(0.5)
        out[0, E] = amp * (_horner(t["E_P0"], u) + 1j * _horner(t["E_Q0"], u) / ze) * ph
        out[1, E] = amp * (_horner(t["E_P1"], u) + 1j * _horner(t["E_Q1"], u) / ze) * ph * (-1j)
    return out


def report(t):
    zs = np.concatenate([np.geomspace(1e-3, 1e4, 4000), np.linspace(3.5, 8.5, 1001)])
    got = eval_f64(t, zs)
    worst = {}
    for q, z in enumerate(zs):
        reg = "A" if z < ZA else ("B" if z < ZC else ("C" if z < ZD else ("D" if z < ZE else "E")))
        for n in (0, 1):
            ref = complex(mp.besselj(n, z) + 1j * mp.bessely(n, z))
            e = abs(got[n, q] - ref) / abs(ref)
            worst[(reg, n)] = max(worst.get((reg, n), 0.0), e)
    return worst


def emit(t, path):
    def arr(vals):
        return ",\n        ".join(mp.nstr(v, 21, min_fixed=-1, max_fixed=-1) for v in vals)

    names = ("A_J0", "A_J1", "A_R0", "A_R1", "C_P0", "C_Q0", "C_P1", "C_Q1", "D_P0", "D_Q0", "D_P1",
             "D_Q1", "E_P0", "E_Q0", "E_P1", "E_Q1", "T_SIN", "T_COS", "T_CW")
    flat = []
    for row in t["B"]:
        for f in row:
            flat.extend(f)
    lines = ["// Generated by gen_bessel_coeffs.py from mpmath (40 digits). Do not edit.",
             "// Polynomial coefficients are listed from degree 0 upwards.",
             "#pragma once", "",
             "namespace bm_bessel_coef {", "",
             f"constexpr double ZA = {ZA!r};   // series region: 0 < z < ZA",
             f"constexpr double ZC = {ZC!r};   // large-argument region C: ZC <= z < ZD",
             f"constexpr double ZD = {ZD!r};  // large-argument region D: ZD <= z < ZE",
             f"constexpr double ZE = {ZE!r};  // large-argument region E: z >= ZE",
             f"constexpr double HB = {HB!r};   // width of the piecewise intervals in [ZA, ZC)",
             f"constexpr int NB = {len(t['B'])};        // number of intervals",
             f"constexpr int DB = {DEG_B + 1};       // coefficients per interval polynomial",
             f"constexpr int NA = {DEG_A + 1};       // coefficients of the series-region polynomials",
             f"constexpr int NC = {DEG_C + 1};       // coefficients of the region-C polynomials",
             f"constexpr int ND = {DEG_D + 1};        // coefficients of the region-D polynomials",
             f"constexpr int NE = {DEG_E + 1};        // coefficients of the region-E polynomials",
             f"constexpr int NT = {DEG_TRIG + 1};        // coefficients of the sine and cosine polynomials", "",
             "// All coefficients in one table; kernels read it through a pointer.",
             "struct Table {"]
    for name in names:
        lines.append(f"    double {name}[{len(t[name])}];")
    lines.append(f"    double B_TAB[{len(flat)}];   // [interval][J0, Y0, J1, Y1 + 2/(pi z)][coefficient in s = z - centre]")
    lines.append("};")
    lines.append("")
    lines.append("constexpr Table kTable = {")
    for name in names:
        lines.append(f"    {{{arr(t[name])}}},")
    lines.append(f"    {{{arr(flat)}}}}};")
    lines.append("")
    lines.append("}  // namespace bm_bessel_coef")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    t = build()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bessel_coeffs.h")
    emit(t, out)
    w = report(t)
    xs = np.linspace(-1e4, 1e4, 200001)
    sm, cm = model_sincos(t, xs)
    werr = max(np.max(np.abs(sm - np.sin(xs))), np.max(np.abs(cm - np.cos(xs))))
    print(f"sine/cosine model on [-1e4, 1e4]: max abs error {werr:.2e}")
    print(f"wrote {out}; float64 model, max relative error of H_n by region:")
    for key in sorted(w):
        print(f"  region {key[0]} H{key[1]}: {w[key]:.2e}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
