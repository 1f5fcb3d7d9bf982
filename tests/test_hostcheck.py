"""CPU checks of the kernels' arithmetic (bessel.hpp, wsbm_pair.hpp,
wsbm_adjoint.hpp) through a host-compiled instance of the same headers
(libbmhss_hostcheck.so, test-only).

Bessel functions are checked against mpmath (40 digits) and the Wronskian;
the 2x2 pair/diagonal blocks against the oracle at the parity bar 1e-10; the
pair and diagonal derivatives of the shape-derivative kernel against
Richardson central differences of the oracle's blocks (1e-8 relative)."""
import ctypes
import os

import mpmath as mp
import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, wsbm
from parity import assert_parity

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2607_00790_amd", "libbmhss_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIB):
        pytest.skip("hostcheck library not built")
    lib = ctypes.CDLL(LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.bmh_bessel01.argtypes = [vp, i64, vp]
    lib.bmh_sincos.argtypes = [vp, i64, vp]
    lib.bmh_system_blocks.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp]
    lib.bmh_system_blocks_f32.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp]
    lib.bmh_id_guard.argtypes = [i64, i64, i64]
    lib.bmh_level_box_geometry.argtypes = [vp, vp, i64, i64, ctypes.c_int, ctypes.c_double, i64, ctypes.c_int,
                                           ctypes.c_double, vp, vp]
    lib.bmh_level_box_geometry.restype = None
    return lib


def bessel(hc, z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty((z.size, 4))
    hc.bmh_bessel01(z.ctypes.data, z.size, out.ctypes.data)
    return out


def test_bessel_against_mpmath(hc):
    mp.mp.dps = 40
    rng = np.random.default_rng(0)
    z = np.concatenate([np.geomspace(1e-4, 1e4, 1500), rng.uniform(3.9, 8.1, 400),
                        [4.0, 8.0, 4.5, 7.999999999999999, 3.9999999999999996]])
    got = bessel(hc, z)
    worst = 0.0
    for q, zz in enumerate(z):
        zm = mp.mpf(zz)
        h0 = complex(mp.besselj(0, zm) + 1j * mp.bessely(0, zm))
        y1 = mp.bessely(1, zm)
        h1 = complex(mp.besselj(1, zm) + 1j * y1)
        g0 = got[q, 0] + 1j * got[q, 1]
        g1 = got[q, 2] + 1j * (got[q, 3] - 2 / (np.pi * zz))
        worst = max(worst, abs(g0 - h0) / abs(h0), abs(g1 - h1) / abs(h1))
        # the pole-free part Y1 + 2/(pi z) itself, relative to |H1| (what N0 - N1 uses)
        y1r = float(y1 + 2 / (mp.pi * zm))
        assert abs(got[q, 3] - y1r) <= 4e-15 * abs(h1) + 1e-300
    assert worst < 4e-15, worst


def test_sincos_against_mpmath(hc):
    """The kernels' own sine/cosine (Cody-Waite reduction + polynomials) against
    40-digit values, over the argument range k r takes (up to 1e4) and near
    multiples of pi/2, where the reduction must not lose digits."""
    mp.mp.dps = 40
    rng = np.random.default_rng(1)
    near = np.array([k * np.pi / 2 + d for k in (1, 2, 3, 7, 100, 6365) for d in (-1e-9, 0.0, 1e-9)])
    x = np.concatenate([rng.uniform(-10, 10, 300), rng.uniform(8, 1e4, 600),
                        np.geomspace(1e-8, 1e4, 200), near, [0.0, np.pi / 4, -np.pi / 4]])
    out = np.empty((x.size, 2))
    hc.bmh_sincos(np.ascontiguousarray(x).ctypes.data, x.size, out.ctypes.data)
    worst = 0.0
    for q, xx in enumerate(x):
        xm = mp.mpf(xx)
        worst = max(worst, abs(out[q, 0] - float(mp.sin(xm))), abs(out[q, 1] - float(mp.cos(xm))))
    assert worst < 3.5e-16, worst


def test_bessel_wronskian(hc):
    z = np.geomspace(1e-3, 1e4, 3000)
    b = bessel(hc, z)
    j0, y0, j1, y1 = b[:, 0], b[:, 1], b[:, 2], b[:, 3] - 2 / (np.pi * z)
    w = j1 * y0 - j0 * y1
    scale = np.hypot(j0, y0) * np.hypot(j1, y1)
    assert np.max(np.abs(w - 2 / (np.pi * z)) / scale) < 1e-14


def host_blocks(hc, nd, media, rows, cols):
    soa = np.ascontiguousarray(np.stack([nd.x[:, 0], nd.x[:, 1], nd.n[:, 0], nd.n[:, 1], nd.w, nd.kappa]))
    curve = np.ascontiguousarray(nd.curve.astype(np.int32))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    md = np.array([media.k0, media.k1, media.eps0, media.eps1])
    out = np.empty((2 * len(rows), 2 * len(cols)), dtype=np.complex128)
    hc.bmh_system_blocks(soa.ctypes.data, curve.ctypes.data, nd.size, rows.ctypes.data, len(rows),
                         cols.ctypes.data, len(cols), md.ctypes.data, out.ctypes.data)
    return out


def nodes_for(curves, sizes):
    xyd, s = sc.sample_curves(curves, sizes)
    return geometry.discretize(xyd, s)


@pytest.mark.parametrize("case", ["circle512", "star1000", "two_curves", "star16384_rows"])
def test_pair_blocks_match_oracle(hc, case):
    if case == "circle512":
        wl = sc.circle_workload(512)
        nd, media = nodes_for(wl.curves, wl.sizes), wl.media
        rows = cols = np.arange(512)
    elif case == "star1000":
        nd, media = nodes_for([sc.star(0.3, 5)], [1000]), sc.media_from_index(50.0, 1.5)
        rows = cols = np.arange(1000)
    elif case == "two_curves":
        nd = nodes_for([sc.star(0.2, 4), sc.star(0.25, 3, 1.0, (3.0, 0.5))], [300, 200])
        media = sc.media_from_index(20.0, 2.0)
        rows = cols = np.arange(500)
    else:
        wl = sc.star_workload()
        nd, media = nodes_for(wl.curves, wl.sizes), wl.media
        rng = np.random.default_rng(1)
        rows = np.concatenate([[0, 1, 16383], rng.integers(0, 16384, 13)])
        cols = np.arange(16384)
    got = host_blocks(hc, nd, media, rows, cols)
    ref = wsbm.system_blocks(nd, media, rows, cols).reshape(2 * len(rows), 2 * len(cols))
    assert_parity(got, ref)


@pytest.mark.parametrize("case", ["star1000", "two_curves", "star16384_rows"])
def test_fp32_pair_blocks_match_oracle(hc, case):
    """The FP32 entry path (wsbm_pair_f32.hpp, compiled for the host) against
    the FP64 oracle: per 2x2 component, max|diff| <= 1e-6 max|ref| -- FP32
    rounding of ~1e-7 relative per entry (r and the phase k r are FP64),
    amplified in the D-type entries of close pairs, which are small."""
    if case == "star1000":
        nd, media = nodes_for([sc.star(0.3, 5)], [1000]), sc.media_from_index(50.0, 1.5)
        rows = cols = np.arange(1000)
    elif case == "two_curves":
        nd = nodes_for([sc.star(0.2, 4), sc.star(0.25, 3, 1.0, (3.0, 0.5))], [300, 200])
        media = sc.media_from_index(20.0, 2.0)
        rows = cols = np.arange(500)
    else:
        wl = sc.star_workload()
        nd, media = nodes_for(wl.curves, wl.sizes), wl.media
        rng = np.random.default_rng(1)
        rows = np.concatenate([[0, 1, 16383], rng.integers(0, 16384, 13)])
        cols = np.arange(16384)
    soa = np.ascontiguousarray(np.stack([nd.x[:, 0], nd.x[:, 1], nd.n[:, 0], nd.n[:, 1], nd.w, nd.kappa]))
    curve = np.ascontiguousarray(nd.curve.astype(np.int32))
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    md = np.array([media.k0, media.k1, media.eps0, media.eps1])
    got = np.empty((2 * len(r), 2 * len(c)), dtype=np.complex128)
    hc.bmh_system_blocks_f32(soa.ctypes.data, curve.ctypes.data, nd.size, r.ctypes.data, len(r), c.ctypes.data,
                             len(c), md.ctypes.data, got.ctypes.data)
    ref = wsbm.system_blocks(nd, media, rows, cols).reshape(2 * len(rows), 2 * len(cols))
    g = got.reshape(len(r), 2, len(c), 2)
    f = ref.reshape(g.shape)
    for a in range(2):
        for b in range(2):
            err = np.abs(g[:, a, :, b] - f[:, a, :, b]).max() / np.abs(f[:, a, :, b]).max()
            assert err <= 1e-6, (a, b, err)
    # cross-curve pairs keep no interior terms: the first row is exactly zero
    if case == "two_curves":
        assert np.all(g[:300, 0, 300:, :] == 0)


def test_id_work_guard_decisions(hc):
    """The ID work guard (host-side planning from sizes): the top-level ID that
    never finished (two boxes of 19096 unknowns x 62236 rows) is stopped; the
    levels the benchmark and the large workload compress are not."""
    g = hc.bmh_id_guard
    assert g(62236, 19096, 2 * 62236 * 19096) == 3
    assert g(684, 188, 72 * 684 * 188) == 0           # leaf level of the batched forest
    assert g(760, 260, 4 * 760 * 260) == 0
    assert g(4000, 1400, 256 * 4000 * 1400) == 0      # the large workload's last compressed level
    assert g(12000, 4096, 64 * 12000 * 4096) == 2     # fine per box, too much for one level
    assert g(2 ** 26, 1, 2 ** 26) == 0 and g(2 ** 26 + 1, 1, 2 ** 26 + 1) == 1
    assert g(0, 0, 0) == 0


def test_level_box_geometry_matches_its_definition(hc):
    """The tree's boxes and proxy circles (paper Sec. III, Fig. 2; the build's
    host planning, hss_plan.hpp) on the nodes of the N = 16384 star, for the
    whole curve and for a body of 5000 nodes starting at node 1000: level l has
    2^l boxes of consecutive nodes that partition the body, each box's centre is
    the mean of its nodes, its proxy radius 1.5 times the largest node distance
    from the centre, so that every node lies strictly inside the circle, and its
    proxy count is P = 64, or with adaptive counts max(P, ceil(2 k r) + 32),
    capped at 2^20 (k = 2e6 reaches the cap on level 1)."""
    xyd, s = sc.sample_curves([sc.star(0.3, 5)], [16384])
    nd = geometry.discretize(xyd, s)
    x = np.ascontiguousarray(nd.x[:, 0])
    y = np.ascontiguousarray(nd.x[:, 1])
    for nlo, nn in ((0, 16384), (1000, 5000)):
        for lev in (1, 4, 8):
            nb = 1 << lev
            bounds = [nlo + (b * nn) // nb for b in range(nb + 1)]
            assert bounds[0] == nlo and bounds[-1] == nlo + nn and min(np.diff(bounds)) > 0
            for adapt, kmax in ((0, 50.0), (1, 75.0), (1, 2e6)):
                bc = np.zeros(3 * nb)
                bp = np.zeros(nb, dtype=np.int32)
                hc.bmh_level_box_geometry(x.ctypes.data, y.ctypes.data, nlo, nn, lev, 1.5, 64, adapt, kmax,
                                          bc.ctypes.data, bp.ctypes.data)
                bc = bc.reshape(nb, 3)
                for b in range(nb):
                    lo, hi = bounds[b], bounds[b + 1]
                    cx, cy = x[lo:hi].mean(), y[lo:hi].mean()
                    dist = np.hypot(x[lo:hi] - bc[b, 0], y[lo:hi] - bc[b, 1])
                    assert abs(bc[b, 0] - cx) <= 1e-14 and abs(bc[b, 1] - cy) <= 1e-14
                    assert abs(bc[b, 2] - 1.5 * np.hypot(x[lo:hi] - cx, y[lo:hi] - cy).max()) <= 1e-13 * bc[b, 2]
                    assert dist.max() < bc[b, 2]
                    want = 64 if not adapt else min(max(64, int(np.ceil(2.0 * kmax * bc[b, 2])) + 32), 2 ** 20)
                    assert bp[b] == want, (nlo, lev, b, adapt, bp[b], want)
            if lev == 1:
                assert (bp == 2 ** 20).all()   # the last case: k = 2e6 on the two largest boxes


# ---------------------------------------------------------------------------
# Shape-derivative building blocks (wsbm_adjoint.hpp) against Richardson
# central differences of the oracle's own pair and diagonal blocks.

def _richardson(f, h):
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def _pair_form(media, tx, tn, sx, sn, sw, lam, ph, interior):
    """lam_i^T A_ij phi_j from the oracle's pair block."""
    blk = wsbm.pair_blocks(tx[None], tn[None], sx[None], sn[None], np.array([sw]), media,
                           interior=np.array([[interior]]))[0, :, 0, :]
    return lam @ blk @ ph


def test_pair_adjoint_matches_oracle_differences(hc):
    hc.bmh_pair_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p]
    media = sc.media_from_index(40.0, 1.5)
    md = np.array([media.k0, media.k1, media.eps0, media.eps1])
    rng = np.random.default_rng(11)
    cases = []
    for r in (1e-3, 0.02, 0.1, 0.3, 1.0, 3.0, 20.0):      # z = k r from 0.04 to 1200
        for interior in (1.0, 0.0):
            ang = rng.uniform(0, 2 * np.pi)
            tx = rng.standard_normal(2)
            sx = tx - r * np.array([np.cos(ang), np.sin(ang)])
            a1, a2 = rng.uniform(0, 2 * np.pi, 2)
            tn, sn = np.array([np.cos(a1), np.sin(a1)]), np.array([np.cos(a2), np.sin(a2)])
            sw = rng.uniform(0.001, 0.01)
            lam = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            ph = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            cases.append((tx, tn, sx, sn, sw, lam, ph, interior))
    inp = np.zeros((len(cases), 16))
    phi = np.zeros((len(cases), 4))
    for q, (tx, tn, sx, sn, sw, lam, ph, it) in enumerate(cases):
        inp[q, :14] = [*tx, *tn, lam[0].real, lam[0].imag, lam[1].real, lam[1].imag, *sx, *sn, sw, it]
        phi[q] = [ph[0].real, ph[0].imag, ph[1].real, ph[1].imag]
    out = np.empty((len(cases), 14))
    hc.bmh_pair_adjoint(inp.ctypes.data, phi.ctypes.data, len(cases), md.ctypes.data, out.ctypes.data)
    got = out[:, 0::2] + 1j * out[:, 1::2]          # d/drho x, y; d/dn_i x, y; d/dn_j x, y; d/dw
    for q, (tx, tn, sx, sn, sw, lam, ph, it) in enumerate(cases):
        r = np.hypot(*(tx - sx))
        F = lambda **kw: _pair_form(media, kw.get("tx", tx), kw.get("tn", tn), kw.get("sx", sx),
                                    kw.get("sn", sn), kw.get("sw", sw), lam, ph, it)
        e = np.eye(2)
        hx, hn = 1e-3 * min(r, 1.0 / media.k1), 1e-4   # small against r and the wavelength
        ref = [_richardson(lambda s, c=c: F(tx=tx + s * e[c]), hx) for c in range(2)]
        ref += [_richardson(lambda s, c=c: F(tn=tn + s * e[c]), hn) for c in range(2)]
        ref += [_richardson(lambda s, c=c: F(sn=sn + s * e[c]), hn) for c in range(2)]
        ref += [F() / sw]                           # the pair is linear in w_j
        src = [_richardson(lambda s, c=c: F(sx=sx + s * e[c]), hx) for c in range(2)]
        ref, src = np.array(ref), np.array(src)
        scale = np.abs(ref).max()
        err = np.abs(got[q] - ref).max()
        assert err <= 1e-8 * scale, (q, r, it, err / scale)
        # the pair depends on x_i - x_j only: d/dx_j = -d/drho
        assert np.abs(src + got[q, :2]).max() <= 1e-8 * scale, (q, r, it)


def test_diag_adjoint_matches_oracle_differences(hc):
    hc.bmh_diag_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p]
    rng = np.random.default_rng(12)
    for media in (sc.media_from_index(40.0, 1.5), sc.table1_media()):
        md = np.array([media.k0, media.k1, media.eps0, media.eps1])
        for w, kap in ((1e-3, 1.0), (0.02, -3.0), (0.3, 0.2)):
            lam = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            ph = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            inp = np.array([w, kap, lam[0].real, lam[0].imag, lam[1].real, lam[1].imag, 0, 0])
            phi = np.array([ph[0].real, ph[0].imag, ph[1].real, ph[1].imag])
            out = np.empty(4)
            hc.bmh_diag_adjoint(inp.ctypes.data, phi.ctypes.data, 1, md.ctypes.data, out.ctypes.data)

            def F(ww, kk):
                nd = geometry.Nodes(np.zeros((1, 2)), np.array([[1.0, 0.0]]), np.array([ww]),
                                    np.array([kk]), np.zeros(1, dtype=np.int64))
                return lam @ wsbm.system_blocks(nd, media, [0], [0]).reshape(2, 2) @ ph

            dw = _richardson(lambda s: F(w + s, kap), 1e-3 * w)
            dk = _richardson(lambda s: F(w, kap + s), 1e-2)
            assert abs(out[0] + 1j * out[1] - dw) <= 1e-9 * abs(dw), (w, kap)
            assert abs(out[2] + 1j * out[3] - dk) <= 1e-9 * max(abs(dk), abs(dw) * w), (w, kap)


def test_shape_derivative_matches_oracle_differences(hc):
    """The kernels' whole per-node derivative (pair sums, diagonal, right-hand
    side, far field, chain rule to the samples) run on the host for one body of
    two curves, against Richardson differences of the oracle's
    L = g.phi + lam.(b - A phi) with respect to every sample of sampled nodes."""
    vp = ctypes.c_void_p
    hc.bmh_shape_derivative.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp, ctypes.c_double,
                                        ctypes.c_double, vp, vp]
    media = sc.media_from_index(8.0, 1.5)
    xyd, s = sc.sample_curves([sc.star(0.2, 3), sc.circle(0.3, (2.5, 0.0))], [48, 40])
    nd = geometry.discretize(xyd, s)
    N = nd.size
    rng = np.random.default_rng(13)
    phi = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    lam = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
    coef = np.array([0.7, -1.3])
    inc, obs = 0.7, 2.9
    soa = np.ascontiguousarray(np.stack([nd.x[:, 0], nd.x[:, 1], nd.n[:, 0], nd.n[:, 1], nd.w, nd.kappa]))
    curve = np.ascontiguousarray(nd.curve.astype(np.int32))
    md = np.array([media.k0, media.k1, media.eps0, media.eps1])
    grad = np.empty((6, N))
    hc.bmh_shape_derivative(soa.ctypes.data, np.ascontiguousarray(xyd).ctypes.data, curve.ctypes.data, N,
                            md.ctypes.data, lam.ctypes.data, phi.ctypes.data, inc, obs, coef.ctypes.data,
                            grad.ctypes.data)

    def L(x):
        n2 = geometry.discretize(x, s)
        g = wsbm.far_field_weights(n2, media, obs)
        b = wsbm.rhs_plane_wave(n2, media, inc)
        return g @ phi + lam @ (b - wsbm.assemble_dense(n2, media) @ phi)

    c = coef[0] + 1j * coef[1]
    for i in (0, 5, 47, 48, 70, 87):
        for r in range(6):
            def f(h):
                x = xyd.copy()
                x[r, i] += h
                return L(x)
            ref = np.real(c * _richardson(f, 1e-5 if r < 4 else 1e-3))
            assert abs(grad[r, i] - ref) <= 1e-7 * np.abs(grad).max(), (i, r, grad[r, i], ref)
