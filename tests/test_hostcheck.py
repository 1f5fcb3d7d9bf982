"""CPU checks of the kernels' arithmetic (bessel.hpp, wsbm_pair.hpp) through a
host-compiled instance of the same headers (libbmhss_hostcheck.so, test-only).

Bessel functions are checked against mpmath (40 digits) and the Wronskian;
the 2x2 pair/diagonal blocks against the oracle at the parity bar 1e-10."""
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
