"""Brute-force WSBM entries in 30-digit arithmetic (mpmath), for tiny inputs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Evaluates, pair by pair, the same definitions as oracle.wsbm (Eq. (5) of the
paper with readings R1-R6) but with mpmath's Bessel functions and arithmetic,
so that a misuse of the double-precision special-function library, or
cancellation in the hypersingular difference N_k0 - N_k1, shows up as a
mismatch.  Only sensible for N <= a few dozen.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def _h(nu, z):
    return mp.besselj(nu, z) + 1j * mp.bessely(nu, z)


def system_matrix(nodes, media, dps=30):
    """Dense node-interleaved 2N x 2N matrix as complex128 (computed at dps digits)."""
    idx = np.arange(nodes.size)
    return system_blocks(nodes, media, idx, idx, dps).reshape(2 * nodes.size, 2 * nodes.size)


def system_blocks(nodes, media, rows, cols, dps=30):
    """Blocks A(rows, cols), shape (len(rows), 2, len(cols), 2), at dps digits."""
    mp.mp.dps = dps
    k0, k1 = mp.mpf(media.k0), mp.mpf(media.k1)
    e0, e1 = mp.mpf(media.eps0), mp.mpf(media.eps1)
    alpha = mp.mpc(0, 1) / k0
    pi = mp.pi
    out = np.empty((len(rows), 2, len(cols), 2), dtype=np.complex128)
    X = [(mp.mpf(float(p[0])), mp.mpf(float(p[1]))) for p in nodes.x]
    Nn = [(mp.mpf(float(p[0])), mp.mpf(float(p[1]))) for p in nodes.n]
    W = [mp.mpf(float(v)) for v in nodes.w]
    K = [mp.mpf(float(v)) for v in nodes.kappa]
    for ii, i in enumerate(rows):
        for jj, j in enumerate(cols):
            if i == j:
                w, kap = W[i], K[i]
                L0 = mp.log(k0 * w / (4 * pi)) + mp.euler
                L1 = mp.log(k1 * w / (4 * pi)) + mp.euler
                S0 = -(w / (2 * pi)) * (L0 - 1j * pi / 2)
                S1 = -(w / (2 * pi)) * (L1 - 1j * pi / 2)
                Dd = -kap * w / (4 * pi)
                ND = -(w / (4 * pi)) * (k0**2 * (L0 - mp.mpf(1) / 2 - 1j * pi / 2)
                                        - k1**2 * (L1 - mp.mpf(1) / 2 - 1j * pi / 2))
                blk = [[Dd + mp.mpf(1) / 2, -e1 * S1],
                       [Dd - mp.mpf(1) / 2 + alpha * ND,
                        -e0 * S0 - alpha * (e0 - e1) * Dd - alpha * (e0 + e1) / 2]]
            else:
                same = nodes.curve[i] == nodes.curve[j]
                rx, ry = X[i][0] - X[j][0], X[i][1] - X[j][1]
                r = mp.sqrt(rx * rx + ry * ry)
                a = rx * Nn[i][0] + ry * Nn[i][1]
                b = rx * Nn[j][0] + ry * Nn[j][1]
                c = Nn[i][0] * Nn[j][0] + Nn[i][1] * Nn[j][1]
                w = W[j]

                def kern(k):
                    z = k * r
                    h0, h1, h2 = _h(0, z), _h(1, z), _h(2, z)
                    S = 1j / 4 * h0 * w
                    D = 1j * k / 4 * h1 * (b / r) * w
                    Ds = -1j * k / 4 * h1 * (a / r) * w
                    Nk = 1j * k / 4 * (h1 * c / r - k * h2 * a * b / r**2) * w
                    return S, D, Ds, Nk

                S0, D0, Ds0, N0 = kern(k0)
                if same:
                    S1, D1, Ds1, N1 = kern(k1)
                else:
                    S1 = D1 = Ds1 = N1 = mp.mpc(0)
                blk = [[D1, -e1 * S1],
                       [D0 + alpha * (N0 - N1), -e0 * S0 - alpha * (e0 * Ds0 - e1 * Ds1)]]
            for p in range(2):
                for q in range(2):
                    out[ii, p, jj, q] = complex(blk[p][q])
    return out
