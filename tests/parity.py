"""Parity bar shared by the CPU and GPU parity tests."""
import numpy as np


def assert_parity(got, ref, tol=1e-10):
    """Per 2x2 component: max|diff| <= tol * max|ref|, and per entry relative
    error <= tol wherever |ref| >= 1e-6 * max|ref| of that component."""
    g = got.reshape(got.shape[0] // 2, 2, got.shape[1] // 2, 2)
    r = ref.reshape(g.shape)
    for p in range(2):
        for q in range(2):
            gg, rr = g[:, p, :, q], r[:, p, :, q]
            m = np.abs(rr).max()
            if m == 0:
                assert np.all(gg == 0)
                continue
            d = np.abs(gg - rr)
            assert d.max() <= tol * m, (p, q, d.max() / m)
            big = np.abs(rr) >= 1e-6 * m
            assert np.all(d[big] <= tol * np.abs(rr[big])), (p, q, (d[big] / np.abs(rr[big])).max())
