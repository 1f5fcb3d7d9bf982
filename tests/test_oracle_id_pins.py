"""Pins of the oracle's interpolative decomposition (oracle/idecomp.py, the ID
of the proxy-surface compression, paper Sec. III) to facts that do not come
from its own code: a worked example computed by hand, exact low-rank
reconstruction, LAPACK's column-pivoted QR (geqp3, through SciPy) as the
special case tol = 0, the rank rule on matrices of known singular values, and
the degenerate cases (zero matrix, zero and tied columns)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import idecomp


def test_worked_example_by_hand():
    """X = [[3, 1, 4], [4, 2, 3]].  Column norms 5, sqrt 5, 5: the tie goes to
    column 0.  Its reflector has alpha = -5, v = (8, 4), beta = 1 / (5 (5 + 3))
    = 1/40, and maps column 1 to (1, 2) - (16/40)(8, 4) = (-2.2, 0.4), column 2
    to (4, 3) - (44/40)(8, 4) = (-4.8, -1.4).  Below row 0 the norms are 0.4
    and 1.4: column 2 is next, alpha = 1.4 (x = -1.4), and the rank is 2
    (1.4 / 5 = 0.28).  R11 = [[-5, -4.8], [0, 1.4]], R12 = (-2.2, -0.4):
    z = R11^-1 R12 = (5/7, -2/7), and indeed 5/7 (3, 4) - 2/7 (4, 3) = (1, 2).
    With tol = 0.3 the second step fails 1.4 > 0.3 * 5: rank 1, and column j
    is R_0j / R_00 times column 0: (1, 2.2/5, 4.8/5)."""
    X = np.array([[3, 1, 4], [4, 2, 3]], dtype=complex)
    r, perm, T, d = idecomp.interp_decomp(X, 1e-10)
    assert r == 2
    assert perm.tolist() == [0, 2, 1]
    np.testing.assert_allclose(d, [-5.0, 1.4], rtol=0, atol=1e-14)
    np.testing.assert_allclose(T, [[1, 0], [5 / 7, -2 / 7], [0, 1]], rtol=0, atol=1e-14)
    r, perm, T, d = idecomp.interp_decomp(X, 0.3)
    assert r == 1
    assert perm.tolist() == [0, 1, 2]
    np.testing.assert_allclose(T[:, 0], [1.0, 0.44, 0.96], rtol=0, atol=1e-14)


@pytest.mark.parametrize("m,n,r", [(60, 40, 8), (40, 60, 1), (136, 128, 53), (30, 30, 17)])
def test_exact_low_rank_is_reconstructed(m, n, r):
    """A product of complex Gaussian m x r and r x n factors has rank r: the
    ID finds r and reproduces every column to rounding."""
    rng = np.random.default_rng(m * 1000 + n + r)
    g = lambda a, b: rng.standard_normal((a, b)) + 1j * rng.standard_normal((a, b))
    X = g(m, r) @ g(r, n)
    k, perm, T, _ = idecomp.interp_decomp(X, 1e-10)
    assert k == r
    np.testing.assert_array_equal(T[perm[:k]], np.eye(k))
    assert np.linalg.norm(X - X[:, perm[:k]] @ T.T) <= 1e-12 * np.linalg.norm(X)
    assert sorted(perm.tolist()) == list(range(n))
    assert perm[k:].tolist() == sorted(perm[k:].tolist())


@pytest.mark.parametrize("m,n", [(50, 30), (30, 50), (136, 128), (7, 7)])
def test_pivots_and_diagonal_match_lapack_geqp3(m, n):
    """With tol = 0 the factorisation is plain column-pivoted QR: LAPACK's
    geqp3 (norm downdating, another code) picks the same columns in the same
    order on a generic complex matrix, and |R_kk| agree to rounding."""
    rng = np.random.default_rng(7 * m + n)
    X = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    k, perm, _, d = idecomp.interp_decomp(X, 0.0)
    assert k == min(m, n)
    _, R, P = scipy.linalg.qr(X, pivoting=True, mode="economic")
    assert P[:k].tolist() == perm[:k].tolist()
    np.testing.assert_allclose(np.abs(d), np.abs(np.diag(R))[:k], rtol=1e-12)


def test_rank_rule_on_a_known_spectrum():
    """X = U diag(s) V^H with s_j = 10^(-j/4) and random unitary U, V: the
    rank at tol is at least the count of s_j > tol s_0 (|R_kk| >= s_k up to a
    factor, |R_00| = the largest column norm <= s_0) and at most four more
    (|R_kk| exceeds s_k by less than a factor 10 here, four steps of the
    decay), and the ID error stays within 100 tol |X|_2."""
    rng = np.random.default_rng(11)
    m, n = 120, 100
    U, _ = np.linalg.qr(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    s = 10.0 ** (-np.arange(n) / 4.0)
    X = (U * s) @ V.conj().T
    for tol in (1e-3, 1e-6, 1e-10):
        k, perm, T, _ = idecomp.interp_decomp(X, tol)
        cnt = int((s > tol * s[0]).sum())
        assert cnt <= k <= cnt + 4, (tol, k, cnt)
        assert np.linalg.norm(X - X[:, perm[:k]] @ T.T, 2) <= 100 * tol * s[0]


def test_degenerate_cases():
    """A zero matrix has rank 0 (perm is the identity, T has no columns); a
    zero column is never a skeleton column of a nonzero matrix; among columns
    of exactly equal norm the lowest index is chosen first."""
    k, perm, T, _ = idecomp.interp_decomp(np.zeros((5, 4), dtype=complex), 1e-10)
    assert k == 0 and perm.tolist() == [0, 1, 2, 3] and T.shape == (4, 0)
    X = np.array([[0, 1, 2], [0, 2, 1], [0, 2, 2]], dtype=complex)   # columns 1 and 2: equal norms 3
    k, perm, T, _ = idecomp.interp_decomp(X, 1e-10)
    assert perm[0] == 1 and 0 not in perm[:k].tolist()
    np.testing.assert_allclose(T[0], 0.0, atol=0)
