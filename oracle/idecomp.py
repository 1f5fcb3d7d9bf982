"""Interpolative decomposition (ID) of a complex matrix by Householder QR with
column pivoting -- the step of the proxy-surface compression that picks a
box's skeleton indices (paper Sec. III, which takes the skeleton indices of
Martinsson and Rokhlin's direct solver).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names the method, not its algorithm.  Readings (the same as the
library's, listed with the others in the design notes):
  I1  the ID is the one obtained from QR with column pivoting (Businger and
      Golub): at step k the remaining column of largest 2-norm over rows
      k, k+1, .. becomes column k (lowest original index on ties), and a
      Householder reflection zeroes it below row k;
  I2  the rank is the number of steps k with |R_kk| > tol |R_00| (a relative
      tolerance on the diagonal of R, which is non-increasing in magnitude);
      the factorisation stops at the first step that fails the test, or after
      min(m, n) steps;
  I3  with the pivot order perm (the k skeleton columns first, then the other
      columns in increasing order) and R = [R11 R12], the interpolation
      matrix T (n x k) has row perm[i] = e_i (i < k) and row perm[k + c] =
      column c of R11^-1 R12, so that X ~= X[:, perm[:k]] @ T.T.

The norms are recomputed from the reflected columns at every step (no norm
downdating).  Plain NumPy in FP64 with explicit column swaps and one
triangular solve from SciPy; no blocking.
"""
import numpy as np
import scipy.linalg


def _householder(x):
    """Reflector H = I - beta v v^H with H x = alpha e_0, alpha = -(x_0/|x_0|) |x|
    (alpha = -|x| when x_0 = 0).  Returns (v, beta, alpha)."""
    xn = np.linalg.norm(x)
    a0 = abs(x[0])
    phase = x[0] / a0 if a0 > 0 else 1.0
    alpha = -phase * xn
    v = x.astype(np.complex128).copy()
    v[0] -= alpha
    beta = 1.0 / (xn * (xn + a0)) if xn > 0 else 0.0
    return v, beta, alpha


def cpqr(X, tol):
    """Column-pivoted Householder QR of X (m x n, complex), readings I1 and I2.
    Returns (rank, order, R): order[k] is the original index of the column
    chosen at step k (the first `rank` entries are meaningful), R the m x n
    upper-trapezoidal factor of X[:, order] (rows >= rank not completed)."""
    A = np.array(X, dtype=np.complex128, copy=True)
    m, n = A.shape
    order = np.arange(n)
    ref = None
    rank = 0
    for k in range(min(m, n)):
        norms = np.linalg.norm(A[k:, k:], axis=0)
        j = k + int(np.argmax(norms))          # first maximum: lowest index on ties
        if ref is None:
            ref = norms[j - k]
        if not (norms[j - k] > tol * ref) or ref == 0:
            break
        A[:, [k, j]] = A[:, [j, k]]
        order[[k, j]] = order[[j, k]]
        v, beta, alpha = _householder(A[k:, k])
        A[k:, k + 1:] -= beta * np.outer(v, v.conj() @ A[k:, k + 1:])
        A[k, k] = alpha
        A[k + 1:, k] = 0.0
        rank = k + 1
    return rank, order, A


def interp_decomp(X, tol):
    """The ID of X (reading I3).  Returns (rank, perm, T, rdiag): perm as the
    library orders it (skeleton first, then the rest in increasing order), T
    (n x rank) and the diagonal R_00 .. R_{rank-1, rank-1}."""
    X = np.asarray(X)
    m, n = X.shape
    rank, order, R = cpqr(X, tol)
    skel = order[:rank]
    rest = np.array(sorted(set(range(n)) - set(skel.tolist())), dtype=np.int64)
    perm = np.concatenate([skel, rest]).astype(np.int64)
    T = np.zeros((n, rank), dtype=np.complex128)
    T[skel, np.arange(rank)] = 1.0
    if rank > 0 and rest.size:
        # R12 in the order of `rest`: the columns of R belonging to those indices
        pos = {int(c): i for i, c in enumerate(order)}
        R12 = R[:rank, [pos[int(c)] for c in rest]]
        Z = scipy.linalg.solve_triangular(R[:rank, :rank], R12, lower=False)
        T[rest, :] = Z.T
    return rank, perm, T, np.diag(R[:rank, :rank]).copy()
