"""GPU tests of the dense inverse the HSS factorisation uses (bm_dense_inverse:
Gauss-Jordan for blocks up to 64 -- by panels of eight columns with the
rank-8 updates on the matrix cores from 48 rows, two elimination steps per
barrier below --, block Gauss-Jordan over 64-column panels with look-ahead up
to 4096, the Schur recursion above), against NumPy's LAPACK inverse, and of
its singular-pivot reporting, directly and through the build's test hook.

The bar: the inverse of a matrix with condition number kappa is determined
to about kappa * eps; these matrices have kappa below ~100 (a Gaussian matrix
scaled to spectral radius ~1 plus 3 I, or for n <= 64 a plain Gaussian matrix,
where partial pivoting runs over every row), and the bar is 1e-11 relative in
the Frobenius norm."""
import os
import sys

import numpy as np
import pytest

import scatterers as sc

pytestmark = pytest.mark.gpu

BAR = 1e-11
ESINGULAR = 4


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gaussian(n, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0 * n)
    return a + shift * np.eye(n)


def gpu_inverse(bm, a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bm.bm_dense_inverse(t)
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 31, 32, 33, 47, 48, 55, 63, 64])
def test_gauss_jordan_blocks_vs_lapack(gpu_lib, n):
    """Blocks up to 64: one workgroup, pivoting over every row (a plain Gaussian
    matrix, no diagonal shift, so the pivot order is not the identity)."""
    bm = gpu_lib
    a = gaussian(n, 100 + n)
    note(f"inverse: n={n}, Gaussian, cond {np.linalg.cond(a):.1f}")
    x = gpu_inverse(bm, a)
    err = rel(x, np.linalg.inv(a))
    note(f"  rel error {err:.2e}")
    assert err <= BAR * max(1.0, np.linalg.cond(a) / 100.0)


@pytest.mark.parametrize("n", [65, 100, 128, 200, 777, 1526])
def test_panel_inverse_vs_lapack(gpu_lib, n):
    """Above 64: 64-column panels, the trailing updates on the matrix cores, the
    second stream's look-ahead; ragged last panels (100, 200, 777, 1526)."""
    bm = gpu_lib
    a = gaussian(n, 200 + n, shift=3.0)
    note(f"inverse: n={n}, Gaussian + 3 I")
    x = gpu_inverse(bm, a)
    err = rel(x, np.linalg.inv(a))
    note(f"  rel error {err:.2e}")
    assert err <= BAR


def test_schur_recursion_inverse_residual(gpu_lib):
    """Above 4096 the Schur recursion (large products in rocBLAS): residual
    |A X - I|_F / sqrt(n) on the device."""
    import torch
    bm = gpu_lib
    n = 4133
    a = gaussian(n, 300, shift=3.0)
    note(f"inverse: n={n} (recursion), Gaussian + 3 I")
    at = torch.from_numpy(a).cuda()
    x = at.clone()
    bm.bm_dense_inverse(x)
    r = at @ x - torch.eye(n, dtype=torch.complex128, device="cuda")
    res = (torch.linalg.matrix_norm(r) / np.sqrt(n)).item()
    note(f"  residual {res:.2e}")
    assert res <= BAR


@pytest.mark.parametrize("n", [5, 40, 56, 64])
def test_singular_block_reported_and_left_unchanged(gpu_lib, n):
    """A zero row: the kernel ends normally with BM_ESINGULAR, the matrix is
    left as it was (no NaN), and the next call on a good matrix succeeds."""
    import torch
    bm = gpu_lib
    a = gaussian(n, 400 + n)
    a[n // 2, :] = 0.0
    note(f"inverse: n={n}, zero row {n // 2}")
    t = torch.from_numpy(a).cuda()
    with pytest.raises(bm.BmError) as ei:
        bm.bm_dense_inverse(t)
    assert ei.value.code == ESINGULAR
    back = t.cpu().numpy()
    assert np.isfinite(back).all()
    assert np.array_equal(back, a)
    good = gaussian(n, 500 + n, shift=3.0)
    assert rel(gpu_inverse(bm, good), np.linalg.inv(good)) <= BAR


def test_tiny_pivot_reported(gpu_lib):
    """A row scaled by 1e-20 leaves a last pivot below 64 eps of the block's
    largest entry: reported as singular rather than inverted into huge
    values."""
    bm = gpu_lib
    n = 48
    a = gaussian(n, 600)
    a[7, :] *= 1e-20
    note("inverse: n=48, row 7 scaled by 1e-20")
    import torch
    t = torch.from_numpy(a).cuda()
    with pytest.raises(bm.BmError) as ei:
        bm.bm_dense_inverse(t)
    assert ei.value.code == ESINGULAR


def test_singular_panel_reported(gpu_lib):
    """A zero row in the second 64-column panel of a 200 x 200 matrix: the
    panel path ends normally with BM_ESINGULAR; the next call succeeds."""
    import torch
    bm = gpu_lib
    n = 200
    a = gaussian(n, 700, shift=3.0)
    a[90, :] = 0.0
    note("inverse: n=200, zero row 90")
    t = torch.from_numpy(a).cuda()
    with pytest.raises(bm.BmError) as ei:
        bm.bm_dense_inverse(t)
    assert ei.value.code == ESINGULAR
    good = gaussian(n, 701, shift=3.0)
    assert rel(gpu_inverse(bm, good), np.linalg.inv(good)) <= BAR


def test_inverse_rejects_bad_arguments(gpu_lib):
    import torch
    bm = gpu_lib
    with pytest.raises(ValueError):
        bm.bm_dense_inverse(torch.zeros((3, 4), dtype=torch.complex128, device="cuda"))
    lib = bm.load()
    t = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    import ctypes
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.bm_dense_inverse(ctypes.c_void_p(t.data_ptr()), 0, 4, s) == 1
    assert lib.bm_dense_inverse(ctypes.c_void_p(t.data_ptr()), 4, 3, s) == 1
    assert lib.bm_dense_inverse(None, 4, 4, s) == 1
    assert lib.bm_dense_inverse(ctypes.c_void_p(t.data_ptr()), 16385, 16385, s) == 1


def test_hss_build_reports_singular_root_through_hook(gpu_lib):
    """BMHSS_TEST_SINGULAR_ROOT=1 zeroes the first row of the dense root before
    its inversion: bm_hss_build returns BM_ESINGULAR (every kernel ends
    normally), and without the hook the same build solves as before."""
    bm = gpu_lib
    media = sc.media_from_index(50.0, 1.5)
    xyd, s = sc.sample_curves([sc.star(0.3, 5)], [2048])
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create(g, media.k0, media.k1, media.eps0, media.eps1)
    b = bm.bm_rhs_plane_wave(p, 0.2)
    note("hss: singular root hook, star N=2048, tuned options")
    os.environ["BMHSS_TEST_SINGULAR_ROOT"] = "1"
    try:
        with pytest.raises(bm.BmError) as ei:
            bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=-1,
                            max_rank_ratio=-1.0)
        assert ei.value.code == ESINGULAR
    finally:
        del os.environ["BMHSS_TEST_SINGULAR_ROOT"]
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=-1, max_rank_ratio=-1.0)
    x = bm.bm_hss_solve(h, b)
    r = bm.bm_matvec(p, x) - b
    import torch
    res = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    note(f"  after the hook: residual {res:.2e}")
    assert res < 1e-6
