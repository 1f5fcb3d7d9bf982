"""GPU tests of the randomized ID's sketch Y = Omega X (bm_sketch: a real
Omega times a complex X on the FP64 matrix cores) against NumPy, on shapes
that take the single-slice path (enough tiles to fill the device), the
split-K path with its partial sums, ragged tiles and the 1 x 1 x 1 corner.
The bar is 1e-13 relative in the Frobenius norm: the products differ only in
summation order (Gaussian entries, K <= 1000)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("l,m,n", [(1, 1, 1), (65, 17, 33), (136, 388, 128), (200, 1000, 300),
                                   (640, 64, 3300), (64, 4096, 31)])
def test_sketch_vs_numpy(gpu_lib, l, m, n):
    import torch
    bm = gpu_lib
    rng = np.random.default_rng(l * 7 + m * 3 + n)
    omega = rng.standard_normal((l, m))
    x = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    note(f"sketch: l={l} m={m} n={n}")
    yt = bm.bm_sketch(torch.from_numpy(omega).cuda(), torch.from_numpy(np.ascontiguousarray(x.T)).cuda())
    y = yt.cpu().numpy().T
    ref = omega @ x
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    note(f"  rel error {err:.2e}")
    assert err <= 1e-13


def test_sketch_rejects_bad_arguments(gpu_lib):
    import ctypes
    import torch
    bm = gpu_lib
    lib = bm.load()
    o = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    x = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    po, px = ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(x.data_ptr())
    assert lib.bm_sketch(po, 4, px, 0, 4, 4, px, s) == 1
    assert lib.bm_sketch(po, 3, px, 4, 4, 4, px, s) == 1
    assert lib.bm_sketch(None, 4, px, 4, 4, 4, px, s) == 1
    with pytest.raises(ValueError):
        bm.bm_sketch(o, torch.zeros((4, 3), dtype=torch.complex128, device="cuda"))
