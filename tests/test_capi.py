"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/bmhss.h declares, and rejects bad arguments on the host (BM_EINVAL)
before any device work is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import scatterers as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmhss.h")
LIB = os.path.join(ROOT, "paper_2607_00790_amd", "libbmhss.so")

BM_EINVAL = 1


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libbmhss.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("bm_geom_create", "bm_problem_create", "bm_assemble_dense", "bm_assemble_block",
                     "bm_assemble_proxy", "bm_rhs_plane_wave", "bm_far_field", "bm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _geom_create(lib, sizes, xyd):
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.bm_geom_create.argtypes = [ctypes.c_int, ctypes.POINTER(i64), vp, ctypes.c_int, vp,
                                   ctypes.POINTER(vp)]
    lib.bm_last_error.restype = ctypes.c_char_p
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    xyd = np.ascontiguousarray(xyd, dtype=np.float64)
    out = vp()
    code = lib.bm_geom_create(len(sizes), sizes.ctypes.data_as(ctypes.POINTER(i64)),
                              xyd.ctypes.data, 0, None, ctypes.byref(out))
    return code, lib.bm_last_error().decode(), out


def test_geom_create_rejects_too_few_nodes(lib):
    xyd, s = sc.sample_curves([sc.circle()], [6])
    code, msg, out = _geom_create(lib, s, xyd)
    assert code == BM_EINVAL and "8 nodes" in msg and not out.value


def test_geom_create_rejects_non_finite(lib):
    xyd, s = sc.sample_curves([sc.circle()], [16])
    xyd[0, 3] = np.nan
    code, msg, _ = _geom_create(lib, s, xyd)
    assert code == BM_EINVAL and "non-finite" in msg


def test_geom_create_rejects_clockwise_curve(lib):
    xyd, s = sc.sample_curves([sc.circle(), sc.star(0.3, 5, 1.0, (4, 0))], [16, 32])
    # reverse the orientation of the second curve: t -> -t flips x' and keeps x''
    xyd[:, 16:] = xyd[:, 16:][:, ::-1]
    xyd[2:4, 16:] *= -1
    code, msg, _ = _geom_create(lib, s, xyd)
    assert code == BM_EINVAL and "curve 1" in msg and "counter-clockwise" in msg


def test_problem_create_rejects_bad_media(lib):
    vp = ctypes.c_void_p

    class Media(ctypes.Structure):
        _fields_ = [("k0", ctypes.c_double), ("k1", ctypes.c_double), ("eps0", ctypes.c_double),
                    ("eps1", ctypes.c_double)]

    lib.bm_problem_create.argtypes = [vp, ctypes.POINTER(Media), ctypes.POINTER(vp)]
    out = vp()
    m = Media(-1.0, 15.0, 1.0, 2.25)
    assert lib.bm_problem_create(vp(1), ctypes.byref(m), ctypes.byref(out)) == BM_EINVAL
    assert lib.bm_problem_create(None, ctypes.byref(m), ctypes.byref(out)) == BM_EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2607_00790_amd._binding as b
    monkeypatch.setattr(b, "_LIB", None)
    monkeypatch.setattr(b, "lib_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        b.load()


def test_new_entry_points_reject_bad_arguments_on_the_host(lib):
    """The adjoint and Fourier entry points validate on the host (no GPU needed)."""
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.bm_fourier_curve.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64, vp,
                                     vp]
    lib.bm_fourier_chain.argtypes = [vp, i64, ctypes.c_int, ctypes.c_double, vp, vp]
    lib.bm_shape_derivative.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    lib.bm_hss_solve_graph.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp]
    lib.bm_hss_solve_transpose.argtypes = [vp, vp, vp, i64, vp]
    lib.bm_far_field_weights.argtypes = [vp, ctypes.c_double, vp, vp]
    dummy = ctypes.c_void_p(16)   # never dereferenced: every call below fails validation first
    assert lib.bm_fourier_curve(dummy, -1, 1.0, 0.0, 0.0, 64, dummy, None) == BM_EINVAL
    assert lib.bm_fourier_curve(dummy, 4, 0.0, 0.0, 0.0, 64, dummy, None) == BM_EINVAL
    assert lib.bm_fourier_curve(dummy, 4, 1.0, 0.0, 0.0, 0, dummy, None) == BM_EINVAL
    assert lib.bm_fourier_curve(None, 4, 1.0, 0.0, 0.0, 64, dummy, None) == BM_EINVAL
    assert lib.bm_fourier_chain(dummy, 64, 0, 1.0, dummy, None) == BM_EINVAL
    assert lib.bm_fourier_chain(None, 64, 4, 1.0, dummy, None) == BM_EINVAL
    assert lib.bm_shape_derivative(None, dummy, dummy, 0.0, 3.0, None, dummy, None) == BM_EINVAL
    assert lib.bm_hss_solve_graph(None, dummy, dummy, 1, 0, None) == BM_EINVAL
    assert lib.bm_hss_solve_transpose(None, dummy, dummy, 1, None) == BM_EINVAL
    assert lib.bm_far_field_weights(None, 0.0, dummy, None) == BM_EINVAL


def test_autotuner_writes_the_fastest_candidate(tmp_path, monkeypatch):
    """The autotuner's selection and header writing, with a stand-in for the GPU timing."""
    import importlib
    at = importlib.import_module("paper_2607_00790_amd.autotune")
    times = {(64, 1e8): 25.0}
    seen = set()

    def fake_measure(b, f, steps, sketch, ratio):
        seen.add((sketch, ratio))
        return times.get((b, f), 26.0 + b / 1000 + f / 1e10)

    # stage 1: (median ms, sketch, ratio, residual, root); the fastest pair (sketch 32,
    # ratio 0.5) has a residual above plain CPQR's and must not be chosen
    stage1 = [(30.0, 0, 0.0, 2e-7, 900), (20.0, 8, 0.6, 1e-8, 1500), (18.0, 32, 0.5, 5e-7, 7000),
              (22.0, 0, 0.6, 7e-9, 1550)]
    monkeypatch.setattr(at, "stage1", lambda builds: stage1)
    monkeypatch.setattr(at, "measure", fake_measure)
    out = tmp_path / "tuned.h"
    monkeypatch.setattr("sys.argv", ["autotune", "--out", str(out), "--repeats", "1"])
    assert at.main() == 0
    text = out.read_text()
    assert "constexpr int kInvBase = 64;" in text
    assert "constexpr double kBlasFlops = 1e+08;" in text
    assert "constexpr long kSketchRows = 8;" in text
    assert "constexpr double kStopRankRatio = 0.6;" in text
    assert seen == {(8, 0.6)}                 # stage 2 runs with the chosen options
    assert "(residual above plain CPQR: excluded)" in text
    assert text.count("median") == 9 + 4 + 2     # one line per candidate, plus the descriptions
    # the committed header parses the same way
    committed = open(os.path.join(ROOT, "paper_2607_00790_amd", "csrc", "tuned_params.h")).read()
    assert re.search(r"constexpr int kInvBase = (32|64|128);", committed)
    assert re.search(r"constexpr long kSketchRows = \d+;", committed)
    assert re.search(r"constexpr double kStopRankRatio = (0|0?\.\d+|1)(\.\d*)?;", committed)


def test_interp_decomp_rejects_bad_arguments_on_the_host(lib):
    """bm_interp_decomp checks its sizes and pointers before any device work:
    an empty batch, a zero size, a size above 4096, tol outside [0, 1) and a
    null pointer are BM_EINVAL (the pointers passed are never dereferenced)."""
    vp = ctypes.c_void_p
    f = lib.bm_interp_decomp
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp]
    lib.bm_last_error.restype = ctypes.c_char_p
    m = np.array([4, 3], dtype=np.int32)
    n = np.array([2, 5], dtype=np.int32)
    ranks = np.zeros(2, dtype=np.int32)
    fake = vp(0x1000)   # a device address stand-in: rejected before use

    def call(nb=2, mm=m, nn=n, x=fake, tol=1e-10, r=ranks, p=fake, t=fake):
        return f(nb, mm.ctypes.data if mm is not None else None, nn.ctypes.data if nn is not None else None,
                 x, tol, r.ctypes.data if r is not None else None, p, t, None)

    assert call(nb=0) == BM_EINVAL
    assert call(nb=70000) == BM_EINVAL
    assert call(mm=np.array([4, 0], dtype=np.int32)) == BM_EINVAL
    assert call(nn=np.array([2, 4097], dtype=np.int32)) == BM_EINVAL
    assert call(tol=1.0) == BM_EINVAL
    assert call(tol=-1e-3) == BM_EINVAL
    assert call(tol=float("nan")) == BM_EINVAL
    assert call(x=None) == BM_EINVAL
    assert call(r=None) == BM_EINVAL
    assert call(mm=None) == BM_EINVAL
    assert b"bm_interp_decomp" in lib.bm_last_error()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 ends with status 2 and says
    why, before anything touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
