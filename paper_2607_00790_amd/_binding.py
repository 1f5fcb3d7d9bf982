"""ctypes marshalling for libbmhss.so (include/bmhss.h).  No arithmetic here."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p


class BmError(RuntimeError):
    """A non-zero status from the library, with bm_last_error()'s message."""

    def __init__(self, code, msg):
        super().__init__(f"bmhss error {code}: {msg}")
        self.code = code


class _Media(ctypes.Structure):
    _fields_ = [("k0", c_dbl), ("k1", c_dbl), ("eps0", c_dbl), ("eps1", c_dbl)]


class _HssOpts(ctypes.Structure):
    _fields_ = [("leaf", c_i64), ("proxy_ratio", c_dbl), ("proxy_points", c_i64),
                ("id_tol", c_dbl), ("sketch", c_i64), ("proxy_adapt", c_i64), ("max_rank_ratio", c_dbl),
                ("kernel_timing", c_i64), ("proxy_fp32", c_i64)]


class _HssStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("compressed_levels", ctypes.c_int32),
                ("root_size", ctypes.c_int32), ("guard_stops", ctypes.c_int32),
                ("max_rank", c_i64), ("entries", c_i64), ("pairs", c_i64),
                ("seconds_generate", c_dbl), ("seconds_compress", c_dbl),
                ("seconds_factor", c_dbl), ("seconds_total", c_dbl),
                ("cpqr_launches", c_i64), ("cpqr_bytes", c_dbl), ("seconds_cpqr", c_dbl),
                ("sketch", c_i64), ("max_rank_ratio", c_dbl),
                ("cpqr_fused_launches", c_i64), ("cpqr_fused_bytes", c_dbl), ("seconds_cpqr_fused", c_dbl),
                ("gemm_launches", c_i64), ("gemm_flops", c_dbl), ("seconds_gemm", c_dbl),
                ("inv_launches", c_i64), ("inv_flops", c_dbl), ("seconds_inv", c_dbl),
                ("sketch_launches", c_i64), ("sketch_flops", c_dbl), ("seconds_sketch", c_dbl),
                ("gen_launches", c_i64), ("gen_pairs", c_dbl), ("seconds_gen", c_dbl)]


class _HssLevel(ctypes.Structure):
    _fields_ = [("boxes", ctypes.c_int32), ("max_unknowns", ctypes.c_int32),
                ("max_rows", ctypes.c_int32), ("id_rows", ctypes.c_int32),
                ("min_rank", ctypes.c_int32), ("max_rank", ctypes.c_int32)]


def lib_path() -> str:
    return os.path.join(_HERE, "libbmhss.so")


def load():
    """Load libbmhss.so (built in-tree by paper_2607_00790_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2607_00790_amd.build`")
    lib = ctypes.CDLL(path)
    sig = {
        "bm_last_error": (ctypes.c_char_p, []),
        "bm_geom_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(c_i64), c_vp, ctypes.c_int,
                                          c_vp, ctypes.POINTER(c_vp)]),
        "bm_geom_destroy": (ctypes.c_int, [c_vp]),
        "bm_geom_size": (c_i64, [c_vp]),
        "bm_geom_nodes": (ctypes.c_int, [c_vp, c_vp, c_vp]),
        "bm_problem_create": (ctypes.c_int, [c_vp, ctypes.POINTER(_Media), ctypes.POINTER(c_vp)]),
        "bm_problem_destroy": (ctypes.c_int, [c_vp]),
        "bm_problem_create_bodies": (ctypes.c_int, [c_vp, ctypes.c_int, c_vp, c_vp, ctypes.POINTER(c_vp)]),
        "bm_rhs_plane_wave": (ctypes.c_int, [c_vp, c_dbl, c_vp, c_vp]),
        "bm_assemble_dense": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp]),
        "bm_rhs_incident": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
        "bm_assemble_block": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, ctypes.c_int, c_vp]),
        "bm_assemble_proxy": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, ctypes.c_int, c_vp,
                                             c_i64, ctypes.c_int, c_vp]),
        "bm_matvec": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp]),
        "bm_matvec_noalloc": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp]),
        "bm_far_field": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp]),
    }
    sig.update({
        "bm_hss_build": (ctypes.c_int, [c_vp, ctypes.POINTER(_HssOpts), c_vp, ctypes.POINTER(c_vp)]),
        "bm_hss_solve": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp]),
        "bm_hss_solve_transpose": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp]),
        "bm_hss_solve_graph": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, ctypes.c_int, c_vp]),
        "bm_far_field_weights": (ctypes.c_int, [c_vp, c_dbl, c_vp, c_vp]),
        "bm_shape_derivative": (ctypes.c_int, [c_vp, c_vp, c_vp, c_dbl, c_dbl, c_vp, c_vp, c_vp]),
        "bm_fourier_curve": (ctypes.c_int, [c_vp, ctypes.c_int, c_dbl, c_dbl, c_dbl, c_i64, c_vp, c_vp]),
        "bm_fourier_chain": (ctypes.c_int, [c_vp, c_i64, ctypes.c_int, c_dbl, c_vp, c_vp]),
        "bm_hss_stats": (ctypes.c_int, [c_vp, ctypes.POINTER(_HssStats)]),
        "bm_hss_level": (ctypes.c_int, [c_vp, ctypes.c_int, ctypes.POINTER(_HssLevel)]),
        "bm_hss_destroy": (ctypes.c_int, [c_vp]),
        "bm_dense_inverse": (ctypes.c_int, [c_vp, c_i64, c_i64, c_vp]),
        "bm_sketch": (ctypes.c_int, [c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_vp, c_vp]),
        "bm_interp_decomp": (ctypes.c_int, [ctypes.c_int32, c_vp, c_vp, c_vp, c_dbl, c_vp, c_vp, c_vp, c_vp]),
    })
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _check(code):
    if code != 0:
        raise BmError(code, _LIB.bm_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_vp(s.cuda_stream)


def _dev_ptr(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return c_vp(t.data_ptr())


class Geometry:
    """Handle of a discretised boundary (bm_geom)."""

    def __init__(self, handle, sizes):
        self._h = handle
        self.sizes = list(sizes)

    @property
    def n(self) -> int:
        return int(_LIB.bm_geom_size(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.bm_geom_destroy(self._h)
            self._h = None


class Problem:
    """Handle of a geometry + media (bm_problem); keeps its geometry alive."""

    def __init__(self, handle, geom, media, nbodies=1):
        self._h = handle
        self.geom = geom
        self.media = media
        self.nbodies = nbodies

    @property
    def n(self) -> int:
        return self.geom.n

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.bm_problem_destroy(self._h)
            self._h = None


class HSS:
    """Handle of a built HSS factorisation (bm_hss); keeps its problem alive."""

    def __init__(self, handle, prob):
        self._h = handle
        self.prob = prob

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.bm_hss_destroy(self._h)
            self._h = None


def bm_geom_create(n_per_curve, xyd, stream=None) -> Geometry:
    """xyd: (6, N) float64, host numpy array or device tensor (see bmhss.h)."""
    load()
    sizes = np.ascontiguousarray(np.asarray(n_per_curve, dtype=np.int64))
    torch = _torch()
    out = c_vp()
    if isinstance(xyd, torch.Tensor) and xyd.is_cuda:
        ptr, on_dev = _dev_ptr(xyd, torch.float64, "xyd"), 1
        keep = xyd
        if tuple(xyd.shape) != (6, int(sizes.sum())):
            raise ValueError("xyd must have shape (6, sum(n_per_curve))")
    else:
        keep = np.ascontiguousarray(np.asarray(xyd, dtype=np.float64))
        if keep.shape != (6, int(sizes.sum())):
            raise ValueError("xyd must have shape (6, sum(n_per_curve))")
        ptr, on_dev = c_vp(keep.ctypes.data), 0
    _check(load().bm_geom_create(len(sizes), sizes.ctypes.data_as(ctypes.POINTER(c_i64)), ptr, on_dev,
                               _stream(stream), ctypes.byref(out)))
    del keep
    return Geometry(out, sizes)


def bm_geom_size(g: Geometry) -> int:
    return g.n


def bm_geom_nodes(g: Geometry, stream=None):
    """(6, N) float64 device tensor: x, y, nx, ny, w, kappa."""
    torch = _torch()
    out = torch.empty((6, g.n), dtype=torch.float64, device="cuda")
    _check(load().bm_geom_nodes(g._h, _dev_ptr(out), _stream(stream)))
    return out


def bm_problem_create(g: Geometry, k0, k1, eps0, eps1) -> Problem:
    load()
    m = _Media(float(k0), float(k1), float(eps0), float(eps1))
    out = c_vp()
    _check(load().bm_problem_create(g._h, ctypes.byref(m), ctypes.byref(out)))
    return Problem(out, g, (float(k0), float(k1), float(eps0), float(eps1)))


def bm_problem_create_bodies(g: Geometry, body_of_curve, media) -> Problem:
    """Independent bodies: body_of_curve[c] = body of curve c (0, .., 0, 1, ..);
    media = one (k0, k1, eps0, eps1) per body."""
    load()
    boc = (ctypes.c_int32 * len(body_of_curve))(*[int(b) for b in body_of_curve])
    nb = len(media)
    arr = (_Media * nb)(*[_Media(*(float(v) for v in m)) for m in media])
    out = c_vp()
    _check(load().bm_problem_create_bodies(g._h, nb, boc, arr, ctypes.byref(out)))
    return Problem(out, g, [tuple(float(v) for v in m) for m in media], nbodies=nb)


def bm_rhs_plane_wave(p: Problem, angle: float, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(2 * p.n, dtype=torch.complex128, device="cuda")
    _check(load().bm_rhs_plane_wave(p._h, float(angle), _dev_ptr(out, torch.complex128, "out"),
                                  _stream(stream)))
    return out


def bm_rhs_incident(p: Problem, uin, dn_uin, out=None, stream=None):
    """Right-hand side of Eq. (3) from u_in and du_in/dn at the nodes
    (each an N-vector, complex128 device tensor)."""
    torch = _torch()
    if uin.numel() != p.n or dn_uin.numel() != p.n:
        raise ValueError("uin and dn_uin need one value per node")
    if out is None:
        out = torch.empty(2 * p.n, dtype=torch.complex128, device="cuda")
    _check(load().bm_rhs_incident(p._h, _dev_ptr(uin, torch.complex128, "uin"),
                                  _dev_ptr(dn_uin, torch.complex128, "dn_uin"),
                                  _dev_ptr(out, torch.complex128, "out"), _stream(stream)))
    return out


def bm_assemble_dense(p: Problem, out=None, stream=None):
    torch = _torch()
    n2 = 2 * p.n
    if out is None:
        out = torch.empty((n2, n2), dtype=torch.complex128, device="cuda")
    if out.dim() != 2 or out.shape[0] != n2 or out.shape[1] < n2:
        raise ValueError("out must be (2N, >=2N)")
    _check(load().bm_assemble_dense(p._h, _dev_ptr(out, torch.complex128, "out"), out.stride(0),
                                  _stream(stream)))
    return out


def bm_assemble_block(p: Problem, rows, cols, out=None, prec=0, stream=None):
    """prec 0: FP64 entries; 1: FP32 arithmetic (stored as complex128)."""
    torch = _torch()
    rows = rows.to(device="cuda", dtype=torch.int64).contiguous()
    cols = cols.to(device="cuda", dtype=torch.int64).contiguous()
    nr, nc = rows.numel(), cols.numel()
    if out is None:
        out = torch.empty((2 * nr, 2 * nc), dtype=torch.complex128, device="cuda")
    _check(load().bm_assemble_block(p._h, _dev_ptr(rows), nr, _dev_ptr(cols), nc,
                                  _dev_ptr(out, torch.complex128, "out"), out.stride(0), int(prec),
                                  _stream(stream)))
    return out


def bm_assemble_proxy(p: Problem, nodes, pts, direction: int, out=None, prec=0, stream=None):
    """pts: (5, P) float64 device tensor (x, y, nx, ny, w); prec as in bm_assemble_block."""
    torch = _torch()
    nodes = nodes.to(device="cuda", dtype=torch.int64).contiguous()
    n, P = nodes.numel(), pts.shape[1]
    shape = (2 * n, 2 * P) if direction == 0 else (2 * P, 2 * n)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
    _check(load().bm_assemble_proxy(p._h, _dev_ptr(nodes), n, _dev_ptr(pts, torch.float64, "pts"), P,
                                  int(direction), _dev_ptr(out, torch.complex128, "out"),
                                  out.stride(0), int(prec), _stream(stream)))
    return out


def bm_matvec(p: Problem, x, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(2 * p.n, dtype=torch.complex128, device="cuda")
    _check(load().bm_matvec(p._h, _dev_ptr(x, torch.complex128, "x"),
                          _dev_ptr(out, torch.complex128, "out"), _stream(stream)))
    return out


def bm_matvec_noalloc(p: Problem, x, out, stream=None):
    """bm_matvec through the library's fixed device buffer (no allocation);
    `out` must be given (2N complex128 device tensor)."""
    torch = _torch()
    _check(load().bm_matvec_noalloc(p._h, _dev_ptr(x, torch.complex128, "x"),
                                    _dev_ptr(out, torch.complex128, "out"), _stream(stream)))
    return out


def bm_dense_inverse(a, stream=None):
    """In-place inverse of a square complex128 device matrix (row-major,
    contiguous); returns a."""
    torch = _torch()
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be a square matrix")
    _check(load().bm_dense_inverse(_dev_ptr(a, torch.complex128, "a"), a.shape[0], a.shape[0], _stream(stream)))
    return a


def bm_sketch(omega, x, out=None, stream=None):
    """Y = omega @ x for a real (l, m) float64 device matrix omega (row-major)
    and a complex (m, n) matrix x stored by columns: pass x as the (n, m)
    complex128 tensor x^T (contiguous), and receive Y^T as an (n, l) tensor."""
    torch = _torch()
    if omega.dim() != 2 or x.dim() != 2 or omega.shape[1] != x.shape[1]:
        raise ValueError("omega must be (l, m) and x^T (n, m)")
    l, m = omega.shape
    n = x.shape[0]
    if out is None:
        out = torch.empty((n, l), dtype=torch.complex128, device="cuda")
    _check(load().bm_sketch(_dev_ptr(omega, torch.float64, "omega"), m, _dev_ptr(x, torch.complex128, "x"), m, n, l,
                            _dev_ptr(out, torch.complex128, "out"), _stream(stream)))
    return out


def bm_interp_decomp(mats, tol, stream=None):
    """Interpolative decomposition of a batch of complex matrices. mats: a list
    of (m_b, n_b) complex128 device tensors (not modified). Returns
    (ranks, perms, Ts): per matrix its rank k, the pivot order (n,) int32
    device tensor, and the (n, k) interpolation matrix T with
    mats[b] ~= mats[b][:, perm[:k]] @ T.T."""
    import numpy as np
    torch = _torch()
    if not mats:
        raise ValueError("mats must not be empty")
    ms = np.array([a.shape[0] for a in mats], dtype=np.int32)
    ns = np.array([a.shape[1] for a in mats], dtype=np.int32)
    for a in mats:
        if a.dim() != 2 or a.dtype != torch.complex128 or not a.is_cuda:
            raise ValueError("every matrix must be a 2-D complex128 device tensor")
    # stored by columns: the transposes, packed
    x = torch.cat([a.t().contiguous().reshape(-1) for a in mats])
    perm = torch.empty(int(ns.sum()), dtype=torch.int32, device="cuda")
    T = torch.empty(int((ns.astype(np.int64) ** 2).sum()), dtype=torch.complex128, device="cuda")
    ranks = np.zeros(len(mats), dtype=np.int32)
    _check(load().bm_interp_decomp(len(mats), ms.ctypes.data, ns.ctypes.data, _dev_ptr(x, torch.complex128, "x"),
                                   float(tol), ranks.ctypes.data, _dev_ptr(perm, torch.int32, "perm"),
                                   _dev_ptr(T, torch.complex128, "T"), _stream(stream)))
    perms, Ts = [], []
    po = to = 0
    for b in range(len(mats)):
        nb, kb = int(ns[b]), int(ranks[b])
        perms.append(perm[po:po + nb])
        Ts.append(T[to:to + nb * kb].reshape(nb, kb))
        po += nb
        to += nb * nb
    return [int(r) for r in ranks], perms, Ts


def bm_far_field(p: Problem, phi, angles, out=None, stream=None):
    torch = _torch()
    angles = angles.to(device="cuda", dtype=torch.float64).contiguous()
    if out is None:
        out = torch.empty(p.nbodies * angles.numel(), dtype=torch.complex128, device="cuda")
    _check(load().bm_far_field(p._h, _dev_ptr(phi, torch.complex128, "phi"), _dev_ptr(angles),
                             angles.numel(), _dev_ptr(out, torch.complex128, "out"), _stream(stream)))
    return out


def bm_hss_build(p: Problem, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10,
                 sketch=0, proxy_adapt=False, max_rank_ratio=0.0, kernel_timing=False, proxy_fp32=False,
                 stream=None) -> HSS:
    """sketch = p > 0: run the ID on a Gaussian sketch of each box's stacked
    matrix with (unknowns + p) rows, when that is fewer than the matrix has.
    proxy_adapt: max(proxy_points, ceil(2 k R_p) + 32) points per proxy circle.
    max_rank_ratio = r > 0: a body stops compressing once a level keeps more
    than r of its unknowns (its skeletons then form its dense root).
    sketch = -1 or max_rank_ratio = -1: the library's tuned value (the build's
    stats report the values used).  kernel_timing: HIP-event timing of every
    batched GEMM and Gauss-Jordan launch (stats gemm_* and inv_*).  proxy_fp32:
    node x proxy blocks in FP32 arithmetic (everything else FP64)."""
    opts = _HssOpts(int(leaf), float(proxy_ratio), int(proxy_points), float(id_tol), int(sketch),
                    int(bool(proxy_adapt)), float(max_rank_ratio), int(bool(kernel_timing)),
                    int(bool(proxy_fp32)))
    out = c_vp()
    _check(load().bm_hss_build(p._h, ctypes.byref(opts), _stream(stream), ctypes.byref(out)))
    return HSS(out, p)


def bm_hss_solve(h: HSS, b, out=None, stream=None):
    """b: (2N,) or (nrhs, 2N) complex128 device tensor (each right-hand side contiguous)."""
    torch = _torch()
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    if out is None:
        out = torch.empty_like(b)
    _check(load().bm_hss_solve(h._h, _dev_ptr(b, torch.complex128, "b"),
                             _dev_ptr(out, torch.complex128, "out"), nrhs, _stream(stream)))
    return out


def bm_hss_stats(h: HSS) -> dict:
    s = _HssStats()
    _check(load().bm_hss_stats(h._h, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in _HssStats._fields_}


def bm_hss_level(h: HSS, level: int) -> dict:
    """Sizes and ranks of compressed level `level` (0 = leaves)."""
    s = _HssLevel()
    _check(load().bm_hss_level(h._h, int(level), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in _HssLevel._fields_}


def bm_hss_solve_transpose(h: HSS, b, out=None, stream=None):
    """x = A^{-T} b with the factors of bm_hss_build; b as in bm_hss_solve."""
    torch = _torch()
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    if out is None:
        out = torch.empty_like(b)
    _check(load().bm_hss_solve_transpose(h._h, _dev_ptr(b, torch.complex128, "b"),
                                       _dev_ptr(out, torch.complex128, "out"), nrhs, _stream(stream)))
    return out


def bm_hss_solve_graph(h: HSS, b, out=None, transpose=False, stream=None):
    """bm_hss_solve (or its transpose) replayed from a HIP graph captured on the
    first call for this (nrhs, transpose); asynchronous on the stream."""
    torch = _torch()
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    if out is None:
        out = torch.empty_like(b)
    _check(load().bm_hss_solve_graph(h._h, _dev_ptr(b, torch.complex128, "b"),
                                     _dev_ptr(out, torch.complex128, "out"), nrhs, int(bool(transpose)),
                                     _stream(stream)))
    return out


def bm_far_field_weights(p: Problem, angle: float, out=None, stream=None):
    """g (2N complex): body b's far field at `angle` is the sum of g_k phi_k over its unknowns."""
    torch = _torch()
    if out is None:
        out = torch.empty(2 * p.n, dtype=torch.complex128, device="cuda")
    _check(load().bm_far_field_weights(p._h, float(angle), _dev_ptr(out, torch.complex128, "out"),
                                     _stream(stream)))
    return out


def bm_shape_derivative(p: Problem, phi, lam, inc_angle: float, obs_angle: float, coef=None, out=None,
                        stream=None):
    """(6, N) float64: Re(coef_b dL_b/d samples), L_b = g_b.phi + lam.(rhs - A phi);
    coef None: coef_b = 2 conj(u_inf,b(obs_angle)), the gradient of sum_b |u_inf,b|^2."""
    torch = _torch()
    if out is None:
        out = torch.empty((6, p.n), dtype=torch.float64, device="cuda")
    cptr = c_vp(None) if coef is None else _dev_ptr(coef, torch.complex128, "coef")
    if coef is not None and coef.numel() != p.nbodies:
        raise ValueError("coef needs one complex value per body")
    _check(load().bm_shape_derivative(p._h, _dev_ptr(phi, torch.complex128, "phi"),
                                    _dev_ptr(lam, torch.complex128, "lam"), float(inc_angle),
                                    float(obs_angle), cptr, _dev_ptr(out, torch.float64, "out"),
                                    _stream(stream)))
    return out


def bm_fourier_curve(coef, n: int, radius: float = 1.0, center=(0.0, 0.0), out=None, stream=None):
    """(6, n) float64 samples of r(t) = 1 + sum_j (a_j cos jt + b_j sin jt);
    coef: device float64 (a_1..a_M, b_1..b_M)."""
    torch = _torch()
    M = coef.numel() // 2
    if coef.numel() != 2 * M:
        raise ValueError("coef must hold a_1..a_M, b_1..b_M")
    if out is None:
        out = torch.empty((6, int(n)), dtype=torch.float64, device="cuda")
    cptr = _dev_ptr(coef, torch.float64, "coef") if M > 0 else c_vp(None)
    _check(load().bm_fourier_curve(cptr, M, float(radius), float(center[0]), float(center[1]), int(n),
                                 _dev_ptr(out, torch.float64, "out"), _stream(stream)))
    return out


def bm_fourier_chain(grad, nmodes: int, radius: float = 1.0, out=None, stream=None):
    """(2 nmodes,) float64: a (6, n) sample gradient turned into d/d(a_1..a_M, b_1..b_M)."""
    torch = _torch()
    if out is None:
        out = torch.empty(2 * int(nmodes), dtype=torch.float64, device="cuda")
    n = grad.shape[-1]
    _check(load().bm_fourier_chain(_dev_ptr(grad, torch.float64, "grad"), int(n), int(nmodes), float(radius),
                                 _dev_ptr(out, torch.float64, "out"), _stream(stream)))
    return out
