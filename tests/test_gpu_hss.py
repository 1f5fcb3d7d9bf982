"""GPU tests of the proxy-surface HSS direct solver (build + solve through the
C-ABI) against the oracle's dense solution.

The HSS solution approximates the dense one to the ID tolerance times a modest
growth factor; with id_tol = 1e-10 the bar here is 1e-7 relative (2-norm).
On the circle the solution must also keep the dense solver's accuracy against
the Mie series (within 2x of the oracle's error)."""
import sys

import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, mie, wsbm

pytestmark = pytest.mark.gpu

HSS_BAR = 1e-7


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def setup(bm, curves, sizes, media):
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create(g, media.k0, media.k1, media.eps0, media.eps1)
    return p, geometry.discretize(xyd, s)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# plain CPQR, a Gaussian sketch with 128 extra rows, and the library's tuned
# options (sketch -1 with stop ratio -1): small sketches put every box of the
# lower levels in the whole-box CPQR kernel
SKETCH = [pytest.param(0, id="cpqr"), pytest.param(128, id="sketch128"), pytest.param(-1, id="tuned")]


# (sketch, stop ratio, adaptive proxy counts) on the benchmark workload:
# plain CPQR on every level and the sketch with 128 extra rows, each with the
# configuration's 64 points on every proxy circle and with adaptive counts
# max(64, ceil(2 k1 R_p) + 32), and the library's tuned options (sketch 8, stop
# ratio 0.6, 64 points).  With 64 points the top two levels' boxes, several
# interior wavelengths wide, are under-resolved: their IDs leave ~2.6e-7
# (still 18x below the discretisation error); adaptive counts, or stopping
# before those levels, bring the error under 1e-7.
GOLDEN_CASES = [pytest.param(0, 0.0, False, id="cpqr_p64"), pytest.param(0, 0.0, True, id="cpqr_adapt"),
                pytest.param(128, 0.0, False, id="sketch128_p64"), pytest.param(128, 0.0, True, id="sketch128_adapt"),
                pytest.param(-1, -1.0, False, id="tuned")]


def _star_bar(ratio, adapt):
    """The HSS bar: 1e-7, except for compression of every level with 64 fixed
    proxy points, which must stay an order below the discretisation error."""
    return HSS_BAR if (adapt or ratio != 0.0) else 5e-7


def ratio_for(sketch):
    return -1.0 if sketch == -1 else 0.0


def check_fused(bm, h, sketch):
    st = bm.bm_hss_stats(h)
    if sketch == -1:
        assert st["cpqr_fused_launches"] >= 1 and st["seconds_cpqr_fused"] > 0
    elif sketch == 0:
        assert st["cpqr_fused_launches"] == 0


@pytest.mark.parametrize("sketch", SKETCH)
def test_hss_circle_plain_workload(gpu_lib, sketch):
    import torch
    bm = gpu_lib
    note(f"hss: circle N=512, k0=10, n=1.5, leaf 64, sketch={sketch}")
    wl = sc.circle_workload(512)
    p, nd = setup(bm, wl.curves, wl.sizes, wl.media)
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=sketch,
                        max_rank_ratio=ratio_for(sketch))
    st = bm.bm_hss_stats(h)
    note(f"  stats {st}")
    assert st["compressed_levels"] >= 1
    check_fused(bm, h, sketch)
    b = bm.bm_rhs_plane_wave(p, 0.0)
    x = bm.bm_hss_solve(h, b).cpu().numpy()
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, wl.media), wsbm.rhs_plane_wave(nd, wl.media, 0.0))
    assert rel(x, ref) < HSS_BAR
    t = 2 * np.pi * np.arange(512) / 512
    u, _ = mie.boundary_values(wl.media, t)
    e_hss = np.linalg.norm(x[0::2].real - u.real) / np.linalg.norm(u.real)
    e_ora = np.linalg.norm(ref[0::2].real - u.real) / np.linalg.norm(u.real)
    assert e_hss <= 2 * e_ora


@pytest.mark.parametrize("sketch", SKETCH)
def test_hss_star_multiple_rhs_in_place(gpu_lib, sketch):
    import torch
    bm = gpu_lib
    note(f"hss: star N=2048, k0=50, n=1.5, 3 right-hand sides, x aliases b, sketch={sketch}")
    media = sc.media_from_index(50.0, 1.5)
    p, nd = setup(bm, [sc.star(0.3, 5)], [2048], media)
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=sketch,
                        max_rank_ratio=ratio_for(sketch))
    note(f"  stats {bm.bm_hss_stats(h)}")
    check_fused(bm, h, sketch)
    angles = [0.0, 1.1, 4.0]
    B = torch.stack([bm.bm_rhs_plane_wave(p, a) for a in angles]).contiguous()
    Bh = B.cpu().numpy()
    bm.bm_hss_solve(h, B, out=B)
    X = B.cpu().numpy()
    A = wsbm.assemble_dense(nd, media)
    for r, a in enumerate(angles):
        ref = wsbm.solve_dense(A, wsbm.rhs_plane_wave(nd, media, a))
        assert np.abs(Bh[r] - wsbm.rhs_plane_wave(nd, media, a)).max() < 1e-12
        assert rel(X[r], ref) < HSS_BAR, (r, rel(X[r], ref))


@pytest.mark.parametrize("sketch", SKETCH)
def test_hss_two_scatterers_ragged_sizes(gpu_lib, sketch):
    bm = gpu_lib
    note(f"hss: two stars N=601+423, k0=20, n=2, sketch={sketch}")
    media = sc.media_from_index(20.0, 2.0)
    p, nd = setup(bm, [sc.star(0.2, 4), sc.star(0.25, 3, 1.0, (3.0, 0.5))], [601, 423], media)
    h = bm.bm_hss_build(p, leaf=40, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=sketch,
                        max_rank_ratio=ratio_for(sketch))
    note(f"  stats {bm.bm_hss_stats(h)}")
    check_fused(bm, h, sketch)
    b = bm.bm_rhs_plane_wave(p, 0.3)
    x = bm.bm_hss_solve(h, b).cpu().numpy()
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_plane_wave(nd, media, 0.3))
    assert rel(x, ref) < HSS_BAR


def test_hss_tiny_problem_is_a_dense_solve(gpu_lib):
    """N below two leaves: no level is compressed, the root is the whole system."""
    bm = gpu_lib
    note("hss: tiny N=40 (root only)")
    media = sc.media_from_index(10.0, 1.5)
    p, nd = setup(bm, [sc.star(0.3, 5)], [40], media)
    h = bm.bm_hss_build(p, leaf=32)
    st = bm.bm_hss_stats(h)
    assert st["compressed_levels"] == 0 and st["root_size"] == 80
    x = bm.bm_hss_solve(h, bm.bm_rhs_plane_wave(p, 0.0)).cpu().numpy()
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_plane_wave(nd, media, 0.0))
    assert rel(x, ref) < 1e-12


@pytest.mark.parametrize("sketch,ratio,adapt", GOLDEN_CASES)
def test_hss_full_size_star_sampled_residual(gpu_lib, sketch, ratio, adapt):
    """Full star workload (N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy points,
    tol 1e-10), the configuration the benchmark times: the residual of the HSS
    solution on 256 sampled rows of the oracle's matrix (below the same bar as
    the solution error), and the per-level sizes.  "tuned" takes the library's
    tuned sketch and stop ratio (value -1), the benchmark's default."""
    bm = gpu_lib
    note(f"hss: star N=16384 (benchmark workload), sampled residual, sketch={sketch}, ratio={ratio}, adapt={adapt}")
    wl = sc.star_workload()
    p, nd = setup(bm, wl.curves, wl.sizes, wl.media)
    h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                        id_tol=wl.id_tol, sketch=sketch, max_rank_ratio=ratio, proxy_adapt=adapt)
    st = bm.bm_hss_stats(h)
    note(f"  stats {st}")
    if sketch == -1:
        assert st["sketch"] >= 0 and 0.0 <= st["max_rank_ratio"] <= 1.0
        sketch = st["sketch"]
    else:
        assert st["sketch"] == sketch and st["max_rank_ratio"] == ratio
    for l in range(st["compressed_levels"]):
        lv = bm.bm_hss_level(h, l)
        note(f"  level {l}: {lv}")
        assert lv["boxes"] == 2 ** (st["levels"] - l)
        assert 0 < lv["min_rank"] <= lv["max_rank"] <= lv["max_unknowns"]
        if sketch:
            assert lv["id_rows"] <= min(lv["max_rows"], lv["max_unknowns"] + sketch)
        else:
            assert lv["id_rows"] == lv["max_rows"]
        assert lv["max_rank"] <= lv["id_rows"]
    with pytest.raises(bm.BmError):
        bm.bm_hss_level(h, st["compressed_levels"])
    b = bm.bm_rhs_plane_wave(p, wl.theta_inc)
    x = bm.bm_hss_solve(h, b).cpu().numpy()
    rows = np.arange(0, wl.n, 64) + 13
    Ar = wsbm.assemble_rows(nd, wl.media, rows)
    br = wsbm.rhs_plane_wave(nd, wl.media, wl.theta_inc).reshape(-1, 2)[rows].reshape(-1)
    res = np.linalg.norm(Ar @ x - br) / np.linalg.norm(br)
    note(f"  sampled relative residual {res:.3e}")
    assert res < _star_bar(ratio, adapt)


def _golden_star16384():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "star16384_dense.json")
    with open(path) as f:
        rec = json.load(f)

    def arr(v):
        a = np.asarray(v)
        return a[:, 0] + 1j * a[:, 1]

    out = {}
    for c in rec["cases"]:
        out[c["n"]] = {"nodes": np.asarray(c["nodes"]), "u": arr(c["u"]), "q": arr(c["q"]),
                       "u_inf": arr(c["u_inf"]), "theta_inc": c["theta_inc"]}
    return out, np.asarray(rec["angles"])


@pytest.mark.parametrize("sketch,ratio,adapt", GOLDEN_CASES)
def test_hss_full_size_star_vs_dense_golden(gpu_lib, sketch, ratio, adapt):
    """The benchmark workload (N = 16384, k0 = 50, n = 1.5, leaf 64, 64 proxy
    points, tol 1e-10) against the oracle's dense LU solution stored in
    tests/golden/star16384_dense.json: u and q at every 16th node and the far
    field at 64 angles, element by element.  The HSS error must stay below
    the bar (1e-7; 5e-7 for every level compressed with 64 fixed proxy points)
    and an order of magnitude below the discretisation error, estimated by the
    change of the dense solution from N = 8192 to N = 16384 (4.8e-6 at the
    O(h^3) rate)."""
    import torch
    bm = gpu_lib
    gold, angles = _golden_star16384()
    g16, g8 = gold[16384], gold[8192]
    disc = np.linalg.norm(g16["u"] - g8["u"]) / np.linalg.norm(g16["u"])
    note(f"hss: star N=16384 vs dense golden, sketch={sketch}, ratio={ratio}, adapt={adapt} "
         f"(discretisation change 8192 -> 16384: {disc:.2e})")
    wl = sc.star_workload()
    assert abs(wl.theta_inc - g16["theta_inc"]) < 1e-15
    xyd, s = wl.xyd()
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create(g, wl.media.k0, wl.media.k1, wl.media.eps0, wl.media.eps1)
    h = bm.bm_hss_build(p, leaf=wl.leaf, proxy_ratio=wl.proxy_ratio, proxy_points=wl.proxy_points,
                        id_tol=wl.id_tol, sketch=sketch, max_rank_ratio=ratio, proxy_adapt=adapt)
    st = bm.bm_hss_stats(h)
    x = bm.bm_hss_solve(h, bm.bm_rhs_plane_wave(p, wl.theta_inc))
    ff = bm.bm_far_field(p, x, torch.from_numpy(angles)).cpu().numpy()
    x = x.cpu().numpy()
    idx = g16["nodes"]
    errs = {"u": rel(x[2 * idx], g16["u"]), "q": rel(x[2 * idx + 1], g16["q"]), "u_inf": rel(ff, g16["u_inf"])}
    emax = {"u": np.abs(x[2 * idx] - g16["u"]).max() / np.abs(g16["u"]).max(),
            "q": np.abs(x[2 * idx + 1] - g16["q"]).max() / np.abs(g16["q"]).max()}
    note(f"  levels {st['compressed_levels']}, root {st['root_size']}; relative errors {errs}, max-norm {emax}")
    bar = _star_bar(ratio, adapt)
    for k, v in errs.items():
        assert v < bar, (k, v)
        assert v < disc / 10, (k, v, disc)
    for k, v in emax.items():
        assert v < bar, (k, v)


def test_hss_point_source_circle_vs_mie(gpu_lib):
    """An incident field other than a plane wave, through bm_rhs_incident: a
    point source at distance 3 from the circle of the plain dense workload
    (k0 = 10, n = 1.5, N = 512).  The HSS solution matches the oracle's dense
    solution to the HSS bar and the separation-of-variables solution within 2x
    of the oracle's own error."""
    import torch
    bm = gpu_lib
    note("hss: circle N=512, point-source incidence, vs dense oracle and Mie")
    wl = sc.circle_workload(512)
    p, nd = setup(bm, wl.curves, wl.sizes, wl.media)
    rho, th = 3.0, 0.8
    uin, dn = wsbm.point_source_field(nd, wl.media.k0, (rho * np.cos(th), rho * np.sin(th)))
    b = bm.bm_rhs_incident(p, torch.from_numpy(uin).cuda(), torch.from_numpy(dn).cuda())
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10)
    x = bm.bm_hss_solve(h, b).cpu().numpy()
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, wl.media), wsbm.rhs_incident(nd, wl.media, uin, dn))
    assert rel(x, ref) < HSS_BAR
    u, q = mie.boundary_values(wl.media, 2 * np.pi * np.arange(512) / 512, theta_inc=th, src=rho)
    e_hss, e_ora = rel(x[0::2], u), rel(ref[0::2], u)
    note(f"  error vs Mie: HSS {e_hss:.2e}, oracle {e_ora:.2e}")
    assert e_hss <= 2 * e_ora


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10])
def test_hss_fp32_proxies_error_vs_oracle(gpu_lib, tol):
    """FP32 proxy blocks (opts.proxy_fp32; near, skeleton, diagonal blocks and
    the factors stay FP64) against the oracle's dense solution, reported beside
    the all-FP64 build at the same tolerance, on the plain dense workload's
    circle (N = 512, k0 = 10) and a star (N = 2048, k0 = 50).  At tolerance
    1e-6 the FP32 proxies must keep the FP64 build's accuracy (within a factor
    5, or 5 tol).  Below it their rounding noise (~1e-7 of each entry) reaches
    the tolerance and the IDs keep more skeletons (the leaves are not
    compressed at 1e-8).  At 1e-8 the error is bounded by 5 times the FP64
    build's or ten times that noise level (1e-6), whichever is larger.  At
    1e-10 the IDs of the upper levels fit the noise (their interpolation
    matrices amplify it): the error, up to ~1e-5, is reported and bounded by
    1e-4 -- FP32 proxies are for tolerances at or above their noise."""
    bm = gpu_lib
    for name, curves, sizes, media in (("circle512", [sc.circle()], [512], sc.media_from_index(10.0, 1.5)),
                                       ("star2048", [sc.star(0.3, 5)], [2048], sc.media_from_index(50.0, 1.5))):
        p, nd = setup(bm, curves, sizes, media)
        ref = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_plane_wave(nd, media, 0.3))
        b = bm.bm_rhs_plane_wave(p, 0.3)
        res = {}
        for fp32 in (False, True):
            h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=tol, proxy_fp32=fp32)
            st = bm.bm_hss_stats(h)
            x = bm.bm_hss_solve(h, b).cpu().numpy()
            lv0 = bm.bm_hss_level(h, 0) if st["compressed_levels"] > 0 else {"max_rank": -1}
            res[fp32] = (rel(x, ref), lv0["max_rank"], st["root_size"])
        note(f"  {name} tol {tol:g}: FP64 proxies error {res[False][0]:.2e} (leaf rank {res[False][1]}, root "
             f"{res[False][2]}); FP32 proxies error {res[True][0]:.2e} (leaf rank {res[True][1]}, root {res[True][2]})")
        if tol >= 1e-6:
            assert res[True][0] <= 5 * max(res[False][0], tol)
        elif tol >= 1e-8:
            assert res[True][0] <= max(5 * res[False][0], 1e-6)
        else:
            assert res[True][0] <= 1e-4


def test_hss_adaptive_proxy_count_high_wavenumber(gpu_lib):
    """A star at k0 = 79.8, n = 1.98 (k1 = 158): 64 points per proxy circle
    cannot represent the far field of the larger boxes; the adaptive count
    max(64, ceil(2 k R_p) + 32) restores the ID tolerance's accuracy."""
    bm = gpu_lib
    note("hss: high-wavenumber star N=3774, fixed vs adaptive proxy counts")
    media = sc.media_from_index(79.8, 158.4 / 79.8)
    p, nd = setup(bm, [sc.star(0.223, 7)], [3774], media)
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, media), wsbm.rhs_plane_wave(nd, media, 0.0))
    errs = {}
    for adapt in (False, True):
        h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, proxy_adapt=adapt)
        x = bm.bm_hss_solve(h, bm.bm_rhs_plane_wave(p, 0.0)).cpu().numpy()
        errs[adapt] = rel(x, ref)
        note(f"  proxy_adapt={adapt}: stats {bm.bm_hss_stats(h)}, error {errs[adapt]:.2e}")
    assert errs[True] < HSS_BAR
    assert errs[True] < errs[False]


def test_hss_stops_compressing_when_ranks_stay_high(gpu_lib):
    """max_rank_ratio: a body whose level keeps more than the given fraction of
    its unknowns stops compressing; its skeletons form a dense root (inverted
    through the Schur recursion, whose large products go to rocBLAS).  Two stars
    in one body, N = 1400, k0 = 40."""
    import torch
    bm = gpu_lib
    note("hss: stop rule on the rank ratio, two stars, N=1400")
    media = sc.media_from_index(40.0, 1.5)
    curves = [sc.star(0.2, 4), sc.star(0.25, 3, 1.0, (3.0, 0.0))]
    p, nd = setup(bm, curves, [800, 600], media)
    A = wsbm.assemble_dense(nd, media)
    ref = wsbm.solve_dense(A, wsbm.rhs_plane_wave(nd, media, 0.5))
    b = bm.bm_rhs_plane_wave(p, 0.5)
    full = bm.bm_hss_build(p, leaf=32, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, proxy_adapt=True)
    cut = bm.bm_hss_build(p, leaf=32, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, proxy_adapt=True,
                          max_rank_ratio=0.3)
    sf, st = bm.bm_hss_stats(full), bm.bm_hss_stats(cut)
    note(f"  without the rule: {sf['compressed_levels']} levels, root {sf['root_size']}; "
         f"with 0.3: {st['compressed_levels']} levels, root {st['root_size']}")
    assert 1 <= st["compressed_levels"] < sf["compressed_levels"]
    assert st["root_size"] > sf["root_size"]
    bh = b.cpu().numpy()
    for h in (full, cut):
        x = bm.bm_hss_solve(h, b).cpu().numpy()
        assert rel(x, ref) < HSS_BAR
        xt = bm.bm_hss_solve_transpose(h, b).cpu().numpy()
        assert np.linalg.norm(A.T @ xt - bh) <= 1e-7 * np.linalg.norm(bh)


@pytest.mark.parametrize("transpose", [False, True])
def test_hss_solve_graph_replays_match_eager(gpu_lib, transpose):
    """bm_hss_solve_graph: the solve captured into a HIP graph on the first call
    and replayed; every replay (with eager solves and synchronisations in
    between) must give the eager result.  Two stars, N = 2300, two shapes
    (nrhs 2 and 1), three replays each."""
    import torch
    bm = gpu_lib
    note(f"hss: graph-replayed solve, transpose={transpose}")
    media = sc.media_from_index(20.0, 1.5)
    p, nd = setup(bm, [sc.star(0.3, 5), sc.star(0.2, 3, 1.0, (3.0, 0.5))], [1500, 800], media)
    h = bm.bm_hss_build(p, leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10)
    eager = bm.bm_hss_solve_transpose if transpose else bm.bm_hss_solve
    rng = np.random.default_rng(9)
    for nrhs in (2, 1):
        for rep in range(3):
            B = rng.standard_normal((nrhs, 2 * p.n)) + 1j * rng.standard_normal((nrhs, 2 * p.n))
            Bt = torch.from_numpy(B[0] if nrhs == 1 else B).cuda().contiguous()
            ref = eager(h, Bt)
            torch.cuda.synchronize()
            got = bm.bm_hss_solve_graph(h, Bt, transpose=transpose)
            other = eager(h, Bt.flip(-1).contiguous())      # eager work between replays
            torch.cuda.synchronize()
            d = (got - ref).abs().max().item()
            note(f"  nrhs {nrhs} replay {rep}: max |graph - eager| {d:.2e}")
            assert d <= 1e-13 * ref.abs().max().item()
            assert other.abs().max().item() > 0
    # the first right-hand side against the dense oracle as well
    A = wsbm.assemble_dense(nd, media)
    b = rng.standard_normal(2 * p.n) + 1j * rng.standard_normal(2 * p.n)
    x = bm.bm_hss_solve_graph(h, torch.from_numpy(b).cuda(), transpose=transpose).cpu().numpy()
    ref = np.linalg.solve(A.T if transpose else A, b)
    assert rel(x, ref) < HSS_BAR


def test_hss_rejects_bad_options(gpu_lib):
    bm = gpu_lib
    media = sc.media_from_index(10.0, 1.5)
    p, _ = setup(bm, [sc.circle()], [64], media)
    for kw in ({"leaf": 2}, {"proxy_ratio": 1.0}, {"proxy_points": 4}, {"id_tol": 0.0}):
        with pytest.raises(bm.BmError):
            bm.bm_hss_build(p, **kw)
    with pytest.raises(bm.BmError):
        bm.bm_hss_build(p, sketch=-2)
    for r in (-0.1, -2.0, 1.5, float("nan")):
        with pytest.raises(bm.BmError):
            bm.bm_hss_build(p, max_rank_ratio=r)
    # the same through the C-ABI directly: nothing is built
    import ctypes
    from paper_2607_00790_amd import _binding as B
    opts = B._HssOpts(64, 1.5, 64, 1e-10, -5)
    out = ctypes.c_void_p()
    assert B._LIB.bm_hss_build(p._h, ctypes.byref(opts), None, ctypes.byref(out)) == 1
    assert out.value is None


def test_hss_kernel_timing_counts_launches(gpu_lib):
    """opts.kernel_timing: every batched GEMM, Gauss-Jordan, sketch and entry-generation launch of the build
    is event-timed; the counts, flops and times are positive, the solution is the
    same as without timing, and the fields stay zero when timing is off."""
    bm = gpu_lib
    note("hss: per-launch kernel timing, star N=2048")
    media = sc.media_from_index(50.0, 1.5)
    p, nd = setup(bm, [sc.star(0.3, 5)], [2048], media)
    b = bm.bm_rhs_plane_wave(p, 0.2)
    opts = dict(leaf=64, proxy_ratio=1.5, proxy_points=64, id_tol=1e-10, sketch=-1, max_rank_ratio=-1.0)
    plain = bm.bm_hss_build(p, **opts)
    timed = bm.bm_hss_build(p, kernel_timing=True, **opts)
    s0, s1 = bm.bm_hss_stats(plain), bm.bm_hss_stats(timed)
    note(f"  gemm {s1['gemm_launches']} launches {s1['seconds_gemm'] * 1e3:.3f} ms {s1['gemm_flops']:.3e} flops; "
         f"inv {s1['inv_launches']} launches {s1['seconds_inv'] * 1e3:.3f} ms {s1['inv_flops']:.3e} flops; "
         f"sketch {s1['sketch_launches']} launches {s1['seconds_sketch'] * 1e3:.3f} ms; "
         f"gen {s1['gen_launches']} launches {s1['seconds_gen'] * 1e3:.3f} ms {s1['gen_pairs']:.3e} pairs")
    for k in ("gemm_launches", "gemm_flops", "seconds_gemm", "inv_launches", "inv_flops", "seconds_inv",
              "sketch_launches", "sketch_flops", "seconds_sketch", "gen_launches", "gen_pairs", "seconds_gen"):
        assert s0[k] == 0
        assert s1[k] > 0
    x0 = bm.bm_hss_solve(plain, b).cpu().numpy()
    x1 = bm.bm_hss_solve(timed, b).cpu().numpy()
    assert np.abs(x1 - x0).max() <= 1e-13 * np.abs(x0).max()
