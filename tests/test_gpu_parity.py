"""GPU parity of the HIP entry-generation path against the CPU oracle, called
through the C-ABI (Python binding of include/bmhss.h).

Bar (FP64): per 2x2 component of a block, max|diff| <= 1e-10 max|ref|, and
per-entry relative error <= 1e-10 wherever |ref| >= 1e-6 max|ref|.  Sizes span
several 256-wide tiles with ragged tails; the full-size star workload
(N = 16384, k0 = 50, n = 1.5) is checked on sampled rows."""
import sys

import numpy as np
import pytest

import scatterers as sc
from oracle import geometry, mie, wsbm

from parity import assert_parity

pytestmark = pytest.mark.gpu


def case(curves, sizes):
    xyd, s = sc.sample_curves(curves, sizes)
    return xyd, s, geometry.discretize(xyd, s)


def gpu_problem(bm, xyd, sizes, media):
    g = bm.bm_geom_create(sizes, xyd)
    return bm.bm_problem_create(g, media.k0, media.k1, media.eps0, media.eps1)


def to_np(t):
    return t.detach().cpu().numpy()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_geometry_nodes(gpu_lib):
    bm = gpu_lib
    note("geometry: star + circle")
    xyd, s, nd = case([sc.star(0.3, 5), sc.circle(0.4, (3, 0))], [777, 64])
    g = bm.bm_geom_create(s, xyd)
    soa = to_np(bm.bm_geom_nodes(g))
    ref = np.stack([nd.x[:, 0], nd.x[:, 1], nd.n[:, 0], nd.n[:, 1], nd.w, nd.kappa])
    np.testing.assert_allclose(soa, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("name", ["circle512", "star1000", "two_curves_ragged"])
def test_dense_matches_oracle(gpu_lib, name):
    bm = gpu_lib
    note(f"dense parity: {name}")
    if name == "circle512":
        wl = sc.circle_workload(512)
        xyd, s, nd = case(wl.curves, wl.sizes)
        media = wl.media
    elif name == "star1000":
        xyd, s, nd = case([sc.star(0.3, 5)], [1000])
        media = sc.media_from_index(50.0, 1.5)
    else:
        xyd, s, nd = case([sc.star(0.2, 4), sc.star(0.25, 3, 1.0, (3.0, 0.5))], [301, 197])
        media = sc.media_from_index(20.0, 2.0)
    p = gpu_problem(bm, xyd, s, media)
    A = to_np(bm.bm_assemble_dense(p))
    ref = wsbm.assemble_dense(nd, media)
    assert_parity(A, ref)


def test_dense_full_size_star_sampled_rows(gpu_lib):
    """Full star workload, same launch as the benchmark's dense sweep."""
    import torch
    bm = gpu_lib
    note("dense parity: star N=16384 sampled rows")
    wl = sc.star_workload()
    xyd, s, nd = case(wl.curves, wl.sizes)
    p = gpu_problem(bm, xyd, s, wl.media)
    A = bm.bm_assemble_dense(p)
    rng = np.random.default_rng(7)
    nodes = np.unique(np.concatenate([[0, 1, 255, 256, 8191, 16383], rng.integers(0, 16384, 26)]))
    rows = torch.from_numpy(np.sort(np.concatenate([2 * nodes, 2 * nodes + 1]))).cuda()
    got = to_np(A.index_select(0, rows))
    ref = wsbm.assemble_rows(nd, wl.media, nodes)
    assert_parity(got, ref)


def test_block_index_lists(gpu_lib):
    import torch
    bm = gpu_lib
    note("block parity: index lists with diagonal pairs, ragged")
    xyd, s, nd = case([sc.star(0.3, 5)], [2000])
    media = sc.media_from_index(50.0, 1.5)
    p = gpu_problem(bm, xyd, s, media)
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(100, 140), rng.integers(0, 2000, 27)])
    cols = np.concatenate([np.arange(90, 150), rng.integers(0, 2000, 300)])
    got = to_np(bm.bm_assemble_block(p, torch.from_numpy(rows), torch.from_numpy(cols)))
    ref = wsbm.system_blocks(nd, media, rows, cols).reshape(2 * len(rows), 2 * len(cols))
    assert_parity(got, ref)
    # empty lists are a no-op
    out = bm.bm_assemble_block(p, torch.zeros(0, dtype=torch.int64), torch.from_numpy(cols))
    assert out.shape == (0, 2 * len(cols))


def test_block_index_lists_across_bodies(gpu_lib):
    """Two bodies with their own media: pairs within a body are that body's
    entries (diagonal pairs corrected), pairs across bodies are zero blocks."""
    import torch
    bm = gpu_lib
    note("block parity: two bodies, cross-body zero blocks")
    curves = [sc.star(0.3, 5), sc.star(0.2, 3, 1.0, (3.0, 0.5))]
    sizes = [400, 300]
    media = [sc.media_from_index(30.0, 1.5), sc.media_from_index(12.0, 1.8)]
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create_bodies(g, [0, 1], [(m.k0, m.k1, m.eps0, m.eps1) for m in media])
    rng = np.random.default_rng(4)
    rows = np.concatenate([np.arange(390, 420), rng.integers(0, 700, 41)])
    cols = np.concatenate([np.arange(380, 430), rng.integers(0, 700, 157)])
    got = to_np(bm.bm_assemble_block(p, torch.from_numpy(rows), torch.from_numpy(cols)))
    ref = np.zeros((len(rows), 2, len(cols), 2), dtype=np.complex128)
    lo = [0, 400, 700]
    for b in range(2):
        nd = geometry.discretize(*sc.sample_curves([curves[b]], [sizes[b]]))
        ri = np.nonzero((rows >= lo[b]) & (rows < lo[b + 1]))[0]
        ci = np.nonzero((cols >= lo[b]) & (cols < lo[b + 1]))[0]
        blk = wsbm.system_blocks(nd, media[b], rows[ri] - lo[b], cols[ci] - lo[b])
        ref[np.ix_(ri, [0, 1], ci, [0, 1])] = blk
    assert_parity(got, ref.reshape(2 * len(rows), 2 * len(cols)))


def fp32_error(got, ref):
    """Largest |diff| / max|ref| over the four 2x2 components."""
    g = got.reshape(got.shape[0] // 2, 2, got.shape[1] // 2, 2)
    r = ref.reshape(g.shape)
    return max(np.abs(g[:, a, :, b] - r[:, a, :, b]).max() / np.abs(r[:, a, :, b]).max()
               for a in range(2) for b in range(2))


# FP32 arithmetic: per 2x2 component, max|diff| <= FP32_BAR max|ref| (entries
# carry ~1e-7 relative rounding; the near-singular D-type entries, which are
# small, lose more, which the component-wise max norm allows).
FP32_BAR = 1e-6


def test_block_index_lists_fp32(gpu_lib):
    import torch
    bm = gpu_lib
    note("block parity, FP32 arithmetic (prec 1)")
    xyd, s, nd = case([sc.star(0.3, 5)], [2000])
    media = sc.media_from_index(50.0, 1.5)
    p = gpu_problem(bm, xyd, s, media)
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(100, 140), rng.integers(0, 2000, 27)])
    cols = np.concatenate([np.arange(90, 150), rng.integers(0, 2000, 300)])
    got = to_np(bm.bm_assemble_block(p, torch.from_numpy(rows), torch.from_numpy(cols), prec=1))
    ref = wsbm.system_blocks(nd, media, rows, cols).reshape(2 * len(rows), 2 * len(cols))
    err = fp32_error(got, ref)
    note(f"  FP32 block: max component error {err:.2e} of max|A|")
    assert err <= FP32_BAR


@pytest.mark.parametrize("direction", [0, 1])
def test_proxy_blocks(gpu_lib, direction):
    import torch
    bm = gpu_lib
    note(f"proxy parity: dir {direction}")
    xyd, s, nd = case([sc.star(0.3, 5)], [4096])
    media = sc.media_from_index(50.0, 1.5)
    p = gpu_problem(bm, xyd, s, media)
    box = np.arange(1000, 1128)
    c = nd.x[box].mean(0)
    R = np.max(np.hypot(*(nd.x[box] - c).T))
    P = 70
    th = 2 * np.pi * np.arange(P) / P
    px = c[None, :] + 1.5 * R * np.stack([np.cos(th), np.sin(th)], 1)
    pn = np.stack([np.cos(th), np.sin(th)], 1)
    pw = np.full(P, 2 * np.pi * 1.5 * R / P)
    pts = torch.from_numpy(np.stack([px[:, 0], px[:, 1], pn[:, 0], pn[:, 1], pw])).cuda()
    got = to_np(bm.bm_assemble_proxy(p, torch.from_numpy(box), pts, direction))
    if direction == 0:
        ref = wsbm.pair_blocks(nd.x[box], nd.n[box], px, pn, pw, media)
        ref = ref.reshape(2 * len(box), 2 * P)
    else:
        ref = wsbm.pair_blocks(px, pn, nd.x[box], nd.n[box], nd.w[box], media)
        ref = ref.reshape(2 * P, 2 * len(box))
    assert_parity(got, ref)
    got32 = to_np(bm.bm_assemble_proxy(p, torch.from_numpy(box), pts, direction, prec=1))
    err = fp32_error(got32, ref)
    note(f"  FP32 proxy dir {direction}: max component error {err:.2e} of max|A|")
    assert err <= FP32_BAR


def test_rhs_incident_point_source(gpu_lib):
    """bm_rhs_incident from a point source's field and normal derivative (the
    oracle's values) against the oracle's right-hand side, on two bodies."""
    import torch
    bm = gpu_lib
    note("rhs parity: point-source incident field, two bodies")
    curves = [sc.star(0.3, 5), sc.circle(0.5, (3.0, 0.0))]
    sizes = [700, 129]
    media = [sc.media_from_index(30.0, 1.5), sc.media_from_index(15.0, 1.2)]
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    p = bm.bm_problem_create_bodies(g, [0, 1], [(m.k0, m.k1, m.eps0, m.eps1) for m in media])
    ref, uins, dns = [], [], []
    for b in range(2):
        nd = geometry.discretize(*sc.sample_curves([curves[b]], [sizes[b]]))
        uin, dn = wsbm.point_source_field(nd, media[b].k0, (1.2, 2.1))
        uins.append(uin)
        dns.append(dn)
        ref.append(wsbm.rhs_incident(nd, media[b], uin, dn))
    ref = np.concatenate(ref)
    uin = torch.from_numpy(np.concatenate(uins)).cuda()
    dn = torch.from_numpy(np.concatenate(dns)).cuda()
    got = to_np(bm.bm_rhs_incident(p, uin, dn))
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    with pytest.raises(bm.BmError) as ei:
        bm.bm_rhs_incident(p, uin, dn, out=uin)
    assert ei.value.code == 1


def test_rhs_matvec_far_field(gpu_lib):
    import torch
    bm = gpu_lib
    note("rhs / matvec / far field parity")
    xyd, s, nd = case([sc.star(0.3, 5)], [700])
    media = sc.media_from_index(30.0, 1.5)
    p = gpu_problem(bm, xyd, s, media)
    rhs = to_np(bm.bm_rhs_plane_wave(p, 0.7))
    ref = wsbm.rhs_plane_wave(nd, media, 0.7)
    assert np.abs(rhs - ref).max() <= 1e-13 * np.abs(ref).max()
    rng = np.random.default_rng(5)
    x = rng.standard_normal(1400) + 1j * rng.standard_normal(1400)
    y = to_np(bm.bm_matvec(p, torch.from_numpy(x).cuda()))
    yref = wsbm.assemble_dense(nd, media) @ x
    assert np.abs(y - yref).max() <= 1e-12 * np.abs(yref).max()
    ang = np.linspace(0, 2 * np.pi, 37)
    ff = to_np(bm.bm_far_field(p, torch.from_numpy(x).cuda(), torch.from_numpy(ang)))
    ffref = wsbm.far_field(nd, media, x, ang)
    assert np.abs(ff - ffref).max() <= 1e-12 * np.abs(ffref).max()


def test_dense_solution_vs_oracle_and_mie(gpu_lib):
    """Plain dense workload: GPU-assembled matrix, LU on the device; the
    solution matches the oracle's to 1e-10 and its Mie error is within 2x."""
    import torch
    bm = gpu_lib
    note("dense solve: circle N=512 vs oracle and Mie")
    wl = sc.circle_workload(512)
    xyd, s, nd = case(wl.curves, wl.sizes)
    p = gpu_problem(bm, xyd, s, wl.media)
    A = bm.bm_assemble_dense(p)
    b = bm.bm_rhs_plane_wave(p, 0.0)
    phi = to_np(torch.linalg.solve(A, b))
    ref = wsbm.solve_dense(wsbm.assemble_dense(nd, wl.media), wsbm.rhs_plane_wave(nd, wl.media, 0.0))
    assert np.linalg.norm(phi - ref) <= 1e-10 * np.linalg.norm(ref)
    t = 2 * np.pi * np.arange(512) / 512
    u, _ = mie.boundary_values(wl.media, t)
    e_gpu = np.linalg.norm(phi[0::2].real - u.real) / np.linalg.norm(u.real)
    e_ora = np.linalg.norm(ref[0::2].real - u.real) / np.linalg.norm(u.real)
    assert e_gpu <= 2 * e_ora


def test_invalid_arguments_enqueue_nothing(gpu_lib):
    import torch
    bm = gpu_lib
    xyd, s, _ = case([sc.circle()], [64])
    p = gpu_problem(bm, xyd, s, sc.media_from_index(10, 1.5))
    with pytest.raises((bm.BmError, ValueError)):
        bm.bm_assemble_dense(p, out=torch.empty((128, 100), dtype=torch.complex128, device="cuda"))
    with pytest.raises(bm.BmError):
        bm.bm_assemble_proxy(p, torch.arange(4), torch.zeros((5, 3), dtype=torch.float64).cuda(), 2)
    with pytest.raises(bm.BmError):
        bm.bm_assemble_block(p, torch.arange(4), torch.arange(4), prec=2)


def test_fp64_fma_probe_values(gpu_lib):
    """The benchmark's FMA probe (libbmhss_probe.so, not part of the product
    library) computes what it claims: per thread, 16 chains of
    a <- a x + y from a_c = 1e-3 (c + 1), x = 1 + 1e-9 (t mod 1024), y = 1e-12 (t mod 256);
    after n steps a_n = a_0 x^n + y (x^n - 1)/(x - 1) (x = 1: a_0 + n y)."""
    import torch
    import bench
    blocks, iters = 4, 300
    out = bench.fma_probe(blocks, iters, torch.empty(blocks * 256, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for t in (0, 1, 255, 256, 1023, 1024 - 1, blocks * 256 - 1):
        x = 1.0 + 1e-9 * (t & 1023)
        y = 1e-12 * (t % 256)
        a0 = 1e-3 * np.arange(1, 17)
        if x == 1.0:
            ref = np.sum(a0 + iters * y)
        else:
            xn = x ** iters
            ref = np.sum(a0 * xn + y * (xn - 1.0) / (x - 1.0))
        assert abs(out[t] - ref) <= 1e-12 * abs(ref), (t, out[t], ref)
