"""The allocation-free product bm_matvec_noalloc against bm_matvec, through the
C-ABI: two calls in a row (the second on a smaller, two-body problem, so the
fixed buffer holds the first call's partial sums when the second starts), each
compared with bm_matvec on the same input -- the same kernels in the same
order, so the results must agree bit for bit -- and a problem whose partial
sums exceed the fixed buffer, which must be rejected before anything runs."""
import sys

import numpy as np
import pytest

import scatterers as sc

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(bm, curves, sizes, media, bodies=None):
    xyd, s = sc.sample_curves(curves, sizes)
    g = bm.bm_geom_create(s, xyd)
    if bodies is None:
        return bm.bm_problem_create(g, media[0].k0, media[0].k1, media[0].eps0, media[0].eps1)
    return bm.bm_problem_create_bodies(g, bodies, [(m.k0, m.k1, m.eps0, m.eps1) for m in media])


def test_matvec_noalloc_matches_matvec(gpu_lib):
    import torch
    bm = gpu_lib
    rng = np.random.default_rng(11)
    cases = [
        ("one star, N = 5000 (3 source tiles, ragged)", [sc.star(0.3, 5)], [5000],
         [sc.media_from_index(40.0, 1.5)], None),
        ("two bodies, N = 1200 + 700", [sc.star(0.2, 4), sc.circle(0.6, (3.0, 0.0))], [1200, 700],
         [sc.media_from_index(20.0, 1.3), sc.media_from_index(35.0, 1.8)], [0, 1]),
    ]
    for name, curves, sizes, media, bodies in cases:
        note(f"no-alloc matvec: {name}")
        p = _problem(bm, curves, sizes, media, bodies)
        n2 = 2 * p.n
        x = torch.from_numpy(rng.standard_normal(n2) + 1j * rng.standard_normal(n2)).cuda()
        y = torch.empty(n2, dtype=torch.complex128, device="cuda")
        bm.bm_matvec_noalloc(p, x, y)
        yref = bm.bm_matvec(p, x)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert torch.equal(y, yref), (torch.abs(y - yref).max() / torch.abs(yref).max()).item()


def test_matvec_noalloc_rejects_problems_beyond_its_buffer(gpu_lib):
    import torch
    bm = gpu_lib
    note("no-alloc matvec: N = 40000 exceeds the fixed buffer")
    p = _problem(bm, [sc.star(0.3, 5)], [40000], [sc.media_from_index(10.0, 1.5)])
    x = torch.zeros(2 * p.n, dtype=torch.complex128, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(bm.BmError) as ei:
        bm.bm_matvec_noalloc(p, x, y)
    assert ei.value.code == 1
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
