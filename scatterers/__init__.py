"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* scatterers and draws random parameters: it samples
an analytic closed curve r(theta) (and its first two parameter derivatives) at
equispaced parameter values, and it turns a workload description (wavenumber,
refractive index) into the material constants of the transmission problem.
It holds none of the solver's arithmetic: normals, quadrature weights,
curvature, kernels, corrections and solves are computed independently by the
oracle and by the HIP library from the raw samples produced here.

Conventions (paper, Sec. II and Sec. IV):
  * a curve is parametrised counter-clockwise by t in [0, 2*pi) and sampled
    at t_j = 2*pi*j/N, j = 0..N-1 (equispaced trapezoidal nodes);
  * the sample array ``xyd`` is float64 with shape (6, N_total) holding
    x, y, x', y', x'', y'' (derivatives with respect to t); several curves are
    concatenated along the second axis;
  * k_j = omega*sqrt(eps_j*mu_j) with mu_0 = mu_1 = 1 (Sec. II); a workload
    given by an exterior wavenumber k_ext and a refractive index n therefore has
    eps_0 = 1, eps_1 = n**2, k_1 = n*k_ext.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "RadialCurve", "circle", "star", "fourier_curve", "sample_curves",
    "Media", "media_from_index", "table1_media", "Workload",
    "circle_workload", "star_workload", "batched_star_workloads",
    "fourier_workload", "grid_of_stars_workload",
]


@dataclasses.dataclass(frozen=True)
class RadialCurve:
    """Closed star-shaped curve x(t) = c + R*r(t)*(cos t, sin t).

    r(t) = 1 + sum_j (a_j cos(j t) + b_j sin(j t)); ``a`` and ``b`` hold the
    coefficients for j = 1..len(a).
    """

    a: Tuple[float, ...] = ()
    b: Tuple[float, ...] = ()
    radius: float = 1.0
    center: Tuple[float, float] = (0.0, 0.0)

    def radial(self, t: np.ndarray):
        """r(t), r'(t), r''(t) (unscaled)."""
        r = np.ones_like(t)
        dr = np.zeros_like(t)
        ddr = np.zeros_like(t)
        for j, (aj, bj) in enumerate(zip(self.a, self.b), start=1):
            c, s = np.cos(j * t), np.sin(j * t)
            r += aj * c + bj * s
            dr += j * (-aj * s + bj * c)
            ddr += -j * j * (aj * c + bj * s)
        return r, dr, ddr

    def sample(self, n: int) -> np.ndarray:
        """Return the (6, n) array x, y, x', y', x'', y'' at t_j = 2*pi*j/n."""
        t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
        r, dr, ddr = self.radial(t)
        r, dr, ddr = self.radius * r, self.radius * dr, self.radius * ddr
        c, s = np.cos(t), np.sin(t)
        x = self.center[0] + r * c
        y = self.center[1] + r * s
        dx = dr * c - r * s
        dy = dr * s + r * c
        ddx = ddr * c - 2.0 * dr * s - r * c
        ddy = ddr * s + 2.0 * dr * c - r * s
        return np.stack([x, y, dx, dy, ddx, ddy])


def circle(radius: float = 1.0, center=(0.0, 0.0)) -> RadialCurve:
    return RadialCurve((), (), float(radius), (float(center[0]), float(center[1])))


def star(amp: float, m: int, radius: float = 1.0, center=(0.0, 0.0)) -> RadialCurve:
    """r(theta) = radius*(1 + amp*cos(m*theta))."""
    a = [0.0] * int(m)
    a[int(m) - 1] = float(amp)
    return RadialCurve(tuple(a), (0.0,) * int(m), float(radius),
                       (float(center[0]), float(center[1])))


def fourier_curve(a: Sequence[float], b: Sequence[float]) -> RadialCurve:
    """r(theta) = 1 + sum_j (a_j cos j theta + b_j sin j theta), j = 1..len(a)."""
    assert len(a) == len(b)
    return RadialCurve(tuple(float(v) for v in a), tuple(float(v) for v in b))


def sample_curves(curves: Sequence[RadialCurve], sizes: Sequence[int]):
    """Concatenate the samples of several curves.

    Returns (xyd float64 (6, sum(sizes)), sizes int64 array)."""
    parts = [c.sample(int(n)) for c, n in zip(curves, sizes)]
    return np.ascontiguousarray(np.concatenate(parts, axis=1)), np.asarray(sizes, dtype=np.int64)


@dataclasses.dataclass(frozen=True)
class Media:
    """Wavenumbers and permittivities of the exterior (0) and interior (1)."""

    k0: float
    k1: float
    eps0: float
    eps1: float


def media_from_index(k_ext: float, n: float) -> Media:
    """eps_0 = 1, eps_1 = n^2, mu = 1, so k_1 = n*k_ext (Sec. II, k_j = w sqrt(eps_j mu_j))."""
    return Media(float(k_ext), float(n) * float(k_ext), 1.0, float(n) ** 2)


def table1_media() -> Media:
    """Material constants of the paper's Table I: eps0=1, eps1=5, mu0=mu1=1, omega=10."""
    omega, eps0, eps1 = 10.0, 1.0, 5.0
    return Media(omega * math.sqrt(eps0), omega * math.sqrt(eps1), eps0, eps1)


@dataclasses.dataclass
class Workload:
    name: str
    curves: List[RadialCurve]
    sizes: List[int]
    media: Media
    theta_inc: float
    leaf: int = 64
    proxy_ratio: float = 1.5
    proxy_points: int = 64
    id_tol: float = 1e-10

    @property
    def n(self) -> int:
        return int(sum(self.sizes))

    def xyd(self):
        return sample_curves(self.curves, self.sizes)


def circle_workload(n: int = 512, k_ext: float = 10.0, index: float = 1.5,
                    radius: float = 1.0, theta_inc: float = 0.0) -> Workload:
    """Plain dense method: dielectric circle, plane wave at angle 0."""
    return Workload(f"circle_a{radius:g}_k{k_ext:g}_n{index:g}_N{n}", [circle(radius)], [n],
                    media_from_index(k_ext, index), theta_inc)


def star_workload(n: int = 16384, k_ext: float = 50.0, index: float = 1.5, amp: float = 0.3,
                  m: int = 5, seed: int = 0, leaf: int = 64, proxy_points: int = 64,
                  id_tol: float = 1e-10) -> Workload:
    """Plain HSS workload: star r = 1 + amp*cos(m*theta); incidence angle drawn U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    theta = float(rng.uniform(0.0, 2.0 * np.pi))
    return Workload(f"star_a{amp:g}_m{m}_N{n}_k{k_ext:g}_n{index:g}", [star(amp, m)], [n],
                    media_from_index(k_ext, index), theta, leaf=leaf, proxy_points=proxy_points,
                    id_tol=id_tol)


def batched_star_workloads(count: int = 256, seed: int = 0) -> List[Workload]:
    """Independent stars: a~U[0.1,0.3], m~U{3..8}, N~U{1024..8192}, k_ext~U[10,80],
    n~U[1.2,2.0], drawn per scatterer in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        amp = float(rng.uniform(0.1, 0.3))
        m = int(rng.integers(3, 9))
        n = int(rng.integers(1024, 8193))
        k_ext = float(rng.uniform(10.0, 80.0))
        index = float(rng.uniform(1.2, 2.0))
        out.append(Workload(f"batch{s}", [star(amp, m)], [n], media_from_index(k_ext, index), 0.0))
    return out


def fourier_workload(n: int = 8192, k_ext: float = 40.0, index: float = 1.5, modes: int = 32,
                     sigma: float = 0.01, seed: int = 0) -> Workload:
    """Random smooth boundary with Fourier coefficients ~ N(0, sigma^2) (a_1..a_M, then b_1..b_M)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, sigma, modes)
    b = rng.normal(0.0, sigma, modes)
    return Workload(f"fourier{modes}_N{n}_k{k_ext:g}", [fourier_curve(a, b)], [n],
                    media_from_index(k_ext, index), 0.0)


def grid_of_stars_workload(per_curve: int = 16384, k_ext: float = 200.0, index: float = 2.0,
                           grid: int = 4, spacing: float = 3.0, seed: int = 0, leaf: int = 128,
                           proxy_points: int = 96) -> Workload:
    """Disjoint unit stars centred on a grid x spacing; a~U[0.1,0.3], m~U{3..8} per star."""
    rng = np.random.default_rng(seed)
    curves = []
    for i in range(grid):
        for j in range(grid):
            amp = float(rng.uniform(0.1, 0.3))
            m = int(rng.integers(3, 9))
            curves.append(star(amp, m, 1.0, (spacing * i, spacing * j)))
    return Workload(f"grid{grid}x{grid}_stars_N{per_curve * grid * grid}_k{k_ext:g}", curves,
                    [per_curve] * len(curves), media_from_index(k_ext, index), 0.0, leaf=leaf,
                    proxy_points=proxy_points)
