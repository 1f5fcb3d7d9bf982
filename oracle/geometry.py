"""Boundary discretisation for the Nystrom method (paper Sec. II; Sec. I on the
one-point corrected trapezoidal rule).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Each closed curve Gamma_c is parametrised counter-clockwise by t in [0, 2pi)
and sampled at N_c equispaced values t_j = 2 pi j / N_c.  From the samples of
x(t), x'(t), x''(t):
  * speed          s_j = |x'(t_j)|
  * weight         w_j = (2 pi / N_c) s_j          (trapezoidal rule)
  * outward normal n_j = (x2', -x1') / s_j          (ccw curve, Sec. II: n points
                                                      out of the scatterer)
  * curvature      kappa_j = (x1' x2'' - x2' x1'') / s_j^3
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Nodes:
    x: np.ndarray       # (N, 2) positions
    n: np.ndarray       # (N, 2) outward unit normals
    w: np.ndarray       # (N,) quadrature weights
    kappa: np.ndarray   # (N,) signed curvature (1/a on a circle of radius a)
    curve: np.ndarray   # (N,) index of the closed curve each node belongs to

    @property
    def size(self) -> int:
        return int(self.w.shape[0])


def discretize(xyd: np.ndarray, sizes) -> Nodes:
    xyd = np.asarray(xyd, dtype=np.float64)
    sizes = np.asarray(sizes, dtype=np.int64)
    assert xyd.shape == (6, int(sizes.sum()))
    x, y, dx, dy, ddx, ddy = xyd
    per_node_n = np.repeat(sizes, sizes).astype(np.float64)
    s = np.sqrt(dx * dx + dy * dy)
    w = (2.0 * np.pi / per_node_n) * s
    normal = np.stack([dy / s, -dx / s], axis=1)
    kappa = (dx * ddy - dy * ddx) / s**3
    curve = np.repeat(np.arange(len(sizes)), sizes)
    return Nodes(np.stack([x, y], axis=1), normal, w, kappa, curve)
