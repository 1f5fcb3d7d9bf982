"""torch.autograd.Function for shape gradients of the backscattered intensity.

J(c) = |u_inf(theta_inc + pi)|^2 for the boundary r(t) = 1 + sum_j (a_j cos jt
+ b_j sin jt), c = (a_1..a_M, b_1..b_M), discretised by n trapezoidal nodes
and solved with the proxy-surface HSS factorisation.  The backward pass is the
adjoint method on the same factors: far-field weights g, the transposed solve
A^T lam = g, the pair-derivative contraction and the chain rule to c, each a
C-ABI call (include/bmhss.h); this module only passes tensors between them.
The class is created on first use, so importing the package does not import
torch.
"""
from __future__ import annotations

import math

from . import _binding as _b

_FN = None


def _function_class():
    global _FN
    if _FN is not None:
        return _FN
    import torch

    class BackscatterIntensity(torch.autograd.Function):
        """apply(coef, n, (k0, k1, eps0, eps1), theta_inc, hss_opts) -> J."""

        @staticmethod
        def forward(ctx, coef, n, media, theta_inc, hss_opts):
            coef = coef.detach().contiguous()
            xyd = _b.bm_fourier_curve(coef, n)
            g = _b.bm_geom_create([n], xyd)
            p = _b.bm_problem_create(g, *media)
            h = _b.bm_hss_build(p, **hss_opts)
            rhs = _b.bm_rhs_plane_wave(p, theta_inc)
            phi = _b.bm_hss_solve(h, rhs)
            obs = theta_inc + math.pi
            u = _b.bm_far_field(p, phi, torch.tensor([obs], dtype=torch.float64))
            ctx.h, ctx.p, ctx.phi = h, p, phi
            ctx.theta_inc, ctx.obs, ctx.nmodes = theta_inc, obs, coef.numel() // 2
            return (u.real ** 2 + u.imag ** 2)[0]

        @staticmethod
        def backward(ctx, grad_out):
            gw = _b.bm_far_field_weights(ctx.p, ctx.obs)
            lam = _b.bm_hss_solve_transpose(ctx.h, gw)
            g6 = _b.bm_shape_derivative(ctx.p, ctx.phi, lam, ctx.theta_inc, ctx.obs)
            gc = _b.bm_fourier_chain(g6, ctx.nmodes)
            return grad_out * gc, None, None, None, None

    _FN = BackscatterIntensity
    return _FN


def backscatter_intensity(coef, n: int, k0: float, k1: float, eps0: float, eps1: float,
                          theta_inc: float = 0.0, **hss_opts):
    """J(coef) as a differentiable scalar tensor (coef: device float64, 2M values);
    hss_opts go to bm_hss_build (leaf, proxy_ratio, proxy_points, id_tol, ...)."""
    return _function_class().apply(coef, int(n), (float(k0), float(k1), float(eps0), float(eps1)),
                                   float(theta_inc), dict(hss_opts))


def __getattr__(name):
    if name == "BackscatterIntensity":
        return _function_class()
    raise AttributeError(name)
