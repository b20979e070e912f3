"""torch.autograd.Function over the library's hand-written reverse pass.

forward() calls sps_logl_grad when theta requires a gradient (the exact gradient
is computed together with logL and kept), sps_logl otherwise; backward() returns
grad_out[:, None] * d logL / d theta.  Gradient-based samplers (the paper's NUTS
and variational engines, Sec. 4.3) consume it through ordinary torch autograd.
"""
from __future__ import annotations

import torch

from . import sps


class SpsLogL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, library, obs, precision):
        if theta.requires_grad:
            ll, g = sps.logl_grad(library, obs, theta.detach().contiguous(), precision)
            ctx.save_for_backward(g)
        else:
            ll = sps.logl(library, obs, theta.detach().contiguous(), precision)
            ctx.save_for_backward(None)
        return ll

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        if g is None:
            return None, None, None, None
        return grad_out[:, None] * g, None, None, None


def logl(library, obs, theta, precision="fp32"):
    """Differentiable logL [B] of theta [B, P] (float64 CUDA tensor)."""
    return SpsLogL.apply(theta, library, obs, precision)
