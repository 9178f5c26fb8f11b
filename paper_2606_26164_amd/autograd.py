"""torch.autograd.Function around the fused value/adjoint kernel.

forward evaluates f at the rows of X with the adjoint kernel, which produces
grad f in the same pass; backward scales the stored gradient by the incoming
gradient.  No torch arithmetic touches the objective itself.
"""
from __future__ import annotations

import torch

from . import _lib as L


class ChisaoLogDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: torch.Tensor, opt) -> torch.Tensor:
        f, G = opt.eval(X.detach(), grad_mode=L.GRAD_ADJOINT, want_f=True, want_g=X.requires_grad)
        if G is not None:
            ctx.save_for_backward(G)
        return f

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (G,) = ctx.saved_tensors
        return grad_out.to(G.dtype)[:, None] * G, None


def log_density(X: torch.Tensor, opt) -> torch.Tensor:
    return ChisaoLogDensity.apply(X, opt)
