"""Differentiable forward SHT.

``SHTForward`` wraps the plan's forward transform; its backward calls the
library's adjoint (``sht_backward``: transposed phi DFT without the 1/M
factor, transposed ALT without quadrature weights).  The forward SHT is
complex-linear, f = S beta, so in PyTorch's gradient convention the
vector-Jacobian product is grad_beta = S^H grad_f.
"""
from __future__ import annotations

import torch

from .sht import Plan, materialize


class SHTForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(materialize(beta))

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        return ctx.plan.backward(materialize(grad_f)), None


def sht_forward(beta: torch.Tensor, plan: Plan) -> torch.Tensor:
    """f = S beta with autograd support (gradient via the adjoint kernels)."""
    return SHTForward.apply(beta, plan)
