"""Learned-feature data term: float patch cost behind torch.autograd.

PatchCost wraps ff_cost_f32_fwd / ff_cost_f32_bwd (hand-written HIP
kernels): forward gives the squared-difference cost of the subsampled patch
for every entry (x, y, fx, fy); backward gives the gradients with respect to
both feature maps (deterministic, fixed-point accumulation).
"""
from __future__ import annotations

import torch

from .ffi import check, lib
from .flowfields import _ptr, _stream


def cost_f32(f1: torch.Tensor, f2: torch.Tensor, entries: torch.Tensor, n: int = 1, radius: int = 3):
    H, W, C = f1.shape
    if C != 16 or tuple(f2.shape) != (H, W, 16):
        raise ValueError("features must be float32 [H, W, 16]")
    count = entries.shape[0]
    cost = torch.empty(count, dtype=torch.float32, device=f1.device)
    check(lib().ff_cost_f32_fwd(_ptr(f1, torch.float32, "f1"), _ptr(f2, torch.float32, "f2"), W, H, n, radius,
                                _ptr(entries, torch.int32, "entries"), count, _ptr(cost), _stream()),
          "ff_cost_f32_fwd")
    return cost


def cost_f32_grad(f1, f2, entries, grad_cost, n: int = 1, radius: int = 3):
    H, W, _ = f1.shape
    acc = torch.empty((2, H, W, 16), dtype=torch.int64, device=f1.device)
    g1 = torch.empty_like(f1)
    g2 = torch.empty_like(f2)
    check(lib().ff_cost_f32_bwd(_ptr(f1, torch.float32, "f1"), _ptr(f2, torch.float32, "f2"), W, H, n, radius,
                                _ptr(entries, torch.int32, "entries"), entries.shape[0],
                                _ptr(grad_cost, torch.float32, "grad_cost"), _ptr(acc), _ptr(g1), _ptr(g2),
                                _stream()), "ff_cost_f32_bwd")
    return g1, g2


class PatchCost(torch.autograd.Function):
    """cost[e] = sum over the (2r+1)^2 subsampled patch of |f1 - f2(+flow)|^2."""

    @staticmethod
    def forward(ctx, f1, f2, entries, n: int = 1, radius: int = 3):
        f1 = f1.contiguous()
        f2 = f2.contiguous()
        entries = entries.contiguous()
        ctx.save_for_backward(f1, f2, entries)
        ctx.n, ctx.radius = n, radius
        return cost_f32(f1, f2, entries, n, radius)

    @staticmethod
    def backward(ctx, grad_cost):
        f1, f2, entries = ctx.saved_tensors
        g1, g2 = cost_f32_grad(f1, f2, entries, grad_cost.contiguous().float(), ctx.n, ctx.radius)
        return g1, g2, None, None, None


def patch_cost(f1, f2, entries, n: int = 1, radius: int = 3):
    return PatchCost.apply(f1, f2, entries, n, radius)
