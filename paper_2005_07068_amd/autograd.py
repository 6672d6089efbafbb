"""``torch.autograd.Function`` over the library's adjoint kernel.

Forward runs ``ht_eval_particles_grad`` (cost and dE/dh in one pass) and keeps the gradient;
backward scales it by the incoming gradient of the costs.
"""
from __future__ import annotations

import torch


class HandCost(torch.autograd.Function):
    """E(h, O) per particle, differentiable with respect to the poses h.

    ``HandCost.apply(poses, ctx, frame_slots, pixel_mask=None)`` with poses [F, P, D] or [P, D]
    float32 on the GPU returns costs [F, P] or [P]."""

    @staticmethod
    def forward(fctx, poses, ctx, frame_slots, pixel_mask=None):
        cost, grad = ctx.eval_grad(poses.detach(), frame_slots, pixel_mask)
        fctx.save_for_backward(grad)
        return cost

    @staticmethod
    def backward(fctx, g_cost):
        (grad,) = fctx.saved_tensors
        return g_cost.unsqueeze(-1) * grad, None, None, None
