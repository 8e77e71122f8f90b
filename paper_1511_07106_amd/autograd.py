"""torch.autograd wrapper of the differentiable raycast (hand-written HIP
forward and backward kernels in libmvf)."""
from __future__ import annotations

import numpy as np
import torch

from .api import Context, pose_retract, pose_right_jacobian


class DiffRaycast(torch.autograd.Function):
    """depth = DiffRaycast.apply(F, xi, W, ctx, origin, voxel_size, T0, K, width, height[, generation])

    F: (nz, ny, nx) float32 TSDF on the device (truncation units), W: weights
    of the same shape (uint16/int16; 0 = unobserved), xi: 6-vector (rho,
    omega) of the right pose perturbation T = T0 Exp(xi).  The backward gives
    dL/dF and dL/dxi: the kernel's gradient g for a right perturbation at T
    is mapped through the right Jacobian of Exp at xi (dL/dxi = J_r(xi)^T g,
    equal to g at xi = 0).  The crossing found by the forward is held fixed.
    generation (default 0: rebuild every call) lets the forward reuse the
    library's brick-layout copy of (F, W) while F and W stay unchanged; bump
    it whenever either changes.
    """

    @staticmethod
    def forward(ctx, F, xi, W, mvf: Context, origin, voxel_size, T0, K, width, height, generation=0):
        T = pose_retract(T0, xi.detach().double().cpu().numpy())
        depth, record = mvf.diffray_forward(F.detach(), W, origin, voxel_size, T, K, width, height,
                                            generation=generation)
        ctx.save_for_backward(F, W, record)
        ctx.mvf = mvf
        ctx.params = (origin, voxel_size, T, K)
        ctx.jr = pose_right_jacobian(xi.detach().double().cpu().numpy())
        ctx.xi_dtype = xi.dtype
        ctx.xi_device = xi.device
        ctx.mark_non_differentiable(record)
        return depth

    @staticmethod
    def backward(ctx, grad_depth):
        F, W, record = ctx.saved_tensors
        origin, voxel_size, T, K = ctx.params
        grad_F = torch.zeros_like(F) if ctx.needs_input_grad[0] else None
        gxi = ctx.mvf.diffray_backward(F.detach(), W, origin, voxel_size, T, K,
                                       grad_depth.float().contiguous(), record, grad_F)
        if ctx.needs_input_grad[1]:
            g = gxi.cpu().numpy() @ ctx.jr  # J_r^T g
            gxi = torch.from_numpy(g).to(device=ctx.xi_device, dtype=ctx.xi_dtype)
        else:
            gxi = None
        return grad_F, gxi, None, None, None, None, None, None, None, None, None


def depth_loss(pred, target, gate: float = 0.05):
    """L = 1/(2|P|) sum_P (z - z_target)^2 over the pixels P valid in both
    maps whose residual is below `gate` metres (pixels where prediction and
    target see different surfaces are outliers, not alignment signal)."""
    valid = (pred > 0) & (target > 0) & ((pred - target).abs() < gate)
    n = valid.sum().clamp(min=1)
    r = torch.where(valid, pred - target, torch.zeros_like(pred))
    return 0.5 * (r * r).sum() / n
