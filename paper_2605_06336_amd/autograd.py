"""torch.autograd wrappers of the projector with hand-written backward passes.

ProjectFn:  y = A(theta) x.  backward: grad_x = A(theta)^T grad_y (nlrmm_backproject) and
            grad_theta_v = <dA/dtheta_v x, grad_y_v> computed by the fused per-view reduction
            of nlrmm_project_dtheta (the derivative sinogram is never written).
StreamingDataLoss: L(x, theta) = 1/2 sum_j ||A_j(theta_j) x - b_j||^2 over measurement
            blocks (contiguous view ranges, Section 2.4 / Alg. "s_nl_rmmgks_final").  Only
            (x, theta, b) are saved; each block's residual sinogram is recomputed in
            backward (checkpointing of the sinogram intermediates).
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import ops


class ProjectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, g, frames=None):
        ctx.g = g
        ctx.frames = frames
        ctx.save_for_backward(x, theta)
        y = ops.project(x.contiguous(), theta.contiguous(), g, frames)
        return y.view(*x.shape[:-3], theta.numel(), g.nbins)

    @staticmethod
    def backward(ctx, gy):
        x, theta = ctx.saved_tensors
        g, frames = ctx.g, ctx.frames
        gy = gy.contiguous()
        V, nb = theta.numel(), g.nbins
        cols = gy.numel() // (V * nb)
        gx = gth = None
        if ctx.needs_input_grad[0]:
            gx = ops.backproject(gy, theta, g, frames).view_as(x)
        if ctx.needs_input_grad[1]:
            xs = x.contiguous().reshape(cols, -1)
            gys = gy.reshape(cols, V, nb)
            gth = torch.zeros(V, dtype=torch.float64, device=x.device)
            for c in range(cols):
                res = ops.project_dtheta(xs[c].contiguous(), theta, g, frames, want_dy=False,
                                         gres=gys[c].contiguous(), want_gdot=True)
                gth = gth + res["gdot"][0]
        return gx, gth, None, None


def project(x: torch.Tensor, theta: torch.Tensor, g: ops.Geom, frames=None) -> torch.Tensor:
    """Differentiable y = A(theta) x; x [..., F, ny, nx] or [ny, nx] float32, theta float64."""
    if x.dim() == 2:
        return ProjectFn.apply(x.unsqueeze(0), theta, g, frames)
    return ProjectFn.apply(x, theta, g, frames)


class StreamingDataLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, b, g, block_off: Sequence[int]):
        ctx.g = g
        ctx.block_off = list(block_off)
        ctx.save_for_backward(x, theta, b)
        nb = g.nbins
        total = torch.zeros((), dtype=torch.float64, device=x.device)
        xs = x.contiguous().view(-1)
        for j in range(len(ctx.block_off) - 1):
            v0, v1 = ctx.block_off[j], ctx.block_off[j + 1]
            _, rn = ops.project_residual(xs, theta[v0:v1].contiguous(),
                                         b.view(-1, nb)[v0:v1].contiguous(), g, want_r=False)
            total = total + rn.sum()
        return 0.5 * total

    @staticmethod
    def backward(ctx, gl):
        x, theta, b = ctx.saved_tensors
        g = ctx.g
        nb = g.nbins
        xs = x.contiguous().view(-1)
        gx = torch.zeros_like(xs).view(1, 1, g.ny, g.nx)
        gth = torch.zeros_like(theta)
        for j in range(len(ctx.block_off) - 1):
            v0, v1 = ctx.block_off[j], ctx.block_off[j + 1]
            th = theta[v0:v1].contiguous()
            r, _ = ops.project_residual(xs, th, b.view(-1, nb)[v0:v1].contiguous(), g,
                                        want_rnorm2=False)
            res = ops.project_dtheta(xs, th, g, want_dy=False, gres=r, want_gdot=True)
            gth[v0:v1] = res["gdot"][0]
            ops.backproject_into(r, th, g, gx, accumulate=(j > 0))
        scale = gl.to(torch.float64)
        return (gx.view_as(x) * scale.to(x.dtype)), gth * scale, None, None, None


def streaming_data_loss(x, theta, b, g, block_off):
    """1/2 ||A(theta) x - b||^2 evaluated block by block without storing sinograms."""
    return StreamingDataLoss.apply(x, theta, b, g, block_off)
