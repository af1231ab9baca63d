"""Occupancy loss with gradients for calibration and background refinement.

``occupancy_loss`` wraps the library's differentiable forward (bilinear
sampling of every view's log(2*SLM) map at the projected voxel centres, mean
binary cross-entropy with logits against 0/1 labels) and its hand-written
adjoint in a ``torch.autograd.Function``. Gradients flow to the background
means and variances of every view and to the 3x4 camera matrices; images and
labels get none. Projections are recomputed in the backward, not stored.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _lib as L
from .api import LOG_U_DEFAULT, Plan


class _View:
    def __init__(self, width, height, P):
        self.width, self.height, self.P = width, height, P


class OccupancyLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, plan, images, labels, sub, *bg):
        n = len(images)
        means, vars_ = bg[:n], bg[n:]
        Ph = P.detach().to("cpu", torch.float32).numpy().reshape(n, 3, 4).copy()
        cams = [_View(c.width, c.height, Ph[k]) for k, c in enumerate(plan.sizes)]
        bg_m, bg_v = [m.detach() for m in means], [v.detach() for v in vars_]
        plan.set_cameras(cams)
        plan.set_backgrounds(bg_m, bg_v)
        logits, loss, ws = plan.diff_forward(images, labels, sub)
        # The plan is shared: another forward may re-set its cameras and
        # backgrounds before this backward runs, so keep this call's own
        # (host FP32 matrices, the background tensors) and re-set them there.
        ctx.plan, ctx.images, ctx.sub, ctx.ws = plan, images, sub, ws
        ctx.cams, ctx.bg = cams, (bg_m, bg_v)
        ctx.p_device = P.device
        ctx.save_for_backward(labels, logits)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        labels, logits = ctx.saved_tensors
        ctx.plan.set_cameras(ctx.cams)
        ctx.plan.set_backgrounds(*ctx.bg)
        gmeans, gvars, gP = ctx.plan.diff_backward(ctx.images, labels, logits, grad_loss, ctx.ws, ctx.sub)
        return (gP.to(ctx.p_device), None, None, None, None, *gmeans, *gvars)


class DiffPlan(Plan):
    """A plan whose cameras are re-set from a parameter tensor on each call."""

    def __init__(self, sizes: Sequence, grid, prior=0.5, log_u=LOG_U_DEFAULT):
        super().__init__(None, grid, prior=prior, log_u=log_u, sampling=L.BILINEAR)
        self.sizes = list(sizes)


def occupancy_loss(P: torch.Tensor, means: Sequence[torch.Tensor], vars_: Sequence[torch.Tensor],
                   images: Sequence[torch.Tensor], labels: torch.Tensor, plan: DiffPlan,
                   sub: Optional[Sequence[int]] = None) -> torch.Tensor:
    """Mean BCE-with-logits occupancy loss; differentiable in P ([n][3][4]),
    means and variances (each [H][W][3], on the GPU)."""
    if P.shape != (len(images), 3, 4):
        raise ValueError(f"P must be [{len(images)}, 3, 4], got {tuple(P.shape)}")
    return OccupancyLoss.apply(P, plan, list(images), labels, None if sub is None else list(sub),
                               *means, *vars_)
