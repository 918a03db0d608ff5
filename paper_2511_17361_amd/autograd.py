"""torch.autograd.Function over sq_build_index / sq_render_fwd / sq_render_bwd.

The index is rebuilt inside forward from the current means and is not
differentiated (the voxel lists are piecewise constant in m); gradients reach
m only through the occupancy p_o (Sec. 3.3 "Backward Pass")."""
from __future__ import annotations

import torch

from . import api


class SQRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every=8,
                tuning=None):
        prims = api.Prims(*(t.contiguous() for t in (means, quats, scales, eps, opacity, logits)))
        rays = api.Rays(origins.contiguous(), dirs.contiguous())
        index = api.build_index(grid, prims)
        out = api.render_fwd(grid, index, prims, rays, march, ckpt_every=ckpt_every, probs=False, tuning=tuning)
        ctx.grid, ctx.march, ctx.ckpt_every, ctx.tuning = grid, march, ckpt_every, tuning
        ctx.index = index
        ctx.save_for_backward(*(getattr(prims, k) for k in ("means", "quats", "scales", "eps", "opacity", "logits")),
                              rays.origins, rays.dirs, out["ckpt"])
        return out["depth"], out["sem"]

    @staticmethod
    def backward(ctx, g_depth, g_sem):
        means, quats, scales, eps, opacity, logits, origins, dirs, ckpt = ctx.saved_tensors
        prims = api.Prims(means, quats, scales, eps, opacity, logits)
        rays = api.Rays(origins, dirs)
        gd = None if g_depth is None else g_depth.contiguous().float()
        gs = None if g_sem is None else g_sem.contiguous().float()
        g = api.render_bwd(ctx.grid, ctx.index, prims, rays, ctx.march, ckpt, ctx.ckpt_every, gd, gs,
                           tuning=ctx.tuning)
        return (g["means"], g["quats"], g["scales"], g["eps"], g["opacity"], g["logits"],
                None, None, None, None, None, None)


def render(means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every=8, tuning=None):
    """Differentiable (depth [cams,H,W], sem [cams,C,H,W])."""
    return SQRenderFn.apply(means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every,
                            tuning)
