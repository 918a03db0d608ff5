"""torch.autograd.Function over sq_build_index and the one-scene forward and
backward of the batched ABI (api.render_train_fwd / render_train_bwd: the
checkpoints, the per-tile stops and, given an api.StashPool, the per-sample
stash).

The index is rebuilt inside forward from the current means and is not
differentiated (the voxel lists are piecewise constant in m); gradients reach
m only through the occupancy p_o (Sec. 3.3 "Backward Pass")."""
from __future__ import annotations

import torch

from . import api


class SQRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every=8,
                tuning=None, stash=None):
        prims = api.Prims(*(t.contiguous() for t in (means, quats, scales, eps, opacity, logits)))
        rays = api.Rays(origins.contiguous(), dirs.contiguous())
        index = api.build_index(grid, prims)
        st = api.render_train_fwd(grid, index, prims, rays, march, ckpt_every=ckpt_every, tuning=tuning,
                                  stash=stash)
        # the state holds the inputs, checkpoints, stops and stash until
        # backward; the inputs are also saved so that autograd catches an
        # in-place change to them before then
        ctx.st = st
        ctx.save_for_backward(*(getattr(prims, k) for k in ("means", "quats", "scales", "eps", "opacity", "logits")),
                              rays.origins, rays.dirs)
        return st["depth"], st["sem"]

    @staticmethod
    def backward(ctx, g_depth, g_sem):
        ctx.saved_tensors  # (the version check)
        gd = None if g_depth is None else g_depth.contiguous().float()
        gs = None if g_sem is None else g_sem.contiguous().float()
        g = api.render_train_bwd(ctx.st, gd, gs)
        ctx.st = None
        return (g["means"], g["quats"], g["scales"], g["eps"], g["opacity"], g["logits"],
                None, None, None, None, None, None, None)


def render(means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every=8, tuning=None,
           stash=None):
    """Differentiable (depth [cams,H,W], sem [cams,C,H,W]).  `stash`: an
    api.StashPool to reuse across steps (the backward then skips its
    recompute pass); None renders without one."""
    return SQRenderFn.apply(means, quats, scales, eps, opacity, logits, origins, dirs, grid, march, ckpt_every,
                            tuning, stash)
