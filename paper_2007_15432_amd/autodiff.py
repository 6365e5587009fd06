"""Differentiable soft kick and a checkpointed leapfrog built on it.

SoftKick is the soft kick v' = v + h a_soft(x, m) of the P3T splitting (eq.
(HamiltonSol)) as a torch.autograd.Function whose backward is the library's
hand-written adjoint (p3t_soft_kick_adjoint): the pair cut-offs r_out and the
tree's interaction lists are held fixed, which is what the forward computes
for a given state.  The forward and the backward both rebuild the tree from
the saved state, so a backward long after its forward (or inside a
checkpointed recomputation) still sees exactly the forward's lists.

leapfrog() integrates kick-drift-kick steps in which the soft kicks go
through SoftKick and the central star's kick and the drift are plain torch
operations; with checkpoint_every = k only every k-th state is kept and each
segment is recomputed during the backward pass.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

__all__ = ["SoftKick", "soft_kick", "star_acc", "leapfrog"]


class SoftKick(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, v, m, r_out, r_search, ctx, h):
        x, v, m = x.detach().contiguous(), v.detach().contiguous(), m.detach().contiguous()
        ctx.build_tree(x, v, m, r_out, r_search)
        a = ctx.compute_soft_force()
        fctx.save_for_backward(x, v, m, r_out, r_search)
        fctx.ctx, fctx.h = ctx, float(h)
        return v + fctx.h * a

    @staticmethod
    def backward(fctx, g_v):
        x, v, m, r_out, r_search = fctx.saved_tensors
        c = fctx.ctx
        # same state -> same tree and lists as the forward
        c.build_tree(x, v, m, r_out, r_search)
        c.compute_soft_force()
        gx, gm = c.soft_kick_adjoint(g_v.contiguous(), fctx.h)
        return gx, g_v, gm, None, None, None, None


def soft_kick(x, v, m, r_out, r_search, ctx, h):
    return SoftKick.apply(x, v, m, r_out, r_search, ctx, h)


def star_acc(x, GM: float = 1.0):
    """Acceleration from the central star, -GM x / |x|^3 (torch ops)."""
    r2 = (x * x).sum(0, keepdim=True)
    return -GM * x * r2.rsqrt() / r2


def _kdk(x, v, m, r_out, r_search, ctx, h, GM, steps):
    for _ in range(steps):
        v = soft_kick(x, v, m, r_out, r_search, ctx, 0.5 * h)
        v = v + (0.5 * h) * star_acc(x, GM)
        x = x + h * v
        v = v + (0.5 * h) * star_acc(x, GM)
        v = soft_kick(x, v, m, r_out, r_search, ctx, 0.5 * h)
    return x, v


def leapfrog(x, v, m, r_out, r_search, ctx, h: float, n_steps: int, checkpoint_every: int = 0, GM: float = 1.0):
    """n_steps kick-drift-kick steps of size h; returns (x, v).  With
    checkpoint_every = k > 0 the steps run in segments of k whose inner
    states are recomputed in the backward pass."""
    if checkpoint_every <= 0:
        return _kdk(x, v, m, r_out, r_search, ctx, h, GM, n_steps)
    done = 0
    while done < n_steps:
        k = min(checkpoint_every, n_steps - done)
        x, v = checkpoint(_kdk, x, v, m, r_out, r_search, ctx, h, GM, k, use_reentrant=False)
        done += k
    return x, v
