"""torch.autograd.Function over the library's rollout and its hand-written adjoint.

Forward runs stamp_rollout_fwd and keeps either the full tape or, with
``ckpt_every = K > 0``, one state every K steps of each push phase; backward runs
stamp_rollout_adj, which replays each K-step segment from its checkpoint into a
scratch buffer and reverses it (the gradient is bit-identical to the full-tape
adjoint).  Gradients flow to theta only; the scene and cost weights are
constants.  All work is on torch's current stream.
"""
from __future__ import annotations

import torch

from . import Context, CostW, Scene


class StampRollout(torch.autograd.Function):
    """cost = StampRollout.apply(theta [d][N] float32 cuda, ctx, scene, w, ckpt_every)."""

    @staticmethod
    def forward(fctx, theta: torch.Tensor, ctx: Context, scene: Scene, w: CostW, ckpt_every: int = 32):
        theta = theta.detach().contiguous()
        N = theta.shape[1]
        tape = torch.empty(Context.tape_floats(scene, N, ckpt_every), dtype=torch.float32, device=theta.device)
        cost = ctx.rollout_fwd(scene, w, theta, tape=tape, ckpt_every=ckpt_every)
        fctx.save_for_backward(theta, tape)
        fctx.stamp = (ctx, scene, w, ckpt_every)
        return cost

    @staticmethod
    def backward(fctx, cost_bar: torch.Tensor):
        theta, tape = fctx.saved_tensors
        ctx, scene, w, ckpt_every = fctx.stamp
        grad = ctx.rollout_adj(scene, w, theta, tape, ckpt_every=ckpt_every,
                               cost_bar=cost_bar.detach().to(torch.float32).contiguous())
        return grad, None, None, None, None


def rollout_cost(theta, ctx, scene, w, ckpt_every: int = 32):
    return StampRollout.apply(theta, ctx, scene, w, ckpt_every)


def tape_bytes(scene: Scene, N: int, ckpt_every: int) -> int:
    """Bytes the differentiation keeps between forward and backward (tape plus
    the segment replay buffer of the checkpointed mode)."""
    return 4 * Context.tape_floats(scene, N, ckpt_every) + Context.adj_workspace_bytes(scene, N, ckpt_every)
