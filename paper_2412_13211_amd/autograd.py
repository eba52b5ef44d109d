"""Differentiable rollouts over the C ABI: ``torch.autograd.Function`` with
checkpointing.

The forward pass runs T control steps (``ms_step``) and keeps only every
k-th state.  The backward pass walks the segments in reverse: it recomputes
the k states of a segment from its checkpoint, then chains
``ms_step_backward`` through them (each call itself recomputes the substeps
of its control step).  Memory: T/k + k states instead of T.
"""
from __future__ import annotations

import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, U, mb, every):
        T = U.shape[0]
        k = max(1, int(every))
        ckpt = {0: x0.detach().clone()}
        x = x0.detach()
        for t in range(T):
            x = mb.step(x, U[t].contiguous())
            if (t + 1) % k == 0 and t + 1 < T:
                ckpt[t + 1] = x.clone()
        ctx.mb = mb
        ctx.k = k
        ctx.ckpt = ckpt
        ctx.save_for_backward(U)
        return x

    @staticmethod
    def backward(ctx, gx):
        (U,) = ctx.saved_tensors
        mb, k, ckpt = ctx.mb, ctx.k, ctx.ckpt
        T = U.shape[0]
        gU = torch.zeros_like(U)
        g = gx.contiguous().clone()
        starts = sorted(ckpt.keys())
        for s0 in reversed(starts):
            s1 = min(s0 + k, T)
            # recompute the states of the segment [s0, s1)
            xs = [ckpt[s0]]
            for t in range(s0, s1 - 1):
                xs.append(mb.step(xs[-1], U[t].contiguous()))
            for t in range(s1 - 1, s0 - 1, -1):
                g, gu = mb.step_backward(xs[t - s0], U[t].contiguous(), g, gx_in=g)
                gU[t].copy_(gu)
        return g, gU, None, None


def rollout(mb, x0, U, every=10):
    """Final state after ``U.shape[0]`` control steps from ``x0``;
    differentiable with respect to ``x0`` and ``U`` ([T, S, 16])."""
    return _Rollout.apply(x0, U, mb, every)
