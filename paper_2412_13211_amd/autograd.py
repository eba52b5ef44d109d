"""Differentiable rollouts over the C ABI: ``torch.autograd.Function``.

Two ways to keep what the backward pass needs:

* ``records=True``: every forward step runs ``ms_step_record`` and keeps its
  record (substep states, contact lists, Gauss-Seidel tape; ``sizes.record``
  bytes per step, resident in device memory) and its start state; the
  backward pass chains ``ms_step_backward_recorded`` and runs no step again.
* ``records=False`` (checkpointing): the forward pass keeps only every k-th
  state; the backward pass recomputes the k states of a segment from its
  checkpoint and chains ``ms_step_backward`` through them (each call runs its
  control step again to record it).  Memory: T/k + k states.

Both give the same gradients bit for bit.
"""
from __future__ import annotations

import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, U, mb, every, records):
        T = U.shape[0]
        ctx.mb = mb
        ctx.records = bool(records)
        ctx.save_for_backward(U)
        x = x0.detach()
        if ctx.records:
            xs, recs = [], []
            for t in range(T):
                rec = mb.new_record()
                xs.append(x)
                x = mb.step_record(x, U[t].contiguous(), rec)
                recs.append(rec)
            ctx.xs, ctx.recs = xs, recs
            return x
        k = max(1, int(every))
        ckpt = {0: x.clone()}
        for t in range(T):
            x = mb.step(x, U[t].contiguous())
            if (t + 1) % k == 0 and t + 1 < T:
                ckpt[t + 1] = x.clone()
        ctx.k = k
        ctx.ckpt = ckpt
        return x

    @staticmethod
    def backward(ctx, gx):
        (U,) = ctx.saved_tensors
        mb = ctx.mb
        T = U.shape[0]
        gU = torch.zeros_like(U)
        g = gx.contiguous().clone()
        if ctx.records:
            for t in range(T - 1, -1, -1):
                g, gu = mb.step_backward_recorded(ctx.xs[t], U[t].contiguous(), ctx.recs[t], g, gx_in=g)
                gU[t].copy_(gu)
            ctx.xs = ctx.recs = None
            return g, gU, None, None, None
        k, ckpt = ctx.k, ctx.ckpt
        for s0 in reversed(sorted(ckpt.keys())):
            s1 = min(s0 + k, T)
            # recompute the states of the segment [s0, s1)
            xs = [ckpt[s0]]
            for t in range(s0, s1 - 1):
                xs.append(mb.step(xs[-1], U[t].contiguous()))
            for t in range(s1 - 1, s0 - 1, -1):
                g, gu = mb.step_backward(xs[t - s0], U[t].contiguous(), g, gx_in=g)
                gU[t].copy_(gu)
        return g, gU, None, None, None


def rollout(mb, x0, U, every=10, records=False):
    """Final state after ``U.shape[0]`` control steps from ``x0``;
    differentiable with respect to ``x0`` and ``U`` ([T, S, 16]).
    ``records=True`` keeps every step's record instead of checkpoints."""
    return _Rollout.apply(x0, U, mb, every, records)
