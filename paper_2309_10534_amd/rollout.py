"""Differentiable multi-step rollouts with checkpointed recomputation.

A rollout advances W0 by n S2O4 steps, each with the CFL step of its state
computed on the device and recorded; the reverse pass holds those steps and
every stencil selection fixed (the selections are recomputed from the same
state bits, so they are the forward's).  Only every `every`-th state is kept;
the reverse pass recomputes the states of one segment at a time from its
checkpoint and runs tgks_step_adjoint backwards through it.  Memory: n/every
checkpoints plus every + 1 states of one segment.

Every step and every reverse step runs in the library's kernels; this module
only orders the calls.
"""
from __future__ import annotations

import torch

from . import tgks


def rollout(ctx, W0, n_steps, cfl=0.5, dts=None, every=20):
    """Advance a copy of W0.  dts: None (CFL steps, recorded) or a device
    tensor of n_steps fixed steps.  Returns (W_n, dts, checkpoints) with
    checkpoints[k] the state after k * every steps."""
    if every < 1:
        raise ValueError("every must be >= 1")
    W = W0.contiguous().clone()
    rec = dts is None
    if rec:
        dts = torch.zeros(n_steps, dtype=torch.float64, device=W.device)
    elif dts.numel() != n_steps or not dts.is_contiguous():
        raise ValueError("dts must hold n_steps contiguous values")
    ckpt = [W.clone()]
    nxt = torch.empty_like(W)
    for k in range(n_steps):
        dk = dts[k:k + 1]
        if rec:
            tgks.tgks_cfl_dt(ctx, W, cfl, 0.0, 0.0, dk)
        tgks.tgks_step(ctx, W, nxt, dk)
        W, nxt = nxt, W
        if (k + 1) % every == 0 and k + 1 < n_steps:
            ckpt.append(W.clone())
    return W, dts, ckpt


def rollout_adjoint(ctx, ckpt, dts, gW, every=20):
    """Cotangent of W0 given the cotangent gW of W_n (reverse of rollout)."""
    n_steps = dts.numel()
    g = gW.contiguous().clone()
    g2 = torch.empty_like(g)
    nseg = (n_steps + every - 1) // every
    for s in reversed(range(nseg)):
        k0, k1 = s * every, min((s + 1) * every, n_steps)
        # the segment's states and the intermediate states W* of its steps
        # (the last step's W* is recomputed by the reverse step itself)
        states, stars = [ckpt[s]], []
        for k in range(k0, k1 - 1):
            nxt, star = torch.empty_like(states[-1]), torch.empty_like(states[-1])
            tgks.tgks_step(ctx, states[-1], nxt, dts[k:k + 1], None, star)
            states.append(nxt)
            stars.append(star)
        stars.append(None)
        for k in reversed(range(k0, k1)):
            tgks.tgks_step_adjoint(ctx, states[k - k0], dts[k:k + 1], g, g2, W_star=stars[k - k0])
            g, g2 = g2, g
    return g


class GKSRollout(torch.autograd.Function):
    """W_n = GKSRollout.apply(W0, ctx, n_steps, cfl, every[, dts]) with a
    hand-written backward (checkpointed recomputation every `every` steps)."""

    @staticmethod
    def forward(fctx, W0, ctx, n_steps, cfl=0.5, every=20, dts=None):
        with torch.no_grad():
            W, dts_used, ckpt = rollout(ctx, W0, n_steps, cfl, dts, every)
        fctx.gks = (ctx, every)
        fctx.ckpt = ckpt
        fctx.dts = dts_used
        return W

    @staticmethod
    def backward(fctx, gW):
        ctx, every = fctx.gks
        with torch.no_grad():
            g0 = rollout_adjoint(ctx, fctx.ckpt, fctx.dts, gW, every)
        return g0, None, None, None, None, None
