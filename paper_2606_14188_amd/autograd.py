"""torch.autograd.Function over libcord's rollout and adjoint kernels.

Two output modes of `rollout(sim, s0, u, ...)`:

* ``mode="full"``  -> the whole trajectory (flat, sum (T+1) n_s); the
  backward pass reads the stored states.
* ``mode="final"`` -> only s_T (flat, sum n_s); the forward pass keeps one
  checkpoint every ``ckpt_every`` steps and the backward kernel recomputes
  each segment from its checkpoint (bitwise equal to the stored states).

The backward pass is the implicit-differentiation adjoint of the paper's
eq. (diff-sim), evaluated in libcord's kernels.
"""
from __future__ import annotations

import torch

from . import _lib as L


class CordRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, s0, u, mode: str = "full", ckpt_every: int = 10):
        s0c = s0.detach().contiguous()
        uc = u.detach().contiguous()
        ctx.sim = sim
        ctx.mode = mode
        ctx.ckpt_every = ckpt_every
        if mode == "full":
            traj = sim.rollout(s0c, uc, store=L.STORE_FULL)
            # the step internals this rollout wrote serve its backward only
            # while no later FULL rollout has overwritten them
            ctx.aux_gen = sim.aux_generation()
            ctx.save_for_backward(uc, traj)
            return traj
        if mode != "final":
            raise ValueError("mode must be 'full' or 'final'")
        sT = torch.empty(sim.info.s_floats, dtype=torch.float32, device=s0c.device)
        ck = sim.rollout(s0c, uc, store=L.STORE_CKPT, ckpt_every=ckpt_every, final_state=sT)
        ctx.save_for_backward(uc, ck)
        return sT

    @staticmethod
    def backward(ctx, g):
        u, saved = ctx.saved_tensors
        sim = ctx.sim
        g = g.contiguous()
        if ctx.mode == "full":
            with sim.aux_if_current(ctx.aux_gen):
                s0_bar, u_bar = sim.backward(u, saved, traj_bar=g, store=L.STORE_FULL)
        else:
            s0_bar, u_bar = sim.backward(u, saved, sT_bar=g, store=L.STORE_CKPT, ckpt_every=ctx.ckpt_every)
        return None, s0_bar, u_bar, None, None


def rollout(sim, s0, u, mode: str = "full", ckpt_every: int = 10):
    """Differentiable rollout through libcord (see module docstring)."""
    return CordRollout.apply(sim, s0, u, mode, ckpt_every)
