"""The oracle's step as a differentiable layer, for analytical policy
gradients (Sec. 4.3) in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward: q+ = f_{kappa_fwd}(q, u) by the oracle's step; backward: the VJP of
f_{kappa_bwd} at the same (q, u) (eq. diff-sim), i.e. the paper's surrogate
gradient when kappa_fwd = 0 < kappa_bwd and the exact gradient when they are
equal.  Any torch policy and loss can then be differentiated through a
closed-loop rollout with torch's own reverse mode.
"""
from __future__ import annotations

import numpy as np
import torch

from . import model
from .derivatives import StepDerivative
from .step import Layout, split_state, step


class OracleStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, u, insts):
        ctx.insts = insts
        ctx.save_for_backward(s, u)
        out = torch.zeros_like(s)
        for b, inst in enumerate(insts):
            sb = s[b].detach().numpy()
            x, v, g = split_state(inst, sb)
            r = step(inst, x, v, u[b].detach().numpy(), inst.kappa_fwd, model.elements(inst), Layout(inst), g=g)
            n = inst.n
            nxt = np.concatenate([r.x.ravel(), r.v.ravel()] + ([r.g.ravel()] if r.g is not None else []))
            out[b] = torch.from_numpy(nxt)
        return out

    @staticmethod
    def backward(ctx, gout):
        s, u = ctx.saved_tensors
        sbar = torch.zeros_like(s)
        ubar = torch.zeros_like(u)
        for b, inst in enumerate(ctx.insts):
            d = StepDerivative(inst, s[b].detach().numpy(), u[b].detach().numpy(), inst.kappa_bwd)
            a, c = d.vjp_s(gout[b].detach().numpy())
            sbar[b] = torch.from_numpy(a)
            ubar[b] = torch.from_numpy(c)
        return sbar, ubar, None


def oracle_step(insts):
    """step(s, u) for batches (B, n_s), (B, n_u) of float64 CPU tensors."""
    def f(s, u):
        return OracleStep.apply(s, u, insts)
    return f


# ---------------------------------------------------------------- lift task, written out plainly
def lift_features(s, n, t, T):
    """Policy input of the lift task for states s (B, n_s) = [x | v | g0 g1]
    (grippers of nodes 0 and n-1): per environment the two gripper-to-node
    offsets, the two gripper heights, the two end-node heights, the mean
    node height and t / T (12 numbers)."""
    rows = []
    for b in range(s.shape[0]):
        x = s[b, :3 * n].reshape(n, 3)
        g = s[b, 6 * n:6 * n + 6].reshape(2, 3)
        f = [g[0] - x[0], g[1] - x[n - 1], g[:, 2], torch.stack([x[0, 2], x[n - 1, 2]]),
             x[:, 2].mean().reshape(1), torch.tensor([t / T], dtype=s.dtype)]
        rows.append(torch.cat(f))
    return torch.stack(rows)


def mlp(params, o, u_max):
    """u = u_max tanh(W2 tanh(W1 o + b1) + b2), params = (W1, b1, W2, b2)."""
    W1, b1, W2, b2 = params
    return u_max * torch.tanh(torch.tanh(o @ W1.T + b1) @ W2.T + b2)


def lift_objective(insts, params, s0, n, T, height, u_max, u_weight=1e-4):
    """The lift task's loss of a closed-loop rollout through the oracle:
    mean squared end-node height error at T plus the control penalty."""
    f = oracle_step(insts)
    s = s0
    pen = 0.0
    for t in range(T):
        u = mlp(params, lift_features(s, n, t, T), u_max)
        pen = pen + (u * u).sum(1).mean()
        s = f(s, u)
    x = s[:, :3 * n].reshape(-1, n, 3)
    e0 = x[:, 0, 2] - height
    e1 = x[:, n - 1, 2] - height
    return (e0 * e0 + e1 * e1).mean() + u_weight * pen
