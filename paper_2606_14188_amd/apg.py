"""Analytical policy gradients (APG) through the simulator (Sec. 4.3,
"Accelerating Model-Based RL via Analytical Policy Gradients").

A control policy is trained by differentiating the task loss through the
contact-smoothed simulator used as a differentiable layer (eq. diff-sim):
the policy closes the loop between steps, every step is one launch of the
batched rollout kernel over all environments (a simulator of B instances
with T = 1, in `CordRollout`'s final-state mode), and the backward pass
runs the adjoint kernel step by step in reverse.  In the paper's mode the
forward dynamics are the nonsmooth ones (kappa_fwd = 0) and the gradients
those of the smoothed model (kappa_bwd > 0).

The policy and the loss are small torch modules on the device; the
simulation, its adjoint and its smoothing run in libcord's kernels.

Task used here (the paper's lift-rope task, synthetic): two penalty
grippers (smoothed activation, so the gradient pulls them into contact)
must lift the end nodes of a rope lying on the ground to a target height.
"""
from __future__ import annotations

import torch

from .autograd import rollout


def lift_observation(s, n, t, T):
    """Features of states s (B, n_s) with s = [x | v | g_0 g_1], grippers
    for nodes 0 and n - 1: gripper-node offsets (6), gripper heights (2),
    end-node heights (2), mean rope height (1), time (1)."""
    x = s[:, :3 * n].reshape(-1, n, 3)
    g = s[:, 6 * n:6 * n + 6].reshape(-1, 2, 3)
    ends = torch.stack([x[:, 0], x[:, n - 1]], dim=1)
    tt = torch.full((s.shape[0], 1), t / T, dtype=s.dtype, device=s.device)
    return torch.cat([(g - ends).reshape(-1, 6), g[:, :, 2], ends[:, :, 2], x[:, :, 2].mean(1, keepdim=True), tt],
                     dim=1)


class MLPPolicy(torch.nn.Module):
    """u = u_max tanh(W2 tanh(W1 o + b1) + b2)."""

    def __init__(self, n_obs=12, n_hidden=32, n_u=6, u_max=0.5):
        super().__init__()
        self.l1 = torch.nn.Linear(n_obs, n_hidden)
        self.l2 = torch.nn.Linear(n_hidden, n_u)
        self.u_max = u_max

    def forward(self, o):
        return self.u_max * torch.tanh(self.l2(torch.tanh(self.l1(o))))


def lift_loss(sT, us, n, height, u_weight=1e-4):
    """Mean over environments of the squared height errors of the two end
    nodes at the final step plus a small control penalty."""
    x = sT[:, :3 * n].reshape(-1, n, 3)
    err = torch.stack([x[:, 0, 2], x[:, n - 1, 2]], dim=1) - height
    return (err * err).sum(1).mean() + u_weight * sum((u * u).sum(1).mean() for u in us)


def policy_rollout(step, policy, s0, n, T):
    """Closed-loop rollout: `step(s, u)` advances the batch (B, n_s) by one
    step under controls (B, n_u).  Returns the final state and the controls."""
    s = s0
    us = []
    for t in range(T):
        u = policy(lift_observation(s, n, t, T))
        us.append(u)
        s = step(s, u)
    return s, us


def sim_step(sim):
    """One differentiable step of every environment through libcord (the
    simulator's instances have T = 1)."""
    B = sim.B

    def step(s, u):
        return rollout(sim, s.reshape(-1), u.reshape(-1), mode="final").reshape(B, -1)
    return step


def train(sim, policy, s0, n, T, height, iters=40, lr=1e-2):
    """Adam on the policy's parameters with the analytical policy gradient.
    Returns the loss of every iteration."""
    opt = torch.optim.Adam(policy.parameters(), lr=lr)
    step = sim_step(sim)
    losses = []
    for _ in range(iters):
        opt.zero_grad()
        sT, us = policy_rollout(step, policy, s0, n, T)
        loss = lift_loss(sT, us, n, height)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    return losses
