"""Reference planner: projected gradient descent on a batch of candidate
control sequences, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): the tests and the
benchmark's CPU baseline use it; the HIP library never does.

The paper obtains the nominal trajectory (z, v) of its SLS program (Sec. 4.2,
stage (1) of the decomposition) by gradient-based trajectory optimization
through the differentiable simulator (Sec. 1; Sec. 4.1 "Differentiating
Through Simulation"), but names neither the cost nor the update.  The
reading used here:

* cost  J(u) = |x_T[goal_node] - goal|^2 + u_reg * sum_t |u_t|^2,
  with x_T the final positions of a rollout from s0 under u (relaxation
  kappa_fwd);
* gradient  dJ/du = u_bar of the rollout's adjoint (relaxation kappa_bwd) for
  the terminal cotangent 2 (x_T[goal_node] - goal) on that node's position,
  plus 2 u_reg u;
* update  u <- clip(u - step * dJ/du, -u_max, u_max), componentwise, a fixed
  step per request (plain projected gradient descent);
* choice  after the last update every candidate is rolled out once more and
  the lowest J wins; ties go to the lowest candidate index.
"""
from __future__ import annotations

import numpy as np

from .derivatives import rollout_backward
from .step import rollout


def cost(inst, u, goal_node, goal, u_reg):
    """J(u) and the rollout it was evaluated on: (J, traj (T+1, n_s))."""
    u = np.asarray(u, dtype=np.float64).reshape(inst.T, inst.n_u)
    traj, _ = rollout(inst, s0=inst.s0, u=u)
    d = traj[-1, 3 * goal_node:3 * goal_node + 3] - np.asarray(goal, dtype=np.float64)
    return float(d @ d + u_reg * np.sum(u * u)), traj


def cost_gradient(inst, u, goal_node, goal, u_reg):
    """(J, dJ/du (T, n_u), traj): the terminal cotangent of J pulled back
    through the rollout's adjoint, plus the regulariser's gradient."""
    u = np.asarray(u, dtype=np.float64).reshape(inst.T, inst.n_u)
    J, traj = cost(inst, u, goal_node, goal, u_reg)
    d = traj[-1, 3 * goal_node:3 * goal_node + 3] - np.asarray(goal, dtype=np.float64)
    sT_bar = np.zeros(inst.n_s)
    sT_bar[3 * goal_node:3 * goal_node + 3] = 2.0 * d
    _, u_bar = rollout_backward(inst.replace(u=u), traj, sT_bar=sT_bar)
    return J, u_bar + 2.0 * u_reg * u, traj


def projected_step(u, grad, step, u_max):
    """One projected gradient step, clipped componentwise to [-u_max, u_max]."""
    return np.clip(np.asarray(u, dtype=np.float64) - step * np.asarray(grad, dtype=np.float64), -u_max, u_max)


def argmin_lowest(costs):
    """Index of the smallest cost; among equal costs the lowest index."""
    best = 0
    for c in range(1, len(costs)):
        if costs[c] < costs[best]:
            best = c
    return best


def plan(inst, u_init, goal_node, goal, iters, step, u_max, u_reg):
    """Run `iters` projected gradient steps on every candidate of
    u_init (C, T, n_u), then pick the winner.  Returns a dict with the final
    controls of every candidate, their costs, the winner's index, controls and
    trajectory."""
    u_all = [np.asarray(u0, dtype=np.float64).reshape(inst.T, inst.n_u).copy() for u0 in u_init]
    for _ in range(iters):
        for c in range(len(u_all)):
            _, g, _ = cost_gradient(inst, u_all[c], goal_node, goal, u_reg)
            u_all[c] = projected_step(u_all[c], g, step, u_max)
    costs, trajs = [], []
    for uc in u_all:
        J, tr = cost(inst, uc, goal_node, goal, u_reg)
        costs.append(J)
        trajs.append(tr)
    b = argmin_lowest(costs)
    return {"u": np.array(u_all), "costs": np.array(costs), "best": b, "u_best": u_all[b], "traj_best": trajs[b]}
