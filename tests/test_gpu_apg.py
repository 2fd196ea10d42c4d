"""Analytical policy gradients on the GPU (Sec. 4.3) in the paper's
surrogate mode (hard-contact forward, smoothed gradients, penalty grippers
with smoothed activation) on the synthetic lift-rope task: the policy
gradient of a closed-loop rollout through libcord against the same rollout
through the oracle's step (FP64), and a short training run that lowers the
task loss."""
import numpy as np
import pytest

import workloads as W
from oracle.apg import lift_objective
from tests.parity import GRAD_TOL, rel_l2

pytestmark = pytest.mark.gpu


def test_policy_gradient_matches_oracle():
    import torch
    from paper_2606_14188_amd import Sim
    from paper_2606_14188_amd.apg import MLPPolicy, lift_loss, policy_rollout, sim_step
    torch.manual_seed(3)
    n, T, h, umax = 12, 10, 0.02, 0.5
    insts = W.lift_rope_envs(4, n=n, seed=1010)
    sim = Sim(insts)
    policy = MLPPolicy(u_max=umax).to(sim.device)
    s0 = sim.pack_states([i.s0 for i in insts]).reshape(len(insts), -1)
    sT, us = policy_rollout(sim_step(sim), policy, s0, n, T)
    loss = lift_loss(sT, us, n, h)
    loss.backward()
    torch.cuda.synchronize()
    params = [p.detach().cpu().double().clone().requires_grad_(True)
              for p in (policy.l1.weight, policy.l1.bias, policy.l2.weight, policy.l2.bias)]
    ref = lift_objective(insts, params, torch.from_numpy(np.stack([i.s0 for i in insts])), n, T, h, umax)
    ref.backward()
    print(f"loss gpu {loss.item():.8e} oracle {ref.item():.8e}", flush=True)
    assert abs(loss.item() - ref.item()) <= 1e-4 * ref.item()
    for name, p, q in zip(["W1", "b1", "W2", "b2"],
                          (policy.l1.weight, policy.l1.bias, policy.l2.weight, policy.l2.bias), params):
        e = rel_l2(p.grad.cpu().numpy(), q.grad.numpy())
        print(f"dL/d{name}: relative error {e:.2e}", flush=True)
        assert e <= GRAD_TOL


def test_policy_training_lowers_the_loss():
    import torch
    from paper_2606_14188_amd import Sim
    from paper_2606_14188_amd.apg import MLPPolicy, train
    torch.manual_seed(4)
    n, T, h = 12, 20, 0.02
    insts = W.lift_rope_envs(64, n=n, seed=1011)
    sim = Sim(insts)
    policy = MLPPolicy(u_max=0.5).to(sim.device)
    s0 = sim.pack_states([i.s0 for i in insts]).reshape(len(insts), -1)
    losses = train(sim, policy, s0, n, T, h, iters=40, lr=1e-2)
    print("losses", [f"{x:.3e}" for x in losses[::5]], losses[-1], flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] <= 0.5 * losses[0]
