"""Pin of the oracle's differentiable step (Sec. 4.3 analytical policy
gradients): with the smoothed forward (kappa_fwd = kappa_bwd) the policy
gradient of a closed-loop lift-rope rollout through the oracle equals
central differences of the loss in the policy parameters."""
import numpy as np
import torch

import workloads as W
from oracle.apg import lift_objective


def test_policy_gradient_matches_central_differences():
    torch.manual_seed(0)
    insts = W.lift_rope_envs(2, n=5, seed=21)
    insts = [i.replace(kappa_fwd=i.kappa_bwd) for i in insts]
    n, T, h, umax = 5, 3, 0.02, 0.5
    params = [torch.randn(8, 12, dtype=torch.float64) * 0.3, torch.randn(8, dtype=torch.float64) * 0.1,
              torch.randn(6, 8, dtype=torch.float64) * 0.3, torch.randn(6, dtype=torch.float64) * 0.1]
    for p in params:
        p.requires_grad_(True)
    s0 = torch.from_numpy(np.stack([i.s0 for i in insts]))
    L = lift_objective(insts, params, s0, n, T, h, umax)
    L.backward()
    rng = np.random.default_rng(1)
    hstep = 1e-6
    for pi, p in enumerate(params):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, d)) for d in p.shape)
            with torch.no_grad():
                old = p[idx].item()
                p[idx] = old + hstep
                lp = lift_objective(insts, params, s0, n, T, h, umax).item()
                p[idx] = old - hstep
                lm = lift_objective(insts, params, s0, n, T, h, umax).item()
                p[idx] = old
            fd = (lp - lm) / (2 * hstep)
            g = p.grad[idx].item()
            assert abs(g - fd) <= 1e-5 * max(abs(fd), 1e-6) + 1e-9, (pi, idx, g, fd)
