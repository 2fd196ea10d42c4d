"""Conformal calibration on the GPU (Sec. 4.4) against the oracle: the
nonconformity scores of a synthetic calibration set of rope transitions
(one-step rollouts of 200 pairs in one launch), and the radius: the GPU
selects exactly the order statistic the oracle's rule selects on the same
FP32 scores, and its value is within tolerance of the oracle's FP64
radius; an infinite radius when the index exceeds n."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import conformal

pytestmark = pytest.mark.gpu


def test_cp_scores_and_radius_match_oracle():
    import torch
    from paper_2606_14188_amd import Sim, cp_radius
    cal = W.calibration_set(200, seed=1007)
    insts = [c[0] for c in cal]
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    s_next = sim.pack_states([np.concatenate([c[1].ravel(), np.zeros(3 * c[0].n)]) for c in cal])
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    sc = sim.cp_scores(s0, u, s_next, status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    got = sc.cpu().numpy().astype(np.float64)
    ref = conformal.scores(insts, [i.s0[:3 * i.n].reshape(-1, 3) for i in insts], [i.u[0] for i in insts],
                           [c[1] for c in cal])
    err = np.max(np.abs(got - ref) / ref)
    print(f"scores: max relative error {err:.2e}, range {ref.min():.3e}..{ref.max():.3e}", flush=True)
    assert err <= 1e-4
    for delta, T in ((0.1, 1), (0.2, 10), (0.05, 1), (0.5, 30)):
        r, idx = cp_radius(sc, delta, T)
        torch.cuda.synchronize()
        r, idx = float(r.item()), int(idx.item())
        r_or, k = conformal.radius(ref, delta, T)
        # the same rule on the GPU's own FP32 scores selects that score (bitwise)
        r_same, _ = conformal.radius(got, delta, T)
        print(f"delta {delta} T {T}: k {k} radius gpu {r:.6e} oracle {r_or:.6e}", flush=True)
        assert r == np.float32(r_same)
        assert idx >= 0 and got[idx] == r_same
        assert abs(r - r_or) <= 1e-4 * r_or
    r, idx = cp_radius(sc[:9], 0.05, 1)           # k = ceil(10 * 0.95) = 10 > 9
    torch.cuda.synchronize()
    assert math.isinf(r.item()) and int(idx.item()) == -1


@pytest.mark.parametrize("n", [1, 17, 10000, 65536])
def test_cp_radius_order_statistic_with_ties_and_nan(n):
    """The radius kernel on FP32 scores with many exact ties and 2 % NaN
    (a failed rollout's score orders last), up to the largest accepted n:
    the value the oracle's rule selects, and the index of that position in
    the order (score, index), NaN as +inf."""
    import torch
    from paper_2606_14188_amd import cp_radius
    rng = np.random.default_rng(1030 + n)
    s = np.round(rng.gamma(2.0, 1e-3, size=n), 5).astype(np.float32)
    if n > 1:
        s[rng.choice(n, size=max(1, n // 50), replace=False)] = np.nan
    dev = torch.from_numpy(s).cuda()
    key = np.where(np.isnan(s), np.inf, s.astype(np.float64))
    order = np.argsort(key, kind="stable")
    for delta, T in ((0.1, 1), (0.02, 1), (0.5, 2), (0.9, 1), (0.3, 30)):
        r, idx = cp_radius(dev, delta, T)
        torch.cuda.synchronize()
        r, idx = float(r.item()), int(idx.item())
        r_or, k = conformal.radius(s, delta, T)
        print(f"n {n} delta {delta} T {T}: k {k} radius gpu {r} oracle {r_or} index {idx}", flush=True)
        if k > n:
            assert math.isinf(r) and idx == -1
            continue
        assert idx == order[k - 1]
        assert (math.isnan(r) and math.isnan(r_or)) or r == np.float32(r_or)
