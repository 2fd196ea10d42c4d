"""The checkpointed adjoint without device allocation
(cord_rollout_backward_noalloc), called through the C ABI: bitwise the
outputs of cord_rollout_backward on two calls in a row, the second on a
smaller batch (the static scratch keeps the first call's contents), in
checkpointed and full storage; a request beyond the scratch's 64 MiB is
refused with CORD_ETOOBIG."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _call_noalloc(sim, u, traj, sT, store, K):
    import torch
    from paper_2606_14188_amd import _lib as L
    from paper_2606_14188_amd.api import _ptr, _stream
    s0_bar = torch.full((sim.info.s_floats,), float("nan"), dtype=torch.float32, device=sim.device)
    u_bar = torch.full((max(sim.info.u_floats, 1),), float("nan"), dtype=torch.float32, device=sim.device)
    o = L.BackwardOpts()
    o.store, o.ckpt_every = store, K
    o.sT_bar = _ptr(sT)
    rc = sim.lib.cord_rollout_backward_noalloc(sim._h, _ptr(u), _ptr(traj), None, _ptr(s0_bar), _ptr(u_bar), None,
                                               ctypes.byref(o), _stream())
    return rc, s0_bar, u_bar[:sim.info.u_floats]


def _case(insts, seed):
    import torch
    from paper_2606_14188_amd import Sim, _lib as L
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([W.random_cotangent(i.n_s, seed + j) for j, i in enumerate(insts)])
    full = sim.rollout(s0, u)
    for store, K in ((L.STORE_CKPT, 7), (L.STORE_CKPT, 1), (L.STORE_FULL, 1)):
        traj = sim.rollout(s0, u, store=L.STORE_CKPT, ckpt_every=K) if store == L.STORE_CKPT else full
        ref = sim.backward(u, traj, sT_bar=sT, store=store, ckpt_every=K)
        rc, s0b, ub = _call_noalloc(sim, u, traj, sT, store, K)
        torch.cuda.synchronize()
        assert rc == L.CORD_OK, sim.lib.cord_last_error()
        print(f"{len(insts)} instances store={store} K={K}: bitwise", flush=True)
        assert torch.equal(s0b, ref[0]) and torch.equal(ub, ref[1])


def test_noalloc_backward_matches_and_second_call_smaller():
    big = W.small_rope_batch(6, 64, 23, seed=1501) + W.small_cloth_batch(2, 9, 7, 23, seed=1502) \
        + W.small_rope_batch(2, 130, 12, seed=1503)
    small = W.small_rope_batch(2, 20, 9, seed=1504)
    _case(big, 1600)
    _case(small, 1700)


def test_noalloc_refuses_beyond_the_scratch():
    import torch
    from paper_2606_14188_amd import Sim, _lib as L
    insts = W.small_cloth_batch(8, 48, 48, 3, seed=1505)      # 8 x 13824 floats x K = 200 -> 88 MB
    sim = Sim(insts)
    u = sim.pack_controls([i.u for i in insts])
    traj = torch.zeros(sim.ckpt_floats(200), dtype=torch.float32, device=sim.device)
    sT = torch.zeros(sim.info.s_floats, dtype=torch.float32, device=sim.device)
    rc, _, _ = _call_noalloc(sim, u, traj, sT, L.STORE_CKPT, 200)
    assert rc == L.CORD_ETOOBIG
    assert b"scratch" in sim.lib.cord_last_error()
