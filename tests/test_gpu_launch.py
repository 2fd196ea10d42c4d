"""Launch modes (grouped, per instance, persistent work queue, hipGraph),
repeated graph replays, autotuner and a mixed uneven batch (C4-style)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.step import rollout as orollout
from tests.parity import GRAD_TOL, JAC_TOL, STATE_TOL, check, gradient_block_errors, state_errors, tangent_block_errors

pytestmark = pytest.mark.gpu


def _mixed(seed=600):
    insts = []
    for j, n in enumerate((16, 40, 100, 200)):
        insts += W.small_rope_batch(2, n, 12 + 3 * j, seed=seed + j)
    for j, side in enumerate((5, 10, 20, 32)):
        insts += W.small_cloth_batch(1, side, side, 10 + 2 * j, seed=seed + 10 + j)
    return insts


def _setup(insts):
    import torch
    from paper_2606_14188_amd import Sim
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([W.random_cotangent(i.n_s, 40 + j) for j, i in enumerate(insts)])
    return sim, s0, u, sT


def test_launch_modes_bitwise():
    import torch
    from paper_2606_14188_amd import _lib as L
    insts = _mixed()
    sim, s0, u, sT = _setup(insts)
    print("classes", sim.classes())
    ref = sim.rollout(s0, u)
    rb = sim.backward(u, ref, sT_bar=sT)
    torch.cuda.synchronize()
    for mode in (L.LAUNCH_PER_INSTANCE, L.LAUNCH_PERSISTENT, L.LAUNCH_GRAPH):
        sim.set_launch(mode)
        for rep in range(2):
            tr = sim.rollout(s0, u)
            b = sim.backward(u, tr, sT_bar=sT)
            torch.cuda.synchronize()
            assert torch.equal(tr, ref), (mode, rep)
            assert torch.equal(b[0], rb[0]) and torch.equal(b[1], rb[1]), (mode, rep)


def test_graph_replays_with_eager_work_between():
    import torch
    from paper_2606_14188_amd import _lib as L
    insts = _mixed(seed=700)
    sim, s0, u, sT = _setup(insts)
    eager = sim.rollout(s0, u).clone()
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    out = torch.empty_like(eager)
    sim.set_launch(L.LAUNCH_GRAPH)
    for rep in range(4):
        out.fill_(float("nan"))            # eager work between replays
        sim.rollout(s0, u, out=out, status=st)
        x = torch.randn(1 << 20, device=sim.device).sum()   # more eager work
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert (st.cpu().numpy() == 0).all()
        st.fill_(-1)


def test_autotune_and_cache(tmp_path):
    import torch
    insts = _mixed(seed=800)
    sim, s0, u, sT = _setup(insts)
    path = str(tmp_path / "tune.json")
    cls = sim.autotune(s0, u, sample=8, cache_path=path)
    print("tuned", cls)
    data = json.load(open(path))
    assert len(data["entries"]) == len(cls)
    # the chosen configurations still match the oracle
    tr = sim.rollout(s0, u)
    torch.cuda.synchronize()
    parts = sim.split(tr, "traj")
    for i in (0, 5, 8):
        ref, _ = orollout(insts[i])
        ex, ev = state_errors(parts[i], ref, insts[i].n)
        assert ex <= STATE_TOL and ev <= STATE_TOL, (i, ex, ev)
    # a second simulator reads the cache and picks the same configurations
    sim2, *_ = _setup(insts)
    cls2 = sim2.autotune(s0, u, sample=8, cache_path=path)
    assert cls2 == cls


def test_c4_mixed_batch_graph():
    """4096 uneven instances (ropes 16..256 nodes, cloths 8x8..48x48, T
    30..120) in one graph launch; sampled instances against the oracle, and
    one instance alone vs inside the mix (bitwise)."""
    import torch
    from paper_2606_14188_amd import _lib as L, Sim
    insts = W.config_c4()
    sim, s0, u, sT = _setup(insts)
    sim.set_launch(L.LAUNCH_GRAPH)
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    tr = sim.rollout(s0, u, status=st)
    b = sim.backward(u, tr, sT_bar=sT)
    torch.cuda.synchronize()
    stc = st.cpu().numpy()
    print("classes", sim.classes(), "status", np.bincount(stc, minlength=5))
    assert (stc == 0).all()
    parts = sim.split(tr, "traj")
    s0p, up = sim.split(b[0], "s"), sim.split(b[1], "u")
    cots = sim.split(sT, "s")
    order = sorted(range(len(insts)), key=lambda i: insts[i].n * insts[i].T)
    ropes = [i for i in order if insts[i].kind == "rope"]
    cloths = [i for i in order if insts[i].kind == "cloth"]
    # across the n T range: the smallest, a middle one and the largest rope
    # (256 nodes, 119 steps); the smallest and a middle cloth and the
    # largest cloth the oracle finishes in about a minute (47 x 47 nodes
    # over 34 steps; a 48 x 48 cloth over 60 or more steps would take it
    # several minutes)
    big = max((i for i in cloths if insts[i].T <= 35), key=lambda i: insts[i].n)
    picks = [ropes[0], ropes[len(ropes) // 2], ropes[-1], cloths[0], cloths[len(cloths) // 2], big]
    for i in picks:
        print(f"C4 instance {i} {insts[i].kind} n={insts[i].n} T={insts[i].T}", flush=True)
    from tests.oracle_pool import fp32_storage_drift, references
    refs = references([insts[i] for i in picks], [cots[i] for i in picks], [parts[i] for i in picks])
    for i, (ref, rst, s0r, ur) in zip(picks, refs):
        inst = insts[i]
        assert rst.max() == 0
        ex, ev = state_errors(parts[i], ref, inst.n)
        print(f"C4 instance {i}: x {ex:.2e} v {ev:.2e}", flush=True)
        if not (ex <= STATE_TOL and ev <= STATE_TOL):
            # a sensitive trajectory over a long horizon (the heavy 256-node
            # rope over 119 steps, a cloth over 94): the oracle's own steps
            # drift this far when the state is rounded to FP32 between
            # steps; the GPU must stay within three times that drift
            sx, sv = fp32_storage_drift(inst, ref)
            print(f"C4 instance {i}: oracle drift with FP32 state rounding x {sx:.2e} v {sv:.2e}", flush=True)
            assert ex <= max(STATE_TOL, 3 * sx) and ev <= max(STATE_TOL, 3 * sv)
        # the derivative along the GPU's own trajectory
        check(gradient_block_errors(s0p[i], up[i], s0r, ur, inst.n), GRAD_TOL, f"C4 instance {i} gradient")
    j = picks[0]
    alone = Sim([insts[j]])
    ta = alone.rollout(alone.pack_states([insts[j].s0]), alone.pack_controls([insts[j].u]))
    torch.cuda.synchronize()
    assert np.array_equal(alone.split(ta, "traj")[0], parts[j])


def test_c4_largest_instances_sampled_steps():
    """The largest cloth (48 x 48 nodes, T = 120) and the largest rope (256
    nodes, T = 119) of the mixed batch, in its graph launch, over their
    whole horizons: at sampled steps the oracle's step from the GPU's state
    at t gives the GPU's state at t + 1, and the oracle's step derivative
    applied to seeded tangents gives the GPU's JVP tangents there (the
    per-step maps whose transposes the adjoint chains).  A whole-horizon
    oracle rollout of the cloth would take it several minutes; the sampled
    steps take seconds."""
    import torch
    from oracle.derivatives import StepDerivative
    from oracle.step import split_state, step as ostep
    from paper_2606_14188_amd import _lib as L
    insts = W.config_c4()
    big = [max((i for i in insts if i.kind == kind), key=lambda i: (i.n, i.T)) for kind in ("cloth", "rope")]
    assert (big[0].n, big[0].T) == (2304, 120) and (big[1].n, big[1].T) == (256, 119)
    sim, s0, u, _ = _setup(big)
    sim.set_launch(L.LAUNCH_GRAPH)
    st = torch.full((len(big),), -1, dtype=torch.int32, device=sim.device)
    tr = sim.rollout(s0, u, status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    parts = sim.split(tr, "traj")
    k = 2
    rng = np.random.default_rng(1031)
    ds = [rng.normal(size=(i.T, k, i.n_s)) for i in big]
    du = [rng.normal(size=(i.T, k, i.n_u)) for i in big]
    st.fill_(-1)
    _, _, jv = sim.linearize(tr, u, dense=False, want_B=False, jvp_k=k,
                             jvp_ds=sim.pack_states([d.ravel() for d in ds]),
                             jvp_du=sim.pack_states([d.ravel() for d in du]), status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    h = jv.cpu().numpy()
    off = 0
    for j, inst in enumerate(big):
        ns = inst.n_s
        traj = parts[j].reshape(inst.T + 1, ns).astype(np.float64)
        blk = h[off:off + inst.T * k * ns].reshape(inst.T, k, ns)
        off += inst.T * k * ns
        for t in (0, inst.T // 3, 2 * inst.T // 3, inst.T - 1):
            print(f"{inst.kind} n={inst.n} T={inst.T} step {t}", flush=True)
            x, v, _ = split_state(inst, traj[t])
            r = ostep(inst, x, v, inst.u[t], inst.kappa_fwd)
            assert r.status == 0
            ex, ev = state_errors(traj[t + 1], np.concatenate([r.x.ravel(), r.v.ravel()]), inst.n)
            print(f"  one step: x {ex:.2e} v {ev:.2e}", flush=True)
            assert ex <= STATE_TOL and ev <= STATE_TOL
            d = StepDerivative(inst, traj[t], inst.u[t], inst.kappa_bwd)
            check(tangent_block_errors(blk[t], d.jvp_s(ds[j][t].T, du[j][t].T).T, inst.n), JAC_TOL,
                  f"  {inst.kind} JVP at step {t}")
