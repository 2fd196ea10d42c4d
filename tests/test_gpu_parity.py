"""GPU parity: libcord (HIP, FP32, through the C ABI) against the FP64 oracle
on the same seeded inputs.  Sizes span several workgroup tiles and ragged
tails; full-size configurations are checked on sampled instances."""
import numpy as np
import pytest

import workloads as W
from oracle.derivatives import StepDerivative, rollout_backward
from oracle.step import rollout as orollout
from tests.parity import (GRAD_TOL, JAC_TOL, STATE_TOL, check, gradient_block_errors, jacobian_block_errors,
                          state_errors, tangent_block_errors)

pytestmark = pytest.mark.gpu


def _sim(insts):
    from paper_2606_14188_amd import Sim
    return Sim(insts)


def _run(insts, **kw):
    import torch
    sim = _sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    traj = sim.rollout(s0, u, status=st, **kw)
    torch.cuda.synchronize()
    return sim, s0, u, traj, st.cpu().numpy()


def _check_states(sim, traj, insts, idx=None):
    """States against the oracle; returns the oracle trajectories by index."""
    parts = sim.split(traj, "traj")
    idx = range(len(insts)) if idx is None else idx
    refs = {}
    for i in idx:
        inst = insts[i]
        ref, st = orollout(inst)
        assert st.max() == 0
        ex, ev = state_errors(parts[i], ref, inst.n)
        print(f"instance {i} ({inst.kind} n={inst.n} T={inst.T}): state err x {ex:.2e} v {ev:.2e}", flush=True)
        assert ex <= STATE_TOL and ev <= STATE_TOL, (i, ex, ev)
        refs[i] = ref
    return refs


def test_c1_forward_and_gradient():
    import torch
    inst = W.config_c1()
    sim, s0, u, traj, st = _run([inst])
    assert st.tolist() == [0]
    _check_states(sim, traj, [inst])
    n = inst.n
    ref, _ = orollout(inst)
    d = ref[-1, 3 * (n - 1):3 * n] - W.gen.C1_GOAL
    sb = np.zeros(6 * n)
    sb[3 * (n - 1):3 * n] = d / np.linalg.norm(d)
    s0b_or, ub_or = rollout_backward(inst, ref, sT_bar=sb)
    sT_bar = torch.tensor(sb, dtype=torch.float32, device=sim.device)
    s0b, ub = sim.backward(u, traj, sT_bar=sT_bar)
    torch.cuda.synchronize()
    check(gradient_block_errors(s0b.cpu().numpy(), ub.cpu().numpy(), s0b_or, ub_or, n), GRAD_TOL, "C1 gradient")


@pytest.mark.parametrize("ns", [(64,), (16, 37, 64, 100)])
def test_rope_batch_forward(ns):
    insts = []
    for j, n in enumerate(ns):
        insts += W.small_rope_batch(2, n, 30, seed=200 + j)
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all(), st
    _check_states(sim, traj, insts)


@pytest.mark.parametrize("dims", [((8, 8),), ((6, 5), (9, 7), (16, 16))])
def test_cloth_batch_forward(dims):
    insts = []
    for j, (nx, ny) in enumerate(dims):
        insts += W.small_cloth_batch(1, nx, ny, 20, seed=300 + j)
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all(), st
    _check_states(sim, traj, insts)


def _backward_parity(insts, store="full", K=7):
    import torch
    from paper_2606_14188_amd import _lib as L
    sim, s0, u, traj, st = _run(insts)
    cots = [W.random_cotangent(i.n_s, 900 + j) for j, i in enumerate(insts)]
    sT = sim.pack_states(cots)
    s0b, ub = sim.backward(u, traj, sT_bar=sT)
    torch.cuda.synchronize()
    s0bp = sim.split(s0b, "s")
    ubp = sim.split(ub, "u")
    refs = [orollout(i)[0] for i in insts]
    for j, inst in enumerate(insts):
        s0r, ur = rollout_backward(inst, refs[j], sT_bar=cots[j])
        check(gradient_block_errors(s0bp[j], ubp[j], s0r, ur, inst.n), GRAD_TOL,
              f"instance {j} ({inst.kind} n={inst.n}) gradient")
    return sim, s0, u, traj, sT, s0b, ub


def test_rope_backward():
    insts = W.small_rope_batch(2, 64, 25, seed=401) + W.small_rope_batch(1, 23, 25, seed=402)
    _backward_parity(insts)


def test_cloth_backward():
    insts = W.small_cloth_batch(1, 8, 8, 15, seed=411) + W.small_cloth_batch(1, 7, 5, 15, seed=412)
    _backward_parity(insts)


def test_smallest_cloths():
    """Cloths of 2x2, 3x2 and 2x5 nodes (two corners gripped, so two to
    eight free particles; no bend springs along a side of two nodes):
    states and gradients against the oracle."""
    insts = (W.small_cloth_batch(1, 2, 2, 12, seed=492) + W.small_cloth_batch(1, 3, 2, 12, seed=502)
             + W.small_cloth_batch(1, 2, 5, 12, seed=495))
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all(), st
    _check_states(sim, traj, insts)
    _backward_parity(insts)


def test_degenerate_and_largest_ropes():
    """Ropes at the edges of what the simulator accepts, side by side in one
    ragged batch: a single free particle (no spring, no gripper, no
    controls) that falls onto the ground, ropes of two and three nodes (one
    spring; one bending centre), and a rope of 256 nodes (the largest size
    class), and a horizon of one step.  States and gradients against the
    oracle."""
    import torch
    part = W.rope(1, T=30, grip_nodes=(), k=0.0, k_bend=0.0, h=0.01,
                  s0=np.array([0.1, 0.2, 0.004, 0.3, -0.1, -0.5]))
    insts = ([part] + W.small_rope_batch(1, 2, 20, seed=611) + W.small_rope_batch(1, 3, 20, seed=612)
             + W.small_rope_batch(1, 256, 6, seed=613) + W.small_rope_batch(1, 20, 1, seed=614))
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all(), st
    _check_states(sim, traj, insts)
    cots = [W.random_cotangent(i.n_s, 960 + j) for j, i in enumerate(insts)]
    s0b, ub = sim.backward(u, traj, sT_bar=sim.pack_states(cots))
    torch.cuda.synchronize()
    s0bp, ubp = sim.split(s0b, "s"), sim.split(ub, "u")
    for j, inst in enumerate(insts):
        s0r, ur = rollout_backward(inst, orollout(inst)[0], sT_bar=cots[j])
        check(gradient_block_errors(s0bp[j], ubp[j], s0r, ur, inst.n), GRAD_TOL,
              f"instance {j} (rope n={inst.n}) gradient")


def test_checkpointed_backward_bitwise():
    import torch
    from paper_2606_14188_amd import _lib as L
    insts = W.small_rope_batch(3, 40, 23, seed=421) + W.small_cloth_batch(1, 6, 6, 23, seed=422)
    sim, s0, u, traj, st = _run(insts)
    sT = sim.pack_states([W.random_cotangent(i.n_s, 950 + j) for j, i in enumerate(insts)])
    s0b, ub = sim.backward(u, traj, sT_bar=sT)
    for K in (1, 7, 23, 50):
        ck = sim.rollout(s0, u, store=L.STORE_CKPT, ckpt_every=K)
        s0k, ubk = sim.backward(u, ck, sT_bar=sT, store=L.STORE_CKPT, ckpt_every=K)
        torch.cuda.synchronize()
        assert torch.equal(s0k, s0b) and torch.equal(ubk, ub), K
        # checkpoints are bitwise the stored states
        full = sim.split(traj, "traj")
        cks = sim.split(ck, "ckpt", K)
        for j, inst in enumerate(insts):
            tr = full[j].reshape(inst.T + 1, -1)
            c = cks[j].reshape(-1, inst.n_s)
            slots = list(range(0, inst.T, K)) + [inst.T]
            assert np.array_equal(c, tr[slots])


def test_determinism_and_mix_invariance():
    import torch
    insts = W.small_rope_batch(6, 64, 20, seed=431)
    sim, s0, u, traj, st = _run(insts)
    traj2 = sim.rollout(s0, u)
    torch.cuda.synchronize()
    assert torch.equal(traj, traj2)
    alone, _, _, t1, _ = _run([insts[3]])
    assert np.array_equal(sim.split(traj, "traj")[3], alone.split(t1, "traj")[0])


def test_nonfinite_input_flags_only_that_instance():
    insts = W.small_rope_batch(3, 20, 5, seed=441)
    bad = insts[1].s0.copy()
    bad[7] = np.nan
    insts[1] = insts[1].replace(s0=bad)
    sim, s0, u, traj, st = _run(insts)
    assert st[1] == 4 and st[0] == 0 and st[2] == 0, st


@pytest.mark.parametrize("kind", ["rope", "rope_tiny", "cloth"])
def test_linearize_dense(kind):
    import torch
    if kind == "rope_tiny":
        # ropes whose free DoFs (3, 6, 12) are fewer than the band is wide
        # (and a horizon of one step)
        insts = (W.small_rope_batch(1, 2, 3, seed=456) + W.small_rope_batch(1, 3, 3, seed=457)
                 + W.small_rope_batch(1, 5, 2, seed=458) + W.small_rope_batch(1, 33, 1, seed=459))
    elif kind == "rope":
        # one rope per size class of the direct kernel (32, 64, 128 nodes)
        # plus a ragged one; T differs so the (instance, step) grid is ragged
        insts = (W.small_rope_batch(1, 10, 4, seed=451) + W.small_rope_batch(1, 7, 4, seed=452)
                 + W.small_rope_batch(1, 40, 3, seed=454) + W.small_rope_batch(1, 100, 2, seed=455))
    else:
        insts = W.small_cloth_batch(1, 4, 4, 3, seed=453)
    sim, s0, u, traj, st = _run(insts)
    A, Bm, _ = sim.linearize(traj, u)
    torch.cuda.synchronize()
    Ap, Bp = sim.split(A, "A"), sim.split(Bm, "B")
    tp = sim.split(traj, "traj")
    for j, inst in enumerate(insts):
        ns, nu = inst.n_s, inst.n_u
        Aj = Ap[j].reshape(inst.T, ns, ns)
        Bj = Bp[j].reshape(inst.T, ns, nu)
        tr = tp[j].reshape(inst.T + 1, ns).astype(np.float64)
        for t in range(inst.T):
            Ar, Br = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd).dense()
            check(jacobian_block_errors(Aj[t], Ar, Bj[t], Br, inst.n), JAC_TOL, f"{kind} {j} t={t}")


def test_jvp_tangents():
    import torch
    insts = W.small_cloth_batch(1, 6, 5, 4, seed=461) + W.small_rope_batch(1, 30, 4, seed=462)
    sim, s0, u, traj, st = _run(insts)
    k = 3
    rng = np.random.default_rng(5)
    ds = [rng.normal(size=(i.T, k, i.n_s)) for i in insts]
    du = [rng.normal(size=(i.T, k, i.n_u)) for i in insts]
    dst = sim.pack_states([d.ravel() for d in ds])
    dut = sim.pack_states([d.ravel() for d in du])
    _, _, out = sim.linearize(traj, u, dense=False, want_B=False, jvp_k=k, jvp_ds=dst, jvp_du=dut)
    torch.cuda.synchronize()
    h = out.cpu().numpy()
    tp = sim.split(traj, "traj")
    off = 0
    for j, inst in enumerate(insts):
        blk = h[off:off + inst.T * k * inst.n_s].reshape(inst.T, k, inst.n_s)
        off += inst.T * k * inst.n_s
        tr = tp[j].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        for t in range(inst.T):
            d = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd)
            n3 = 3 * inst.n
            dxn, dvn = d.jvp(ds[j][t].T[:n3], ds[j][t].T[n3:], du[j][t].T)
            ref = np.vstack([dxn, dvn]).T
            check(tangent_block_errors(blk[t], ref, inst.n), JAC_TOL, f"{inst.kind} t={t} jvp")


def test_autograd_function():
    import torch
    from paper_2606_14188_amd import rollout
    insts = W.small_rope_batch(2, 32, 12, seed=471)
    sim = _sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts]).requires_grad_(True)
    u = sim.pack_controls([i.u for i in insts]).requires_grad_(True)
    traj = rollout(sim, s0, u, mode="full")
    w = torch.randn_like(traj)
    (traj * w).sum().backward()
    s0b, ub = sim.backward(u.detach(), traj.detach(), traj_bar=w)
    torch.cuda.synchronize()
    assert torch.equal(s0.grad, s0b) and torch.equal(u.grad, ub)
    # final-state mode with checkpoints
    s0.grad = None
    u.grad = None
    sT = rollout(sim, s0, u, mode="final", ckpt_every=5)
    wT = torch.randn_like(sT)
    (sT * wT).sum().backward()
    full_sT = torch.cat([p[-6 * i.n:] for p, i in zip(torch.split(traj.detach(), [(i.T + 1) * i.n_s for i in insts]), insts)])
    assert torch.equal(sT.detach(), full_sT)
    s0b2, ub2 = sim.backward(u.detach(), traj.detach(), sT_bar=wT)
    torch.cuda.synchronize()
    assert torch.equal(s0.grad, s0b2) and torch.equal(u.grad, ub2)


def test_autograd_two_graphs_before_backward():
    """With step internals kept, two differentiable rollouts are built before
    the first one's backward runs: the second rollout has overwritten the
    internals, so that backward solves its steps again and gives bitwise the
    gradient of a simulator without step internals (and the second graph's
    backward still uses the internals it owns)."""
    import torch
    from paper_2606_14188_amd import Sim, rollout
    insts = W.small_rope_batch(3, 32, 10, seed=475)
    sim = Sim(insts)
    sim.use_aux(True)
    plain = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u1 = sim.pack_controls([i.u for i in insts]).requires_grad_(True)
    u2 = (u1.detach() * 1.5).requires_grad_(True)
    tr1 = rollout(sim, s0, u1, mode="full")
    tr2 = rollout(sim, s0, u2, mode="full")
    w = torch.randn_like(tr1)
    (tr1 * w).sum().backward()
    (tr2 * w).sum().backward()
    r1 = plain.backward(u1.detach(), tr1.detach(), traj_bar=w)
    r2 = plain.backward(u2.detach(), tr2.detach(), traj_bar=w)
    torch.cuda.synchronize()
    assert torch.equal(u1.grad, r1[1]) and torch.equal(u2.grad, r2[1])
    # the first gradient against the oracle
    tp, gp = sim.split(tr1.detach(), "traj"), sim.split(u1.grad, "u")
    wp = sim.split(w, "traj")
    for j in (0, 2):
        inst = insts[j]
        tr = tp[j].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        _, ur = rollout_backward(inst.replace(u=sim.split(u1.detach(), "u")[j].reshape(inst.T, -1).astype(np.float64)),
                                 tr, traj_bar=wp[j].reshape(inst.T + 1, inst.n_s).astype(np.float64))
        check({"u_bar": float(np.linalg.norm(gp[j] - ur.ravel()) / np.linalg.norm(ur))}, GRAD_TOL, f"graph 1 rope {j}")


def _c2_bench_sim():
    """The full-size rope batch as the benchmark runs it: step internals
    kept by the rollout for the adjoint and the linearization."""
    import torch
    from paper_2606_14188_amd import Sim
    insts = W.config_c2()
    sim = Sim(insts)
    sim.use_aux(True)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    traj = sim.rollout(s0, u, status=st)
    torch.cuda.synchronize()
    return insts, sim, s0, u, traj, st.cpu().numpy()


def test_c2_full_size_sampled():
    """C2 at full size (1024 ropes of 64 nodes, 100 steps) in the launches
    the benchmark times (rollout keeping its step internals, adjoint of the
    benchmark's terminal cotangents); sampled instances' states and
    gradients against the oracle."""
    import torch
    insts, sim, s0, u, traj, st = _c2_bench_sim()
    print("status counts", np.bincount(st, minlength=5))
    assert (st == 0).all()
    cots = [W.random_cotangent(i.n_s, 7000 + j) for j, i in enumerate(insts)]
    s0b, ub = sim.backward(u, traj, sT_bar=sim.pack_states(cots))
    torch.cuda.synchronize()
    refs = _check_states(sim, traj, insts, idx=[0, 341, 682, 1023])
    s0p, up = sim.split(s0b, "s"), sim.split(ub, "u")
    for j in (0, 1023):
        s0r, ur = rollout_backward(insts[j], refs[j], sT_bar=cots[j])
        check(gradient_block_errors(s0p[j], up[j], s0r, ur, insts[j].n), GRAD_TOL, f"instance {j} gradient")


def test_c3_full_size_sampled():
    """C3 at full size (256 cloths of 32x32, 60 steps) in the launches the
    cloth benchmark times: a full rollout keeping its step internals, the
    checkpointed (every 10 steps) rollout and adjoint, and 6 JVP tangents
    per step (unit control directions, the B_t columns).  One sampled
    instance's states, gradient and tangents (three steps) against the
    oracle."""
    import torch
    from paper_2606_14188_amd import Sim, _lib as L
    insts = W.config_c3()
    sim = Sim(insts)
    sim.use_aux(True)
    B, T = len(insts), insts[0].T
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    st = torch.full((B,), -1, dtype=torch.int32, device=sim.device)
    traj = sim.rollout(s0, u, status=st)
    cots = [W.random_cotangent(i.n_s, 8000 + j) for j, i in enumerate(insts)]
    ck = sim.rollout(s0, u, store=L.STORE_CKPT, ckpt_every=10)
    s0b, ub = sim.backward(u, ck, sT_bar=sim.pack_states(cots), store=L.STORE_CKPT, ckpt_every=10)
    k = 6
    du = np.zeros((B, T, k, 6), np.float32)
    du[:, :, np.arange(6), np.arange(6)] = 1.0
    _, _, jv = sim.linearize(traj, u, dense=False, want_B=False, jvp_k=k,
                             jvp_du=torch.from_numpy(du.ravel()).to(sim.device))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    print("status counts", np.bincount(st, minlength=5), flush=True)
    assert (st == 0).all()
    j = 255
    inst = insts[j]
    ref = _check_states(sim, traj, insts, idx=[j])[j]
    s0r, ur = rollout_backward(inst, ref, sT_bar=cots[j])
    check(gradient_block_errors(sim.split(s0b, "s")[j], sim.split(ub, "u")[j], s0r, ur, inst.n), GRAD_TOL,
          f"instance {j} gradient")
    ns, n3 = inst.n_s, 3 * inst.n
    blk = jv.cpu().numpy()[j * T * k * ns:(j + 1) * T * k * ns].reshape(T, k, ns)
    tr = sim.split(traj, "traj")[j].reshape(T + 1, ns).astype(np.float64)
    for t in (0, 29, 59):
        d = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd)
        dxn, dvn = d.jvp(np.zeros((n3, k)), np.zeros((n3, k)), np.eye(6))
        check(tangent_block_errors(blk[t], np.vstack([dxn, dvn]).T, inst.n), JAC_TOL, f"instance {j} t={t} jvp")


def test_c1_linearize_in_contact():
    """Dense A_t/B_t along C1, where the rope lands on the ground and drapes
    over the sphere: every step against the oracle at the same state."""
    import torch
    inst = W.config_c1()
    sim, s0, u, traj, st = _run([inst])
    A, Bm, _ = sim.linearize(traj, u)
    torch.cuda.synchronize()
    ns, nu, T = inst.n_s, inst.n_u, inst.T
    Aj = A.cpu().numpy().reshape(T, ns, ns)
    Bj = Bm.cpu().numpy().reshape(T, ns, nu)
    tr = traj.cpu().numpy().reshape(T + 1, ns).astype(np.float64)
    worst = 0.0
    for t in range(T):
        d = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd)
        Ar, Br = d.dense()
        errs = jacobian_block_errors(Aj[t], Ar, Bj[t], Br, inst.n)
        print(f"C1 t={t}: max lam {d.res.lam.max():.2e} min gap {d.res.gap.min():.2e}", flush=True)
        check(errs, JAC_TOL, f"C1 t={t}")


def test_linearize_b_only_and_with_jvp():
    """B_t alone (no A_t) and A_t together with JVP tangents: the same B_t
    and the same tangents as the separate calls, within the Jacobian
    tolerance, and B_t against the oracle."""
    import torch
    insts = W.small_rope_batch(1, 24, 3, seed=471) + W.small_rope_batch(1, 50, 3, seed=472)
    sim, s0, u, traj, st = _run(insts)
    k = 2
    rng = np.random.default_rng(9)
    ds = [rng.normal(size=(i.T, k, i.n_s)) for i in insts]
    du = [rng.normal(size=(i.T, k, i.n_u)) for i in insts]
    dst = sim.pack_states([d.ravel() for d in ds])
    dut = sim.pack_states([d.ravel() for d in du])
    status = torch.zeros(len(insts), dtype=torch.int32, device=sim.device)
    A, B1, o1 = sim.linearize(traj, u, jvp_k=k, jvp_ds=dst, jvp_du=dut, status=status)
    _, B2, _ = sim.linearize(traj, u, dense=False)
    _, _, o2 = sim.linearize(traj, u, dense=False, want_B=False, jvp_k=k, jvp_ds=dst, jvp_du=dut)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    assert torch.equal(o1, o2)
    b1, b2 = B1.cpu().numpy(), B2.cpu().numpy()
    assert np.linalg.norm(b1 - b2) <= JAC_TOL * np.linalg.norm(b2)
    Bp = sim.split(B1, "B")
    tp = sim.split(traj, "traj")
    for j, inst in enumerate(insts):
        tr = tp[j].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        for t in range(inst.T):
            Ar, Br = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd).dense()
            Bj = Bp[j].reshape(inst.T, inst.n_s, inst.n_u)[t]
            errs = {k: v for k, v in jacobian_block_errors(Ar, Ar, Bj, Br, inst.n).items() if k.startswith("B")}
            check(errs, JAC_TOL, f"rope {inst.n} t={t} B")


def test_linearize_scratch_and_in_place_agree(monkeypatch):
    """The direct rope linearization keeps each column's intermediate vector
    in the scratch table indexed by the hardware workgroup slot, or (without
    the table) inside A_t.  Both run the same arithmetic: A_t and B_t agree
    bitwise, for ropes of all three direct size classes in one batch, and the
    default path matches the oracle."""
    import torch
    insts = (W.small_rope_batch(3, 30, 6, seed=481) + W.small_rope_batch(3, 64, 5, seed=482)
             + W.small_rope_batch(2, 100, 4, seed=483))
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all()
    A1, B1, _ = sim.linearize(traj, u)
    torch.cuda.synchronize()
    monkeypatch.setenv("CORD_LINEARIZE_NO_SCRATCH", "1")
    A2, B2, _ = sim.linearize(traj, u)
    torch.cuda.synchronize()
    assert torch.equal(A1, A2) and torch.equal(B1, B2)
    Ap, Bp, tp = sim.split(A1, "A"), sim.split(B1, "B"), sim.split(traj, "traj")
    for j in (0, 3, 7):
        inst = insts[j]
        tr = tp[j].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        t = inst.T - 1
        Ar, Br = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd).dense()
        Aj = Ap[j].reshape(inst.T, inst.n_s, inst.n_s)[t]
        Bj = Bp[j].reshape(inst.T, inst.n_s, inst.n_u)[t]
        check(jacobian_block_errors(Aj, Ar, Bj, Br, inst.n), JAC_TOL, f"rope {inst.n} t={t}")


def test_linearize_concurrent_streams():
    """Two simulators linearizing at the same time on two streams (each with
    its own scratch table; workgroups of both kernels share the CUs and the
    hardware slots) give bitwise the results of running them one after the
    other."""
    import torch
    ia = W.small_rope_batch(48, 64, 12, seed=495)
    ib = W.small_rope_batch(40, 50, 16, seed=496)
    runs = []
    for insts in (ia, ib):
        sim, s0, u, traj, st = _run(insts)
        assert (st == 0).all()
        runs.append((sim, u, traj))
    ref = []
    for sim, u, traj in runs:
        A, Bm, _ = sim.linearize(traj, u)
        torch.cuda.synchronize()
        ref.append((A.clone(), Bm.clone()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = []
    torch.cuda.synchronize()
    for (sim, u, traj), sm in zip(runs, streams):
        with torch.cuda.stream(sm):
            out.append(sim.linearize(traj, u)[:2])
    torch.cuda.synchronize()
    for (A1, B1), (A2, B2) in zip(ref, out):
        assert torch.equal(A1, A2) and torch.equal(B1, B2)
    for sim, _, _ in runs:
        assert sim.lin_stats()["slot_overlaps"] == 0


def test_backward_and_linearize_overlap_on_two_sims():
    """The adjoint and the linearization of one rollout run at the same time
    on two streams through two simulators over the same instances that share
    the step-internals buffer; the results are bitwise those of running both
    on one simulator one after the other."""
    import torch
    from paper_2606_14188_amd import Sim
    insts = W.small_rope_batch(40, 64, 12, seed=497)
    rng = np.random.default_rng(498)
    sim = Sim(insts)
    sim.use_aux(True)
    sim_lin = Sim(insts)
    sim_lin.use_aux(True, buffer=sim.aux)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([rng.normal(size=i.n_s) for i in insts])
    st = torch.zeros(len(insts), dtype=torch.int32, device=sim.device)
    traj = sim.rollout(s0, u, status=st)
    s0b, ub = sim.backward(u, traj, sT_bar=sT)
    A, Bm, _ = sim.linearize(traj, u)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    ref = [t.clone() for t in (traj, s0b, ub, A, Bm)]
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()
    for _ in range(2):
        traj2 = sim.rollout(s0, u)
        side.wait_stream(main)
        with torch.cuda.stream(side):
            A2, B2, _ = sim_lin.linearize(traj2, u)
        s0b2, ub2 = sim.backward(u, traj2, sT_bar=sT)
        main.wait_stream(side)
        torch.cuda.synchronize()
        for nm, a, b in zip(["traj", "s0_bar", "u_bar", "A", "B"], ref, (traj2, s0b2, ub2, A2, B2)):
            assert torch.equal(a, b), nm
    with pytest.raises(ValueError):
        sim_lin.use_aux(True, buffer=sim.aux[:10])


def test_c2_linearize_full_size_sampled():
    """Dense A_t/B_t for the full 1024 x 64-node x 100-step rope batch in one
    launch (60 GB of A_t), with the step internals kept as the benchmark
    runs it; sampled (instance, step) blocks against the oracle."""
    import torch
    insts, sim, s0, u, traj, st = _c2_bench_sim()
    assert (st == 0).all()
    status = torch.zeros(len(insts), dtype=torch.int32, device=sim.device)
    A, Bm, _ = sim.linearize(traj, u, status=status)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    # no two resident workgroups shared a scratch slot, and no step needed
    # the row-by-row kernel
    stats = sim.lin_stats()
    print("linearization counters", stats, flush=True)
    assert stats == {"slot_overlaps": 0, "steps_redone": 0}
    offA, offB, offT = sim.offsets()["A"], sim.offsets()["B"], sim.offsets()["traj"]
    for j, t in [(0, 0), (1, 99), (517, 50), (1023, 7), (700, 93)]:
        inst = insts[j]
        ns, nu = inst.n_s, inst.n_u
        a0 = int(offA[j]) + t * ns * ns
        b0 = int(offB[j]) + t * ns * nu
        Aj = A[a0:a0 + ns * ns].cpu().numpy().reshape(ns, ns)
        Bj = Bm[b0:b0 + ns * nu].cpu().numpy().reshape(ns, nu)
        tr = traj[int(offT[j]) + t * ns:int(offT[j]) + (t + 1) * ns].cpu().numpy().astype(np.float64)
        Ar, Br = StepDerivative(inst, tr, inst.u[t], inst.kappa_bwd).dense()
        check(jacobian_block_errors(Aj, Ar, Bj, Br, inst.n), JAC_TOL, f"C2 inst {j} t={t}")


def test_cloth_48x48_forward_and_gradient():
    """A 48 x 48 cloth (2304 nodes, the three-particles-per-thread
    configuration) over 4 steps: states and gradient against the oracle."""
    import torch
    insts = W.small_cloth_batch(1, 48, 48, 4, seed=481)
    sim, s0, u, traj, st = _run(insts)
    assert (st == 0).all()
    _check_states(sim, traj, insts)
    inst = insts[0]
    cot = W.random_cotangent(inst.n_s, 482)
    s0b, ub = sim.backward(u, traj, sT_bar=sim.pack_states([cot]))
    torch.cuda.synchronize()
    tr = sim.split(traj, "traj")[0].reshape(inst.T + 1, inst.n_s).astype(np.float64)
    sb_ref, ub_ref = rollout_backward(inst, tr, sT_bar=cot)
    check(gradient_block_errors(s0b.cpu().numpy(), ub.cpu().numpy(), sb_ref, ub_ref, inst.n), GRAD_TOL,
          "cloth 48x48 gradient")


def test_hard_contact_forward_and_surrogate_gradient():
    """Surrogate mode: hard contact (kappa_fwd = 0) drives the rollout and the
    gradient uses kappa_bwd at the hard trajectory's states.  C1 (the rope
    lands on the ground and drapes over the sphere) and a small rope batch."""
    import torch
    c1 = W.config_c1()
    insts = [c1.replace(kappa_fwd=0.0)] + [i.replace(kappa_fwd=0.0) for i in W.small_rope_batch(2, 30, 20, seed=491)]
    sim, s0, u, traj, st = _run(insts)
    print("status", st, flush=True)
    assert (st == 0).all()
    parts = sim.split(traj, "traj")
    for i, inst in enumerate(insts):
        ref, rst = orollout(inst)
        assert rst.max() == 0
        ex, ev = state_errors(parts[i], ref, inst.n)
        print(f"hard rope {i} n={inst.n} T={inst.T}: state err x {ex:.2e} v {ev:.2e}", flush=True)
        assert ex <= STATE_TOL and ev <= STATE_TOL
    rng = np.random.default_rng(17)
    cot = [rng.normal(size=i.n_s) for i in insts]
    s0b, ub = sim.backward(u, traj, sT_bar=sim.pack_states(cot))
    torch.cuda.synchronize()
    sp, up, tp = sim.split(s0b, "s"), sim.split(ub, "u"), sim.split(traj, "traj")
    for i, inst in enumerate(insts):
        tr = tp[i].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        sb_ref, ub_ref = rollout_backward(inst, tr, sT_bar=cot[i])
        check(gradient_block_errors(sp[i], up[i], sb_ref, ub_ref, inst.n), GRAD_TOL, f"hard rope {i} n={inst.n} gradient")


@pytest.mark.parametrize("graph", [False, True])
def test_step_internals_bitwise(graph):
    """With the step-internals buffer the adjoint and the linearizations
    skip re-solving each step.  Batch: ropes of the direct-linearization classes and of the
    iterative one, a cloth, a penalty-grasp rope and a rope whose forward
    and gradient relaxations differ (always re-solved)."""
    import torch
    from paper_2606_14188_amd import Sim, _lib as L
    insts = (W.small_rope_batch(1, 60, 6, seed=701) + W.small_rope_batch(1, 100, 5, seed=702)
             + W.small_rope_batch(1, 200, 4, seed=703) + W.small_cloth_batch(1, 6, 5, 5, seed=704)
             + [W.penalty_grasp(W.small_rope_batch(1, 30, 6, seed=705)[0], seed=3)])
    r = W.small_rope_batch(1, 40, 5, seed=706)[0]
    insts.append(r.replace(kappa_fwd=0.5 * r.kappa_bwd))
    rng = np.random.default_rng(41)
    cot = [rng.normal(size=i.n_s) for i in insts]
    k = 2
    ds = [rng.normal(size=(i.T, k, i.n_s)) for i in insts]
    du = [rng.normal(size=(i.T, k, i.n_u)) for i in insts]
    outs = []
    for aux in (False, True):
        sim = Sim(insts)
        if graph:
            sim.set_launch(L.LAUNCH_GRAPH)
        if aux:
            sim.use_aux(True)
        s0 = sim.pack_states([i.s0 for i in insts])
        u = sim.pack_controls([i.u for i in insts])
        sT = sim.pack_states(cot)
        st = torch.zeros(len(insts), dtype=torch.int32, device=sim.device)
        traj = sim.rollout(s0, u, status=st)
        s0b, ub = sim.backward(u, traj, sT_bar=sT)
        A, Bm, jv = sim.linearize(traj, u, jvp_k=k, jvp_ds=sim.pack_states([d.ravel() for d in ds]),
                                  jvp_du=sim.pack_states([d.ravel() for d in du]))
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        outs.append([traj, s0b, ub, A, Bm, jv])
    # the adjoint restores exactly the state the rollout solved (bitwise);
    # a re-solve inside the linearization kernels repeats that arithmetic in
    # another kernel (other reduction widths and contractions), so there the
    # two paths agree to FP32 rounding
    names = ["traj", "s0_bar", "u_bar"]
    for nm, a, b in zip(names, outs[0][:3], outs[1][:3]):
        assert torch.equal(a, b), nm
    for nm, a, b in zip(["A", "B", "jvp"], outs[0][3:], outs[1][3:]):
        e = (torch.linalg.norm(a - b) / torch.linalg.norm(a)).item()
        print(f"{nm}: relative difference with / without step internals {e:.2e}", flush=True)
        assert e <= 1e-5, nm
