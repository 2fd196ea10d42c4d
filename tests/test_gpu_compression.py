"""Compression guard on the GPU: straight ropes compressed to 70-78 % of their
rest length, where the exact dF/dq* of the step is indefinite (the stage-1
root is a saddle of the incremental potential).  The forward pass (projected
Newton direction, exact root) matches the oracle; the adjoint, the dense
A_t/B_t and the JVP tangents solve with the indefinite matrix -- the
conjugate gradient meets negative curvature and the minimum residual method
takes over, and the band Cholesky of the direct linearization meets a
negative pivot and its step is done again by the iterative kernel -- and
match the oracle's LU solves.  Neither side flags the instances.  A rope of
normal tension in the same size class shares the launches."""
import numpy as np
import pytest

import workloads as W
from oracle.derivatives import StepDerivative, rollout_backward
from oracle.step import rollout as orollout
from tests.parity import (GRAD_TOL, JAC_TOL, STATE_TOL, check, gradient_block_errors, jacobian_block_errors,
                          state_errors, tangent_block_errors)

pytestmark = pytest.mark.gpu


def _batch():
    return [W.compressed_rope(n=10, T=6), W.compressed_rope(n=24, ratio=0.7, T=5),
            W.compressed_rope(n=40, ratio=0.78, T=4)] + W.small_rope_batch(1, 20, 5, seed=1401)


def test_compressed_rope_forward_gradient_and_jacobians():
    import torch
    from paper_2606_14188_amd import Sim
    insts = _batch()
    for inst in insts:
        print(f"rope n={inst.n} T={inst.T}", flush=True)
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    st = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    traj = sim.rollout(s0, u, status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    parts = sim.split(traj, "traj")
    refs = []
    for j, inst in enumerate(insts):
        ref, rst = orollout(inst)
        assert rst.max() == 0
        refs.append(ref)
        ex, ev = state_errors(parts[j], ref, inst.n)
        print(f"rope {j} n={inst.n}: state err x {ex:.2e} v {ev:.2e}", flush=True)
        assert ex <= STATE_TOL and ev <= STATE_TOL
    # the compressed ropes stay straight on the GPU too: their Hessian is indefinite
    for j in range(3):
        xs = parts[j].reshape(insts[j].T + 1, -1)[:, :3 * insts[j].n].reshape(insts[j].T + 1, -1, 3)
        assert np.max(np.abs(xs[:, :, :2])) == 0.0
        d = StepDerivative(insts[j], refs[j][1], insts[j].u[1], insts[j].kappa_bwd)
        assert np.linalg.eigvalsh(d.Hff.toarray()).min() < 0.0

    # gradient
    rng = np.random.default_rng(1402)
    cot = [rng.normal(size=i.n_s) for i in insts]
    st.fill_(-1)
    s0b, ub = sim.backward(u, traj, sT_bar=sim.pack_states(cot), status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    sp, up = sim.split(s0b, "s"), sim.split(ub, "u")
    for j, inst in enumerate(insts):
        tr = parts[j].reshape(inst.T + 1, inst.n_s).astype(np.float64)
        s0r, ur = rollout_backward(inst, tr, sT_bar=cot[j])
        check(gradient_block_errors(sp[j], up[j], s0r, ur, inst.n), GRAD_TOL, f"rope {j} n={inst.n} gradient")

    # dense A_t / B_t and JVP tangents at every step
    k = 2
    ds = [rng.normal(size=(i.T, k, i.n_s)) for i in insts]
    du = [rng.normal(size=(i.T, k, i.n_u)) for i in insts]
    status = torch.full((len(insts),), -1, dtype=torch.int32, device=sim.device)
    A, Bm, jv = sim.linearize(traj, u, jvp_k=k, jvp_ds=sim.pack_states([d.ravel() for d in ds]),
                              jvp_du=sim.pack_states([d.ravel() for d in du]), status=status)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all(), status
    # every step of the three compressed ropes met a non-positive pivot in
    # the band factorization and was done again by the row-by-row kernel
    stats = sim.lin_stats()
    print("linearization counters", stats, flush=True)
    assert stats["slot_overlaps"] == 0 and stats["steps_redone"] == sum(i.T for i in insts[:3])
    Ap, Bp = sim.split(A, "A"), sim.split(Bm, "B")
    h = jv.cpu().numpy()
    off = 0
    for j, inst in enumerate(insts):
        ns, nu = inst.n_s, inst.n_u
        tr = parts[j].reshape(inst.T + 1, ns).astype(np.float64)
        blk = h[off:off + inst.T * k * ns].reshape(inst.T, k, ns)
        off += inst.T * k * ns
        for t in range(inst.T):
            d = StepDerivative(inst, tr[t], inst.u[t], inst.kappa_bwd)
            Ar, Br = d.dense()
            errs = jacobian_block_errors(Ap[j].reshape(inst.T, ns, ns)[t], Ar, Bp[j].reshape(inst.T, ns, nu)[t],
                                         Br, inst.n)
            errs.update(tangent_block_errors(blk[t], d.jvp_s(ds[j][t].T, du[j][t].T).T, inst.n))
            check(errs, JAC_TOL, f"rope {j} n={inst.n} t={t}")
