"""Oracle references computed in worker processes (started with "spawn", so
nothing of the parent's GPU state is inherited; the workers import only the
oracle and numpy).  Used where one test needs the oracle on several large
instances at once."""
import concurrent.futures
import multiprocessing

import numpy as np


def _reference(inst, cot, traj):
    from oracle.derivatives import rollout_backward
    from oracle.step import rollout
    ref, st = rollout(inst)
    s0r, ur = rollout_backward(inst, np.asarray(traj, dtype=np.float64).reshape(inst.T + 1, inst.n_s),
                               sT_bar=np.asarray(cot, dtype=np.float64))
    return ref, st, s0r, ur


def references(insts, cots, trajs, workers=6):
    """[(oracle trajectory, status per step, s0_bar, u_bar)] of each
    instance: its own rollout, and the adjoint of its cotangent of the final
    state along the given trajectory (the GPU's), in parallel."""
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(workers, len(insts)), mp_context=ctx) as ex:
        return list(ex.map(_reference, insts, cots, trajs))


def fp32_storage_drift(inst, ref):
    """Position and velocity errors (as in the parity tests), against the
    oracle's rollout `ref`, of the oracle's own steps when the inputs and
    every step's state are rounded to FP32 in between (the state a FP32
    implementation carries from step to step).  On a well-conditioned
    trajectory this stays near FP32 rounding; on a sensitive one (a heavy
    256-node rope over 119 steps, contacts) it shows how far any FP32
    computation of the trajectory must drift."""
    from oracle import model
    from oracle.step import Layout, split_state, step
    from tests.parity import state_errors
    el, lay = model.elements(inst), Layout(inst)
    n = inst.n
    tr = np.zeros_like(ref)
    tr[0] = np.asarray(inst.s0, dtype=np.float32)
    u = np.asarray(inst.u, dtype=np.float32).astype(np.float64)
    for t in range(inst.T):
        x, v, g = split_state(inst, tr[t])
        r = step(inst, x, v, u[t], inst.kappa_fwd, el, lay, g=g)
        tr[t + 1, :3 * n] = r.x.ravel().astype(np.float32)
        tr[t + 1, 3 * n:6 * n] = r.v.ravel().astype(np.float32)
        if r.g is not None:
            tr[t + 1, 6 * n:] = r.g.ravel().astype(np.float32)
    return state_errors(tr, ref, n)
