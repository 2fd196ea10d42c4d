"""Oracle references computed in worker processes (started with "spawn", so
nothing of the parent's GPU state is inherited; the workers import only the
oracle and numpy).  Used where one test needs the oracle on several large
instances at once."""
import concurrent.futures
import multiprocessing

import numpy as np


def _reference(inst, cot):
    from oracle.derivatives import rollout_backward
    from oracle.step import rollout
    ref, st = rollout(inst)
    s0r, ur = rollout_backward(inst, ref, sT_bar=np.asarray(cot, dtype=np.float64))
    return ref, st, s0r, ur


def references(insts, cots, workers=6):
    """[(trajectory, status per step, s0_bar, u_bar)] of each instance under
    its cotangent of the final state, by the oracle, in parallel."""
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=min(workers, len(insts)), mp_context=ctx) as ex:
        return list(ex.map(_reference, insts, cots))
