"""The block-wise parity helpers catch what a whole-matrix norm misses.

A step Jacobian of a 64-node rope (C2 material, dt = 5 ms) from the oracle:
dv+/dx = (dx+/dx - I)/dt holds nearly all of its Frobenius norm, so zeroing
dx+/dv or scaling dx+/dx by 1.01 passes a single relative Frobenius check at
1e-3 but fails the per-block check.  The same holds for the velocity part of
a state cotangent and of a tangent.
"""
import numpy as np

import workloads as W
from oracle.derivatives import StepDerivative, rollout_backward
from oracle.step import rollout
from tests.parity import (GRAD_TOL, JAC_TOL, gradient_block_errors, jacobian_block_errors,
                          tangent_block_errors, worst)


def _rope_step():
    inst = W.config_c2(B=1, seed=1002)[0].replace(T=3)
    inst = inst.replace(u=inst.u[:3])
    traj, st = rollout(inst)
    assert st.max() == 0
    d = StepDerivative(inst, traj[2], inst.u[2], inst.kappa_bwd)
    return inst, traj, d


def test_jacobian_blocks_catch_planted_errors():
    inst, _, d = _rope_step()
    A, B = d.dense()
    n = inst.n
    x, v = slice(0, 3 * n), slice(3 * n, 6 * n)
    assert worst(jacobian_block_errors(A, A, B, B, n)) == 0.0
    # dv+/dx dominates the matrix norm
    assert np.linalg.norm(A[v, x]) > 0.999 * np.linalg.norm(A)

    def whole(M):
        return np.linalg.norm(M - A) / np.linalg.norm(A)

    zero_xv = A.copy()
    zero_xv[x, v] = 0.0
    scale_xx = A.copy()
    scale_xx[x, x] *= 1.01
    scale_vv = A.copy()
    scale_vv[v, v] *= 1.01
    for M in (zero_xv, scale_xx, scale_vv):
        assert whole(M) <= JAC_TOL                      # the old check would pass
        assert worst(jacobian_block_errors(M, A, B, B, n)) > JAC_TOL
    bad_b = B.copy()
    bad_b[x] *= 1.01
    assert worst(jacobian_block_errors(A, A, bad_b, B, n)) > JAC_TOL


def test_tangent_and_gradient_blocks_catch_planted_errors():
    inst, traj, d = _rope_step()
    n = inst.n
    rng = np.random.default_rng(3)
    ds = rng.normal(size=(inst.n_s, 4))
    du = rng.normal(size=(inst.n_u, 4))
    out = d.jvp_s(ds, du).T
    assert worst(tangent_block_errors(out, out, n)) == 0.0
    bad = out.copy()
    bad[:, :3 * n] *= 1.01
    assert np.linalg.norm(bad - out) / np.linalg.norm(out) <= JAC_TOL
    assert worst(tangent_block_errors(bad, out, n)) > JAC_TOL
    cot = W.random_cotangent(inst.n_s, 5)
    s0b, ub = rollout_backward(inst, traj, sT_bar=cot)
    assert worst(gradient_block_errors(s0b, ub, s0b, ub, n)) == 0.0
    bad_s = s0b.copy()
    bad_s[3 * n:] *= 1.03
    assert np.linalg.norm(bad_s - s0b) / np.linalg.norm(s0b) <= GRAD_TOL
    assert worst(gradient_block_errors(bad_s, ub, s0b, ub, n)) > GRAD_TOL
