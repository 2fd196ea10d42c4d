"""Pins of the oracle's penalty grasp (holonomic penalty of eq.
(dynamics-first-stage) with the smoothed activation of the Contact
Smoothing paragraph), CPU only.

* closed form: a single node pulled by its gripper, no springs, gravity or
  contact, solves a scalar linear equation per axis;
* hard activation: inside r_g the node is pulled, outside it moves freely;
* D_max -> infinity: the penalty step converges to the Dirichlet step at
  rate 1/D_max;
* the step Jacobian over the full state (x, v, g) and u, including the
  derivative of the activation, against central differences, with contact;
* JVP / VJP dot product and a rollout gradient against directional
  differences.
"""
import numpy as np
import pytest

import workloads as W
from oracle import STATUS_OK
from oracle.derivatives import StepDerivative, rollout_backward
from oracle.step import rollout, split_state, step


def _two_nodes(D_max, kappa_h, r_g, offset):
    """Two unconnected nodes (k = k_b = 0), no gravity, no obstacles; the
    gripper of node 0 sits at x_0 + offset."""
    inst = W.rope(2, mass=0.01, dt=0.005, gamma=0.3, T=1, grip_nodes=(0,), ground=False,
                  k=0.0, k_bend=0.0, h=0.05, gravity=(0.0, 0.0, 0.0))
    n = inst.n
    s = inst.s0.copy()
    s[3 * n:6 * n] = np.array([0.2, -0.1, 0.05, 0.0, 0.1, 0.0])
    g0 = s[:3] + np.asarray(offset)
    return inst.replace(grip_mode="penalty", D_max=D_max, kappa_h=kappa_h, r_g=r_g,
                        s0=np.concatenate([s[:6 * n], g0]))


@pytest.mark.parametrize("kappa_h,r_g,offset", [(0.01, 0.0, (0.003, -0.002, 0.001)),
                                                (0.0, 0.005, (0.002, 0.0, 0.001)),
                                                (0.0, 0.005, (0.006, 0.0, 0.001))])
def test_penalty_closed_form(kappa_h, r_g, offset):
    inst = _two_nodes(400.0, kappa_h, r_g, offset)
    u = np.array([0.1, 0.0, -0.2])
    x, v, g = split_state(inst, inst.s0)
    r = step(inst, x, v, u, 0.0, g=g)
    assert r.status == STATUS_OK
    dt, m = inst.dt, inst.mass
    c = np.linalg.norm(x[0] - g[0])
    if kappa_h > 0:
        D = 400.0 * np.exp(-c / kappa_h)
    else:
        D = 400.0 if c <= r_g else 0.0
    xhat = x + dt * (1 - inst.gamma) * v
    gp = g[0] + dt * u
    # m (y - xhat)/dt^2 + D (y - g+) = 0, per axis
    y0 = (m / dt ** 2 * xhat[0] + D * gp) / (m / dt ** 2 + D)
    np.testing.assert_allclose(r.x[0], y0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r.x[1], xhat[1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(r.v[0], (y0 - x[0]) / dt, rtol=0, atol=1e-10)
    np.testing.assert_allclose(r.g[0], gp, rtol=0, atol=1e-15)


def test_penalty_to_dirichlet_limit():
    """Gripper on its node (activation 1): as D_max grows the penalty step
    tends to the Dirichlet step, with error ~ 1/D_max."""
    base = W.small_rope_batch(1, 8, 1, seed=91)[0]
    n = base.n
    u = base.u[0]
    x, v, _ = split_state(base, base.s0)
    rd = step(base, x, v, u, base.kappa_bwd)
    errs = []
    for scale in (1e2, 1e4, 1e6):
        inst = W.penalty_grasp(base, offset_scale=0.0, D_max=scale * base.mass / base.dt ** 2)
        _, _, g = split_state(inst, inst.s0)
        rp = step(inst, x, v, u, inst.kappa_bwd, g=g)
        assert rp.status == STATUS_OK
        errs.append(np.max(np.abs(rp.x - rd.x)))
    assert errs[2] < 1e-6 * inst.h
    assert 50.0 < errs[0] / errs[1] < 200.0 and 50.0 < errs[1] / errs[2] < 200.0


def _fd_full(inst, s, u, kappa, h):
    def f(ss, uu):
        x, v, g = split_state(inst, ss)
        rr = step(inst, x, v, uu, kappa, g=g)
        return np.concatenate([rr.x.ravel(), rr.v.ravel(), rr.g.ravel()])
    A = np.stack([(f(s + h * e, u) - f(s - h * e, u)) / (2 * h) for e in np.eye(len(s))], axis=1)
    B = np.stack([(f(s, u + h * e) - f(s, u - h * e)) / (2 * h) for e in np.eye(len(u))], axis=1)
    return A, B


def _contact_rope(kappa_h, r_g, offset_scale, seed):
    """6-node rope 0.4 mm above the ground, falling, a sphere under node 3;
    penalty gripper near node 0."""
    inst = W.rope(6, length=0.05, z0=0.0004, T=1, grip_nodes=(0,),
                  spheres=[[0.03, 0.0, 0.0004 - 0.0103, 0.01]])
    n = inst.n
    s = inst.s0.copy()
    s[3 * n + 2::3] = -0.05
    inst = inst.replace(s0=s)
    return W.penalty_grasp(inst, offset_scale=offset_scale, kappa_h=kappa_h, r_g=r_g, seed=seed)


@pytest.mark.parametrize("kappa_h,r_g", [(0.01, 0.0), (0.0, 0.005)])
def test_penalty_step_jacobian_fd(kappa_h, r_g):
    inst = _contact_rope(kappa_h, r_g, 0.002, seed=5)
    s = inst.s0.copy()
    u = np.array([0.05, -0.02, 0.03])
    d = StepDerivative(inst, s, u, inst.kappa_bwd)
    assert d.res.status == STATUS_OK
    assert np.max(d.res.lam) > 1e-3                 # contact carries force
    assert d.pen.D[0] > 1.0                          # the grasp is active
    A, B = d.dense()
    assert A.shape == (inst.n_s, inst.n_s) and B.shape == (inst.n_s, 3)
    Afd, Bfd = _fd_full(inst, s, u, inst.kappa_bwd, 1e-7)
    assert np.linalg.norm(A - Afd) <= 1e-5 * np.linalg.norm(A)
    assert np.linalg.norm(B - Bfd) <= 1e-5 * np.linalg.norm(B)
    # the activation derivative matters: dropping it breaks the match
    if kappa_h > 0:
        d.pen.dD[:] = 0.0
        A0, _ = d.dense()
        assert np.linalg.norm(A0 - Afd) > 1e-3 * np.linalg.norm(A)


def test_penalty_dot_product():
    inst = _contact_rope(0.01, 0.0, 0.002, seed=6)
    rng = np.random.default_rng(3)
    u = np.array([0.02, 0.01, -0.03])
    d = StepDerivative(inst, inst.s0, u, inst.kappa_bwd)
    w = rng.normal(size=inst.n_s)
    ds = rng.normal(size=inst.n_s)
    du = rng.normal(size=3)
    lhs = w @ d.jvp_s(ds[:, None], du[:, None])[:, 0]
    sb, ub = d.vjp_s(w)
    np.testing.assert_allclose(lhs, sb @ ds + ub @ du, rtol=1e-11)


def test_penalty_rollout_gradient_fd():
    """Terminal distance of the last node through a 6-step penalty-grasp
    rollout: adjoint gradient against directional central differences."""
    inst = W.penalty_grasp(W.small_rope_batch(1, 8, 6, seed=93)[0], offset_scale=0.002, seed=2)
    n = inst.n
    goal = np.array([0.5, 0.1, 0.05])

    def loss(s0, u):
        tr, _ = rollout(inst.replace(s0=s0, u=u), kappa=inst.kappa_bwd)
        dlt = tr[-1, 3 * (n - 1):3 * n] - goal
        return float(dlt @ dlt), tr

    L0, tr = loss(inst.s0, inst.u)
    sT = np.zeros(inst.n_s)
    sT[3 * (n - 1):3 * n] = 2.0 * (tr[-1, 3 * (n - 1):3 * n] - goal)
    sb, ub = rollout_backward(inst, tr, sT_bar=sT, kappa=inst.kappa_bwd)
    rng = np.random.default_rng(4)
    for _ in range(3):
        ds = rng.normal(size=inst.n_s)
        du = rng.normal(size=inst.u.shape)
        h = 1e-6
        fd = (loss(inst.s0 + h * ds, inst.u + h * du)[0] - loss(inst.s0 - h * ds, inst.u - h * du)[0]) / (2 * h)
        an = sb @ ds + np.sum(ub * du)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-8)
