"""Pins of the oracle's friction cone (eq. contact-constraint, mu > 0):
the stick/slip threshold tan(theta) = mu of a particle on a plane under
tilted gravity with Anitescu's normal lift mu |y_t| in the slip regime
(closed form), the smoothed step of that particle against a general-purpose
minimiser of the barrier objective written out here, the reduction to the
frictionless stage 2 at mu = 0, the cone and complementarity conditions on
a dragged rope, the smoothed-to-hard limit, and the step Jacobian against
central differences (with a planted mistake that must fail)."""
import numpy as np
import pytest
import scipy.optimize

import workloads as W
from oracle import derivatives as OD
from oracle import step as OS


def _particle(mu, theta, kappa, gamma=1.0):
    g = 9.81 * np.array([np.sin(theta), 0.0, -np.cos(theta)])
    inst = W.rope(1, grip_nodes=(), gravity=tuple(g), gamma=gamma, z0=0.0, T=1, u=np.zeros((1, 0)))
    return inst.replace(mu=mu, kappa_fwd=kappa, kappa_bwd=kappa)


@pytest.mark.parametrize("theta", [0.1, 0.25, 0.35, 0.6, 1.0])
def test_tilted_plane_stick_slip(theta):
    """A particle at rest on the ground under gravity tilted by theta: with
    hard contact it sticks iff tan(theta) <= mu; sliding, its tangential step
    is a (sin - mu cos)/(1 + mu^2) and it lifts by mu times that (the
    projection of the stage-1 point onto the dual cone), a = dt^2 |g|."""
    mu = 0.3
    inst = _particle(mu, theta, 0.0)
    r = OS.step(inst, np.zeros((1, 3)), np.zeros((1, 3)), np.zeros(0), 0.0)
    assert r.status == 0
    a = inst.dt ** 2 * 9.81
    slide = max(0.0, a * (np.sin(theta) - mu * np.cos(theta)) / (1.0 + mu * mu))
    assert (slide == 0.0) == (np.tan(theta) <= mu)
    assert r.x[0, 0] == pytest.approx(slide, abs=1e-6 * a)
    assert r.x[0, 2] == pytest.approx(mu * slide, abs=1e-6 * a)
    assert r.x[0, 1] == 0.0


def test_threshold_is_tan_theta_equal_mu():
    mu = 0.5
    th = np.arctan(mu)
    a = 0.005 ** 2 * 9.81
    for t, moves in ((th - 0.03, False), (th + 0.03, True)):
        inst = _particle(mu, t, 0.0)
        r = OS.step(inst, np.zeros((1, 3)), np.zeros((1, 3)), np.zeros(0), 0.0)
        assert (r.x[0, 0] > 1e-3 * a) == moves


def test_smoothed_particle_is_the_barrier_minimiser():
    """kappa > 0: the step minimises 1/2 (m/dt^2) |D|^2 - kappa/2 log(y_n^2 -
    mu^2 |y_t|^2) with y_n = phi(y*) + D_z, y_t = (y* - x + D)_xy."""
    mu, theta = 0.4, 0.5
    kappa = 2e-5
    inst = _particle(mu, theta, kappa)
    x = np.array([[0.0, 0.0, 0.001]])
    v = np.array([[0.02, -0.01, 0.0]])
    r = OS.step(inst, x, v, np.zeros(0), kappa)
    assert r.status == 0
    ys = r.y[0]
    w = inst.mass / inst.dt ** 2

    def obj(D):
        yn = ys[2] + D[2]
        yt = (ys - x[0] + D)[:2]
        q = yn * yn - mu * mu * (yt @ yt)
        if yn <= 0 or q <= 0:
            return 1e30
        return 0.5 * w * (D @ D) - 0.5 * kappa * np.log(q)

    D0 = r.delta[0] * 0.9 + np.array([0.0, 0.0, 1e-4])
    res = scipy.optimize.minimize(obj, D0, method="Nelder-Mead",
                                  options=dict(xatol=1e-13, fatol=1e-20, maxiter=20000, maxfev=40000))
    np.testing.assert_allclose(r.delta[0], res.x, atol=1e-9)


def _dragged_rope(mu=0.4, kappa=None, n=8):
    rng = np.random.default_rng(5)
    inst = W.rope(n, length=0.3, z0=0.001, T=1, grip_nodes=(0,), spheres=[[0.15, 0.0, -0.02, 0.025]])
    inst = inst.replace(mu=mu)
    if kappa is not None:
        inst = inst.replace(kappa_fwd=kappa, kappa_bwd=kappa)
    s = inst.s0.copy()
    s[3 * n:6 * n] = 0.05 * rng.normal(size=3 * n)
    s[2:3 * n:3] += 0.0005 * rng.normal(size=n)
    return inst, s, np.array([0.3, 0.1, 0.0])


def _stage2_inputs(inst, s, u):
    x, v, _ = OS.split_state(inst, s)
    r = OS.step(inst, x, v, u, inst.kappa_fwd)
    lay = OS.Layout(inst)
    P = OS.psi_hessian_ff(inst, OS.model.elements(inst), lay, r.y, project=False)
    fscale = inst.mass / inst.dt ** 2 * inst.h + inst.mass * 9.81
    return x, r, lay, P, fscale


@pytest.mark.parametrize("kappa", [4e-4, 0.0])
def test_mu_zero_is_the_frictionless_stage2(kappa):
    inst, s, u = _dragged_rope(mu=0.0, kappa=kappa)
    x, r, lay, P, fscale = _stage2_inputs(inst, s, u)
    D, y, lam, _, ok = OS.friction_stage2(P, lay, r.pair_node, r.phi, r.normal, (r.y - x)[r.pair_node], 0.0,
                                          kappa, fscale, inst.h)
    assert ok
    # step() took the frictionless interior point (and crossover) for mu = 0
    np.testing.assert_allclose(D, r.delta[lay.free_nodes].ravel(), rtol=0, atol=1e-10 * inst.h)
    np.testing.assert_allclose(np.einsum("ci,ci->c", lam, r.normal), r.lam, atol=1e-8 * fscale)


def test_cone_and_complementarity_on_a_dragged_rope():
    inst, s, u = _dragged_rope(mu=0.4)
    kappa = inst.kappa_fwd
    x, r, lay, P, fscale = _stage2_inputs(inst, s, u)
    assert r.status == 0 and r.force is not None
    mu = inst.mu
    # force balance P D = sum_c lam_c at the free nodes
    f = np.zeros((inst.n, 3))
    np.add.at(f, r.pair_node, r.force)
    np.testing.assert_allclose(P @ r.delta[lay.free_nodes].ravel(), f[lay.free_nodes].ravel(), atol=1e-11 * fscale)
    some_slip = False
    for c, p in enumerate(r.pair_node):
        nrm = r.normal[c]
        lam = r.force[c]
        ln = lam @ nrm
        lt = lam - ln * nrm
        yn = r.phi[c] + nrm @ r.delta[p]
        disp = r.x[p] - x[p]
        yt = disp - (disp @ nrm) * nrm
        assert np.linalg.norm(lt) <= mu * ln * (1 + 1e-9)            # lam in F_mu
        assert yn >= mu * np.linalg.norm(yt) * (1 - 1e-9)            # y in F_mu^*
        assert yn * ln + yt @ lt == pytest.approx(kappa, rel=1e-7)   # smoothed complementarity
        # friction opposes the tangential displacement
        if np.linalg.norm(yt) > 1e-9:
            assert lt @ yt <= 0.0
            some_slip |= np.linalg.norm(lt) > 1e-3 * ln
    assert some_slip


def test_smoothed_to_hard_limit():
    inst, s, u = _dragged_rope(mu=0.4)
    x, v, _ = OS.split_state(inst, s)
    hard = OS.step(inst, x, v, u, 0.0)
    assert hard.status == 0
    errs = []
    for kappa in (4e-4, 4e-5, 4e-6, 4e-7, 4e-8, 4e-9):
        errs.append(np.max(np.abs(OS.step(inst, x, v, u, kappa).x - hard.x)))
    # monotone, and linear in kappa once the smoothing width is below the
    # gaps (the last decade)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.15 * errs[-2] and errs[-1] < 1e-3 * errs[0]


def _jacobian_errors(inst, s, u):
    n = inst.n
    kap = inst.kappa_bwd
    d = OD.StepDerivative(inst, s, u, kap)
    A, B = d.dense()

    def f(sv, uv):
        x, v, _ = OS.split_state(inst, sv)
        r = OS.step(inst, x, v, uv, kap)
        return np.concatenate([r.x.ravel(), r.v.ravel()])

    hs = np.r_[np.full(3 * n, 1e-7), np.full(3 * n, 1e-5)]
    Afd = np.zeros_like(A)
    for i in range(inst.n_s):
        e = np.zeros(inst.n_s)
        e[i] = hs[i]
        Afd[:, i] = (f(s + e, u) - f(s - e, u)) / (2 * hs[i])
    Bfd = np.zeros_like(B)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1e-5
        Bfd[:, i] = (f(s, u + e) - f(s, u - e)) / 2e-5
    errs = {}
    for rn, rs in (("x", slice(0, 3 * n)), ("v", slice(3 * n, 6 * n))):
        for cn, cs in (("x", slice(0, 3 * n)), ("v", slice(3 * n, 6 * n))):
            errs["A" + rn + cn] = np.linalg.norm(A[rs, cs] - Afd[rs, cs]) / np.linalg.norm(Afd[rs, cs])
        errs["B" + rn] = np.linalg.norm(B[rs] - Bfd[rs]) / np.linalg.norm(Bfd[rs])
    return errs, d


def test_friction_step_jacobian_matches_central_differences(monkeypatch):
    inst, s, u = _dragged_rope(mu=0.4, n=6)
    errs, d = _jacobian_errors(inst, s, u)
    assert max(errs.values()) <= 1e-4, errs
    rng = np.random.default_rng(7)
    ds, du, sb = rng.normal(size=inst.n_s), rng.normal(size=3), rng.normal(size=inst.n_s)
    jv = d.jvp_s(ds[:, None], du[:, None])[:, 0]
    sbar, ubar = d.vjp_s(sb)
    assert sb @ jv == pytest.approx(sbar @ ds + ubar @ du, rel=1e-10)
    # planted mistake: drop the direct dependence on x (tangential displacement)
    real = OD.friction_blocks

    def no_lx(r, x, mu, kappa):
        Kc, Ly, Lx = real(r, x, mu, kappa)
        return Kc, Ly, 0.0 * Lx

    monkeypatch.setattr(OD, "friction_blocks", no_lx)
    bad, _ = _jacobian_errors(inst, s, u)
    assert bad["Axx"] > 1e-3
