"""Pins of the FP64 oracle against what the paper and the mathematics fix.

The paper prints no worked simulator example (its tables hold timings and an
accuracy figure on a hardware dataset), so every pin here is a closed form,
an invariant, an independent solve, or brute force:

P1 free fall, P2 isolated contact (hard projection and smoothed closed form),
P3 spring oscillator (exact discrete amplification matrix), P4 hanging rope
(independent linear solve), P5 momentum / energy, P6 equivariance,
P7 smoothed -> hard limit, P8 linear bending-only step, P9 finite
differences of the step and of the rollout gradient, dot-product test,
independent QP / barrier solves of stage 2, complex-step of the element and
SDF derivatives.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so

import workloads as W
from oracle import STATUS_OK, model, sdf
from oracle.derivatives import StepDerivative, rollout_backward, rollout_jvp
from oracle.step import Layout, contact_pairs, psi_hessian_ff, rollout, step

G = np.array([0.0, 0.0, -9.81])


def particle(z=0.05, vz=0.0, dt=0.005, gamma=0.0, mass=0.01, spheres=(), ground=True,
             width=1e-3, kappa=None, gravity=G):
    kap = W.contact_kappa(mass, dt, width) if kappa is None else kappa
    s0 = np.array([0.1, 0.2, z, 0.3, -0.1, vz])
    return W.rope(1, mass=mass, dt=dt, gamma=gamma, T=1, grip_nodes=(), ground=ground,
                  spheres=spheres, kappa_fwd=kap, kappa_bwd=kap, s0=s0, gravity=gravity,
                  k=0.0, k_bend=0.0, h=0.01)


# ---------------------------------------------------------------- complex step
def cs_grad(f, x, h=1e-30):
    g = np.zeros(x.shape)
    for i in np.ndindex(x.shape):
        xc = x.astype(complex)
        xc[i] += 1j * h
        g[i] = np.imag(f(xc)) / h
    return g


def test_element_derivatives_complex_step():
    rng = np.random.default_rng(0)
    inst = W.cloth(4, 3, T=1)
    el = model.elements(inst)
    y = inst.s0[:3 * inst.n].reshape(-1, 3) + 0.004 * rng.normal(size=(inst.n, 3))
    g = model.gradient(el, y)
    np.testing.assert_allclose(cs_grad(lambda z: model.energy(el, z), y), g, rtol=1e-12, atol=1e-13)
    H = model.hessian(el, y).toarray()
    for j in range(3 * inst.n):
        e = np.zeros(3 * inst.n); e[j] = 1e-30
        col = np.imag(model.gradient(el, y + 1j * e.reshape(-1, 3))).ravel() / 1e-30
        np.testing.assert_allclose(H[:, j], col, rtol=1e-11, atol=1e-9)
    dy = rng.normal(size=y.shape) * 1e-3
    Wm = model.third(el, y, dy).toarray()
    Wcs = np.imag(model.hessian(el, y + 1e-30j * dy).toarray()) / 1e-30
    np.testing.assert_allclose(Wm, Wcs, rtol=1e-10, atol=1e-8)
    # rope with the bending term
    rp = W.rope(7, T=1)
    elr = model.elements(rp)
    yr = rp.s0[:21].reshape(-1, 3) + 0.003 * rng.normal(size=(7, 3))
    np.testing.assert_allclose(cs_grad(lambda z: model.energy(elr, z), yr),
                               model.gradient(elr, yr), rtol=1e-12, atol=1e-13)
    Hr = model.hessian(elr, yr).toarray()
    for j in range(21):
        e = np.zeros(21); e[j] = 1e-30
        col = np.imag(model.gradient(elr, yr + 1j * e.reshape(-1, 3))).ravel() / 1e-30
        np.testing.assert_allclose(Hr[:, j], col, rtol=1e-11, atol=1e-9)
    # energy difference formula vs plain difference (well separated points)
    y1 = y + 0.01 * rng.normal(size=y.shape)
    np.testing.assert_allclose(model.energy_difference(el, y, y1),
                               model.energy(el, y1) - model.energy(el, y), rtol=1e-9)


def test_projected_hessian_is_psd_and_exact_in_tension():
    rng = np.random.default_rng(1)
    inst = W.rope(6, T=1)
    el = model.elements(inst)
    y = inst.s0[:18].reshape(-1, 3) * 0.7 + 0.001 * rng.normal(size=(6, 3))   # compressed
    Hp = model.hessian(el, y, project=True).toarray()
    assert np.linalg.eigvalsh(Hp).min() > -1e-9
    y2 = inst.s0[:18].reshape(-1, 3) * 1.2                                     # stretched
    np.testing.assert_allclose(model.hessian(el, y2, project=True).toarray(),
                               model.hessian(el, y2).toarray(), rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("kind", ["sphere", "box_out", "box_in", "box_edge", "ground"])
def test_sdf_complex_step(kind):
    rng = np.random.default_rng(2)
    if kind == "sphere":
        fn = lambda p: sdf.sphere(p, np.array([0.1, -0.2, 0.05]), 0.07)  # noqa: E731
        pts = np.array([0.1, -0.2, 0.05]) + 0.12 * rng.normal(size=(5, 3))
    elif kind == "ground":
        fn = sdf.ground
        pts = rng.normal(size=(5, 3))
    else:
        c, h = np.array([0.2, 0.1, 0.04]), np.array([0.05, 0.03, 0.04])
        fn = lambda p: sdf.box(p, c, h, 0.005)  # noqa: E731
        if kind == "box_out":
            pts = c + np.array([[0.09, 0.01, 0.0], [0.0, -0.07, 0.01], [0.0, 0.0, 0.09]])
        elif kind == "box_in":
            pts = c + np.array([[0.03, 0.01, 0.0], [0.0, -0.02, 0.01], [0.001, 0.0, 0.03]])
        else:
            pts = c + np.array([[0.07, 0.05, 0.0], [0.07, -0.05, 0.06]])
    phi, n, H = fn(pts)
    for i in range(len(pts)):
        g = cs_grad(lambda q: fn(q[None])[0][0], pts[i])
        np.testing.assert_allclose(n[i], g, rtol=1e-12, atol=1e-12)
        for a in range(3):
            e = np.zeros(3); e[a] = 1e-30
            col = np.imag(fn((pts[i] + 1j * e)[None])[1][0]) / 1e-30
            np.testing.assert_allclose(H[i][:, a], col, rtol=1e-10, atol=1e-10)
    if kind == "box_out":
        # distance to a face / rounded edge, straight from the geometry
        np.testing.assert_allclose(phi[0], 0.09 - 0.05, atol=1e-15)
        np.testing.assert_allclose(phi[2], 0.09 - 0.04, atol=1e-15)
    if kind == "sphere":
        d = np.linalg.norm(pts - np.array([0.1, -0.2, 0.05]), axis=1)
        np.testing.assert_allclose(phi, d - 0.07, atol=1e-15)


# ---------------------------------------------------------------- P1 / P2
@pytest.mark.parametrize("gamma", [0.0, 0.02, 0.5, 1.0])
def test_p1_free_fall(gamma):
    inst = particle(z=1.0, vz=-0.4, gamma=gamma, ground=False)
    r = step(inst, inst.s0[:3], inst.s0[3:], np.zeros(0), 0.0)
    v0 = inst.s0[3:]
    v1 = (1 - gamma) * v0 + inst.dt * G
    np.testing.assert_allclose(r.v.ravel(), v1, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r.x.ravel(), inst.s0[:3] + inst.dt * v1, rtol=0, atol=1e-15)
    assert r.status == STATUS_OK


@pytest.mark.parametrize("vz", [-2.0, -0.3, 0.0, 0.5])
def test_p2_isolated_ground_contact(vz):
    z0 = 0.002
    hard = particle(z=z0, vz=vz, kappa=0.0)
    soft = particle(z=z0, vz=vz, width=1e-3)
    dt = hard.dt
    zs = z0 + dt * vz + dt * dt * G[2]
    rh = step(hard, hard.s0[:3], hard.s0[3:], np.zeros(0), 0.0)
    np.testing.assert_allclose(rh.x[0, 2], max(zs, 0.0), atol=1e-13)
    rs = step(soft, soft.s0[:3], soft.s0[3:], np.zeros(0), soft.kappa_fwd)
    c = soft.kappa_fwd * dt * dt / soft.mass
    np.testing.assert_allclose(rs.x[0, 2], 0.5 * (zs + math.sqrt(zs * zs + 4 * c)), rtol=1e-12)
    # tangential motion is untouched by frictionless contact
    np.testing.assert_allclose(rs.x[0, :2], soft.s0[:2] + dt * soft.s0[3:5], atol=1e-15)
    # derivative of the smoothed correction: 1/2 (1 + z*/sqrt(z*^2 + 4c))
    A, _ = StepDerivative(soft, soft.s0, np.zeros(0), soft.kappa_bwd).dense()
    j2 = 0.5 * (1 + zs / math.sqrt(zs * zs + 4 * c))
    np.testing.assert_allclose(A[2, 2], j2, rtol=1e-10)
    np.testing.assert_allclose(A[2, 5], j2 * dt, rtol=1e-10)


def test_p2_isolated_sphere_contact():
    c, r = np.array([0.1, 0.2, -0.5]), 0.55
    hard = particle(z=0.05, vz=-1.0, kappa=0.0, ground=False, spheres=[[*c, r]])
    rh = step(hard, hard.s0[:3], hard.s0[3:], np.zeros(0), 0.0)
    ys = hard.s0[:3] + hard.dt * hard.s0[3:] + hard.dt ** 2 * G
    assert np.linalg.norm(ys - c) < r                      # penetrating before stage 2
    # hard projection with P = m/dt^2 I onto the sphere: closest point
    np.testing.assert_allclose(rh.x[0], c + r * (ys - c) / np.linalg.norm(ys - c), atol=1e-12)


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("gamma", [0.0, 0.02, 1.0])
def test_p3_spring_oscillator(gamma):
    k, m, dt, l0 = 500.0, 0.01, 0.005, 0.1
    y0 = 0.013
    s0 = np.array([0, 0, 1.0, l0 + y0, 0, 1.0, 0, 0, 0, 0.2, 0, 0])
    inst = W.rope(2, k=k, k_bend=0.0, mass=m, dt=dt, gamma=gamma, T=20, grip_nodes=(0,),
                  ground=False, gravity=(0, 0, 0), s0=s0, h=l0)
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    w2 = k / m
    c = 1.0 / (1.0 + w2 * dt * dt)
    y, v = y0, 0.2
    for t in range(inst.T):
        y, v = c * (y + dt * (1 - gamma) * v), c * (-w2 * dt * y + (1 - gamma) * v)
        np.testing.assert_allclose(traj[t + 1][3] - l0, y, atol=1e-14)
        np.testing.assert_allclose(traj[t + 1][9], v, atol=1e-11)
        np.testing.assert_allclose(traj[t + 1][[4, 5, 10, 11]], [0, 1.0, 0, 0], atol=1e-14)
    A, B = StepDerivative(inst, traj[3], np.zeros(3), 0.0).dense()
    amp = np.array([[c, c * dt * (1 - gamma)], [(c - 1) / dt, c * (1 - gamma)]])
    np.testing.assert_allclose(A[np.ix_([3, 9], [3, 9])], amp, rtol=1e-10)


def test_p3_continuous_limit_frequency():
    """Undamped, dt -> 0: amplitude follows cos(w t) with O(dt) error."""
    k, m, l0, y0 = 200.0, 0.02, 0.1, 0.01
    w = math.sqrt(k / m)
    errs = []
    for dt in (2e-4, 1e-4):
        Tn = int(round(2 * math.pi / w / dt))
        s0 = np.array([0, 0, 0, l0 + y0, 0, 0, 0, 0, 0, 0, 0, 0.0])
        inst = W.rope(2, k=k, k_bend=0.0, mass=m, dt=dt, gamma=0.0, T=Tn, grip_nodes=(0,),
                      ground=False, gravity=(0, 0, 0), s0=s0, h=l0)
        traj, _ = rollout(inst)
        tt = np.arange(Tn + 1) * dt
        errs.append(np.max(np.abs(traj[:, 3] - l0 - y0 * np.cos(w * tt))))
    assert 0.4 < errs[1] / errs[0] < 0.6


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("kb", [0.0, 5.0])
@pytest.mark.parametrize("gamma", [0.02, 1.0])
def test_p4_hanging_rope_fixed_point(kb, gamma):
    n, k, m, l0 = 8, 400.0, 0.01, 0.05
    g = 9.81
    # independent equilibrium along z: unknown z_1..z_{n-1}, z_0 fixed.
    # spring i joins i-1, i: tension k (z_{i-1} - z_i - l0); bending stencil k_b (1,-2,1)
    nf = n - 1
    Amat = np.zeros((nf, nf))
    rhs = np.full(nf, m * g)            # A z = -(constant forces); gravity -m g moves over
    z0 = 1.0
    for i in range(1, n):
        # spring above node i (between i-1 and i) pulls node i up: +k(z_{i-1} - z_i - l0)
        r = i - 1
        Amat[r, r] += -k
        if i - 1 >= 1:
            Amat[r, r - 1] += k
        else:
            rhs[r] -= k * z0
        rhs[r] -= -k * l0
        if i + 1 < n:       # spring below node i pulls down: -k(z_i - z_{i+1} - l0)
            Amat[r, r] += -k
            Amat[r, r + 1] += k
            rhs[r] -= k * l0
    # bending: E = 1/2 kb sum (z_{a} - 2 z_b + z_c)^2 ; force = -dE/dz
    D2 = np.zeros((n - 2, n))
    for j in range(n - 2):
        D2[j, j:j + 3] = [1, -2, 1]
    Kb = kb * D2.T @ D2
    Amat -= Kb[1:, 1:]
    rhs += Kb[1:, 0] * z0
    zf = np.linalg.solve(Amat, rhs)
    z = np.concatenate([[z0], zf])
    if kb == 0.0:
        seg = z[:-1] - z[1:]
        np.testing.assert_allclose(seg, l0 + (n - np.arange(1, n)) * m * g / k, rtol=1e-12)
    pos = np.stack([np.zeros(n), np.zeros(n), z], axis=1)
    s0 = np.concatenate([pos.ravel(), np.zeros(3 * n)])
    inst = W.rope(n, k=k, k_bend=kb, mass=m, gamma=gamma, T=3, ground=False, s0=s0, h=l0)
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    for t in range(1, 4):
        np.testing.assert_allclose(traj[t][:3 * n], traj[0][:3 * n], atol=1e-12)
        np.testing.assert_allclose(traj[t][3 * n:], 0.0, atol=1e-9)


# ---------------------------------------------------------------- P5
def _free_rope(dt, T, gamma=0.0, gravity=(0, 0, 0), seed=3, smooth=False):
    rng = np.random.default_rng(seed)
    n, l0 = 10, 0.05
    pos = np.stack([np.arange(n) * l0 * 1.05, np.zeros(n), np.full(n, 0.5)], axis=1)
    if smooth:
        # low-frequency motion only: rigid spin about z plus the first bending shape
        c = pos.mean(0)
        th = np.linspace(0.0, math.pi, n)
        vel = 2.0 * np.cross(np.array([0, 0, 1.0]), pos - c) + 0.2 * np.stack(
            [np.zeros(n), np.zeros(n), np.sin(th)], axis=1)
        k = 50.0
    else:
        pos += 0.002 * rng.normal(size=pos.shape)
        vel = 0.3 * rng.normal(size=pos.shape)
        k = 300.0
    s0 = np.concatenate([pos.ravel(), vel.ravel()])
    return W.rope(n, k=k, k_bend=2.0, mass=0.01, dt=dt, gamma=gamma, T=T, grip_nodes=(),
                  ground=False, gravity=gravity, s0=s0, h=l0)


def test_p5_momentum():
    inst = _free_rope(0.005, 40, gamma=0.02, gravity=G)
    traj, st = rollout(inst)
    n, m = inst.n, inst.mass
    P = [m * traj[t][3 * n:].reshape(n, 3).sum(0) for t in range(inst.T + 1)]
    for t in range(inst.T):
        np.testing.assert_allclose(P[t + 1], (1 - inst.gamma) * P[t] + inst.dt * n * m * G,
                                   atol=1e-11)
    # quasi-static mode: the centre of mass moves by dt^2 g per step
    qs = _free_rope(0.005, 5, gamma=1.0, gravity=G)
    tq, _ = rollout(qs)
    com = [tq[t][:3 * n].reshape(n, 3).mean(0) for t in range(6)]
    for t in range(5):
        np.testing.assert_allclose(com[t + 1] - com[t], qs.dt ** 2 * G, atol=1e-13)


def _energy(inst, s):
    el = model.elements(inst)
    n = inst.n
    x = s[:3 * n].reshape(n, 3)
    v = s[3 * n:]
    return float(model.energy(el, x)) + 0.5 * inst.mass * float(v @ v)


def _angmom(inst, s):
    n = inst.n
    x = s[:3 * n].reshape(n, 3)
    v = s[3 * n:].reshape(n, 3)
    return inst.mass * np.cross(x, v).sum(0)


def test_p5_energy_and_angular_momentum():
    Tsim = 0.2
    drifts, adrifts = [], []
    for dt in (1e-3, 5e-4, 2.5e-4):
        inst = _free_rope(dt, int(round(Tsim / dt)), smooth=True)
        traj, st = rollout(inst)
        E = np.array([_energy(inst, s) for s in traj])
        assert np.all(np.diff(E) <= 1e-12)          # implicit Euler never gains energy
        drifts.append(E[0] - E[-1])
        L = np.array([_angmom(inst, s) for s in traj])
        adrifts.append(np.linalg.norm(L[-1] - L[0]))
    assert 0.4 < drifts[1] / drifts[0] < 0.65 and 0.4 < drifts[2] / drifts[1] < 0.65
    assert adrifts[2] < adrifts[1] < adrifts[0]


# ---------------------------------------------------------------- P6
def _rot_z(th):
    c, s = math.cos(th), math.sin(th)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


@pytest.mark.parametrize("kind", ["rope", "cloth"])
def test_p6_equivariance(kind):
    if kind == "rope":
        inst = W.small_rope_batch(1, 12, 12, seed=11)[0]
    else:
        inst = W.small_cloth_batch(1, 5, 4, 8, seed=12)[0]
    traj, _ = rollout(inst)
    n = inst.n
    for name, Rm, tvec in (("translate", np.eye(3), np.array([0.3, -0.2, 0.0])),
                           ("rotate", _rot_z(0.7), np.zeros(3)),
                           ("mirror", np.diag([1.0, -1.0, 1.0]), np.zeros(3))):
        def tf_state(s):
            x = s[:3 * n].reshape(n, 3) @ Rm.T + tvec
            v = s[3 * n:].reshape(n, 3) @ Rm.T
            return np.concatenate([x.ravel(), v.ravel()])
        sph = inst.spheres.copy()
        sph[:, :3] = sph[:, :3] @ Rm.T + tvec
        boxes = inst.boxes.copy()
        if len(boxes):
            if name == "rotate":
                continue                        # axis-aligned boxes are not rotation-invariant
            boxes[:, :3] = boxes[:, :3] @ Rm.T + tvec
        u = (inst.u.reshape(inst.T, -1, 3) @ Rm.T).reshape(inst.T, -1)
        other = inst.replace(s0=tf_state(inst.s0), u=u, spheres=sph, boxes=boxes)
        t2, _ = rollout(other)
        for t in range(inst.T + 1):
            ref = tf_state(traj[t])
            # velocities are (x+ - x)/dt: rounding is amplified by 1/dt
            np.testing.assert_allclose(t2[t][:3 * n], ref[:3 * n], rtol=0, atol=1e-10, err_msg=name)
            np.testing.assert_allclose(t2[t][3 * n:], ref[3 * n:], rtol=0, atol=1e-8, err_msg=name)


# ---------------------------------------------------------------- P7
def test_p7_smoothed_to_hard_limit():
    base = W.config_c1()
    base = base.replace(T=25, u=base.u[:25])
    th, _ = rollout(base, kappa=0.0)
    errs = []
    for w in (4e-4, 2e-4, 1e-4):
        kap = W.contact_kappa(base.mass, base.dt, w)
        ts, _ = rollout(base, kappa=kap)
        errs.append(np.max(np.abs(ts[:, :60] - th[:, :60])))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.6 * errs[1] and errs[1] < 0.6 * errs[0]
    # isolated particle at phi = 0: gap is exactly the width
    p = particle(z=0.0, vz=0.0, gravity=(0, 0, 0), width=3e-4)
    r = step(p, p.s0[:3], p.s0[3:], np.zeros(0), p.kappa_fwd)
    np.testing.assert_allclose(r.x[0, 2], 3e-4, rtol=1e-12)


# ---------------------------------------------------------------- P8
def test_p8_linear_bending_only_jacobian():
    n, kb, m, dt, gamma = 7, 30.0, 0.02, 0.004, 0.1
    rng = np.random.default_rng(5)
    inst = W.rope(n, k=0.0, k_bend=kb, mass=m, dt=dt, gamma=gamma, T=1, ground=False,
                  gravity=(0, 0, 0))
    s = inst.s0 + 0.01 * rng.normal(size=inst.s0.shape)
    A, B = StepDerivative(inst, s, np.array([0.1, 0.0, -0.2]), 0.0).dense()
    D2 = np.zeros((n - 2, n))
    for j in range(n - 2):
        D2[j, j:j + 3] = [1, -2, 1]
    Kb = np.kron(kb * D2.T @ D2, np.eye(3))
    Mh = m / dt ** 2
    f = np.arange(3, 3 * n)
    g = np.arange(0, 3)
    Hff = Mh * np.eye(len(f)) + Kb[np.ix_(f, f)]
    Gx = np.zeros((3 * n, 3 * n))
    Gx[np.ix_(f, f)] = np.linalg.solve(Hff, Mh * np.eye(len(f)))
    Gx[np.ix_(f, g)] = -np.linalg.solve(Hff, Kb[np.ix_(f, g)])
    Gx[np.ix_(g, g)] = np.eye(3)
    Pf = np.diag([0.0] * 3 + [1.0] * (3 * n - 3))
    I = np.eye(3 * n)
    Aref = np.block([[Gx, dt * (1 - gamma) * Gx @ Pf], [(Gx - I) / dt, (1 - gamma) * Gx @ Pf]])
    np.testing.assert_allclose(A, Aref, rtol=1e-10, atol=1e-10)
    Gu = dt * Gx[:, g]
    Bref = np.vstack([Gu, Gu / dt])
    np.testing.assert_allclose(B, Bref, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------- stage 2 independent solves
def _stage2_problem(kappa):
    """A 6-node rope (12 mm spacing) laid over a sphere, its last node below
    the ground, so that sphere and ground pairs are both active."""
    inst = W.small_rope_batch(1, 6, 1, seed=21)[0]
    c = inst.spheres[0, :3]
    r = inst.spheres[0, 3]
    n, h = inst.n, 0.012
    x = np.stack([c[0] + (np.arange(n) - 2.5) * h, np.full(n, c[1]),
                  np.full(n, c[2] + r * 0.98)], axis=1)
    x[-1, 2] = -0.002
    s = np.concatenate([x.ravel(), np.zeros(3 * n)])
    inst = inst.replace(s0=s, h=h, grip_nodes=(0,), u=np.zeros((1, 3)), kappa_fwd=kappa,
                        kappa_bwd=kappa)
    return inst, s


@pytest.mark.parametrize("kappa", [0.0, 4e-4])
def test_stage2_against_scipy(kappa):
    inst, s = _stage2_problem(kappa)
    n = inst.n
    r = step(inst, s[:3 * n], s[3 * n:], np.zeros(3), kappa)
    assert r.status == STATUS_OK
    lay = Layout(inst)
    el = model.elements(inst)
    P = psi_hessian_ff(inst, el, lay, r.y, project=False).toarray()
    pn, po, phi, nrm, _ = contact_pairs(inst, lay, r.y)
    Nm = np.zeros((len(phi), P.shape[0]))
    for c in range(len(phi)):
        Nm[c, 3 * lay.fpos[pn[c]]:3 * lay.fpos[pn[c]] + 3] = nrm[c]
    D = r.delta.ravel()[lay.fidx]
    if kappa == 0.0:
        res = so.minimize(lambda d: 0.5 * d @ P @ d, np.zeros(P.shape[0]), jac=lambda d: P @ d,
                          constraints=[{"type": "ineq", "fun": lambda d: phi + Nm @ d,
                                        "jac": lambda d: Nm}], method="SLSQP",
                          options={"ftol": 1e-16, "maxiter": 500})
        np.testing.assert_allclose(D, res.x, atol=1e-8)
        assert np.min(phi + Nm @ D) > -1e-12
    else:
        def f(d):
            gp = phi + Nm @ d
            return 0.5 * d @ P @ d - kappa * np.sum(np.log(gp)) if np.all(gp > 0) else np.inf

        def gr(d):
            return P @ d - Nm.T @ (kappa / (phi + Nm @ d))

        def hs(d):
            gp = phi + Nm @ d
            return P + Nm.T @ np.diag(kappa / gp ** 2) @ Nm
        # stationarity of the strictly convex barrier objective = its unique minimiser
        assert np.linalg.eigvalsh(P).min() > 0
        assert np.max(np.abs(gr(D))) < 1e-10
        d0 = D + 1e-5
        res = so.minimize(f, d0, jac=gr, hess=hs, method="Newton-CG",
                          options={"xtol": 1e-14, "maxiter": 200})
        np.testing.assert_allclose(D, res.x, atol=1e-10)
        np.testing.assert_allclose(r.lam * r.gap, kappa, rtol=1e-9)


# ---------------------------------------------------------------- P9
def _fd_jacobian(inst, s, u, kappa, h):
    n = inst.n
    cols = []
    def f(ss, uu):
        rr = step(inst, ss[:3 * n], ss[3 * n:], uu, kappa)
        return np.concatenate([rr.x.ravel(), rr.v.ravel()])
    for j in range(len(s)):
        e = np.zeros(len(s)); e[j] = h
        cols.append((f(s + e, u) - f(s - e, u)) / (2 * h))
    A = np.stack(cols, axis=1)
    ucols = []
    for j in range(len(u)):
        e = np.zeros(len(u)); e[j] = h
        ucols.append((f(s, u + e) - f(s, u - e)) / (2 * h))
    return A, np.stack(ucols, axis=1)


@pytest.mark.parametrize("case", ["rope_soft", "cloth_soft", "rope_hard"])
def test_p9_step_jacobian_fd(case):
    if case.startswith("rope"):
        kap = 0.0 if case == "rope_hard" else None
        inst, s = _stage2_problem(4e-4 if kap is None else 0.0)
        u = np.array([0.05, -0.02, 0.03])
        kappa = inst.kappa_bwd
    else:
        # 4x4 cloth (1 cm cells) resting 0.4 mm above a rounded box, one row
        # hanging past the box edge onto a small sphere, moving down
        top = 0.04
        inst = W.cloth(4, 4, size=0.03, T=1, boxes=[[0.0153, 0.0, 0.02, 0.02, 0.02, 0.02, 0.005]],
                       spheres=[[0.02, 0.03, top + 0.0004 - 0.0105, 0.01]], z0=top + 0.0004)
        n = inst.n
        s = inst.s0.copy()
        s[3 * n + 2::3] = -0.05
        inst = inst.replace(s0=s)
        u = np.array([0.01, 0.0, 0.02, -0.01, 0.0, 0.01])
        kappa = inst.kappa_bwd
    d = StepDerivative(inst, s, u, kappa)
    assert d.res.status == STATUS_OK
    A, B = d.dense()
    Afd, Bfd = _fd_jacobian(inst, s, u, kappa, 1e-5)
    assert np.linalg.norm(A - Afd) <= 1e-5 * np.linalg.norm(A)
    assert np.linalg.norm(B - Bfd) <= 1e-5 * np.linalg.norm(B)
    if case == "rope_hard":
        assert d.res.active.sum() >= 2
    else:
        assert np.max(d.res.lam) > 1e-2       # a pair carries real force


def test_dot_product_jvp_vjp():
    inst = W.small_cloth_batch(1, 4, 3, 1, seed=41)[0]
    rng = np.random.default_rng(7)
    s = inst.s0 + 0.001 * rng.normal(size=inst.s0.shape)
    d = StepDerivative(inst, s, inst.u[0], inst.kappa_bwd)
    n = inst.n
    w = rng.normal(size=6 * n)
    ds = rng.normal(size=6 * n)
    du = rng.normal(size=6)
    dxn, dvn = d.jvp(ds[:3 * n], ds[3 * n:], du)
    lhs = w @ np.concatenate([dxn.ravel(), dvn.ravel()])
    xb, vb, ub = d.vjp(w[:3 * n], w[3 * n:])
    rhs = np.concatenate([xb, vb]) @ ds + ub @ du
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_p9_rollout_gradient_directional_fd():
    """C1: gradient of the terminal distance-to-goal wrt all controls,
    checked along random directions by central differences."""
    c1 = W.config_c1()
    inst = c1.replace(T=20, u=c1.u[:20])
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    n = inst.n
    goal = W.gen.C1_GOAL

    def loss(u):
        tr, _ = rollout(inst.replace(u=u))
        return np.linalg.norm(tr[-1, 3 * (n - 1):3 * n] - goal)

    dvec = traj[-1, 3 * (n - 1):3 * n] - goal
    sb = np.zeros(6 * n)
    sb[3 * (n - 1):3 * n] = dvec / np.linalg.norm(dvec)
    s0b, ub = rollout_backward(inst, traj, sT_bar=sb)
    rng = np.random.default_rng(9)
    for _ in range(2):
        du = rng.normal(size=inst.u.shape)
        h = 1e-4
        fd = (loss(inst.u + h * du) - loss(inst.u - h * du)) / (2 * h)
        np.testing.assert_allclose(np.sum(ub * du), fd, rtol=2e-6)
    # forward-mode tangent agrees with the adjoint
    du = rng.normal(size=inst.u.shape)
    tang = rollout_jvp(inst, traj, np.zeros(6 * n), du)
    np.testing.assert_allclose(sb @ tang[-1][:, 0], np.sum(ub * du), rtol=1e-10)


# ---------------------------------------------------------------- P13
def test_p13_surrogate_mode():
    """kappa_fwd = 0 < kappa_bwd: the step Jacobian used by the backward pass is
    the finite-difference Jacobian of the smoothed step, taken at the states
    of the hard trajectory."""
    c1 = W.config_c1()
    inst = c1.replace(T=30, u=c1.u[:30])
    kap = inst.kappa_bwd
    hard = inst.replace(kappa_fwd=0.0)
    traj, st = rollout(hard)
    assert st.max() == STATUS_OK
    t = 29
    d = StepDerivative(hard, traj[t], hard.u[t], kap)
    A, B = d.dense()
    Afd, Bfd = _fd_jacobian(hard, traj[t], hard.u[t], kap, 1e-5)
    assert np.linalg.norm(A - Afd) <= 1e-5 * np.linalg.norm(A)
    # and the hard trajectory itself rests on the ground / sphere without penetration
    n = inst.n
    z = traj[:, 2:3 * n:3]
    assert z.min() > -1e-12
