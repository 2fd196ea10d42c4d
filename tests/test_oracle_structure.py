"""More pins of the FP64 oracle, each against something other than itself.

* Cloth lattice (Sec. 4.1 nodal system; a mass-spring cloth of structural,
  shear and bend springs): the element lists equal a brute-force enumeration
  of node pairs by grid offset, with the expected count per class (1984
  structural, 1922 shear and 1920 bend springs at 32 x 32), and a cloth
  hanging from its top row, brought to equilibrium by a separate solver of
  an energy written out here, is a fixed point of the oracle's step.
* Compression guard (P14): a straight rope compressed to 75 % of its rest
  length stays straight, so the stage-1 root is a saddle of the incremental
  potential and the exact Hessian there is indefinite (but not singular).
  The oracle converges to it without flagging, and its step Jacobian
  (eq. diff-sim with the exact, indefinite dF/dq*) matches central
  differences of the root continued by a local root finder.
* Planner: the reference gradient of the planning cost matches central
  differences of the cost through the oracle's rollout; the projected step
  clips; ties go to the lowest candidate index.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so

import workloads as W
from oracle import STATUS_OK, model, planner
from oracle.derivatives import StepDerivative
from oracle.step import Layout, psi_gradient, psi_hessian_ff, rollout, step

G = np.array([0.0, 0.0, -9.81])


# ---------------------------------------------------------------- cloth lattice
def _brute_pairs(nx, ny):
    """All node pairs of the grid by their offset: structural |d| = (1,0) or
    (0,1); shear (1,1); bend (2,0) or (0,2)."""
    out = {"struct": set(), "shear": set(), "bend": set()}
    nodes = [(ix, iy) for iy in range(ny) for ix in range(nx)]
    for a in range(len(nodes)):
        for b in range(a + 1, len(nodes)):
            dx = abs(nodes[b][0] - nodes[a][0])
            dy = abs(nodes[b][1] - nodes[a][1])
            if (dx, dy) in ((1, 0), (0, 1)):
                out["struct"].add((a, b))
            elif (dx, dy) == (1, 1):
                out["shear"].add((a, b))
            elif (dx, dy) in ((2, 0), (0, 2)):
                out["bend"].add((a, b))
    return out


@pytest.mark.parametrize("nx,ny", [(32, 32), (5, 4), (2, 2), (3, 2), (2, 5), (7, 1 + 2)])
def test_cloth_lattice_against_brute_force(nx, ny):
    inst = W.cloth(nx, ny, T=1)
    el = model.elements(inst)
    h = inst.h
    got = {"struct": set(), "shear": set(), "bend": set()}
    for a, b, r, k in zip(el.sa, el.sb, el.rest, el.k):
        key = (int(min(a, b)), int(max(a, b)))
        if abs(r - h) < 1e-12 * h:
            cls, kk = "struct", inst.k_struct
        elif abs(r - h * math.sqrt(2.0)) < 1e-12 * h:
            cls, kk = "shear", inst.k_shear
        else:
            assert abs(r - 2.0 * h) < 1e-12 * h
            cls, kk = "bend", inst.k_bend
        assert k == kk
        assert key not in got[cls]
        got[cls].add(key)
    ref = _brute_pairs(nx, ny)
    assert got == ref
    assert len(el.sa) == sum(len(v) for v in ref.values())
    assert len(ref["struct"]) == ny * (nx - 1) + nx * (ny - 1)
    assert len(ref["shear"]) == 2 * (nx - 1) * (ny - 1)
    assert len(ref["bend"]) == ny * max(nx - 2, 0) + nx * max(ny - 2, 0)
    if (nx, ny) == (32, 32):
        assert (len(ref["struct"]), len(ref["shear"]), len(ref["bend"])) == (1984, 1922, 1920)
    assert len(el.ba) == 0          # the cloth bends through its bend springs only


def _hanging_equilibrium(nx, ny, h, k_s, k_sh, k_b, m, z_top):
    """Equilibrium of a cloth hanging in the x-z plane from its top row,
    found by a root solve of the gradient of
        U(p) = sum_pairs 1/2 k (|p_b - p_a| - l0)^2 + sum_free m g z,
    with the pairs enumerated by grid offset (independent of the oracle)."""
    pairs = []
    for cls, (kk, l0) in {"struct": (k_s, h), "shear": (k_sh, h * math.sqrt(2.0)),
                          "bend": (k_b, 2.0 * h)}.items():
        for a, b in _brute_pairs(nx, ny)[cls]:
            pairs.append((a, b, kk, l0))
    n = nx * ny
    rest = np.array([[ix * h, 0.0, z_top - iy * h] for iy in range(ny) for ix in range(nx)])
    free = np.array([i >= nx for i in range(n)])

    def grad(pf):
        p = rest.copy()
        p[free] = pf.reshape(-1, 3)
        g = np.zeros((n, 3))
        for a, b, kk, l0 in pairs:
            e = p[b] - p[a]
            L = math.sqrt(e @ e)
            f = kk * (L - l0) / L * e
            g[b] += f
            g[a] -= f
        g[:, 2] += m * 9.81
        return g[free].ravel()

    sol = so.root(grad, rest[free].ravel(), method="hybr", options={"xtol": 1e-15})
    p = rest.copy()
    p[free] = sol.x.reshape(-1, 3)
    p[:, 1] = 0.0          # in-plane forces only; the solver leaves ~1e-16 of y
    return p, float(np.max(np.abs(grad(p[free].ravel()))))


@pytest.mark.parametrize("gamma", [0.02, 1.0])
def test_hanging_cloth_fixed_point(gamma):
    nx, ny, h, m = 5, 4, 0.05, 0.01
    k_s, k_sh, k_b = 500.0, 250.0, 5.0
    p, res = _hanging_equilibrium(nx, ny, h, k_s, k_sh, k_b, m, 0.5)
    assert res <= 1e-12
    assert np.max(np.abs(p[:, 1])) == 0.0
    # the cloth sags and narrows: a genuinely 2-D equilibrium
    assert p[-1, 2] < 0.5 - (ny - 1) * h - 1e-4
    assert abs(p[-1, 0] - p[-nx, 0]) < (nx - 1) * h - 1e-5
    s0 = np.concatenate([p.ravel(), np.zeros(3 * nx * ny)])
    inst = W.cloth(nx, ny, size=(nx - 1) * h, k_struct=k_s, k_shear=k_sh, k_bend=k_b, mass=m, gamma=gamma,
                   T=3, grip_nodes=tuple(range(nx)), ground=False, s0=s0)
    assert abs(inst.h - h) < 1e-15
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    for t in range(1, 4):
        np.testing.assert_allclose(traj[t][:3 * inst.n], traj[0][:3 * inst.n], rtol=0, atol=1e-11)
        np.testing.assert_allclose(traj[t][3 * inst.n:], 0.0, atol=1e-8)


def test_hanging_cloth_detects_a_dropped_spring():
    """The fixed point above is sensitive to every spring: removing one shear
    diagonal from the independent energy moves the equilibrium by far more
    than the fixed-point tolerance."""
    nx, ny, h, m = 5, 4, 0.05, 0.01
    p, _ = _hanging_equilibrium(nx, ny, h, 500.0, 250.0, 5.0, m, 0.5)
    s0 = np.concatenate([p.ravel(), np.zeros(3 * nx * ny)])
    inst = W.cloth(nx, ny, size=(nx - 1) * h, mass=m, T=1, grip_nodes=tuple(range(nx)), ground=False, s0=s0)
    el = model.elements(inst)
    g_all = model.gradient(el, p)
    keep = np.ones(len(el.sa), dtype=bool)
    keep[np.nonzero(np.abs(el.rest - h * math.sqrt(2.0)) < 1e-12)[0][3]] = False
    el2 = model.Elements(el.n, el.sa[keep], el.sb[keep], el.rest[keep], el.k[keep], el.ba, el.bb, el.bc, el.kb)
    g_drop = model.gradient(el2, p)
    assert np.max(np.abs(g_all - g_drop)) > 1e-4


# ---------------------------------------------------------------- P14 compression guard
compressed_rope = W.compressed_rope


def test_p14_root_is_a_straight_saddle():
    inst = compressed_rope()
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    n = inst.n
    xs = traj[:, :3 * n].reshape(-1, n, 3)
    assert np.max(np.abs(xs[:, :, :2])) == 0.0
    el, lay = model.elements(inst), Layout(inst)
    for t in range(inst.T):
        x = traj[t, :3 * n].reshape(n, 3)
        v = traj[t, 3 * n:].reshape(n, 3)
        r = step(inst, x, v, inst.u[t], inst.kappa_fwd, el, lay)
        assert r.status == STATUS_OK
        F = psi_gradient(inst, el, lay, r.y, r.xhat)
        assert np.max(np.abs(F)) <= 1e-9
        H = psi_hessian_ff(inst, el, lay, r.y, project=False).toarray()
        ev = np.linalg.eigvalsh(H)
        assert ev.min() < -100.0                       # indefinite
        assert np.min(np.abs(ev)) > 1e-6 * np.max(np.abs(ev))   # not singular
        # the projected Hessian (Newton's direction) stays positive definite
        assert np.linalg.eigvalsh(psi_hessian_ff(inst, el, lay, r.y, project=True).toarray()).min() > 0.0


def _root_continuation_step(inst, x, v, u, y_start):
    """x+ and v+ of the step for (x, v, u) by a local root solve of F(y) = 0
    started at y_start (the neighbouring root), not by the oracle's Newton."""
    el, lay = model.elements(inst), Layout(inst)
    n, dt = inst.n, inst.dt
    xhat = x + dt * (1.0 - inst.gamma) * v
    b = x.copy()
    uu = u.reshape(-1, 3)
    for kk, j in enumerate(inst.grip_nodes):
        b[j] = x[j] + dt * uu[kk]

    def F(yf):
        y = b.copy()
        y[lay.free] = yf.reshape(-1, 3)
        return psi_gradient(inst, el, lay, y, xhat)[lay.free].ravel()

    sol = so.root(F, y_start[lay.free].ravel(), method="hybr", options={"xtol": 1e-14})
    assert np.max(np.abs(F(sol.x))) <= 1e-10
    y = b.copy()
    y[lay.free] = sol.x.reshape(-1, 3)
    vn = (y - x) / dt
    for kk, j in enumerate(inst.grip_nodes):
        vn[j] = uu[kk]
    return np.concatenate([y.ravel(), vn.ravel()])


def test_p14_step_jacobian_matches_root_continuation():
    inst = compressed_rope(n=6, T=3)
    traj, st = rollout(inst)
    assert st.max() == STATUS_OK
    n, t = inst.n, 2
    s, u = traj[t], inst.u[t]
    d = StepDerivative(inst, s, u, inst.kappa_bwd)
    A, B = d.dense()
    y0 = d.res.y
    hs = 1e-6
    Afd = np.zeros_like(A)
    for j in range(inst.n_s):
        e = np.zeros(inst.n_s)
        e[j] = hs
        sp_, sm_ = s + e, s - e
        fp = _root_continuation_step(inst, sp_[:3 * n].reshape(n, 3), sp_[3 * n:].reshape(n, 3), u, y0)
        fm = _root_continuation_step(inst, sm_[:3 * n].reshape(n, 3), sm_[3 * n:].reshape(n, 3), u, y0)
        Afd[:, j] = (fp - fm) / (2 * hs)
    Bfd = np.zeros_like(B)
    x, v = s[:3 * n].reshape(n, 3), s[3 * n:].reshape(n, 3)
    for j in range(inst.n_u):
        e = np.zeros(inst.n_u)
        e[j] = hs
        fp = _root_continuation_step(inst, x, v, u + e, y0)
        fm = _root_continuation_step(inst, x, v, u - e, y0)
        Bfd[:, j] = (fp - fm) / (2 * hs)
    x_, v_ = slice(0, 3 * n), slice(3 * n, 6 * n)
    for rs in (x_, v_):
        for cs in (x_, v_):
            np.testing.assert_allclose(A[rs, cs], Afd[rs, cs], rtol=0,
                                       atol=2e-6 * max(np.abs(Afd[rs, cs]).max(), 1e-3))
        np.testing.assert_allclose(B[rs], Bfd[rs], rtol=0, atol=2e-6 * max(np.abs(Bfd[rs]).max(), 1e-3))
    # along the axis (z) the oracle's own step stays on the straight branch:
    # its central differences agree too
    for j in [3 * 2 + 2, 3 * n + 3 * 3 + 2]:
        e = np.zeros(inst.n_s)
        e[j] = hs
        rp = step(inst, (s + e)[:3 * n].reshape(n, 3), (s + e)[3 * n:].reshape(n, 3), u, inst.kappa_fwd)
        rm = step(inst, (s - e)[:3 * n].reshape(n, 3), (s - e)[3 * n:].reshape(n, 3), u, inst.kappa_fwd)
        col = (np.concatenate([rp.x.ravel(), rp.v.ravel()]) - np.concatenate([rm.x.ravel(), rm.v.ravel()])) / (2 * hs)
        np.testing.assert_allclose(A[:, j], col, rtol=0, atol=2e-6 * np.abs(col).max())
    # the transverse columns need the exact (indefinite) Hessian: with the
    # projected one in its place the derivative is wrong
    el, lay = model.elements(inst), Layout(inst)
    Hp = psi_hessian_ff(inst, el, lay, y0, project=True).toarray()
    H = psi_hessian_ff(inst, el, lay, y0, project=False).toarray()
    assert np.linalg.norm(Hp - H) > 0.1 * np.linalg.norm(H)


# ---------------------------------------------------------------- planner
def _plan_rope():
    inst = W.small_rope_batch(1, 6, 5, seed=1234)[0]
    return inst, np.array([0.2, 0.1, 0.05])


def test_planner_gradient_matches_central_differences():
    inst, goal = _plan_rope()
    gn, reg = inst.n - 1, 1e-3
    u = inst.u + 0.1
    J, g, _ = planner.cost_gradient(inst, u, gn, goal, reg)
    fd = np.zeros_like(u)
    h = 1e-5      # the step's Newton tolerance leaves ~1e-13 of noise in J
    for idx in np.ndindex(u.shape):
        e = np.zeros_like(u)
        e[idx] = h
        fd[idx] = (planner.cost(inst, u + e, gn, goal, reg)[0] - planner.cost(inst, u - e, gn, goal, reg)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=2e-6 * np.abs(fd).max())
    assert J == planner.cost(inst, u, gn, goal, reg)[0]


def test_planner_step_ties_and_descent():
    inst, goal = _plan_rope()
    gn, reg = inst.n - 1, 1e-3
    u = np.array([[0.3, -0.7, 0.1]])
    g = np.array([[-1.0, 1.0, 2.0]])
    np.testing.assert_array_equal(planner.projected_step(u, g, 0.5, 0.5), [[0.5, -0.5, -0.5]])
    assert planner.argmin_lowest([3.0, 1.0, 1.0, 2.0]) == 1
    assert planner.argmin_lowest([1.0, 1.0]) == 0
    # two identical candidates tie; the lower index wins
    starts = np.stack([inst.u + 0.05, inst.u, inst.u])
    r = planner.plan(inst, starts, gn, goal, iters=1, step=0.05, u_max=0.5, u_reg=reg)
    assert r["costs"][1] == r["costs"][2]
    assert r["best"] in (0, 1)
    # zero iterations: the costs of the starts; one small step descends
    r0 = planner.plan(inst, starts, gn, goal, iters=0, step=0.05, u_max=0.5, u_reg=reg)
    for c in range(3):
        assert r0["costs"][c] == planner.cost(inst, starts[c], gn, goal, reg)[0]
    J0, g0, _ = planner.cost_gradient(inst, inst.u, gn, goal, reg)
    step = 1e-2 / max(np.abs(g0).max(), 1e-12)
    J1 = planner.cost(inst, planner.projected_step(inst.u, g0, step, 0.5), gn, goal, reg)[0]
    assert J1 < J0


def test_singular_flag_only_for_a_singular_hessian():
    """The step flags NOT_PD only when dF/dq* is singular (its derivative
    is then undefined), not when it is merely indefinite."""
    import scipy.sparse as sp
    from oracle.step import singular
    assert not singular(sp.csc_matrix(np.diag([3.0, -2.0, 1.0])))
    assert not singular(sp.csc_matrix(np.array([[0.0, 1.0], [1.0, 0.0]])))
    assert singular(sp.csc_matrix(np.array([[1.0, 2.0], [2.0, 4.0]])))
    assert singular(sp.csc_matrix(np.diag([1.0, 1e-15, 1.0])))
