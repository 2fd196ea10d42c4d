"""One simulator step q+ = f(q, u) and rollouts, in FP64 (Sec. 4.1).

The step follows the paper's two-stage solver (paragraph "Simulation
Solver"), with the readings stated below where the paper is silent.

1. Grippers (eq. holonomic-constraint).  Dirichlet mode (the grasp in its
   D -> infinity limit): gripper k holds node j; x+_j = x_j + dt u_k,
   v+_j = u_k, and node j is removed from the unknowns.  Penalty mode
   (eq. dynamics-first-stage with the holonomic penalty and the smoothed
   activation of the Contact Smoothing paragraph): the gripper position g_k
   is part of the state, g+_k = g_k + dt u_k, node j stays free, and
   F gains D_k (y_j - g+_k) with D_k = D_max exp(-|c_k| / kappa_h),
   c_k = x_j - g_k (the constraint evaluated at the current state; for
   kappa_h = 0 the indicator D_max [|c_k| <= r_g]).  D_k I enters P too.
2. Predictor: x_hat = x + dt (1 - gamma) v.  gamma = 1 is exactly the paper's
   quasi-static eq. (dynamics) with M (q+ - q)/dt^2; gamma < 1 keeps a
   fraction of the velocity (damped implicit Euler).
3. Stage 1 (eq. dynamics-first-stage): find y* with
   F(y) = M (y - x_hat)/dt^2 + dE/dy - M g = 0 over the free nodes.  F is the
   gradient of Psi(y) = |y - x_hat|_M^2 / (2 dt^2) + E(y) - (M g)^T y, so the
   Newton iteration is a minimisation: direction from the spring-projected
   Hessian, Armijo backtracking on Psi, stop at |F|_inf <= 1e-10 (1 + |M g|_inf).
4. Stage 2 (eq. dynamics-second-stage) at y*: P = dF/dy (y*) (the exact
   Hessian of Psi, consistent with the stage-1 units), one contact pair per
   (free node, obstacle), signed distance phi_c and normal n_c at y*.
   * kappa > 0 (Contact Smoothing paragraph): P D = sum_c n_c lam_c with
     lam_c gap_c = kappa, gap_c = phi_c + n_c . D_p > 0, lam_c > 0;
   * kappa = 0: the QP min 1/2 D^T P D s.t. phi_c + n_c . D_p >= 0.
   Both are solved by a primal-dual interior-point iteration on
   (D, lam, gap); the hard case then fixes the active set and solves the
   equality-constrained KKT system exactly.
5. x+ = y* + D on free nodes, v+ = (x+ - x)/dt.

Friction (mu > 0, eq. contact-constraint with Anitescu's relaxation): each
pair's constraint value is y_c = [phi_c + n_c . D_p ; t_c . (s_p + D_p)]
with s = y* - x the stage-1 displacement, i.e. the normal row linearised at
y* as in eq. (dynamics-second-stage) and the tangential rows measuring the
node's whole displacement over the step, x+_p - x_p, as in eq.
(contact-constraint).  (Measured from y*, as the stage-2 equation prints
it, the tangential rows would vanish at D = 0 and a projection onto the
cone could never move a node tangentially: friction would do nothing.)
The cone is F_mu = {lam : |lam_t| <= mu lam_n}, its dual F_mu^* =
{y : y_n >= mu |y_t|}.  Smoothed (kappa > 0): the central-path point of
min 1/2 D^T P D - kappa sum_c psi(y_c), psi(y) = 1/2 log(y_n^2 - mu^2
|y_t|^2), whose stationarity gives lam_c = kappa grad psi(y_c) in F_mu,
y_c in F_mu^* and y_c . lam_c = kappa, the paper's smoothed
complementarity.  Hard (kappa = 0): the same problem followed along a
decreasing kappa to 1e-16 fscale h.  With mu = 0 both reduce to the
frictionless problem above.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import (STATUS_NEWTON_NOCONV, STATUS_NONFINITE, STATUS_NOT_PD, STATUS_OK,
               STATUS_QP_NOCONV, model, sdf)


@dataclass
class StepResult:
    x: np.ndarray          # (n, 3) next positions
    v: np.ndarray          # (n, 3) next velocities
    y: np.ndarray          # (n, 3) stage-1 solution y* (gripped nodes at their targets)
    delta: np.ndarray      # (n, 3) stage-2 correction (0 on gripped nodes)
    xhat: np.ndarray       # (n, 3) predictor
    pair_node: np.ndarray  # (nc,) node of each contact pair
    pair_obs: np.ndarray   # (nc,) obstacle of each contact pair
    phi: np.ndarray        # (nc,) signed distance at y*
    normal: np.ndarray     # (nc, 3) SDF gradient at y*
    curv: np.ndarray       # (nc, 3, 3) SDF Hessian at y*
    lam: np.ndarray        # (nc,) contact force magnitudes
    gap: np.ndarray        # (nc,) phi + n . delta
    active: np.ndarray     # (nc,) hard mode: pairs held at gap 0
    kappa: float
    status: int = STATUS_OK
    newton_iters: int = 0
    ipm_iters: int = 0
    extra: dict = field(default_factory=dict)
    g: np.ndarray = None   # (n_g, 3) next gripper positions (penalty mode)
    pen: object = None     # Penalty data of the step (penalty mode)
    force: np.ndarray = None   # (nc, 3) contact forces with friction (mu > 0)
    mu: float = 0.0


@dataclass
class Penalty:
    """Penalty grasp of one step: gripper k pulls node nodes[k] towards
    gplus[k] with stiffness D[k]; dD[k] = dD_k / dc_k, c_k = x_j - g_k."""
    nodes: np.ndarray
    D: np.ndarray
    dD: np.ndarray
    gplus: np.ndarray


def grasp_activation(inst, x, g):
    """D_k and dD_k/dc_k for every gripper (c_k = x_j - g_k).  The
    derivative of |c| at c = 0 is taken as 0; the hard indicator has zero
    derivative."""
    ng = len(inst.grip_nodes)
    D = np.zeros(ng)
    dD = np.zeros((ng, 3))
    for k, j in enumerate(inst.grip_nodes):
        c = x[j] - g[k]
        r = float(np.sqrt(c @ c))
        if inst.kappa_h > 0.0:
            D[k] = inst.D_max * np.exp(-r / inst.kappa_h)
            if r > 0.0:
                dD[k] = -D[k] / inst.kappa_h * c / r
        else:
            D[k] = inst.D_max if r <= inst.r_g else 0.0
    return D, dD


class Layout:
    """Free/gripped bookkeeping for one instance."""

    def __init__(self, inst):
        n = inst.n
        self.n = n
        self.penalty = getattr(inst, "grip_mode", "dirichlet") == "penalty"
        self.grip_of = -np.ones(n, dtype=np.int64)
        if not self.penalty:
            for k, j in enumerate(inst.grip_nodes):
                self.grip_of[j] = k
        self.free = self.grip_of < 0
        self.free_nodes = np.nonzero(self.free)[0]
        self.grip_nodes = np.array(inst.grip_nodes, dtype=np.int64)
        dof = np.arange(3 * n).reshape(n, 3)
        self.fidx = dof[self.free].ravel()
        self.gidx = dof[~self.free].ravel()
        self.fpos = -np.ones(n, dtype=np.int64)
        self.fpos[self.free_nodes] = np.arange(len(self.free_nodes))


def mass_diag(inst, lay: Layout) -> np.ndarray:
    """Diagonal of M/dt^2 on the free DoFs."""
    return np.full(len(lay.fidx), inst.mass / inst.dt ** 2)


def gripper_targets(inst, lay: Layout, x, u_t):
    """b_j = x_j + dt u_k for every gripped node j held by gripper k."""
    b = np.zeros((inst.n, 3))
    u = np.asarray(u_t).reshape(-1, 3)
    for k, j in enumerate(inst.grip_nodes):
        b[j] = x[j] + inst.dt * u[k]
    return b


def psi_gradient(inst, el, lay, y, xhat, pen=None):
    """F(y) of eq. (dynamics-first-stage) on the free nodes, zero elsewhere."""
    F = model.gradient(el, y)
    F = F + inst.mass / inst.dt ** 2 * (y - xhat) - inst.mass * inst.gravity[None, :]
    if pen is not None:
        for k, j in enumerate(pen.nodes):
            F[j] += pen.D[k] * (y[j] - pen.gplus[k])
    F[~lay.free] = 0.0
    return F


def psi_difference(inst, el, lay, y0, y1, xhat, pen=None):
    """Psi(y1) - Psi(y0) in cancellation-free form."""
    dE = model.energy_difference(el, y0, y1)
    f = lay.free
    dy = (y1 - y0)[f]
    dM = inst.mass / (2.0 * inst.dt ** 2) * np.sum(dy * (y1[f] + y0[f] - 2.0 * xhat[f]))
    dG = -inst.mass * np.sum(dy @ inst.gravity)
    dP = 0.0
    if pen is not None:
        for k, j in enumerate(pen.nodes):
            dP += 0.5 * pen.D[k] * float((y1[j] - y0[j]) @ (y1[j] + y0[j] - 2.0 * pen.gplus[k]))
    return dE + dM + dG + dP


def psi_hessian_ff(inst, el, lay, y, project, pen=None):
    """d^2 Psi / dy^2 restricted to the free DoFs (sparse)."""
    H = model.hessian(el, y, project=project)
    d = mass_diag(inst, lay).copy()
    if pen is not None:
        for k, j in enumerate(pen.nodes):
            d[3 * lay.fpos[j]:3 * lay.fpos[j] + 3] += pen.D[k]
    Hff = H[lay.fidx][:, lay.fidx] + sp.diags(d)
    return Hff.tocsc()


def stage1(inst, el, lay, y0, xhat, max_iter=100, pen=None):
    """Newton's method on F(y) = 0 (minimising Psi) from y0."""
    y = y0.copy()
    scale = 1.0 + inst.mass * float(np.max(np.abs(inst.gravity)))
    tol = 1e-10 * scale
    it = 0
    for it in range(max_iter):
        F = psi_gradient(inst, el, lay, y, xhat, pen)
        if not np.all(np.isfinite(F)):
            return y, STATUS_NONFINITE, it
        if np.max(np.abs(F), initial=0.0) <= tol:
            return y, STATUS_OK, it
        Hp = psi_hessian_ff(inst, el, lay, y, project=True, pen=pen)
        g = F.ravel()[lay.fidx]
        d = spla.spsolve(Hp, -g)
        D = np.zeros(3 * inst.n)
        D[lay.fidx] = d
        D = D.reshape(inst.n, 3)
        gTd = float(g @ d)
        alpha = 1.0
        for _ in range(60):
            if psi_difference(inst, el, lay, y, y + alpha * D, xhat, pen) <= 1e-4 * alpha * gTd:
                break
            alpha *= 0.5
        y = y + alpha * D
        if np.max(np.abs(alpha * D)) <= 1e-16 * (1.0 + np.max(np.abs(y))):
            break
    F = psi_gradient(inst, el, lay, y, xhat, pen)
    ok = np.max(np.abs(F), initial=0.0) <= 1e3 * tol
    return y, (STATUS_OK if ok else STATUS_NEWTON_NOCONV), it + 1


def singular(P, rtol=1e-13):
    """True if the exact Hessian P = dF/dy at y* is singular (to rtol).

    The derivatives of eq. (diff-sim) need (dF/dq*)^{-1}; they exist
    whenever P is nonsingular, positive definite or not.  Compression makes
    P indefinite at a stationary point of Psi that is not a minimum (a
    straight compressed rope), which is a valid root of F; only a singular
    P leaves the step's derivative undefined.  Test: a sparse LU with
    partial pivoting whose smallest pivot is below rtol times the largest
    (or which reports an exactly singular factor)."""
    try:
        lu = spla.splu(sp.csc_matrix(P))
    except RuntimeError:
        return True
    piv = np.abs(lu.U.diagonal())
    return not (np.all(np.isfinite(piv)) and piv.min() > rtol * piv.max())


def contact_pairs(inst, lay, y):
    """All (free node, obstacle) pairs with phi, n and SDF Hessian at y."""
    nodes, obs, phis, ns, Hs = [], [], [], [], []
    pts = y[lay.free_nodes]
    for o, fn in enumerate(sdf.obstacles(inst)):
        phi, nrm, H = fn(pts)
        nodes.append(lay.free_nodes.copy())
        obs.append(np.full(len(pts), o))
        phis.append(phi); ns.append(nrm); Hs.append(H)
    if not nodes:
        z = np.zeros(0)
        return (np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), z,
                np.zeros((0, 3)), np.zeros((0, 3, 3)))
    return (np.concatenate(nodes), np.concatenate(obs), np.concatenate(phis),
            np.concatenate(ns), np.concatenate(Hs))


def normal_matrix(lay, pair_node, normal):
    """N: one row n_c^T per pair, placed at the free DoFs of its node."""
    nc = len(pair_node)
    rows = np.repeat(np.arange(nc), 3)
    cols = (3 * lay.fpos[pair_node][:, None] + np.arange(3)[None]).ravel()
    return sp.csr_matrix((normal.ravel(), (rows, cols)), shape=(nc, 3 * len(lay.free_nodes)))


def interior_point(P, N, phi, kappa, fscale, xscale, max_iter=300):
    """Primal-dual Newton on  P D - N^T lam = 0,  gap - phi - N D = 0,
    lam * gap = mu,  with gap, lam > 0 (infeasible start).  For kappa > 0
    mu = kappa throughout; for kappa = 0 mu is driven to ~0."""
    nc = len(phi)
    ndof = P.shape[0]
    D = np.zeros(ndof)
    if nc == 0:
        return D, np.zeros(0), np.zeros(0), 0, True
    pii = np.asarray((N @ P).multiply(N).sum(axis=1)).ravel()
    hard = kappa <= 0.0
    mu = kappa if not hard else max(1e-2 * float(np.mean(pii * phi ** 2)), 1e-12)
    gap = 0.5 * (phi + np.sqrt(phi ** 2 + 4.0 * mu / pii))
    lam = mu / gap
    NT = N.T.tocsr()
    for it in range(max_iter):
        rd = P @ D - NT @ lam
        rp = gap - phi - N @ D
        rc = lam * gap - mu
        done_res = (np.max(np.abs(rd)) <= 1e-13 * fscale and np.max(np.abs(rp)) <= 1e-13 * xscale)
        if not hard:
            if done_res and np.max(np.abs(rc)) <= 1e-12 * kappa:
                return D, lam, gap, it, True
        else:
            if done_res and np.max(lam * gap) <= 1e-14 * fscale * xscale:
                return D, lam, gap, it, True
            mu = max(0.1 * float(np.mean(lam * gap)), 1e-18 * fscale * xscale)
            rc = lam * gap - mu
        w = lam / gap
        Kip = (P + NT @ sp.diags(w) @ N).tocsc()
        rhs = -rd + NT @ ((-rc + lam * rp) / gap)
        dD = spla.spsolve(Kip, rhs)
        dgap = N @ dD - rp
        dlam = (-rc - lam * dgap) / gap
        alpha = 1.0
        neg = dgap < 0
        if np.any(neg):
            alpha = min(alpha, 0.995 * float(np.min(-gap[neg] / dgap[neg])))
        neg = dlam < 0
        if np.any(neg):
            alpha = min(alpha, 0.995 * float(np.min(-lam[neg] / dlam[neg])))
        D = D + alpha * dD
        gap = gap + alpha * dgap
        lam = lam + alpha * dlam
    return D, lam, gap, max_iter, False


def hard_crossover(P, N, phi, D, lam, gap, fscale, xscale):
    """Fix the active set {lam > pi gap} and solve the KKT system
    [[P, -N_A^T], [N_A, 0]] [D; lam_A] = [0; -phi_A] exactly (dense, least
    squares so degenerate normals are allowed)."""
    pii = np.asarray((N @ P).multiply(N).sum(axis=1)).ravel()
    act = lam > pii * gap
    Pd = P.toarray()
    Nd = N.toarray()
    NA = Nd[act]
    na = NA.shape[0]
    ndof = Pd.shape[0]
    Kk = np.block([[Pd, -NA.T], [NA, np.zeros((na, na))]])
    rhs = np.concatenate([np.zeros(ndof), -phi[act]])
    sol = np.linalg.lstsq(Kk, rhs, rcond=None)[0]
    D2 = sol[:ndof]
    lamA = sol[ndof:]
    gap2 = phi + Nd @ D2
    lam2 = np.zeros_like(lam)
    lam2[act] = lamA
    ok = (np.all(gap2 >= -1e-11 * xscale) and np.all(lamA >= -1e-9 * fscale)
          and np.max(np.abs(Pd @ D2 - Nd.T @ lam2), initial=0.0) <= 1e-9 * fscale)
    return D2, lam2, gap2, act, ok


def tangent_basis(nrm):
    """Unit vectors t1, t2 completing each normal to an orthonormal frame
    (any choice: the cone and its barrier are invariant under rotations
    about n)."""
    a = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = np.cross(nrm, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    return t1, np.cross(nrm, t1)


def cone_barrier(y, mu):
    """psi(y) = 1/2 log(y0^2 - mu^2 (y1^2 + y2^2)) per row of y (nc, 3):
    gradient (nc, 3) and Hessian (nc, 3, 3)."""
    w = np.array([1.0, -mu * mu, -mu * mu])
    Q = y[:, 0] ** 2 - mu * mu * (y[:, 1] ** 2 + y[:, 2] ** 2)
    gr = w[None] * y / Q[:, None]
    H = np.diag(w)[None] / Q[:, None, None] - 2.0 * gr[:, :, None] * gr[:, None, :]
    return gr, H


def in_cone(y, mu):
    return np.all(y[:, 0] > 0.0) and np.all(y[:, 0] ** 2 - mu * mu * (y[:, 1] ** 2 + y[:, 2] ** 2) > 0.0)


def friction_barrier_point(P, J, b, kappa, mu, fscale, xscale, D0=None, y0=None, max_iter=200):
    """Minimiser of 1/2 D^T P D - kappa sum_c psi(y_c) subject to y = J D + b
    (J: 3 rows per pair, b (nc, 3)), by Newton's method from an infeasible
    start on (D, y) with lam = kappa grad psi(y): residuals
    r_D = P D - J^T lam and r_p = y - J D - b; the step solves
    (P + J^T Hb J) dD = -r_D + J^T Hb r_p, dy = J dD - r_p with
    Hb = -kappa Hess psi (positive semidefinite), then halves until y stays
    inside the cone and the scaled residual decreases."""
    nc = b.shape[0]
    D = np.zeros(P.shape[0]) if D0 is None else D0.copy()
    y = y0.copy()
    JT = J.T.tocsr()

    def resid(D, y):
        gr, _ = cone_barrier(y, mu)
        lam = kappa * gr
        rD = P @ D - JT @ lam.ravel()
        rp = (y.ravel() - J @ D - b.ravel())
        return rD, rp, lam

    rD, rp, lam = resid(D, y)
    for it in range(max_iter):
        nrm = np.sqrt(np.sum((rD / fscale) ** 2) + np.sum((rp / xscale) ** 2))
        # the force balance is met to the rounding of the barrier gradient,
        # whose value kappa / (y_n - mu |y_t|) cancels near the cone's surface
        if (np.max(np.abs(rD)) <= 1e-13 * fscale + 1e-9 * np.max(np.abs(lam))
                and np.max(np.abs(rp)) <= 1e-13 * xscale):
            return D, y, lam, it, True
        _, Hs = cone_barrier(y, mu)
        Hb = -kappa * Hs
        Hbd = sp.block_diag(list(Hb), format="csr")
        K = (P + JT @ Hbd @ J).tocsc()
        dD = spla.spsolve(K, -rD + JT @ (Hbd @ rp))
        dy = (J @ dD - rp).reshape(nc, 3)
        alpha = 1.0
        for _ in range(80):
            yn = y + alpha * dy
            if in_cone(yn, mu):
                rD2, rp2, lam2 = resid(D + alpha * dD, yn)
                n2 = np.sqrt(np.sum((rD2 / fscale) ** 2) + np.sum((rp2 / xscale) ** 2))
                if n2 <= (1.0 - 0.01 * alpha) * nrm:
                    break
            alpha *= 0.5
        else:
            return D, y, lam, it, False
        D, y, rD, rp, lam = D + alpha * dD, yn, rD2, rp2, lam2
    return D, y, lam, max_iter, False


def friction_stage2(P, lay, pn, phi, nrm, s, mu, kappa, fscale, xscale):
    """Stage 2 with the friction cone (see the module docstring).  Returns
    D (free DoFs), y (nc, 3) in each pair's frame (n, t1, t2), the contact
    forces lam (nc, 3) in world coordinates, iterations and success."""
    nc = len(phi)
    t1, t2 = tangent_basis(nrm)
    frame = np.stack([nrm, t1, t2], axis=1)                      # (nc, 3, 3), rows n, t1, t2
    rows = np.repeat(np.arange(3 * nc), 3)
    cols = np.tile((3 * lay.fpos[pn][:, None] + np.arange(3)[None]), (1, 3)).ravel()
    J = sp.csr_matrix((frame.reshape(nc, 9).ravel(), (rows, cols)), shape=(3 * nc, P.shape[0]))
    b = np.stack([phi, np.einsum("ci,ci->c", t1, s), np.einsum("ci,ci->c", t2, s)], axis=1)
    pii = np.asarray((J[0::3] @ P).multiply(J[0::3]).sum(axis=1)).ravel()
    hard = kappa <= 0.0
    k0 = kappa if not hard else max(1e-2 * float(np.mean(pii * phi ** 2)), 1e-12 * fscale * xscale)
    # a strictly interior start: the current tangential displacement, a normal
    # value above the cone by the relaxation's own gap scale
    yt = b[:, 1:]
    y = np.concatenate([(np.maximum(phi, 0.0) + mu * np.linalg.norm(yt, axis=1)
                         + np.sqrt(k0 / pii))[:, None], yt], axis=1)
    D = np.zeros(P.shape[0])
    its = 0
    kk = k0
    last = None
    while True:
        D1, y1, lam1, it, ok = friction_barrier_point(P, J, b, kk, mu, fscale, xscale, D, y)
        its += it
        if not ok:
            # a level below the first that does not converge ends the path
            # at the previous one
            if last is not None:
                D, y, lam = last
                ok = True
            break
        D, y, lam = D1, y1, lam1
        last = (D, y, lam)
        if not hard or kk <= 1e-16 * fscale * xscale:
            break
        kk = max(0.05 * kk, 1e-16 * fscale * xscale)
        # move the slack back inside the cone for the smaller relaxation
        y = np.concatenate([np.maximum(y[:, :1], mu * np.linalg.norm(y[:, 1:], axis=1, keepdims=True)
                                       + 1e-3 * np.sqrt(kk / pii)[:, None]), y[:, 1:]], axis=1)
    lam_w = np.einsum("ci,cij->cj", lam, frame)
    return D, y, lam_w, its, ok


def step(inst, x, v, u_t, kappa, el=None, lay=None, g=None) -> StepResult:
    """q+ = f(q, u) with contact relaxation kappa (kappa = 0: hard contact).
    Penalty mode needs the gripper positions g (n_g, 3)."""
    el = model.elements(inst) if el is None else el
    lay = Layout(inst) if lay is None else lay
    dt, gamma = inst.dt, inst.gamma
    x = np.asarray(x, dtype=np.float64).reshape(inst.n, 3)
    v = np.asarray(v, dtype=np.float64).reshape(inst.n, 3)
    u = np.asarray(u_t, dtype=np.float64).reshape(-1, 3)
    pen = None
    if lay.penalty:
        g = np.asarray(g, dtype=np.float64).reshape(-1, 3)
        D, dD = grasp_activation(inst, x, g)
        pen = Penalty(np.array(inst.grip_nodes, dtype=np.int64), D, dD, g + dt * u)
    b = gripper_targets(inst, lay, x, u)
    xhat = x + dt * (1.0 - gamma) * v
    y0 = xhat.copy()
    y0[~lay.free] = b[~lay.free]
    status = STATUS_OK
    if not (np.all(np.isfinite(x)) and np.all(np.isfinite(v)) and np.all(np.isfinite(u))):
        nan = np.full((inst.n, 3), np.nan)
        e = np.zeros(0)
        return StepResult(nan, nan, nan, nan, xhat, e.astype(int), e.astype(int), e,
                          np.zeros((0, 3)), np.zeros((0, 3, 3)), e, e, e.astype(bool),
                          kappa, STATUS_NONFINITE)
    y, st1, it1 = stage1(inst, el, lay, y0, xhat, pen=pen)
    status = max(status, st1)

    pn, po, phi, nrm, curv = contact_pairs(inst, lay, y)
    P = psi_hessian_ff(inst, el, lay, y, project=False, pen=pen)
    fscale = inst.mass / dt ** 2 * inst.h + inst.mass * float(np.max(np.abs(inst.gravity)))
    xscale = inst.h
    delta = np.zeros((inst.n, 3))
    lam = np.zeros(len(phi))
    gap = phi.copy()
    active = np.zeros(len(phi), dtype=bool)
    it2 = 0
    if P.shape[0] and singular(P):
        status = max(status, STATUS_NOT_PD)
    mu = float(getattr(inst, "mu", 0.0))
    force = None
    if len(phi) and mu > 0.0:
        s = (y - x)[pn]
        D, yc, force, it2, ok = friction_stage2(P, lay, pn, phi, nrm, s, mu, kappa, fscale, xscale)
        lam = np.einsum("ci,ci->c", force, nrm)
        gap = yc[:, 0]
        active = np.zeros(len(phi), dtype=bool)
        if not ok:
            status = max(status, STATUS_QP_NOCONV)
        full = np.zeros(3 * inst.n)
        full[lay.fidx] = D
        delta = full.reshape(inst.n, 3)
    elif len(phi):
        N = normal_matrix(lay, pn, nrm)
        D, lam, gap, it2, ok = interior_point(P, N, phi, kappa, fscale, xscale)
        if kappa <= 0.0:
            D, lam, gap, active, ok2 = hard_crossover(P, N, phi, D, lam, gap, fscale, xscale)
            ok = ok and ok2
        if not ok:
            status = max(status, STATUS_QP_NOCONV)
        full = np.zeros(3 * inst.n)
        full[lay.fidx] = D
        delta = full.reshape(inst.n, 3)

    xn = y + delta
    xn[~lay.free] = b[~lay.free]
    vn = (xn - x) / dt
    if not lay.penalty:
        for k, j in enumerate(inst.grip_nodes):
            vn[j] = u[k]
    if not (np.all(np.isfinite(xn)) and np.all(np.isfinite(vn))):
        status = STATUS_NONFINITE
    return StepResult(xn, vn, y, delta, xhat, pn, po, phi, nrm, curv, lam, gap, active,
                      kappa, status, it1, it2, g=None if pen is None else pen.gplus, pen=pen,
                      force=force, mu=mu)


def split_state(inst, s):
    """s = [x | v] (+ [g] in penalty mode) -> x (n, 3), v (n, 3), g (n_g, 3) or None."""
    n = inst.n
    s = np.asarray(s, dtype=np.float64)
    g = s[6 * n:].reshape(-1, 3) if getattr(inst, "grip_mode", "dirichlet") == "penalty" else None
    return s[:3 * n].reshape(n, 3), s[3 * n:6 * n].reshape(n, 3), g


def rollout(inst, kappa=None, s0=None, u=None):
    """Roll out inst.T steps.  Returns (traj (T+1, n_s), status per step)."""
    kappa = inst.kappa_fwd if kappa is None else kappa
    s0 = inst.s0 if s0 is None else s0
    u = inst.u if u is None else u
    el = model.elements(inst)
    lay = Layout(inst)
    n = inst.n
    traj = np.zeros((inst.T + 1, inst.n_s))
    traj[0] = s0
    stat = np.zeros(inst.T, dtype=np.int64)
    for t in range(inst.T):
        x, v, g = split_state(inst, traj[t])
        r = step(inst, x, v, u[t], kappa, el, lay, g=g)
        traj[t + 1, :3 * n] = r.x.ravel()
        traj[t + 1, 3 * n:6 * n] = r.v.ravel()
        if r.g is not None:
            traj[t + 1, 6 * n:] = r.g.ravel()
        stat[t] = r.status
    return traj, stat
