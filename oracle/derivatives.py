"""Implicit derivatives of one step and of a rollout, in FP64.

Follows the paper's "Differentiating Through Simulation" paragraph:

* stage 1: dq*/dtheta = -(dF/dq*)^{-1} dF/dtheta;
* stage 2: dq+/dq* = -[I 0] K^{-1} dG/dq*, K the KKT matrix;
* eq. (diff-sim): the adjoint solves with K^T, applies the VJP of dG/dq*,
  solves with (dF/dq*)^T and applies the VJP of dF/dtheta.

Written out for this model (free DoFs f, gripped DoFs g, b = gripper
targets, H = dF/dy at y*, which is also the stage-2 matrix P):

  W = d^3E[D] (third derivative contracted with the stage-2 correction D)
  C = sum_c lam_c d^2 phi_c        (SDF curvature, block-diagonal)
  smoothed (kappa > 0), with Lam = diag(kappa / gap^2):
    K = P + N^T Lam N,   R = sum_c (kappa/gap_c^2) n_c (d^2 phi_c D_p)^T
    dx+_f = K^{-1} [ (P - W_ff + C - R) dy_f - W_fg db ]
  hard (kappa = 0), active set A:
    [[P, -N_A^T], [N_A, 0]] [dD; dlam] = -[ (W_ff - C) dy_f + W_fg db ; (N_A + R_A) dy_f ]
    with R_A rows (d^2 phi_c D_p)^T,   dx+_f = dy_f + dD
  stage 1: H_ff dy_f = (M/dt^2) dxhat_f - H_fg db,
           dxhat = dx + dt (1 - gamma) dv,   db = dx_g + dt du
  output:  dv+_f = (dx+_f - dx_f)/dt,  dx+_g = db,  dv+_g = du.

Penalty grasp (all nodes free, gripper state g, g+ = g + dt u, stiffness
D_k(c_k), c_k = x_j - g_k): F gains D_k (y_j - g+_k), so dF/dtheta gains
(y_j - g+_k) dD_k - D_k dg+_k at node j, and P gains D_k I, so the stage-2
right-hand side gains -(dD_k) Delta_j at node j:
  H dy = (M/dt^2) dxhat - sum_k e_j [dD_k (y_j - g+_k) - D_k dg+_k]
  K dx+ = J dy - sum_k e_j dD_k Delta_j,   dD_k = D'_k . (dx_j - dg_k)

Friction (mu > 0, smoothed kappa > 0; the step's stage 2 is the
central-path point of the friction-cone barrier, see oracle.step).  Per
pair c at node p, with u = s_p + D_p (s = y* - x), y_n = phi_c + n.D_p,
T = I - n n^T, tau = T u, Q = y_n^2 - mu^2 |tau|^2, a = y_n n - mu^2 tau,
the force is lam_c = kappa a / Q and G = P D - sum_c lam_c = 0.  Its
derivatives:
  K_c  = -dlam/dD  = (kappa/Q) (2 a a^T / Q - (n n^T - mu^2 T))
  Ly_c = dlam/dy*  = (kappa/Q) (A_y - a q_y^T / Q),
     A_y = n (n + Hc D)^T + y_n Hc + mu^2 ((n.u) Hc + n (Hc u)^T - T),
     q_y = 2 y_n (n + Hc D) + 2 mu^2 (n.u) Hc tau - 2 mu^2 tau
  Lx_c = dlam/dx_p = (kappa/Q) (mu^2 T - 2 mu^2 a tau^T / Q)
(Hc the SDF Hessian; dn = Hc dy*, d tau = -(n.u) dn - n (dn.u) + T du).
Then K = P + sum K_c and K dx+ = (K - W + sum Ly_c) dy - W_fg db +
sum Lx_c dx_p: the step now depends on x directly, through the tangential
displacement.  With mu = 0 these blocks reduce to the frictionless ones
(K_c = lam/gap n n^T, Ly_c = lam Hc - lam/gap n (n + Hc D)^T, Lx_c = 0).

Every product above is a plain sparse matrix product; every inverse is a
sparse LU solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model
from .step import Layout, normal_matrix, psi_hessian_ff, rollout, split_state, step


def _blockdiag(lay, pair_node, mats):
    """Sum of per-pair 3x3 blocks placed on the diagonal block of their node."""
    nf = len(lay.free_nodes)
    if len(pair_node) == 0:
        return sp.csr_matrix((3 * nf, 3 * nf))
    ii, jj = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    base = 3 * lay.fpos[pair_node]
    rows = (base[:, None, None] + ii[None]).ravel()
    cols = (base[:, None, None] + jj[None]).ravel()
    return sp.coo_matrix((mats.ravel(), (rows, cols)), shape=(3 * nf, 3 * nf)).tocsr()


def friction_blocks(r, x, mu, kappa):
    """Per-pair 3x3 blocks K_c, Ly_c, Lx_c of the friction-cone stage 2 (see
    the module docstring), from a solved step r and the positions x at the
    start of the step."""
    nc = len(r.pair_node)
    Kc = np.zeros((nc, 3, 3))
    Ly = np.zeros((nc, 3, 3))
    Lx = np.zeros((nc, 3, 3))
    I3 = np.eye(3)
    for c in range(nc):
        p = r.pair_node[c]
        n = r.normal[c]
        Hc = r.curv[c]
        Dp = r.delta[p]
        u = (r.y[p] - x[p]) + Dp
        yn = r.phi[c] + n @ Dp
        T = I3 - np.outer(n, n)
        tau = T @ u
        Q = yn * yn - mu * mu * (tau @ tau)
        a = yn * n - mu * mu * tau
        w = kappa / Q
        nu = n @ u
        Kc[c] = w * (2.0 * np.outer(a, a) / Q - (np.outer(n, n) - mu * mu * T))
        Ay = np.outer(n, n + Hc @ Dp) + yn * Hc + mu * mu * (nu * Hc + np.outer(n, Hc @ u) - T)
        qy = 2.0 * yn * (n + Hc @ Dp) + 2.0 * mu * mu * nu * (Hc @ tau) - 2.0 * mu * mu * tau
        Ly[c] = w * (Ay - np.outer(a, qy) / Q)
        Lx[c] = w * (mu * mu * T - 2.0 * mu * mu * np.outer(a, tau) / Q)
    return Kc, Ly, Lx


class StepDerivative:
    """Linearisation of f_kappa at (s, u): JVP, VJP and dense A, B."""

    def __init__(self, inst, s, u_t, kappa, el=None, lay=None):
        self.inst = inst
        self.el = model.elements(inst) if el is None else el
        self.lay = Layout(inst) if lay is None else lay
        n = inst.n
        self.n = n
        self.x, self.v, self.g = split_state(inst, s)
        self.res = r = step(inst, self.x, self.v, u_t, kappa, self.el, self.lay, g=self.g)
        self.pen = r.pen
        self.kappa = kappa
        lay = self.lay
        fi, gi = lay.fidx, lay.gidx
        Hfull = model.hessian(self.el, r.y)
        self.Hff = psi_hessian_ff(inst, self.el, lay, r.y, project=False, pen=r.pen)
        self.Hfg = Hfull[fi][:, gi].tocsr()
        Wfull = model.third(self.el, r.y, r.delta)
        self.Wff = Wfull[fi][:, fi].tocsr()
        self.Wfg = Wfull[fi][:, gi].tocsr()
        N = normal_matrix(lay, r.pair_node, r.normal)
        self.C = _blockdiag(lay, r.pair_node, r.lam[:, None, None] * r.curv)
        dp = r.delta[r.pair_node]                                   # (nc, 3)
        hd = np.einsum("cij,cj->ci", r.curv, dp)                    # d^2 phi D_p
        self.Hlu = spla.splu(self.Hff)
        self.Lx = None
        if r.mu > 0.0 and len(r.pair_node):
            if not kappa > 0.0:
                raise NotImplementedError("hard-contact derivatives with friction")
            Kc, Ly, Lx = friction_blocks(r, self.x, r.mu, kappa)
            self.K = (self.Hff + _blockdiag(lay, r.pair_node, Kc)).tocsc()
            self.Klu = spla.splu(self.K)
            self.J = (self.K - self.Wff + _blockdiag(lay, r.pair_node, Ly)).tocsr()
            self.Lx = _blockdiag(lay, r.pair_node, Lx)
        elif kappa > 0.0:
            w = kappa / r.gap ** 2
            self.R = _blockdiag(lay, r.pair_node, w[:, None, None] * r.normal[:, :, None] * hd[:, None, :])
            self.K = (self.Hff + N.T @ sp.diags(w) @ N).tocsc()
            self.Klu = spla.splu(self.K)
            self.J = (self.Hff - self.Wff + self.C - self.R).tocsr()
        else:
            act = r.active
            NA = N[act]
            nc = len(r.pair_node)
            RA = sp.csr_matrix((hd.ravel(), (np.repeat(np.arange(nc), 3),
                                             (3 * lay.fpos[r.pair_node][:, None] + np.arange(3)[None]).ravel())),
                               shape=(nc, N.shape[1]))[act]
            self.NA, self.RA = NA.tocsr(), RA.tocsr()
            na = NA.shape[0]
            Kk = np.block([[self.Hff.toarray(), -NA.toarray().T], [NA.toarray(), np.zeros((na, na))]])
            self.Kkkt = Kk
            self.nA = na

    # ------------------------------------------------------------------ JVP
    def jvp(self, dx, dv, du, dg=None):
        """Tangents (3n, m), (3n, m), (n_u, m) [, (3 n_g, m) in penalty mode]
        -> (dx+, dv+), each (3n, m) [, dg+ in penalty mode]."""
        inst, lay = self.inst, self.lay
        dt, gam = inst.dt, inst.gamma
        dx = np.asarray(dx, dtype=np.float64)
        dv = np.asarray(dv, dtype=np.float64)
        du = np.asarray(du, dtype=np.float64)
        if dx.ndim == 1:
            dx, dv, du = dx[:, None], dv[:, None], du[:, None]
        m = dx.shape[1]
        db = np.zeros_like(dx)
        if self.pen is None:
            for k, j in enumerate(inst.grip_nodes):
                db[3 * j:3 * j + 3] = dx[3 * j:3 * j + 3] + dt * du[3 * k:3 * k + 3]
        fi, gi = lay.fidx, lay.gidx
        dxhat_f = dx[fi] + dt * (1.0 - gam) * dv[fi]
        rhs1 = inst.mass / dt ** 2 * dxhat_f - self.Hfg @ db[gi]
        pen2 = np.zeros_like(rhs1)
        if self.pen is not None:
            dg = np.zeros((3 * len(inst.grip_nodes), m)) if dg is None else np.asarray(dg, dtype=np.float64).reshape(-1, m)
            r, P = self.res, self.pen
            for k, j in enumerate(P.nodes):
                sl = slice(3 * j, 3 * j + 3)
                dgp = dg[3 * k:3 * k + 3] + dt * du[3 * k:3 * k + 3]
                dDk = P.dD[k] @ (dx[sl] - dg[3 * k:3 * k + 3])            # (m,)
                rhs1[sl] -= np.outer(r.y[j] - P.gplus[k], dDk) - P.D[k] * dgp
                pen2[sl] -= np.outer(r.delta[j], dDk)
        dy_f = self.Hlu.solve(rhs1)
        if self.Lx is not None:
            dxn_f = self.Klu.solve(self.J @ dy_f - self.Wfg @ db[gi] + pen2 + self.Lx @ dx[fi])
        elif self.kappa > 0.0:
            dxn_f = self.Klu.solve(self.J @ dy_f - self.Wfg @ db[gi] + pen2)
        else:
            top = -((self.Wff - self.C) @ dy_f + self.Wfg @ db[gi]) + pen2
            bot = -((self.NA + self.RA) @ dy_f) if self.nA else np.zeros((0, m))
            sol = np.linalg.solve(self.Kkkt, np.vstack([top, bot])) if self.nA else \
                np.linalg.solve(self.Kkkt, top)
            dxn_f = dy_f + sol[:len(fi)]
        dxn = db.copy()
        dxn[fi] = dxn_f
        dvn = (dxn - dx) / dt
        if self.pen is not None:
            return dxn, dvn, dg + dt * du
        for k, j in enumerate(inst.grip_nodes):
            dvn[3 * j:3 * j + 3] = du[3 * k:3 * k + 3]
        return dxn, dvn

    # ------------------------------------------------------------------ VJP
    def vjp(self, xb, vb, gb=None):
        """Cotangents of (x+, v+) (3n,) [and g+ in penalty mode] -> cotangents
        of (x, v, u) [(x, v, g, u) in penalty mode]."""
        inst, lay = self.inst, self.lay
        dt, gam = inst.dt, inst.gamma
        fi, gi = lay.fidx, lay.gidx
        xb = np.asarray(xb, dtype=np.float64)
        vb = np.asarray(vb, dtype=np.float64)
        xbar = np.zeros(3 * self.n)
        vbar = np.zeros(3 * self.n)
        ubar = np.zeros(3 * len(inst.grip_nodes))
        # v+_f = (x+_f - x_f)/dt ; x+_g = b ; v+_g = u
        xnb_f = xb[fi] + vb[fi] / dt
        xbar[fi] -= vb[fi] / dt
        bbar = np.zeros(3 * self.n)
        bbar[gi] = xb[gi]
        if self.pen is None:
            for k, j in enumerate(inst.grip_nodes):
                ubar[3 * k:3 * k + 3] += vb[3 * j:3 * j + 3]
        # stage 2
        if self.kappa > 0.0 or self.Lx is not None:
            z = self.Klu.solve(xnb_f)
            ybar_f = self.J.T @ z
            bbar[gi] -= self.Wfg.T @ z
            if self.Lx is not None:
                xbar[fi] += self.Lx.T @ z
            a2 = z
        else:
            nf = len(fi)
            rhs = np.concatenate([xnb_f, np.zeros(self.nA)])
            sol = np.linalg.solve(self.Kkkt.T, rhs)
            a, c = sol[:nf], sol[nf:]
            ybar_f = xnb_f - (self.Wff - self.C).T @ a
            if self.nA:
                ybar_f = ybar_f - (self.NA + self.RA).T @ c
            bbar[gi] -= self.Wfg.T @ a
            a2 = a
        # stage 1
        mu = self.Hlu.solve(ybar_f)
        xhatb_f = inst.mass / dt ** 2 * mu
        bbar[gi] -= self.Hfg.T @ mu
        xbar[fi] += xhatb_f
        vbar[fi] += dt * (1.0 - gam) * xhatb_f
        if self.pen is not None:
            r, P = self.res, self.pen
            ng = len(inst.grip_nodes)
            gbar = np.zeros(3 * ng) if gb is None else np.array(gb, dtype=np.float64)
            for k, j in enumerate(P.nodes):
                sl = slice(3 * j, 3 * j + 3)
                Dbar = -(a2[sl] @ r.delta[j]) - (mu[sl] @ (r.y[j] - P.gplus[k]))
                gpbar = P.D[k] * mu[sl] + gbar[3 * k:3 * k + 3]
                xbar[sl] += Dbar * P.dD[k]
                gbar[3 * k:3 * k + 3] = gpbar - Dbar * P.dD[k]
                ubar[3 * k:3 * k + 3] = dt * gpbar
            return xbar, vbar, gbar, ubar
        for k, j in enumerate(inst.grip_nodes):
            xbar[3 * j:3 * j + 3] += bbar[3 * j:3 * j + 3]
            ubar[3 * k:3 * k + 3] += dt * bbar[3 * j:3 * j + 3]
        return xbar, vbar, ubar

    # ------------------------------------------------------ full-state forms
    def jvp_s(self, ds, du):
        """ds (n_s, m), du (n_u, m) -> ds+ (n_s, m), for either grasp mode."""
        n = self.n
        ds = np.asarray(ds, dtype=np.float64)
        if self.pen is None:
            return np.vstack(self.jvp(ds[:3 * n], ds[3 * n:6 * n], du))
        return np.vstack(self.jvp(ds[:3 * n], ds[3 * n:6 * n], du, ds[6 * n:]))

    def vjp_s(self, sb):
        """sb (n_s,) -> (cotangent of s (n_s,), cotangent of u (n_u,))."""
        n = self.n
        sb = np.asarray(sb, dtype=np.float64)
        if self.pen is None:
            xb, vb, ub = self.vjp(sb[:3 * n], sb[3 * n:6 * n])
            return np.concatenate([xb, vb]), ub
        xb, vb, gb, ub = self.vjp(sb[:3 * n], sb[3 * n:6 * n], sb[6 * n:])
        return np.concatenate([xb, vb, gb]), ub

    # ---------------------------------------------------------------- dense
    def dense(self):
        """A = ds+/ds (n_s x n_s), B = ds+/du (n_s x n_u)."""
        ns = self.inst.n_s
        nu = 3 * len(self.inst.grip_nodes)
        A = self.jvp_s(np.eye(ns), np.zeros((nu, ns)))
        B = self.jvp_s(np.zeros((ns, nu)), np.eye(nu))
        return A, B


def rollout_backward(inst, traj, sT_bar=None, traj_bar=None, kappa=None):
    """Reverse-mode gradient of a rollout through f_kappa (default kappa_bwd),
    linearised at the stored states.  Returns (s0_bar (6n,), u_bar (T, n_u))."""
    kappa = inst.kappa_bwd if kappa is None else kappa
    n, T = inst.n, inst.T
    el = model.elements(inst)
    lay = Layout(inst)
    sb = np.zeros(inst.n_s) if sT_bar is None else np.array(sT_bar, dtype=np.float64)
    if traj_bar is not None:
        sb = sb + traj_bar[T]
    ubar = np.zeros((T, 3 * len(inst.grip_nodes)))
    for t in range(T - 1, -1, -1):
        d = StepDerivative(inst, traj[t], inst.u[t], kappa, el, lay)
        sb, ub = d.vjp_s(sb)
        if traj_bar is not None:
            sb = sb + traj_bar[t]
        ubar[t] = ub
    return sb, ubar


def rollout_jvp(inst, traj, ds0, du, kappa=None):
    """Forward-mode tangent of a rollout: ds0 (6n, m), du (T, n_u, m) ->
    ds (T+1, 6n, m)."""
    kappa = inst.kappa_bwd if kappa is None else kappa
    n, T = inst.n, inst.T
    el = model.elements(inst)
    lay = Layout(inst)
    ds0 = np.asarray(ds0, dtype=np.float64)
    if ds0.ndim == 1:
        ds0 = ds0[:, None]
        du = np.asarray(du)[:, :, None]
    out = np.zeros((T + 1,) + ds0.shape)
    out[0] = ds0
    for t in range(T):
        d = StepDerivative(inst, traj[t], inst.u[t], kappa, el, lay)
        out[t + 1] = d.jvp_s(out[t], du[t])
    return out


def rollout_linearize(inst, traj, kappa=None):
    """Dense A_t, B_t along a trajectory: arrays (T, 6n, 6n) and (T, 6n, n_u)."""
    kappa = inst.kappa_bwd if kappa is None else kappa
    el = model.elements(inst)
    lay = Layout(inst)
    As, Bs = [], []
    for t in range(inst.T):
        A, B = StepDerivative(inst, traj[t], inst.u[t], kappa, el, lay).dense()
        As.append(A)
        Bs.append(B)
    return np.array(As), np.array(Bs)


__all__ = ["StepDerivative", "rollout_backward", "rollout_jvp", "rollout_linearize", "rollout"]
