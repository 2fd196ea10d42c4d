"""Elastic model of the nodal system (Sec. 4.1, elastic energy E(q)).

The paper names only "stretching and bending" energies.  The reading used
here:

* rope  - stretch springs between consecutive nodes,
          E_s = 1/2 k (|x_b - x_a| - l0)^2,
          plus a discrete-curvature bending term for every interior node,
          E_b = 1/2 k_b |x_a - 2 x_b + x_c|^2;
* cloth - mass-spring lattice with structural (grid neighbours, rest h),
          shear (cell diagonals, rest h sqrt 2) and bend springs (two nodes
          apart along a grid line, rest 2h), all of the stretch-spring form.

Everything works on node arrays of shape (n, 3) and is written so that it
also evaluates on complex input (complex-step derivative checks): lengths are
sqrt(e . e), never abs().
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Elements:
    n: int
    sa: np.ndarray     # spring first node   (S,)
    sb: np.ndarray     # spring second node  (S,)
    rest: np.ndarray   # spring rest length  (S,)
    k: np.ndarray      # spring stiffness    (S,)
    ba: np.ndarray     # bend triplet nodes  (Bn,)
    bb: np.ndarray
    bc: np.ndarray
    kb: float          # bend stiffness of the discrete-curvature term


def elements(inst) -> Elements:
    """Element lists of a rope or cloth instance (node (ix, iy) -> iy*nx+ix)."""
    nx, ny, h = inst.nx, inst.ny, inst.h
    n = nx * ny
    sa, sb, rest, k = [], [], [], []
    ba, bb, bc = [], [], []
    if inst.kind == "rope":
        for i in range(n - 1):
            sa.append(i); sb.append(i + 1); rest.append(h); k.append(inst.k_struct)
        for i in range(1, n - 1):
            ba.append(i - 1); bb.append(i); bc.append(i + 1)
    else:
        idx = lambda ix, iy: iy * nx + ix  # noqa: E731
        def add(a, b, r, kk):
            sa.append(a); sb.append(b); rest.append(r); k.append(kk)
        for iy in range(ny):
            for ix in range(nx):
                if ix + 1 < nx:
                    add(idx(ix, iy), idx(ix + 1, iy), h, inst.k_struct)
                if iy + 1 < ny:
                    add(idx(ix, iy), idx(ix, iy + 1), h, inst.k_struct)
                if ix + 1 < nx and iy + 1 < ny:
                    add(idx(ix, iy), idx(ix + 1, iy + 1), h * math.sqrt(2.0), inst.k_shear)
                    add(idx(ix + 1, iy), idx(ix, iy + 1), h * math.sqrt(2.0), inst.k_shear)
                if ix + 2 < nx:
                    add(idx(ix, iy), idx(ix + 2, iy), 2.0 * h, inst.k_bend)
                if iy + 2 < ny:
                    add(idx(ix, iy), idx(ix, iy + 2), 2.0 * h, inst.k_bend)
    kb = inst.k_bend if inst.kind == "rope" else 0.0
    return Elements(n=n, sa=np.array(sa, dtype=np.int64), sb=np.array(sb, dtype=np.int64),
                    rest=np.array(rest, dtype=np.float64), k=np.array(k, dtype=np.float64),
                    ba=np.array(ba, dtype=np.int64), bb=np.array(bb, dtype=np.int64),
                    bc=np.array(bc, dtype=np.int64), kb=float(kb))


def _len(e):
    return np.sqrt(np.sum(e * e, axis=-1))


def energy(el: Elements, y) -> complex:
    """E(y): sum of spring and bending energies."""
    e = y[el.sb] - y[el.sa]
    L = _len(e)
    E = 0.5 * np.sum(el.k * (L - el.rest) ** 2)
    if len(el.ba):
        c = y[el.ba] - 2.0 * y[el.bb] + y[el.bc]
        E = E + 0.5 * el.kb * np.sum(c * c)
    return E


def gradient(el: Elements, y) -> np.ndarray:
    """dE/dy, shape (n, 3)."""
    g = np.zeros(y.shape, dtype=y.dtype)
    e = y[el.sb] - y[el.sa]
    L = _len(e)
    f = (el.k * (L - el.rest) / L)[:, None] * e     # k (L - l0) e_hat
    np.add.at(g, el.sb, f)
    np.add.at(g, el.sa, -f)
    if len(el.ba):
        c = el.kb * (y[el.ba] - 2.0 * y[el.bb] + y[el.bc])
        np.add.at(g, el.ba, c)
        np.add.at(g, el.bb, -2.0 * c)
        np.add.at(g, el.bc, c)
    return g


def spring_blocks(el: Elements, y, project: bool) -> np.ndarray:
    """3x3 Hessian block of every spring w.r.t. its edge vector,
    k [e_hat e_hat^T + (1 - l0/L)(I - e_hat e_hat^T)].  With ``project`` the
    transverse factor (1 - l0/L) is clamped at 0, which makes every block
    positive semi-definite (used only for Newton directions)."""
    e = y[el.sb] - y[el.sa]
    L = _len(e)
    eh = e / L[:, None]
    f = 1.0 - el.rest / L
    if project:
        f = np.where(np.real(f) > 0.0, f, 0.0)
    outer = eh[:, :, None] * eh[:, None, :]
    eye = np.eye(3)[None]
    return el.k[:, None, None] * (outer + f[:, None, None] * (eye - outer))


def _assemble_pairs(n, a, b, blocks, dtype):
    """Sparse 3n x 3n matrix with [[K, -K], [-K, K]] on node pair (a, b)."""
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    for (p, q, sgn) in ((a, a, 1.0), (b, b, 1.0), (a, b, -1.0), (b, a, -1.0)):
        rows.append((3 * p[:, None, None] + ii[None]).ravel())
        cols.append((3 * q[:, None, None] + jj[None]).ravel())
        vals.append((sgn * blocks).ravel())
    if not rows or len(a) == 0:
        return sp.csr_matrix((3 * n, 3 * n), dtype=dtype)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * n), dtype=dtype).tocsr()


def bend_matrix(el: Elements) -> sp.csr_matrix:
    """Constant Hessian of the discrete-curvature energy: k_b w w^T (x) I3
    with w = (1, -2, 1) on every triplet."""
    n = el.n
    if len(el.ba) == 0:
        return sp.csr_matrix((3 * n, 3 * n))
    w = (1.0, -2.0, 1.0)
    nodes = (el.ba, el.bb, el.bc)
    rows, cols, vals = [], [], []
    for i in range(3):
        for j in range(3):
            for c in range(3):
                rows.append(3 * nodes[i] + c)
                cols.append(3 * nodes[j] + c)
                vals.append(np.full(len(el.ba), el.kb * w[i] * w[j]))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * n)).tocsr()


def hessian(el: Elements, y, project: bool = False) -> sp.csr_matrix:
    """d^2E/dy^2 as a sparse 3n x 3n matrix (exact, or spring-projected)."""
    K = _assemble_pairs(el.n, el.sa, el.sb, spring_blocks(el, y, project), y.dtype)
    return (K + bend_matrix(el)).tocsr()


def third(el: Elements, y, dy) -> sp.csr_matrix:
    """W = d/de [d^2E/dy^2 (y + e dy)] at e = 0: the third derivative of E
    contracted with dy.  Per spring with edge e and de = dy_b - dy_a:
    k l0 / L^3 [(e.de) I + de e^T + e de^T - 3 (e.de) e_hat e_hat^T].
    The bending term is quadratic and contributes nothing."""
    e = y[el.sb] - y[el.sa]
    de = dy[el.sb] - dy[el.sa]
    L = _len(e)
    eh = e / L[:, None]
    ed = np.sum(e * de, axis=-1)
    c = (el.k * el.rest / L ** 3)
    blocks = c[:, None, None] * (
        ed[:, None, None] * np.eye(3)[None]
        + de[:, :, None] * e[:, None, :]
        + e[:, :, None] * de[:, None, :]
        - 3.0 * ed[:, None, None] * eh[:, :, None] * eh[:, None, :])
    return _assemble_pairs(el.n, el.sa, el.sb, blocks, np.result_type(y, dy))


def energy_difference(el: Elements, y0, y1) -> float:
    """E(y1) - E(y0) summed element by element in a cancellation-free form:
    springs 1/2 k (L1 - L0)(L1 + L0 - 2 l0) with L1 - L0 = (|e1|^2 - |e0|^2)/(L1 + L0),
    bends 1/2 k_b (c1 - c0).(c1 + c0)."""
    e0 = y0[el.sb] - y0[el.sa]
    e1 = y1[el.sb] - y1[el.sa]
    L0, L1 = _len(e0), _len(e1)
    dL = np.sum((e1 - e0) * (e1 + e0), axis=-1) / (L1 + L0)
    dE = 0.5 * np.sum(el.k * dL * (L1 + L0 - 2.0 * el.rest))
    if len(el.ba):
        c0 = y0[el.ba] - 2.0 * y0[el.bb] + y0[el.bc]
        c1 = y1[el.ba] - 2.0 * y1[el.bb] + y1[el.bc]
        dE = dE + 0.5 * el.kb * np.sum((c1 - c0) * (c1 + c0))
    return dE
