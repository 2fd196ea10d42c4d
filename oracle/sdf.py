"""Signed distance functions of the obstacles (Sec. 4.1: contact pair i has a
signed distance phi_i; eq. contact-constraint).

The paper gives no obstacle formulas; the reading used here:

* ground         phi = z,                 n = e_z,                  curvature 0
* sphere (c, r)  phi = |x - c| - r,       n = (x - c)/|x - c|,      curvature (I - n n^T)/|x - c|
                 (at the centre n is taken as e_z)
* rounded box    b = |x - c| - (h - rho) componentwise,
  (c, h, rho)    outside (some b_i > 0): phi = |max(b, 0)| - rho,
                                         n = s * max(b, 0)/|max(b, 0)| with s = sign(x - c),
                                         curvature D (I - m m^T) D / |max(b,0)| over the positive
                                         components (D = diag(s_i [b_i > 0]), m = unit max(b, 0));
                 inside: phi = max_i b_i - rho, n = s_k e_k for the largest b_k (ties: lowest
                                         axis, sign(0) = +1), curvature 0.

Each function takes points of shape (m, 3) and returns (phi (m,), n (m, 3),
curvature (m, 3, 3)).  Complex input is supported for complex-step checks
(branch decisions are taken on the real part).
"""
from __future__ import annotations

import numpy as np


def ground(p):
    m = p.shape[0]
    phi = p[:, 2].copy()
    n = np.zeros((m, 3), dtype=p.dtype)
    n[:, 2] = 1.0
    return phi, n, np.zeros((m, 3, 3), dtype=p.dtype)


def sphere(p, c, r):
    d = p - np.asarray(c)[None, :]
    L = np.sqrt(np.sum(d * d, axis=1))
    zero = np.real(L) == 0.0
    Ls = np.where(zero, 1.0, L)
    n = d / Ls[:, None]
    n[zero] = np.array([0.0, 0.0, 1.0])
    phi = L - r
    H = (np.eye(3)[None] - n[:, :, None] * n[:, None, :]) / Ls[:, None, None]
    H[zero] = 0.0
    return phi, n, H


def box(p, c, half, rho):
    q = p - np.asarray(c)[None, :]
    s = np.where(np.real(q) >= 0.0, 1.0, -1.0)
    aq = s * q
    b = aq - (np.asarray(half)[None, :] - rho)
    pos = np.real(b) > 0.0
    outside = np.any(pos, axis=1)
    m = q.shape[0]
    phi = np.zeros(m, dtype=p.dtype)
    n = np.zeros((m, 3), dtype=p.dtype)
    H = np.zeros((m, 3, 3), dtype=p.dtype)
    for i in range(m):
        if outside[i]:
            mp = np.where(pos[i], b[i], 0.0)
            L = np.sqrt(np.sum(mp * mp))
            phi[i] = L - rho
            mh = mp / L
            n[i] = s[i] * mh
            D = np.diag(np.where(pos[i], s[i], 0.0))
            H[i] = D @ (np.diag(pos[i].astype(float)) - np.outer(mh, mh)) @ D / L
        else:
            k = int(np.argmax(np.real(b[i])))
            phi[i] = b[i, k] - rho
            n[i, k] = s[i, k]
    return phi, n, H


def obstacles(inst):
    """List of callables p -> (phi, n, curvature) in a fixed order:
    ground first (if present), then spheres, then boxes."""
    out = []
    if inst.ground:
        out.append(ground)
    for sph in inst.spheres:
        out.append(lambda p, c=sph[:3].copy(), r=float(sph[3]): sphere(p, c, r))
    for bx in inst.boxes:
        out.append(lambda p, c=bx[:3].copy(), h=bx[3:6].copy(), rho=float(bx[6]): box(p, c, h, rho))
    return out
