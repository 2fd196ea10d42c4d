"""Conformal calibration of the one-step model error, in FP64 (Sec. 4.4,
"Calibrated Reachability Guarantees via Conformal Prediction").

TEST INFRASTRUCTURE ONLY (see the package docstring).

A calibration set holds n perceived-state transitions (q_i, u_i, q_i+).
Each is scored by the distance between the observed next state and the
model's one-step prediction, s_i = |q_i+ - f(q_i, u_i)|_2.  For a
trajectory-level miscoverage delta over a horizon of T steps the per-step
level is delta / T, and the radius is the order statistic
s_(k), k = ceil((n + 1)(1 - delta / T)) (1-based, scores ascending), or
+infinity when k exceeds n.

Readings:
* the configuration q is the positions of the nodes (the paper's perception
  returns the full configuration); the model is the simulator's step in
  its quasi-static form (gamma = 1), where the velocity does not enter the
  step, so f(q, u) needs only the perceived positions;
* k is evaluated in double precision with a margin of 1e-9 below the
  ceiling, so that a level given as a decimal (0.1 = 0.1000...0055 in
  binary) does not move k up by one when (n + 1)(1 - delta / T) is an
  integer in exact arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

from .step import step


def scores(insts, q, u, q_next):
    """s_i = |q_i+ - f(q_i, u_i)|_2 over the positions, one instance per
    calibration pair (its geometry, material and obstacles).  q and q_next
    are lists of (n_i, 3) arrays, u a list of (n_u,) arrays."""
    out = np.zeros(len(insts))
    for i, inst in enumerate(insts):
        x = np.asarray(q[i], dtype=np.float64).reshape(inst.n, 3)
        r = step(inst, x, np.zeros_like(x), np.asarray(u[i], dtype=np.float64), inst.kappa_fwd)
        d = np.asarray(q_next[i], dtype=np.float64).reshape(inst.n, 3) - r.x
        out[i] = math.sqrt(float(np.sum(d * d)))
    return out


def order_index(n, delta, horizon):
    """1-based k = ceil((n + 1)(1 - delta / T)); values above n mean +inf.
    The level delta / T must lie in (0, 1)."""
    if not (0.0 < delta / horizon < 1.0):
        raise ValueError("the per-step miscoverage delta / T must lie in (0, 1)")
    return int(math.ceil((n + 1) * (1.0 - delta / horizon) - 1e-9))


def radius(s, delta, horizon):
    """(r_CP, k): the k-th smallest score (ties in any order give the same
    value), or +inf if k > n."""
    s = np.sort(np.asarray(s, dtype=np.float64))
    k = order_index(len(s), delta, horizon)
    if k > len(s):
        return math.inf, k
    return float(s[k - 1]), k
