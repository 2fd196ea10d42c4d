"""Comparison helpers shared by the GPU parity tests.

Tolerances (FP32 GPU vs FP64 oracle, per instance):
  states      max |dx| / max(|x_or|_inf, 1e-3) <= 1e-4, and the same for the
              velocity block separately (velocities are differences of
              positions divided by dt, so a combined norm would hide them);
  gradients   |g - g_or|_2 / |g_or|_2 <= 1e-3;
  Jacobians   per step |A - A_or|_F / |A_or|_F <= 1e-3.
"""
import numpy as np

STATE_TOL = 1e-4
GRAD_TOL = 1e-3
JAC_TOL = 1e-3
# Hard contact (kappa_fwd = 0): the FP32 interior point stops once
# lam * gap <= 1e-6 fscale h per pair, so a weakly loaded active pair keeps a
# gap of that over lam, which the step divides by dt in v+.  Positions meet
# STATE_TOL; velocities are held to this bound.
HARD_V_TOL = 2.5e-4


def state_errors(traj, ref, n):
    """Position and velocity errors; gripper positions (penalty grasp, after
    the velocity block) count with the positions."""
    traj = np.asarray(traj, dtype=np.float64).reshape(ref.shape)
    x = np.concatenate([traj[..., :3 * n], traj[..., 6 * n:]], axis=-1)
    xr = np.concatenate([ref[..., :3 * n], ref[..., 6 * n:]], axis=-1)
    v, vr = traj[..., 3 * n:6 * n], ref[..., 3 * n:6 * n]
    ex = np.max(np.abs(x - xr)) / max(np.max(np.abs(xr)), 1e-3)
    ev = np.max(np.abs(v - vr)) / max(np.max(np.abs(vr)), 1e-3)
    return float(ex), float(ev)


def rel_l2(g, ref):
    g = np.asarray(g, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(g - ref) / (den if den > 0 else 1.0))
