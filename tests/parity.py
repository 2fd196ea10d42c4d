"""Comparison helpers shared by the GPU parity tests.

Tolerances (FP32 GPU vs FP64 oracle, per instance):
  states      max |dx| / max(|x_or|_inf, 1e-3) <= 1e-4, and the same for the
              velocity block separately (velocities are differences of
              positions divided by dt, so a combined norm would hide them);
  gradients   |g - g_or|_2 / |g_or|_2 <= 1e-3, separately for the cotangent
              of the positions, of the velocities (and of the gripper
              positions in penalty mode) and of the controls;
  Jacobians   per step and per block |A_b - A_or,b|_F / |A_or,b|_F <= 1e-3,
              for every block [x+, v+ (, g+)] x [x, v (, g)] of A_t and the
              x+, v+ (, g+) rows of B_t; JVP tangents likewise per block
              (dx+, dv+ (, dg+)).

Why blocks: in A_t the block dv+/dx = (dx+/dx - I)/dt carries nearly all of
the Frobenius norm (about 99.99 % for a 64-node rope at dt = 5 ms), so one
relative norm over the whole matrix would pass with dx+/dv written as zeros
or dx+/dx off by several percent.  A reference block whose norm is below
1e-6 of the whole matrix (a structural zero, e.g. dg+/dx) is compared
against that floor instead, i.e. it must be zero to 1e-9 of the matrix.
"""
import numpy as np

STATE_TOL = 1e-4
GRAD_TOL = 1e-3
JAC_TOL = 1e-3


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


def _segments(n_s, n):
    """Index ranges of the x, v (and g) parts of a state vector."""
    seg = {"x": slice(0, 3 * n), "v": slice(3 * n, 6 * n)}
    if n_s > 6 * n:
        seg["g"] = slice(6 * n, n_s)
    return seg


def _block_rel(d, r, floor):
    return float(np.linalg.norm(d) / max(np.linalg.norm(r), floor))


def jacobian_block_errors(A, Ar, B, Br, n):
    """Per-block relative errors of A_t (rows x+, v+, g+ by columns x, v, g)
    and of B_t (rows x+, v+, g+): a dict name -> error."""
    A = np.asarray(A, dtype=np.float64)
    Ar = np.asarray(Ar, dtype=np.float64)
    seg = _segments(Ar.shape[0], n)
    out = {}
    fa = 1e-6 * np.linalg.norm(Ar)
    for rn, rs in seg.items():
        for cn, cs in seg.items():
            out[f"A[{rn}+,{cn}]"] = _block_rel(A[rs, cs] - Ar[rs, cs], Ar[rs, cs], fa)
    if B is not None and Br is not None and np.asarray(Br).size:
        B = np.asarray(B, dtype=np.float64)
        Br = np.asarray(Br, dtype=np.float64)
        fb = 1e-6 * np.linalg.norm(Br)
        for rn, rs in seg.items():
            out[f"B[{rn}+]"] = _block_rel(B[rs] - Br[rs], Br[rs], fb)
    return out


def tangent_block_errors(out, ref, n):
    """JVP tangents (k, n_s) or (n_s,) against the oracle, per state block."""
    out = np.asarray(out, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if out.ndim == 1:
        out, ref = out[None], ref[None]
    seg = _segments(ref.shape[-1], n)
    f = 1e-6 * np.linalg.norm(ref)
    return {f"d{k}+": _block_rel(out[:, s] - ref[:, s], ref[:, s], f) for k, s in seg.items()}


def gradient_block_errors(s0_bar, u_bar, s0_ref, u_ref, n):
    """Cotangents of the initial state, per block (x, v, g), and of the
    controls, each as a relative L2 error."""
    s0_bar = np.asarray(s0_bar, dtype=np.float64).ravel()
    s0_ref = np.asarray(s0_ref, dtype=np.float64).ravel()
    seg = _segments(s0_ref.size, n)
    f = 1e-6 * np.linalg.norm(s0_ref)
    out = {f"{k}_bar": _block_rel(s0_bar[s] - s0_ref[s], s0_ref[s], f) for k, s in seg.items()}
    ur = np.asarray(u_ref, dtype=np.float64).ravel()
    if ur.size:
        out["u_bar"] = rel_l2(u_bar, ur)
    return out


def worst(errs):
    return max(errs.values()) if errs else 0.0


def fmt(errs):
    return " ".join(f"{k} {v:.2e}" for k, v in errs.items())


def check(errs, tol, label=""):
    """Print the per-block errors and assert each is within tol."""
    print(f"{label}: {fmt(errs)}", flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, bad)
