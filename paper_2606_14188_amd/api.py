"""Thin Python front end of libcord: builds descriptors, allocates device
tensors with torch, and calls the C ABI on torch's current stream.

Every operation runs in libcord's HIP kernels; torch only provides device
memory and the stream.
"""
from __future__ import annotations

import contextlib
import ctypes
from ctypes import POINTER, byref, c_int64, c_uint32, c_void_p

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def make_desc(inst) -> L.InstanceDesc:
    """Fill a cord_instance_desc from an object with the attributes of
    workloads.Instance (kind, nx, ny, h, mass, k_*, grip_nodes, ground,
    spheres, boxes, dt, gamma, gravity, kappa_fwd, kappa_bwd, T, and
    grip_mode, D_max, kappa_h, r_g for the penalty grasp)."""
    d = L.InstanceDesc()
    d.kind = L.ROPE if inst.kind == "rope" else L.CLOTH
    d.nx, d.ny, d.T = int(inst.nx), int(inst.ny), int(inst.T)
    d.h, d.mass = float(inst.h), float(inst.mass)
    d.k_struct, d.k_shear, d.k_bend = float(inst.k_struct), float(inst.k_shear), float(inst.k_bend)
    grips = list(inst.grip_nodes)
    if len(grips) > L.MAX_GRIP:
        raise ValueError("too many grippers")
    d.n_grip = len(grips)
    for i, g in enumerate(grips):
        d.grip_node[i] = int(g)
    d.ground = 1 if inst.ground else 0
    sph = np.asarray(inst.spheres, dtype=np.float64).reshape(-1, 4)
    box = np.asarray(inst.boxes, dtype=np.float64).reshape(-1, 7)
    if len(sph) > L.MAX_SPHERE or len(box) > L.MAX_BOX:
        raise ValueError("too many obstacles")
    d.n_sphere, d.n_box = len(sph), len(box)
    for i, s in enumerate(sph):
        for c in range(4):
            d.sphere[i][c] = float(s[c])
    for i, b in enumerate(box):
        for c in range(7):
            d.box[i][c] = float(b[c])
    p = d.params
    p.dt, p.gamma = float(inst.dt), float(inst.gamma)
    for c in range(3):
        p.gravity[c] = float(inst.gravity[c])
    p.kappa_fwd, p.kappa_bwd, p.mu = float(inst.kappa_fwd), float(inst.kappa_bwd), float(getattr(inst, "mu", 0.0))
    if getattr(inst, "grip_mode", "dirichlet") == "penalty":
        d.grip_mode = L.GRIP_PENALTY
        d.D_max, d.kappa_h, d.r_g = float(inst.D_max), float(inst.kappa_h), float(inst.r_g)
    return d


class _AuxState:
    """A step-internals buffer and the number of FULL rollouts that have
    written it (shared by the simulators that use the same buffer)."""
    shared = {}     # buffer address -> state

    def __init__(self, buf):
        self.buf = buf
        self.gen = 0


class Sim:
    """A batch of (possibly ragged) rope/cloth instances on the current device."""

    def __init__(self, instances, device=None):
        self.lib = L.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.instances = list(instances)
        B = len(self.instances)
        arr = (L.InstanceDesc * B)(*[make_desc(i) for i in self.instances])
        self._h = c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.cord_sim_create(arr, B, byref(self._h)))
        info = L.SimInfo()
        L.check(self.lib.cord_sim_info(self._h, byref(info)))
        self.info = info
        self.B = B
        self.n = [i.n for i in self.instances]
        self.T = [i.T for i in self.instances]
        self.n_s = [int(i.n_s) for i in self.instances]
        self.n_u = [3 * len(i.grip_nodes) for i in self.instances]
        self._off_cache = {}

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                self.lib.cord_sim_destroy(self._h)
                self._h = c_void_p()
        except Exception:
            pass

    # ------------------------------------------------------------ layout
    def offsets(self, ckpt_every: int = 0):
        """dict of int64 numpy arrays (B + 1 entries): s, u, traj, ckpt, A, B."""
        key = ckpt_every
        if key in self._off_cache:
            return self._off_cache[key]
        arrs = [(c_int64 * (self.B + 1))() for _ in range(6)]
        L.check(self.lib.cord_sim_offsets(self._h, ckpt_every, *[ctypes.cast(a, POINTER(c_int64)) if (i != 3 or ckpt_every > 0) else None
                                                                  for i, a in enumerate(arrs)]))
        out = {k: np.frombuffer(a, dtype=np.int64).copy() for k, a in zip(["s", "u", "traj", "ckpt", "A", "B"], arrs)}
        self._off_cache[key] = out
        return out

    def uniform(self):
        return len(set(self.n)) == 1 and len(set(self.T)) == 1 and len(set(self.n_u)) == 1

    def _empty(self, floats):
        return torch.empty(int(floats), dtype=torch.float32, device=self.device)

    def ckpt_floats(self, K):
        return int(self.offsets(K)["ckpt"][-1])

    # ------------------------------------------------------------ calls
    def rollout(self, s0, u, store: int = L.STORE_FULL, ckpt_every: int = 10, out=None,
                status=None, counters=None, use_kappa_bwd=False, final_state=None):
        """s0: flat float32 cuda tensor (sum n_s), u: flat (sum T n_u).
        Returns the trajectory buffer (flat) in the requested storage."""
        if store == L.STORE_FULL:
            floats = self.info.traj_floats
        elif store == L.STORE_CKPT:
            floats = self.ckpt_floats(ckpt_every)
        else:
            floats = self.info.s_floats
        traj = self._empty(floats) if out is None else out
        o = L.RolloutOpts()
        o.store, o.ckpt_every, o.use_kappa_bwd = store, ckpt_every, int(bool(use_kappa_bwd))
        o.final_state = _ptr(final_state)
        if counters is not None:
            o.counters = ctypes.cast(c_void_p(counters.data_ptr()), POINTER(c_uint32))
        L.check(self.lib.cord_rollout(self._h, _ptr(s0), _ptr(u), _ptr(traj), _ptr(status), byref(o), _stream()))
        st = getattr(self, "_aux_state", None)
        if st is not None and store == L.STORE_FULL:
            st.gen += 1      # the step internals now belong to this trajectory
        return traj

    def backward(self, u, traj, traj_bar=None, sT_bar=None, store: int = L.STORE_FULL, ckpt_every: int = 10,
                 status=None, counters=None, use_kappa_bwd=False):
        s0_bar = self._empty(self.info.s_floats)
        u_bar = self._empty(max(self.info.u_floats, 1))
        o = L.BackwardOpts()
        o.store, o.ckpt_every, o.use_kappa_bwd = store, ckpt_every, int(bool(use_kappa_bwd))
        o.sT_bar = _ptr(sT_bar)
        if counters is not None:
            o.counters = ctypes.cast(c_void_p(counters.data_ptr()), POINTER(c_uint32))
        L.check(self.lib.cord_rollout_backward(self._h, _ptr(u), _ptr(traj), _ptr(traj_bar), _ptr(s0_bar),
                                               _ptr(u_bar), _ptr(status), byref(o), _stream()))
        return s0_bar, u_bar[:self.info.u_floats]

    def linearize(self, traj, u, dense: bool = True, want_B: bool = True, jvp_k: int = 0, jvp_ds=None,
                  jvp_du=None, status=None, A=None, Bm=None):
        if dense and A is None:
            A = self._empty(self.info.A_floats)
        if want_B and Bm is None:
            Bm = self._empty(max(self.info.B_floats, 1))
        jv = None
        out = None
        if jvp_k:
            tns = sum(T * ns for T, ns in zip(self.T, self.n_s))
            out = self._empty(jvp_k * tns)
            jv = L.Jvp()
            jv.k, jv.ds, jv.du, jv.out = jvp_k, _ptr(jvp_ds), _ptr(jvp_du), _ptr(out)
        L.check(self.lib.cord_linearize(self._h, _ptr(traj), _ptr(u), _ptr(A if dense else None),
                                        _ptr(Bm if want_B else None), byref(jv) if jv is not None else None,
                                        _ptr(status), _stream()))
        return (A if dense else None), (Bm if want_B else None), out

    def lin_stats(self):
        """Direct-linearization counters since creation: {"slot_overlaps",
        "steps_redone"} (synchronizes the device)."""
        out = (c_int64 * 2)()
        L.check(self.lib.cord_sim_lin_stats(self._h, out))
        return {"slot_overlaps": int(out[0]), "steps_redone": int(out[1])}

    # ------------------------------------------------------------ conformal calibration
    def cp_scores(self, s_bar, u, s_next, status=None):
        """Nonconformity scores |q+ - f(q, u)|_2 of a calibration set (one
        instance of T = 1 per pair): a float32 tensor of B scores."""
        scores = self._empty(self.B)
        L.check(self.lib.cord_cp_scores(self._h, _ptr(s_bar), _ptr(u), _ptr(s_next), _ptr(scores), _ptr(status),
                                        _stream()))
        return scores

    # ------------------------------------------------------------ step internals
    def use_aux(self, on: bool = True, buffer=None):
        """Keep the internals of every solved step (cord_sim_set_aux): FULL
        rollouts write them, backward (FULL) and linearize read them instead
        of solving each step again.  The buffer is allocated here, or is
        `buffer` (a float32 device tensor of at least info.aux_floats
        floats, e.g. another simulator's `aux` over the same instances, so
        that one simulator's rollout feeds the other's derivatives)."""
        if on:
            if buffer is not None:
                if (buffer.dtype != torch.float32 or buffer.device != self.device or not buffer.is_contiguous()
                        or buffer.numel() < self.info.aux_floats):
                    raise ValueError(f"aux buffer must be a contiguous float32 tensor on {self.device} "
                                     f"with at least {self.info.aux_floats} elements")
                self._aux = buffer
                self._aux_state = _AuxState.shared.get(buffer.data_ptr()) or _AuxState(buffer)
            elif getattr(self, "_aux", None) is None:
                self._aux = self._empty(max(self.info.aux_floats, 1))
                self._aux_state = _AuxState(self._aux)
            _AuxState.shared[self._aux.data_ptr()] = self._aux_state
            L.check(self.lib.cord_sim_set_aux(self._h, _ptr(self._aux)))
        else:
            L.check(self.lib.cord_sim_set_aux(self._h, None))
            self._aux = None
            self._aux_state = None

    def aux_generation(self):
        """Count of FULL rollouts that have written the step internals in use
        (None without a buffer)."""
        st = getattr(self, "_aux_state", None)
        return None if st is None else st.gen

    @contextlib.contextmanager
    def aux_if_current(self, gen):
        """Inside the block the step internals are used only if no FULL
        rollout has overwritten them since generation `gen`; otherwise the
        calls inside solve each step again from the stored states."""
        st = getattr(self, "_aux_state", None)
        if st is None or gen == st.gen:
            yield
            return
        L.check(self.lib.cord_sim_set_aux(self._h, None))
        try:
            yield
        finally:
            L.check(self.lib.cord_sim_set_aux(self._h, _ptr(self._aux)))

    @property
    def aux(self):
        """The step-internals buffer in use (None if none)."""
        return getattr(self, "_aux", None)

    # ------------------------------------------------------------ launch
    def set_launch(self, mode: int):
        """mode: _lib.LAUNCH_GROUPED / PER_INSTANCE / PERSISTENT / GRAPH."""
        L.check(self.lib.cord_sim_set_launch(self._h, int(mode)))

    def autotune(self, s0, u, sample: int = 64, cache_path=None):
        path = cache_path.encode() if cache_path else None
        L.check(self.lib.cord_autotune(self._h, _ptr(s0), _ptr(u), int(sample), path, _stream()))
        return self.classes()

    def classes(self):
        """[(topology, nmax, threads, particles_per_thread, instances)] per size class."""
        cap = 16
        arrs = [(ctypes.c_int32 * cap)() for _ in range(5)]
        cnt = ctypes.c_int32()
        L.check(self.lib.cord_sim_classes(self._h, *[ctypes.cast(a, POINTER(ctypes.c_int32)) for a in arrs], cap,
                                          byref(cnt)))
        return [tuple(int(a[i]) for a in arrs) for i in range(cnt.value)]

    # ------------------------------------------------------------ helpers
    def pack_states(self, states):
        """list of per-instance numpy state vectors -> flat float32 tensor."""
        return torch.from_numpy(np.concatenate([np.asarray(s, dtype=np.float32).ravel() for s in states])).to(self.device)

    def pack_controls(self, controls):
        return torch.from_numpy(np.concatenate([np.asarray(u, dtype=np.float32).ravel() for u in controls]
                                               + [np.zeros(0, np.float32)])).to(self.device)

    def split(self, flat, kind: str, ckpt_every: int = 0):
        """Split a flat buffer into per-instance numpy arrays (kind: s, u, traj, ckpt, A, B)."""
        off = self.offsets(ckpt_every)[kind]
        h = flat.detach().cpu().numpy()
        return [h[off[i]:off[i + 1]] for i in range(self.B)]


def cp_radius(scores, delta: float, horizon: int):
    """Conformal radius of a device tensor of scores for miscoverage `delta`
    over `horizon` steps: (radius, index) as one-element device tensors
    (index -1 with an infinite radius)."""
    lib = L.load()
    radius = torch.empty(1, dtype=torch.float32, device=scores.device)
    index = torch.empty(1, dtype=torch.int32, device=scores.device)
    L.check(lib.cord_cp_radius(_ptr(scores), int(scores.numel()), float(delta), int(horizon), _ptr(radius),
                               _ptr(index), _stream()))
    return radius, index

