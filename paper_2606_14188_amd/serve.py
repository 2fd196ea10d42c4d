"""Python front end of libcord's planning server (cord_server_* / cord_plan_*).

Argument marshalling only: planning (batched rollouts, adjoints, gradient
steps, argmin, linearization) runs on the device inside libcord; the
scheduler is a native thread inside libcord.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int64, c_uint64, c_void_p

import numpy as np

from . import _lib as L
from .api import make_desc


class PlanResult:
    def __init__(self, r: L.PlanResult, want_AB: bool):
        self.status = r.status
        self.sim_status = r.sim_status
        self.best = r.best
        self.cost = r.cost
        T, ns, nu, C = r.T, r.n_s, r.n_u, r.n_cand
        self.u = np.ctypeslib.as_array(r.u, shape=(T * nu,)).reshape(T, nu).copy() if r.u and nu else np.zeros((T, nu))
        self.traj = np.ctypeslib.as_array(r.traj, shape=((T + 1) * ns,)).reshape(T + 1, ns).copy() if r.traj else None
        self.costs = np.ctypeslib.as_array(r.costs, shape=(C,)).copy() if r.costs else None
        self.A = np.ctypeslib.as_array(r.A, shape=(T * ns * ns,)).reshape(T, ns, ns).copy() if (want_AB and r.A) else None
        self.B = np.ctypeslib.as_array(r.B, shape=(T * ns * nu,)).reshape(T, ns, nu).copy() if (want_AB and r.B and nu) else None
        self.t_submit, self.t_admit, self.t_done = r.t_submit, r.t_admit, r.t_done

    @property
    def latency(self):
        return self.t_done - self.t_submit


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 8, queue_cap: int = 100000):
        self.lib = L.load()
        self._h = c_void_p()
        L.check(self.lib.cord_server_create(device, int(hbm_budget), int(max_slots), int(queue_cap), byref(self._h)))
        self._want = {}

    def close(self):
        if self._h and self._h.value:
            self.lib.cord_server_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, inst, goal_node: int, goal, n_cand: int = 128, iters: int = 10, step: float = 0.05,
               u_max: float = 0.5, sigma: float = 0.05, u_reg: float = 1e-3, seed: int = 0, want_AB: bool = False,
               u_warm=None, u_init=None, s0=None):
        r = L.PlanRequest()
        r.inst = make_desc(inst)
        s0a = np.ascontiguousarray(inst.s0 if s0 is None else s0, dtype=np.float32)
        uw = None if u_warm is None else np.ascontiguousarray(u_warm, dtype=np.float32)
        ui = None if u_init is None else np.ascontiguousarray(u_init, dtype=np.float32)
        r.s0 = s0a.ctypes.data
        r.u_warm = uw.ctypes.data if uw is not None else None
        r.u_init = ui.ctypes.data if ui is not None else None
        r.goal_node = int(goal_node)
        for c in range(3):
            r.goal[c] = float(goal[c])
        r.seed, r.n_cand, r.iters = int(seed), int(n_cand), int(iters)
        r.step, r.u_max, r.sigma, r.u_reg = float(step), float(u_max), float(sigma), float(u_reg)
        r.want_AB = int(bool(want_AB))
        t = c_uint64()
        rc = self.lib.cord_plan_submit(self._h, byref(r), byref(t))
        L.check(rc)
        self._want[t.value] = bool(want_AB)
        return t.value

    def poll(self, ticket):
        r = L.PlanResult()
        rc = self.lib.cord_plan_poll(self._h, ticket, byref(r))
        if rc == L.CORD_EAGAIN:
            return None
        L.check(rc)
        return PlanResult(r, self._want.get(ticket, False))

    def wait(self, ticket, timeout_ms: int = -1):
        r = L.PlanResult()
        rc = self.lib.cord_plan_wait(self._h, ticket, int(timeout_ms), byref(r))
        if rc == L.CORD_EAGAIN:
            return None
        L.check(rc)
        return PlanResult(r, self._want.get(ticket, False))

    def release(self, ticket):
        L.check(self.lib.cord_plan_release(self._h, ticket))
        self._want.pop(ticket, None)

    def stats(self):
        a = (c_int64 * 8)()
        L.check(self.lib.cord_server_stats(self._h, a))
        keys = ["submitted", "admitted", "completed", "failed", "queued", "running", "peak_queue", "bytes_in_use"]
        return dict(zip(keys, list(a)))
