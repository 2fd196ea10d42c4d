"""ctypes mirror of include/cord.h and the loader of the in-tree libcord.so.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libcord.  There is no fallback: if the library is missing or does
not load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcord.so")

CORD_OK = 0
CORD_EINVAL = 1
CORD_ENOMEM = 2
CORD_EHIP = 3
CORD_EUNSUPPORTED = 4
CORD_EAGAIN = 5
CORD_ETOOBIG = 6

ST_OK, ST_NEWTON_NOCONV, ST_NOT_PD, ST_QP_NOCONV, ST_NONFINITE = range(5)

MAX_GRIP, MAX_SPHERE, MAX_BOX, MAX_OBST = 4, 4, 2, 4
ROPE, CLOTH = 0, 1
STORE_FULL, STORE_CKPT, STORE_FINAL = 0, 1, 2
GRIP_DIRICHLET, GRIP_PENALTY = 0, 1
LAUNCH_GROUPED, LAUNCH_PER_INSTANCE, LAUNCH_PERSISTENT, LAUNCH_GRAPH = 0, 1, 2, 3
SLS_SERIAL, SLS_SCAN = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("dt", c_float), ("gamma", c_float), ("gravity", c_float * 3),
                ("kappa_fwd", c_float), ("kappa_bwd", c_float), ("mu", c_float)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("nx", c_int32), ("ny", c_int32), ("T", c_int32),
                ("h", c_float), ("mass", c_float), ("k_struct", c_float), ("k_shear", c_float),
                ("k_bend", c_float), ("n_grip", c_int32), ("grip_node", c_int32 * MAX_GRIP),
                ("ground", c_int32), ("n_sphere", c_int32), ("sphere", (c_float * 4) * MAX_SPHERE),
                ("n_box", c_int32), ("box", (c_float * 7) * MAX_BOX), ("params", Params),
                ("grip_mode", c_int32), ("D_max", c_float), ("kappa_h", c_float), ("r_g", c_float)]


class SimInfo(ctypes.Structure):
    _fields_ = [("n_inst", c_int64), ("s_floats", c_int64), ("u_floats", c_int64),
                ("traj_floats", c_int64), ("A_floats", c_int64), ("B_floats", c_int64),
                ("max_n", c_int32), ("max_T", c_int32), ("aux_floats", c_int64)]


class RolloutOpts(ctypes.Structure):
    _fields_ = [("store", c_int32), ("ckpt_every", c_int32), ("use_kappa_bwd", c_int32),
                ("reserved", c_int32), ("counters", POINTER(c_uint32)), ("final_state", c_void_p)]


class BackwardOpts(ctypes.Structure):
    _fields_ = [("store", c_int32), ("ckpt_every", c_int32), ("use_kappa_bwd", c_int32),
                ("reserved", c_int32), ("sT_bar", c_void_p), ("counters", POINTER(c_uint32))]


class Jvp(ctypes.Structure):
    _fields_ = [("k", c_int32), ("ds", c_void_p), ("du", c_void_p), ("out", c_void_p)]


class PlanRequest(ctypes.Structure):
    _fields_ = [("inst", InstanceDesc), ("s0", c_void_p), ("u_warm", c_void_p), ("u_init", c_void_p),
                ("goal_node", c_int32), ("goal", c_float * 3), ("seed", ctypes.c_uint64), ("n_cand", c_int32),
                ("iters", c_int32), ("step", c_float), ("u_max", c_float), ("sigma", c_float), ("u_reg", c_float),
                ("want_AB", c_int32), ("reserved", c_int32)]


class PlanResult(ctypes.Structure):
    _fields_ = [("status", c_int32), ("sim_status", c_int32), ("best", c_int32), ("T", c_int32), ("n_s", c_int32),
                ("n_u", c_int32), ("n_cand", c_int32), ("cost", c_float), ("u", POINTER(c_float)),
                ("traj", POINTER(c_float)), ("A", POINTER(c_float)), ("B", POINTER(c_float)),
                ("costs", POINTER(c_float)), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_STRUCTS = [Params, InstanceDesc, SimInfo, RolloutOpts, BackwardOpts, Jvp]

_EXPORTS = {
    "cord_sim_create": (c_int32, [POINTER(InstanceDesc), c_int32, POINTER(c_void_p)]),
    "cord_sim_destroy": (c_int32, [c_void_p]),
    "cord_sim_info": (c_int32, [c_void_p, POINTER(SimInfo)]),
    "cord_sim_offsets": (c_int32, [c_void_p, c_int32] + [POINTER(c_int64)] * 6),
    "cord_rollout": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               POINTER(RolloutOpts), c_void_p]),
    "cord_rollout_backward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, POINTER(BackwardOpts), c_void_p]),
    "cord_rollout_backward_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                                c_void_p, POINTER(BackwardOpts), c_void_p]),
    "cord_sim_lin_stats": (c_int32, [c_void_p, POINTER(c_int64)]),
    "cord_cp_scores": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cord_cp_radius": (c_int32, [c_void_p, c_int32, ctypes.c_double, c_int32, c_void_p, c_void_p, c_void_p]),
    "cord_linearize": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(Jvp),
                                 c_void_p, c_void_p]),
    "cord_abi_sizes": (c_int32, [POINTER(c_int64), c_int32]),
    "cord_sim_set_launch": (c_int32, [c_void_p, c_int32]),
    "cord_sim_set_aux": (c_int32, [c_void_p, c_void_p]),
    "cord_autotune": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_char_p, c_void_p]),
    "cord_sim_classes": (c_int32, [c_void_p] + [POINTER(c_int32)] * 5 + [c_int32, POINTER(c_int32)]),
    "cord_last_error": (c_char_p, []),
    "cord_server_create": (c_int32, [c_int32, ctypes.c_size_t, c_int32, c_int32, POINTER(c_void_p)]),
    "cord_server_destroy": (c_int32, [c_void_p]),
    "cord_plan_submit": (c_int32, [c_void_p, POINTER(PlanRequest), POINTER(ctypes.c_uint64)]),
    "cord_plan_poll": (c_int32, [c_void_p, ctypes.c_uint64, POINTER(PlanResult)]),
    "cord_plan_wait": (c_int32, [c_void_p, ctypes.c_uint64, c_int32, POINTER(PlanResult)]),
    "cord_plan_release": (c_int32, [c_void_p, ctypes.c_uint64]),
    "cord_server_stats": (c_int32, [c_void_p, POINTER(c_int64)]),
    "cord_sls_create": (c_int32, [c_int32, c_int32, c_int32, c_int32, POINTER(c_void_p)]),
    "cord_sls_destroy": (c_int32, [c_void_p]),
    "cord_sls_kalman": (c_int32, [c_void_p] * 5 + [c_int32] + [c_void_p] * 4),
    "cord_sls_observer": (c_int32, [c_void_p] * 6),
    "cord_sls_state_feedback": (c_int32, [c_void_p] * 7),
    "cord_sls_assemble": (c_int32, [c_void_p] * 11),
    "cord_sls_tubes": (c_int32, [c_void_p] * 10),
}

_lib = None


class CordError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcord error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libcord.so (once) and check that the ctypes mirrors match the
    C structs.  Raises if the library is absent: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcord.so not found at {path}; build it with "
                          "`python -m paper_2606_14188_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    sizes = (c_int64 * 6)()
    lib.cord_abi_sizes(sizes, 6)
    for st, sz in zip(_STRUCTS, sizes):
        if ctypes.sizeof(st) != sz:
            raise ImportError(f"ABI mismatch: {st.__name__} is {ctypes.sizeof(st)} bytes in Python, {sz} in C")
    _lib = lib
    return lib


def check(code: int):
    if code != CORD_OK:
        raise CordError(code, _lib.cord_last_error().decode())
