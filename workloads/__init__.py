"""Seeded synthetic inputs for the rope/cloth simulator.

This package only draws and describes inputs (geometry, material constants,
obstacles, controls, initial states).  It contains none of the simulation's
arithmetic, imports neither the oracle nor the HIP package, and is the only
code that both of them are fed from.
"""
from .gen import (  # noqa: F401
    Instance,
    contact_kappa,
    rope,
    cloth,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    small_rope_batch,
    small_cloth_batch,
    random_cotangent,
    serve_trace,
    penalty_grasp,
    compressed_rope,
    calibration_set,
    lift_rope_envs,
    sls_system,
    friction_ropes,
    friction_cloths,
)
