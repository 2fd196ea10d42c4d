"""MI355X-native batched differentiable rope/cloth simulation (libcord).

The simulation, its adjoint and its linearizations run in hand-written HIP
kernels for gfx950 inside libcord.so (C ABI declared in include/cord.h).
This package is the thin binding: `Sim` (descriptors, buffers, calls on
torch's current stream) and `CordRollout` (torch.autograd.Function).
"""
from ._lib import CordError, load  # noqa: F401

__all__ = ["Sim", "CordRollout", "rollout", "cp_radius", "load", "CordError"]


def __getattr__(name):
    if name in ("Sim", "cp_radius"):
        from . import api
        return getattr(api, name)
    if name in ("CordRollout", "rollout"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
