"""Output-feedback SLS, stage 3 (Sec. 4.2), on the device: thin binding of
the cord_sls_* entry points (argument marshalling only; every step runs in
libcord's kernels, on torch's current stream).

Shapes (float32 CUDA tensors, contiguous): A, E, F (B, N, n, n); Bm (B, N,
n, m); K (B, N+1, m, n); Xi (B, n, n).  C = I: the perception returns the
full state.  Horizon operators are dense (B, (N+1) r, (N+1) n) with block
(k, j) at rows k r, columns j n (r = n for state rows, m for input rows).
"""
from __future__ import annotations

from ctypes import byref, c_void_p

import torch

from . import _lib as L

SERIAL, SCAN = L.SLS_SERIAL, L.SLS_SCAN


def _p(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _st():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class SLS:
    """A handle for B trajectories of N steps, state size n, input size m."""

    def __init__(self, batch, horizon, n, n_u, device="cuda"):
        self._lib = L.load()
        self.B, self.N, self.n, self.m = int(batch), int(horizon), int(n), int(n_u)
        self.device = torch.device(device)
        h = c_void_p()
        with torch.cuda.device(self.device):
            L.check(self._lib.cord_sls_create(self.B, self.N, self.n, self.m, byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cord_sls_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, shape, name):
        if t is None:
            raise ValueError(f"{name} is required")
        if tuple(t.shape) != tuple(shape) or t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name}: expected contiguous float32 CUDA tensor of shape {tuple(shape)}, "
                             f"got {tuple(t.shape)} {t.dtype}")
        return t

    def _empty(self, *shape):
        return torch.empty(shape, dtype=torch.float32, device=self.device)

    @property
    def D(self):
        return (self.N + 1) * self.n

    def kalman(self, A, E, F, Xi, mode=SCAN):
        """(Pi (B, N+1, n, n), L (B, N, n, n) with L[:, j] = L_{j+1}, status (B,))."""
        B, N, n = self.B, self.N, self.n
        for t, s, nm in ((A, (B, N, n, n), "A"), (E, (B, N, n, n), "E"), (F, (B, N, n, n), "F"), (Xi, (B, n, n), "Xi")):
            self._check(t, s, nm)
        Pi = self._empty(B, N + 1, n, n)
        Lg = self._empty(B, N, n, n)
        status = torch.empty(B, dtype=torch.int32, device=self.device)
        L.check(self._lib.cord_sls_kalman(self._h, _p(A), _p(E), _p(F), _p(Xi), int(mode), _p(Pi), _p(Lg),
                                          _p(status), _st()))
        return Pi, Lg, status

    def observer(self, A, Lg):
        """(Phihat^x, Phihat^y), both (B, D, D)."""
        B, N, n = self.B, self.N, self.n
        self._check(A, (B, N, n, n), "A")
        self._check(Lg, (B, N, n, n), "L")
        Phx, Phy = self._empty(B, self.D, self.D), self._empty(B, self.D, self.D)
        L.check(self._lib.cord_sls_observer(self._h, _p(A), _p(Lg), _p(Phx), _p(Phy), _st()))
        return Phx, Phy

    def state_feedback(self, A, Bm, K):
        """(Phibar^x (B, D, D), Phibar^u (B, (N+1) m, D)) of u_j = K_j x_j."""
        B, N, n, m = self.B, self.N, self.n, self.m
        self._check(A, (B, N, n, n), "A")
        self._check(Bm, (B, N, n, m), "Bm")
        self._check(K, (B, N + 1, m, n), "K")
        Pbx, Pbu = self._empty(B, self.D, self.D), self._empty(B, (N + 1) * m, self.D)
        L.check(self._lib.cord_sls_state_feedback(self._h, _p(A), _p(Bm), _p(K), _p(Pbx), _p(Pbu), _st()))
        return Pbx, Pbu

    def assemble(self, A, Pbx, Pbu, Phx, Phy):
        """(Phi^xw, Phi^uw, Phi^xe, Phi^ue)."""
        B, N, n, m, D = self.B, self.N, self.n, self.m, self.D
        self._check(A, (B, N, n, n), "A")
        for t, s, nm in ((Pbx, (B, D, D), "Pbx"), (Pbu, (B, (N + 1) * m, D), "Pbu"), (Phx, (B, D, D), "Phx"),
                         (Phy, (B, D, D), "Phy")):
            self._check(t, s, nm)
        xw, xe = self._empty(B, D, D), self._empty(B, D, D)
        uw, ue = self._empty(B, (N + 1) * m, D), self._empty(B, (N + 1) * m, D)
        L.check(self._lib.cord_sls_assemble(self._h, _p(A), _p(Pbx), _p(Pbu), _p(Phx), _p(Phy), _p(xw), _p(uw),
                                            _p(xe), _p(ue), _st()))
        return xw, uw, xe, ue

    def tubes(self, xw, xe, E, F, uw=None, ue=None):
        """(tau_x (B, N+1, n), tau_u (B, N+1, m) or None)."""
        B, N, n, m, D = self.B, self.N, self.n, self.m, self.D
        self._check(xw, (B, D, D), "Pxw")
        self._check(xe, (B, D, D), "Pxe")
        self._check(E, (B, N, n, n), "E")
        self._check(F, (B, N, n, n), "F")
        tx = self._empty(B, N + 1, n)
        tu = None
        if uw is not None:
            self._check(uw, (B, (N + 1) * m, D), "Puw")
            self._check(ue, (B, (N + 1) * m, D), "Pue")
            tu = self._empty(B, N + 1, m)
        L.check(self._lib.cord_sls_tubes(self._h, _p(xw), _p(xe), _p(uw), _p(ue), _p(E), _p(F), _p(tx), _p(tu),
                                         _st()))
        return tx, tu
