"""The planning server's documented candidate draw, restated from the
published definitions of its generator (SplitMix64) and of the Box-Muller
transform, for tests that reproduce a seeded request."""
import math

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(state):
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): returns the new
    state and the output."""
    state = (state + 0x9E3779B97F4A7C15) & _M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return state, z ^ (z >> 31)


def candidate_starts(u_warm, C, sigma, seed):
    """Candidate starts as the request documentation defines them."""
    w = np.asarray(u_warm, dtype=np.float32).ravel()
    out = np.empty((C, w.size), dtype=np.float32)
    state = seed & _M64
    for c in range(C):
        for i in range(w.size):
            if c == 0:
                z = 0.0
            else:
                state, x1 = splitmix64(state)
                state, x2 = splitmix64(state)
                a1 = ((x1 >> 11) + 0.5) * 2.0 ** -53
                a2 = ((x2 >> 11) + 0.5) * 2.0 ** -53
                z = math.sqrt(-2.0 * math.log(a1)) * math.cos(2.0 * math.pi * a2)
            out[c, i] = w[i] + np.float32(sigma) * np.float32(z)
    return out.reshape((C,) + np.shape(u_warm))
