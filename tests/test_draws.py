"""The test-side SplitMix64 against its published first output for seed 0,
and the candidate starts' basic properties (no GPU)."""
import numpy as np

from tests.draws import candidate_starts, splitmix64


def test_splitmix64_reference_output():
    state, x = splitmix64(0)
    assert state == 0x9E3779B97F4A7C15
    assert x == 0xE220A8397B1DCDAF


def test_candidate_starts():
    w = np.linspace(-0.1, 0.1, 300).reshape(100, 3)
    st = candidate_starts(w, 5, 0.5, 99)
    assert st.dtype == np.float32 and st.shape == (5, 100, 3)
    assert np.array_equal(st[0], w.astype(np.float32))
    z = (st[1:] - st[0]).astype(np.float64).ravel() / 0.5
    assert abs(z.mean()) < 0.15 and abs(z.std() - 1.0) < 0.1
    assert np.array_equal(candidate_starts(w, 5, 0.5, 99), st)
    assert not np.array_equal(candidate_starts(w, 5, 0.5, 100), st)
