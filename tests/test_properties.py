"""Property tests (hypothesis) for the oracle and the host seaweed model: the
plot invariants hold for arbitrary small inputs, and the combing model agrees
with the oracle on them (no GPU)."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from test_seaweed_model import plot_by_count

letters = st.sampled_from([b"AB", b"ACGT", b"ACDEFGHIKLMNPQRSTVWY"])


@st.composite
def plot_inputs(draw):
    alpha = draw(letters)
    w = draw(st.integers(1, 8))
    m = draw(st.integers(0, w + 12))
    n = draw(st.integers(0, w + 12))
    x = bytes(draw(st.lists(st.sampled_from(list(alpha)), min_size=m, max_size=m)))
    y = bytes(draw(st.lists(st.sampled_from(list(alpha)), min_size=n, max_size=n)))
    return x, y, w


@settings(max_examples=150, deadline=None)
@given(plot_inputs())
def test_invariants_any_input(args):
    x, y, w = args
    plot = oracle.wlcs(x, y, w)
    assert plot.shape == (max(len(x) - w, 0), max(len(y) - w, 0))
    if plot.size == 0:
        return
    assert plot.max() <= w
    d = plot.astype(np.int16)
    if d.shape[0] > 1:
        assert np.abs(np.diff(d, axis=0)).max() <= 1
    if d.shape[1] > 1:
        assert np.abs(np.diff(d, axis=1)).max() <= 1
    np.testing.assert_array_equal(oracle.wlcs(y, x, w), plot.T)
    xa, ya = np.frombuffer(x, np.uint8), np.frombuffer(y, np.uint8)
    for i in range(plot.shape[0]):
        for j in range(plot.shape[1]):
            assert plot[i, j] >= int(np.sum(xa[i:i + w] == ya[j:j + w]))


@settings(max_examples=150, deadline=None)
@given(plot_inputs())
def test_seaweed_model_equals_oracle_any_input(args):
    x, y, w = args
    np.testing.assert_array_equal(plot_by_count(x, y, w), oracle.wlcs(x, y, w))
