"""Host-side handling of the learned min-sum weights: the stored sets and the
layered schedule's iteration mapping."""
import numpy as np
import pytest

from paper_2108_08418_amd.train import layered_weights, load_weights


def test_layered_weights_take_every_second_flooding_iteration():
    w = np.arange(30, dtype=np.float32).reshape(10, 3)
    lw = layered_weights(w)
    assert lw.shape == w.shape and lw.dtype == w.dtype and lw.flags.c_contiguous
    for t in range(10):
        np.testing.assert_array_equal(lw[t], w[min(2 * t, 9)])
    np.testing.assert_array_equal(layered_weights(w, 1), w)
    np.testing.assert_array_equal(layered_weights(w, 3)[3], w[9])
    # fractional steps take the nearest flooding iteration (ties to even)
    np.testing.assert_array_equal(layered_weights(w, 1.5)[:5], w[[0, 2, 3, 4, 6]])
    with pytest.raises(ValueError):
        layered_weights(w, 0)


@pytest.mark.parametrize("j", [2, 3])
def test_stored_slice_weights_extend_by_their_last_row(j):
    w = load_weights(f"learned_slice{j}")
    assert w.ndim == 2 and w.shape[1] == 3 and np.all(w > 0)
    e = load_weights(f"learned_slice{j}", extend_to=100)
    assert e.shape == (100, 3)
    np.testing.assert_array_equal(e[: w.shape[0]], w)
    np.testing.assert_array_equal(e[w.shape[0]:], np.repeat(w[-1:], 100 - w.shape[0], axis=0))
    lw = layered_weights(e)
    np.testing.assert_array_equal(lw[: 50], e[0:100:2])
