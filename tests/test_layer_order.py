"""The block-row order of the slice codes (host-side input generation, no GPU):
runs of up to 8 rows with pairwise disjoint columns, the layers a layered
decoder updates together."""
import numpy as np
import pytest

from paper_2108_08418_amd import inputs


def _runs(base, cap):
    """Greedy runs of consecutive rows with pairwise disjoint columns, at most cap
    rows each (the grouping a layered decoder applies to the rows as listed)."""
    runs, first = [], 0
    for i in range(1, base.shape[0] + 1):
        split = i == base.shape[0] or i - first >= cap
        if not split:
            split = any((base[r] & base[i]).any() for r in range(first, i))
        if split:
            runs.append(list(range(first, i)))
            first = i
    return runs


def test_layer_order_is_a_permutation_of_disjoint_runs():
    rng = np.random.default_rng(3)
    for _ in range(20):
        mb, nb = int(rng.integers(4, 60)), int(rng.integers(8, 80))
        base = (rng.random((mb, nb)) < 0.15).astype(np.uint8)
        order = inputs.layer_order(base, group=8)
        assert sorted(order.tolist()) == list(range(mb))
        b = base[order]
        for run in _runs(b, 8):
            cols = b[run].sum(0)
            assert cols.max() <= 1          # no two rows of a run share a column


@pytest.mark.parametrize("j,steps", [(2, 13), (3, 12)])
def test_slice_codes_list_their_block_rows_in_layer_runs(j, steps):
    """At n = 2^16 the slice codes' 104 (slice 2) and 65 (slice 3) block rows form
    13 and 12 runs; every run is column-disjoint; the code is the same for every
    sub-block length (one protograph, shifts per Z)."""
    qc = inputs.slice_code_spec(j, 1 << 16)
    base = (qc.shift >= 0).astype(np.uint8)
    runs = _runs(base, 8)
    assert len(runs) == steps
    for run in runs:
        assert base[run].sum(0).max() <= 1
    other = inputs.slice_code_spec(j, 1 << 12)
    np.testing.assert_array_equal((other.shift >= 0), (qc.shift >= 0))
    np.testing.assert_array_equal(other.block_type, qc.block_type)
