"""CPU checks of bench.py's algorithmic-byte accounting (the roofline numerator)."""
import numpy as np

import bench


def test_frame_decode_bytes_counts_every_iteration_once():
    n, m, E, s = 1024, 512, 3072, 4
    it = np.array([0, 1, 7])
    # per frame: t*(2 s E + 12 n) + (t+1) m + 13 n
    expect = sum(t * (2 * s * E + 12 * n) + (t + 1) * m + 13 * n for t in it)
    assert bench.frame_decode_bytes(it, n, m, E, s) == expect


def test_per_edge_iteration_figure_matches_design_value():
    # lambda(x) code: mean variable degree 3.5703; fp32 messages -> 2*4 + 12/3.57 = 11.4 B
    # per edge-iteration for the message + posterior traffic (the 15.4 B figure adds the
    # 4 B index of explicit codes); n large so that set-up terms vanish
    n = 1 << 16
    E = int(round(3.5703125 * n))
    per = (bench.frame_decode_bytes(np.array([1000]), n, 0, E, 4) - 13 * n) / (1000 * E)
    assert abs(per - (8 + 12 / 3.5703125)) < 1e-6


def test_stage_bytes_check_pass_split():
    n, m, E, s, T = 100, 50, 300, 4, 10
    it = np.array([3, 10])
    chk, full = bench.stage_bytes(it, T, n, m, E, s)
    # frame stopping at 3: 4 tests, updates at t=0..3 (read at t=1..3); at T=10: 11 tests, updates t=0..9
    expect = (4 * (4 * n + m) + (4 + 3) * s * E) + (11 * (4 * n + m) + (10 + 9) * s * E)
    assert chk == expect
    assert full == (3 + 10) * (2 * s * E + 12 * n)


def test_wilson_interval_closed_forms():
    """No failures: the upper end is z^2 / (F + z^2); the interval of F - k
    failures mirrors that of k; it contains the point estimate."""
    z2 = 1.959963984540054 ** 2
    lo, hi = bench.wilson95(0, 2048)
    assert lo == 0.0 and abs(hi - z2 / (2048 + z2)) < 1e-15
    for k, F in ((3, 17), (35, 100), (1, 2)):
        a, b = bench.wilson95(k, F)
        c, d = bench.wilson95(F - k, F)
        assert abs(a - (1 - d)) < 1e-12 and abs(b - (1 - c)) < 1e-12
        assert a <= k / F <= b


def test_key_rate_exp_field_follows_the_key_rate_model():
    """bench's K'_exp field: absent without --s-be; with it, keyrate.k_exp at
    the paper's standard failure probabilities and m = 4 slices."""
    import types
    from paper_2108_08418_amd import keyrate
    assert bench.key_rate_exp(types.SimpleNamespace(s_be=None), 2 ** 27, 0.68, 0.05) is None
    r = bench.key_rate_exp(types.SimpleNamespace(s_be=0.5), 2 ** 27, 0.68, 0.05)
    d_aep = keyrate.delta_aep(4, 2 ** 27, 1.25e-10, 1e-9)
    assert r["bits_per_s"] == keyrate.k_exp(2 ** 27, 0.68, 0.5, d_aep, 2.5e-10, 0.05)
    assert 0 < r["bits_per_s"] < 2 ** 27 * 0.18 / 0.05


def test_reconciliation_efficiency_field():
    """bench's beta at SNR 3 with the slice codes' rates: (4 - 4 + 0.68) / 1."""
    r = bench.efficiency([0.0, 0.0, 0.1875, 0.4921875])
    assert abs(r["beta"] - 0.6796875) < 1e-9 and abs(r["label_entropy_bits"] - 4.0) < 1e-12
    assert 0.95 < r["quantiser_bound"] < 0.97 and r["I_AB_bits"] == 1.0
