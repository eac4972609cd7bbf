"""Pins of the oracle's layered (row-serial) schedule and of its binary32
modes, one iteration at a time.

The layered fp64 mode is pinned to closed forms (a chain of degree-2 checks
after one iteration, which also tells the schedule apart from flooding), to
exact marginals on cycle-free graphs and on a single check, to flooding where
the two schedules coincide (every variable in one check), and to coset
symmetry.  The binary32 modes (flooding and layered), which take the
minimum-selection and binary16-rounding decisions in a binary32 decoder's
precision, are compared with the fp64 definitions one step at a time: from
the same state at every iteration t = 0..14, so that the extrinsic forms
(L_post - c2v in binary32, L_ch + sum over the other checks in fp64) meet
from iteration 1 on."""
import numpy as np
import pytest

import oracle
from paper_2108_08418_amd import inputs as I
from tests.test_oracle_bp import _csr_from_dense, _exact_posteriors, _random_tree

ULP32 = 2.0 ** -24
HALF_TOL = 2.0 ** -10          # two binary16 ulps of the scale


def _chain(N):
    """Checks c_k = {v_k, v_(k+1)}, k = 0..N-1: one layer per check, in order."""
    H = np.zeros((N, N + 1), np.uint8)
    for k in range(N):
        H[k, k] = H[k, k + 1] = 1
    return H, np.arange(N + 1, dtype=np.int32)


@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_chain_of_degree_two_checks_after_one_layered_iteration(algo):
    """Layer k passes v_k's current extrinsic value to v_(k+1), which already
    holds everything the layers before it sent: after one iteration
    L_post[v_k] = L_0 + ... + L_(k-1) + L_k + L_(k+1) (forward sums plus the
    right neighbour), where flooding gives L_(k-1) + L_k + L_(k+1)."""
    N = 9
    H, layers = _chain(N)
    code = _csr_from_dense(H)
    L = np.array([0.625, -1.25, 2.0, 0.375, -0.5, 1.75, 0.25, -0.125, 1.5, 0.875])  # dyadic: sums are exact
    r = oracle.decode_layered(code, L[None, :], None, layers=layers, algo=algo, alpha=1.0, max_iter=1,
                              early_stop=False)
    expect = np.array([L[:k + 1].sum() + (L[k + 1] if k < N else 0.0) for k in range(N + 1)])
    if algo == oracle.NMS:
        np.testing.assert_array_equal(r["post"][0], expect)
    else:
        np.testing.assert_allclose(r["post"][0], expect, rtol=1e-13, atol=1e-13)
    flood = oracle.decode(code, L[None, :], None, algo=algo, alpha=1.0, max_iter=1, early_stop=False)
    expect_f = np.array([L[max(k - 1, 0):k + 2].sum() for k in range(N + 1)])
    np.testing.assert_allclose(flood["post"][0], expect_f, rtol=1e-13, atol=1e-13)
    assert np.abs(r["post"][0] - flood["post"][0]).max() > 1.0


@pytest.mark.parametrize("seed", range(6))
def test_layered_sum_product_on_trees_gives_exact_marginals(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(6, 14))
    H = _random_tree(n, rng)
    code = _csr_from_dense(H)
    L = rng.normal(0.8, 1.5, n)
    s = rng.integers(0, 2, H.shape[0]).astype(np.uint8)
    layers = np.arange(H.shape[0] + 1, dtype=np.int32)                      # one check per layer
    if seed % 2:                                                             # and in reverse order
        perm = np.arange(H.shape[0])[::-1]
        H, s = H[perm], s[perm]
        code = _csr_from_dense(H)
    r = oracle.decode_layered(code, L[None, :], s[None, :], layers=layers, algo=oracle.SP, max_iter=2 * n,
                              early_stop=False)
    ref = _exact_posteriors(H, L, s.astype(np.int64))
    np.testing.assert_allclose(r["post"][0], ref, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("s", [0, 1])
def test_layered_single_check_is_exact_map(s):
    rng = np.random.default_rng(7 + s)
    d = 7
    H = np.ones((1, d), np.uint8)
    code = _csr_from_dense(H)
    L = rng.normal(0.5, 2.0, d)
    r = oracle.decode_layered(code, L[None, :], np.array([[s]], np.uint8), layers=[0, 1], algo=oracle.SP,
                              max_iter=1, early_stop=False)
    np.testing.assert_allclose(r["post"][0], _exact_posteriors(H, L, np.array([s])), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("prec32", [False, True])
@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_layered_equals_flooding_when_every_variable_has_one_check(algo, prec32):
    """Block-diagonal H (rows with disjoint supports), in one layer or several:
    no message of an earlier layer reaches a later one, so in fp64 both
    schedules are the same computation, bit for bit.  In binary32 the layered
    form keeps a running posterior ((L_ch + c) - c is not always L_ch in
    rounding), so the two agree to a few binary32 roundings."""
    rng = np.random.default_rng(3)
    H = np.zeros((6, 24), np.uint8)
    for r in range(6):
        H[r, 4 * r:4 * r + 4] = 1
    code = _csr_from_dense(H)
    L = rng.normal(0.3, 2.0, (4, 24))
    s = rng.integers(0, 2, (4, 6)).astype(np.uint8)
    for layers in ([0, 6], [0, 2, 3, 6]):
        a = oracle.decode_layered(code, L, s, layers=layers, algo=algo, alpha=0.8, max_iter=5, early_stop=False,
                                  prec32=prec32, trace=True)
        b = oracle.decode(code, L, s, algo=algo, alpha=0.8, max_iter=5, early_stop=False, prec32=prec32, trace=True)
        if not prec32:
            for k in ("post", "bits", "iters", "ok", "post_trace", "scale_trace"):
                np.testing.assert_array_equal(a[k], b[k])
        else:
            err = np.abs(a["post_trace"] - b["post_trace"]) / b["scale_trace"]
            assert np.nanmax(err) <= 16 * ULP32
            assert np.abs(a["post_trace"] - b["post_trace"]).max() > 0      # the running sum does round


def test_layers_sharing_a_variable_are_rejected():
    H, _ = _chain(4)
    code = _csr_from_dense(H)
    with pytest.raises(ValueError, match="share a variable"):
        oracle.decode_layered(code, np.zeros((1, 5)), None, layers=[0, 2, 4], max_iter=1)
    with pytest.raises(ValueError, match="rejected"):
        oracle.decode_layered(code, np.zeros((1, 5)), None, layers=[0, 2, 3], max_iter=1)


@pytest.mark.parametrize("prec32", [False, True])
@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_layered_coset_symmetry_is_bit_exact(algo, prec32):
    qc = I.slice_code_spec(3, 1024)
    code = qc.to_csr()
    rng = np.random.default_rng(8)
    F = 4
    bits = rng.integers(0, 2, (F, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(np.zeros_like(bits), 0.5, 12)
    lay = oracle.qc_layers(qc.mb, qc.Z)
    a = oracle.decode_layered(code, llr, np.zeros((F, code.m), np.uint8), layers=lay, algo=algo, max_iter=30,
                              prec32=prec32, store_half=(algo == oracle.NMS))
    sc, _ = oracle.syndrome(code, bits)
    b = oracle.decode_layered(code, llr * (1 - 2 * bits.astype(np.float64)), sc, layers=lay, algo=algo,
                              max_iter=30, prec32=prec32, store_half=(algo == oracle.NMS))
    np.testing.assert_array_equal(b["bits"], a["bits"] ^ bits)
    np.testing.assert_array_equal(b["iters"], a["iters"])
    np.testing.assert_array_equal(np.abs(b["post"]), np.abs(a["post"]))


def test_layered_needs_fewer_iterations_than_flooding_on_a_slice_code():
    """Not a bound the paper states: a sanity check that the layered schedule
    is the faster-converging one on the slice-3 code (serial schedules pass
    each iteration's new messages on within the iteration)."""
    qc = I.slice_code_spec(3, 4096)
    code = qc.to_csr()
    x, y = I.gaussian_pairs(4096 * 6, 3.0, seed=1)
    th = I.equiprobable_thresholds(4, 4 / 3)
    S = oracle.quantize(y, th, 4)
    L = oracle.slice_llr(x, np.sqrt(1 / 3), th, 4, oracle.GRAY, 3, 7, S).reshape(6, -1)
    s, _ = oracle.syndrome(code, S[3].reshape(6, -1))
    f = oracle.decode(code, L, s, algo=oracle.SP, max_iter=100)
    lay = oracle.decode_layered(code, L, s, layers=oracle.qc_layers(qc.mb, qc.Z), algo=oracle.SP, max_iter=100)
    both = (f["ok"] == 1) & (lay["ok"] == 1)
    assert both.sum() >= 4
    assert lay["iters"][both].sum() < 0.8 * f["iters"][both].sum()


# --------------------------------------------------------------------------
# binary32 modes, one step at a time
# --------------------------------------------------------------------------

def _frame(code, sigma2, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, (1, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(bits, sigma2, seed + 1)[0]
    s, _ = oracle.syndrome(code, bits)
    return llr, s[0]


def _scale(code, llr, c2v):
    sc = np.abs(llr).copy()
    np.add.at(sc, code.col_idx, np.abs(c2v))
    return sc


CASES = [(oracle.SP, False, 64 * ULP32, 512 * ULP32), (oracle.NMS, False, 64 * ULP32, 512 * ULP32),
         (oracle.NMS, True, HALF_TOL, HALF_TOL)]


@pytest.mark.parametrize("algo,half,tol_flood,tol_layered", CASES)
def test_binary32_flooding_step_matches_fp64_step_at_every_iteration(algo, half, tol_flood, tol_layered):
    """From the binary32 state c2v(t) at t = 0..14, the fp64 step (v2c written
    as L_ch + sum over the other checks) and the binary32 step (L_post - c2v)
    give posteriors within tol of the scale |L_ch| + sum |c2v|; iterating the
    binary32 step from zero reproduces the binary32 decoder bit for bit."""
    qc = I.lambda_half_rate_spec(2048)
    code = qc.to_csr()
    for seed in (21, 41):
        llr, s = _frame(code, 0.75, seed)
        ref = oracle.decode(code, llr[None, :], s[None, :], algo=algo, alpha=0.8, max_iter=15, early_stop=False,
                            store_half=half, prec32=True, trace=True)
        c = np.zeros(code.n_edges)
        for t in range(15):
            c32, p32 = oracle.flood_step(code, llr, s, c, t, algo=algo, store_half=half, prec32=True, alpha=0.8)
            c64, p64 = oracle.flood_step(code, llr, s, c, t, algo=algo, store_half=half, prec32=False, alpha=0.8)
            assert (np.abs(p32 - p64) / _scale(code, llr, c64)).max() <= tol_flood, (seed, t)
            np.testing.assert_array_equal(p32, ref["post_trace"][0, t + 1])
            c = c32


@pytest.mark.parametrize("algo,half,tol_flood,tol_layered", CASES)
def test_binary32_layered_step_matches_fp64_step_at_every_iteration(algo, half, tol_flood, tol_layered):
    """The same for the layered schedule: the binary32 state is (c2v, running
    posterior); the fp64 step recomputes every extrinsic sum from c2v.  The
    tolerance covers the rounding of the running posterior, which accumulates
    over the iterations (two binary32 roundings per edge and iteration)."""
    qc = I.lambda_half_rate_spec(2048)
    code = qc.to_csr()
    lay = oracle.qc_layers(qc.mb, qc.Z)
    for seed in (21, 41):
        llr, s = _frame(code, 0.75, seed)
        ref32 = oracle.decode_layered(code, llr[None, :], s[None, :], layers=lay, algo=algo, alpha=0.8,
                                      max_iter=15, early_stop=False, store_half=half, prec32=True, trace=True)
        ref64 = oracle.decode_layered(code, llr[None, :], s[None, :], layers=lay, algo=algo, alpha=0.8,
                                      max_iter=15, early_stop=False, store_half=half, trace=True)
        c = np.zeros(code.n_edges)
        L = llr.astype(np.float32).astype(np.float64)
        c64_run = np.zeros(code.n_edges)
        for t in range(15):
            c64, p64 = oracle.layered_step(code, llr, s, c, L, t, layers=lay, algo=algo, store_half=half,
                                           alpha=0.8)
            c, L = oracle.layered_step(code, llr, s, c, L, t, layers=lay, algo=algo, store_half=half, prec32=True,
                                       alpha=0.8)
            assert (np.abs(L - p64) / _scale(code, llr, c64)).max() <= tol_layered, (seed, t)
            np.testing.assert_array_equal(L, ref32["post_trace"][0, t + 1])
            c64_run, p64_run = oracle.layered_step(code, llr, s, c64_run, L, t, layers=lay, algo=algo,
                                                   store_half=half, alpha=0.8)
            np.testing.assert_array_equal(p64_run, ref64["post_trace"][0, t + 1])
