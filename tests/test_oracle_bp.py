"""Pins of the oracle's syndrome and belief-propagation decoder against brute
force (exact MAP marginals on a single check and on cycle-free Tanner graphs),
the tanh rule in 50-digit arithmetic, hand-computed min-sum rows, coset
symmetry, NumPy's binary16 rounding and finite differences of the unrolled
min-sum loss."""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2108_08418_amd import inputs as I


def _csr_from_dense(H, edge_type=None, n_types=1):
    H = np.asarray(H, dtype=np.uint8)
    m, n = H.shape
    rows, cols = np.nonzero(H)
    row_ptr = np.zeros(m + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    et = np.zeros(len(cols), np.uint8) if edge_type is None else np.asarray(edge_type, np.uint8)
    return I.CsrCode(n, m, row_ptr, cols.astype(np.int32), et, n_types)


def _exact_posteriors(H, L, s):
    """ln P(c_v = 0 | L, Hc = s) / P(c_v = 1 | ...) by enumerating all words."""
    m, n = H.shape
    num = np.zeros(n, dtype=object)
    den = np.zeros(n, dtype=object)
    mp.mp.dps = 50
    for w in itertools.product((0, 1), repeat=n):
        c = np.array(w, dtype=np.int64)
        if np.any((H.astype(np.int64) @ c) % 2 != s):
            continue
        # P(c_v) proportional to exp(-c_v L_v)
        lw = mp.e ** (-mp.fsum(mp.mpf(float(L[v])) * int(c[v]) for v in range(n)))
        for v in range(n):
            if c[v]:
                den[v] += lw
            else:
                num[v] += lw
    return np.array([float(mp.log(num[v]) - mp.log(den[v])) for v in range(n)])


# --------------------------------------------------------------------------
# syndrome
# --------------------------------------------------------------------------

def test_syndrome_matches_dense_product_and_is_linear():
    code = I.regular_code(96, 3, 6, seed=4)
    H = code.dense().astype(np.int64)
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2, (5, 96)).astype(np.uint8)
    b = rng.integers(0, 2, (5, 96)).astype(np.uint8)
    sa, ua = oracle.syndrome(code, a)
    sb, _ = oracle.syndrome(code, b)
    sab, _ = oracle.syndrome(code, a ^ b)
    np.testing.assert_array_equal(sa, (a.astype(np.int64) @ H.T) % 2)
    np.testing.assert_array_equal(sab, sa ^ sb)
    np.testing.assert_array_equal(ua, sa.sum(1))
    _, u_self = oracle.syndrome(code, a, sa)
    assert (u_self == 0).all()


# --------------------------------------------------------------------------
# sum-product
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 3, 5, 9, 12])
@pytest.mark.parametrize("s", [0, 1])
def test_single_parity_check_is_exact_map(d, s):
    rng = np.random.default_rng(100 + d + 7 * s)
    H = np.ones((1, d), np.uint8)
    code = _csr_from_dense(H)
    L = rng.normal(0.5, 2.0, d)
    r = oracle.decode(code, L[None, :], np.array([[s]], np.uint8), algo=oracle.SP,
                      max_iter=1, early_stop=False)
    ref = _exact_posteriors(H, L, np.array([s]))
    np.testing.assert_allclose(r["post"][0], ref, rtol=1e-12, atol=1e-12)


def test_phi_form_matches_tanh_rule_in_50_digits():
    rng = np.random.default_rng(3)
    mp.mp.dps = 50
    for trial in range(40):
        d = int(rng.integers(3, 10))
        H = np.ones((1, d), np.uint8)
        code = _csr_from_dense(H)
        L = rng.normal(0, 4, d) * (10 ** rng.uniform(-2, 1, d))
        L = np.clip(L, -45, 45)
        s = int(rng.integers(0, 2))
        r = oracle.decode(code, L[None, :], np.array([[s]], np.uint8), algo=oracle.SP,
                          max_iter=1, early_stop=False)
        c2v = r["post"][0] - L
        for v in range(d):
            prod = mp.mpf(1)
            for k in range(d):
                if k != v:
                    prod *= mp.tanh(mp.mpf(float(L[k])) / 2)
            ref = (1 - 2 * s) * 2 * mp.atanh(prod)
            scale = abs(float(L[v])) + abs(float(ref)) + 1e-300
            assert abs(c2v[v] - float(ref)) <= 1e-12 * max(1.0, scale), (trial, v)


def _random_tree(n_var, rng):
    """Random cycle-free Tanner graph: checks of degree >= 2 joined into a tree."""
    while True:
        H = []
        vars_in = [0]
        nxt = 1
        while nxt < n_var:
            anchor = int(rng.choice(vars_in))
            k = int(min(rng.integers(1, 4), n_var - nxt))
            row = np.zeros(n_var, np.uint8)
            row[anchor] = 1
            row[nxt:nxt + k] = 1
            vars_in.extend(range(nxt, nxt + k))
            nxt += k
            H.append(row)
        H = np.array(H)
        if len(H):
            return H


@pytest.mark.parametrize("seed", range(6))
def test_sum_product_on_trees_gives_exact_marginals(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 14))
    H = _random_tree(n, rng)
    code = _csr_from_dense(H)
    L = rng.normal(0.8, 1.5, n)
    s = rng.integers(0, 2, H.shape[0]).astype(np.uint8)
    r = oracle.decode(code, L[None, :], s[None, :], algo=oracle.SP, max_iter=2 * n, early_stop=False)
    ref = _exact_posteriors(H, L, s.astype(np.int64))
    np.testing.assert_allclose(r["post"][0], ref, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("zero", [0.0, -0.0])
@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_a_zero_input_silences_the_other_edges_of_its_check(zero, algo):
    """tanh(0) = 0 (and min |x| = 0): a check holding an input of magnitude zero,
    of either sign bit, sends exactly zero to its other edges, and to that edge
    the rule over the remaining inputs (tanh product, or scaled minimum)."""
    H = np.ones((1, 4), np.uint8)
    code = _csr_from_dense(H)
    L = np.array([zero, 1.7, -0.6, 3.2])
    for s in (0, 1):
        r = oracle.decode(code, L[None, :], np.array([[s]], np.uint8), algo=algo, max_iter=1,
                          early_stop=False, alpha=0.75)
        c2v = r["post"][0] - L
        assert np.all(np.isfinite(c2v))
        np.testing.assert_array_equal(c2v[1:], 0.0)
        sg = (1 - 2 * s) * -1.0
        if algo == oracle.SP:
            ref = sg * 2 * math.atanh(math.tanh(1.7 / 2) * math.tanh(0.6 / 2) * math.tanh(3.2 / 2))
            assert abs(c2v[0] - ref) <= 1e-13
        else:
            assert c2v[0] == sg * 0.75 * 0.6


def test_degree_two_check_passes_message_through():
    H = np.ones((1, 2), np.uint8)
    code = _csr_from_dense(H)
    for a, b, s in [(1.3, -0.4, 0), (7.0, 2.5, 1), (-0.01, 3.0, 1), (20.0, -30.0, 0)]:
        r = oracle.decode(code, np.array([[a, b]]), np.array([[s]], np.uint8), algo=oracle.SP,
                          max_iter=1, early_stop=False)
        c2v = r["post"][0] - np.array([a, b])
        sg = 1 - 2 * s
        np.testing.assert_allclose(c2v, [sg * b, sg * a], rtol=1e-13, atol=1e-13)


def test_clamp_limits_incoming_messages():
    H = np.ones((1, 3), np.uint8)
    code = _csr_from_dense(H)
    r = oracle.decode(code, np.array([[80.0, 90.0, 1.0]]), None, algo=oracle.SP, max_iter=1,
                      early_stop=False, clamp=50.0)
    c2v = r["post"][0] - np.array([80.0, 90.0, 1.0])
    mp.mp.dps = 50
    # the third variable sees two inputs clamped to 50
    ref = 2 * mp.atanh(mp.tanh(25) * mp.tanh(25))
    assert abs(c2v[2] - float(ref)) < 1e-12


# --------------------------------------------------------------------------
# normalized min-sum
# --------------------------------------------------------------------------

def test_min_sum_hand_computed_row():
    H = np.ones((1, 4), np.uint8)
    code = _csr_from_dense(H)
    L = np.array([2.0, -0.5, 3.0, -1.5])
    r = oracle.decode(code, L[None, :], np.array([[1]], np.uint8), algo=oracle.NMS,
                      max_iter=1, early_stop=False, alpha=0.5)
    c2v = r["post"][0] - L
    # signs: total product of input signs = (+)(-)(+)(-) = +, syndrome 1 flips it
    # v0: others (-0.5, 3, -1.5): sign +, min 0.5 -> -1 * 0.5 * 0.5 = -0.25
    # v1: others (2, 3, -1.5): sign -, min 1.5 -> -1 * -1 * 0.75 = +0.75
    # v2: others (2, -0.5, -1.5): sign +, min 0.5 -> -0.25
    # v3: others (2, -0.5, 3): sign -, min 0.5 -> +0.25
    np.testing.assert_array_equal(c2v, [-0.25, 0.75, -0.25, 0.25])


def test_min_sum_unit_scale_on_degree_two_equals_sum_product():
    H = np.zeros((8, 8), np.uint8)
    for c in range(8):                      # a cycle of degree-2 checks
        H[c, c] = H[c, (c + 1) % 8] = 1
    code = _csr_from_dense(H)
    rng = np.random.default_rng(5)
    L = rng.normal(0.5, 1.0, (3, 8))
    s = rng.integers(0, 2, (3, 8)).astype(np.uint8)
    a = oracle.decode(code, L, s, algo=oracle.SP, max_iter=6, early_stop=False)
    b = oracle.decode(code, L, s, algo=oracle.NMS, alpha=1.0, max_iter=6, early_stop=False)
    np.testing.assert_allclose(a["post"], b["post"], rtol=1e-12, atol=1e-12)


def test_uniform_weights_equal_plain_nms():
    code = I.lambda_half_rate_spec(1024).to_csr()
    rng = np.random.default_rng(2)
    bits = rng.integers(0, 2, (3, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(bits, 0.6, 9)
    s, _ = oracle.syndrome(code, bits)
    a = oracle.decode(code, llr, s, algo=oracle.NMS, alpha=0.8, max_iter=12)
    w = np.full((12, code.n_types), 0.8)
    b = oracle.decode(code, llr, s, algo=oracle.NMS, weights=w, max_iter=12)
    for k in ("bits", "post", "iters", "ok"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_coset_symmetry_is_bit_exact(algo):
    code = I.regular_code(256, 3, 6, seed=11)
    rng = np.random.default_rng(8)
    F = 6
    bits = rng.integers(0, 2, (F, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(np.zeros_like(bits), 0.7, 12)       # all-zero word
    s0 = np.zeros((F, code.m), np.uint8)
    a = oracle.decode(code, llr, s0, algo=algo, max_iter=30)
    sc, _ = oracle.syndrome(code, bits)
    b = oracle.decode(code, llr * (1 - 2 * bits.astype(np.float64)), sc, algo=algo, max_iter=30)
    np.testing.assert_array_equal(b["bits"], a["bits"] ^ bits)
    np.testing.assert_array_equal(b["iters"], a["iters"])
    np.testing.assert_array_equal(b["ok"], a["ok"])
    np.testing.assert_array_equal(np.abs(b["post"]), np.abs(a["post"]))


# --------------------------------------------------------------------------
# binary16 storage emulation
# --------------------------------------------------------------------------

def test_half_rounding_matches_numpy_float16():
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.normal(0, 1, 3000) * 10.0 ** rng.uniform(-9, 5, 3000),
        [0.0, -0.0, 65504.0, 65519.0, 65520.0, 1e6, -1e6, 6e-8, 2.9802322387695312e-08, 1.0 + 2 ** -11],
        (np.arange(2048) + 0.5) * 2.0 ** -24,      # ties on the subnormal grid
        1 + (np.arange(1024) + 0.5) * 2.0 ** -10,   # ties in [1, 2)
    ])
    for x in xs.tolist():
        ref = float(np.float16(np.clip(x, -65504.0, 65504.0)))
        got = oracle.round_half(x)
        assert got == ref or (got == 0 and ref == 0), (x, got, ref)


def test_half_storage_changes_only_by_rounding():
    code = I.regular_code(128, 3, 6, seed=2)
    llr = I.bpsk_llr(np.zeros((2, 128), np.uint8), 0.8, 1)
    a = oracle.decode(code, llr, None, algo=oracle.NMS, max_iter=1, early_stop=False)
    b = oracle.decode(code, llr, None, algo=oracle.NMS, max_iter=1, early_stop=False, store_half=True)
    # one iteration: each posterior differs by at most the rounding of its 3 messages
    assert np.max(np.abs(a["post"] - b["post"])) < 3 * 2 ** -11 * np.max(np.abs(llr))


# --------------------------------------------------------------------------
# early stop bookkeeping
# --------------------------------------------------------------------------

def test_early_stop_and_iteration_count_consistent_with_trace():
    code = I.regular_code(1024, 3, 6, seed=1)
    llr = I.bpsk_llr(np.zeros((20, 1024), np.uint8), 0.56234, 7)
    r = oracle.decode(code, llr, None, algo=oracle.SP, max_iter=50, trace=True)
    for f in range(20):
        t = r["iters"][f]
        ut = r["unsat_trace"][f]
        assert (ut[:t] > 0).all()
        assert (ut[t] == 0) == bool(r["ok"][f])
        np.testing.assert_array_equal(r["post_trace"][f, t], r["post"][f])
        _, u = oracle.syndrome(code, r["bits"][f:f + 1])
        assert (u[0] == 0) == bool(r["ok"][f])
    # the channel word of a clean frame is decoded at t = 0
    r0 = oracle.decode(code, np.full((1, 1024), 5.0), None, algo=oracle.SP, max_iter=50)
    assert r0["iters"][0] == 0 and r0["ok"][0] == 1


# --------------------------------------------------------------------------
# unrolled min-sum derivative
# --------------------------------------------------------------------------

def test_unrolled_nms_forward_matches_decoder():
    code = I.irregular_code(256, 128, I.LAMBDA_NODE_FRACTIONS, seed=3)
    rng = np.random.default_rng(4)
    bits = rng.integers(0, 2, (3, 256)).astype(np.uint8)
    llr = I.bpsk_llr(bits, 0.6, 5)
    s, _ = oracle.syndrome(code, bits)
    w = rng.uniform(0.6, 0.9, (7, code.n_types))
    u = oracle.nms_unrolled(code, llr, s, bits, w)
    d = oracle.decode(code, llr, s, algo=oracle.NMS, weights=w, max_iter=7, early_stop=False)
    np.testing.assert_array_equal(u["post"], d["post"])
    z = -(1 - 2 * bits.astype(np.float64)) * d["post"]
    np.testing.assert_allclose(u["loss"], np.logaddexp(0, z).mean(), rtol=1e-13)


def test_unrolled_nms_gradient_matches_central_differences():
    code = I.irregular_code(256, 128, I.LAMBDA_NODE_FRACTIONS, seed=3)
    rng = np.random.default_rng(6)
    F, T = 4, 20
    bits = rng.integers(0, 2, (F, 256)).astype(np.uint8)
    s2 = I.sigma2_from_ebn0(rng.uniform(1.5, 3.0, F), 0.5)
    llr = I.bpsk_llr(bits, s2, 7)
    s, _ = oracle.syndrome(code, bits)
    w = rng.uniform(0.65, 0.85, (T, code.n_types))
    g = oracle.nms_unrolled(code, llr, s, bits, w, want_dllr=True)
    h = 1e-6
    checked = 0
    for t in range(T):
        for ty in range(code.n_types):
            wp = w.copy(); wp[t, ty] += h
            wm = w.copy(); wm[t, ty] -= h
            gp = oracle.nms_unrolled(code, llr, s, bits, wp)
            gm = oracle.nms_unrolled(code, llr, s, bits, wm)
            # a min/sign switch inside [w-h, w+h] shows up as a jump of the gradient
            if not (np.allclose(gp["dw"], g["dw"], rtol=1e-4, atol=1e-12)
                    and np.allclose(gm["dw"], g["dw"], rtol=1e-4, atol=1e-12)):
                continue
            fd = (gp["loss"] - gm["loss"]) / (2 * h)
            assert abs(fd - g["dw"][t, ty]) <= 1e-6 * max(abs(fd), 1e-8), (t, ty, fd, g["dw"][t, ty])
            checked += 1
    assert checked >= 0.8 * T * code.n_types
    # and with respect to one channel LLR
    v = 17
    lp = llr.copy(); lp[1, v] += h
    lm = llr.copy(); lm[1, v] -= h
    fd = (oracle.nms_unrolled(code, lp, s, bits, w)["loss"] - oracle.nms_unrolled(code, lm, s, bits, w)["loss"]) / (2 * h)
    assert abs(fd - g["dllr"][1, v]) <= 1e-6 * max(abs(fd), 1e-8)


# --------------------------------------------------------------------------
# binary32 mode of the oracle
# --------------------------------------------------------------------------

@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_prec32_values_are_floats_and_close_to_fp64(algo):
    code = I.lambda_half_rate_spec(2048).to_csr()
    rng = np.random.default_rng(21)
    bits = rng.integers(0, 2, (3, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(bits, 0.6, 22)
    s, _ = oracle.syndrome(code, bits)
    a = oracle.decode(code, llr, s, algo=algo, alpha=0.8, max_iter=1, early_stop=False, trace=True)
    b = oracle.decode(code, llr, s, algo=algo, alpha=0.8, max_iter=1, early_stop=False, trace=True, prec32=True)
    # every posterior of the binary32 run is a float
    np.testing.assert_array_equal(b["post"], b["post"].astype(np.float32).astype(np.float64))
    # one iteration: the two agree to a few binary32 roundings of the sum
    err = np.abs(a["post"] - b["post"]) / a["scale_trace"][:, 1]
    assert err.max() < 16 * 2.0 ** -24


@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_prec32_follows_fp64_over_twelve_iterations(algo):
    """From the second iteration on, the binary32 mode forms each variable's
    extrinsic message from its running posterior; the fp64 mode sums the other
    edges directly.  On frames that decode, the two stay within a few hundred
    binary32 roundings of the per-variable scale for 12 iterations (measured
    3e-6), where a stale or missing term in either formulation moves a
    posterior by a sizeable fraction of its scale; the hard decisions, the
    stop iteration and the success flag agree exactly."""
    code = I.lambda_half_rate_spec(2048).to_csr()
    rng = np.random.default_rng(21)
    bits = rng.integers(0, 2, (3, code.n)).astype(np.uint8)
    llr = I.bpsk_llr(bits, 0.6, 22)
    s, _ = oracle.syndrome(code, bits)
    kw = dict(algo=algo, alpha=0.8, max_iter=12, early_stop=False, trace=True)
    a = oracle.decode(code, llr, s, **kw)
    b = oracle.decode(code, llr, s, prec32=True, **kw)
    for t in range(1, 13):
        err = np.abs(a["post_trace"][:, t] - b["post_trace"][:, t]) / a["scale_trace"][:, t]
        assert err.max() < 1e-5, (t, err.max())
    np.testing.assert_array_equal(a["bits"], b["bits"])
    kw["early_stop"] = True
    a = oracle.decode(code, llr, s, **kw)
    b = oracle.decode(code, llr, s, prec32=True, **kw)
    np.testing.assert_array_equal(a["iters"], b["iters"])
    np.testing.assert_array_equal(a["ok"], b["ok"])
    assert a["ok"].all() and (a["iters"] > 1).all()


def test_prec32_min_sum_hand_computed_row():
    H = np.ones((1, 3), np.uint8)
    code = _csr_from_dense(H)
    L = np.array([0.1, -0.3, 2.0])
    r = oracle.decode(code, L[None, :], None, algo=oracle.NMS, max_iter=1, early_stop=False,
                      alpha=0.8, prec32=True)
    f = np.float32
    w = f(0.8)
    Lf = L.astype(np.float32)
    # v0: others (-0.3, 2.0): sign -, min 0.3;  v1: others (0.1, 2.0): +, 0.1;  v2: (0.1, -0.3): -, 0.1
    c2v = np.array([-(w * f(0.3)), w * f(0.1), -(w * f(0.1))], dtype=np.float32)
    expect = (Lf + c2v).astype(np.float64)
    np.testing.assert_array_equal(r["post"][0], expect)


def test_prec32_half_store_is_rounding_of_the_float_message():
    H = np.ones((1, 2), np.uint8)
    code = _csr_from_dense(H)
    L = np.array([[1.0, 1.0 + 3 * 2.0 ** -12]])     # 0.75 * that lies between halves
    r = oracle.decode(code, L, None, algo=oracle.NMS, alpha=0.75, max_iter=1, early_stop=False,
                      prec32=True, store_half=True)
    msg = np.float32(0.75) * np.float32(L[0, 1])
    assert r["post"][0, 0] == np.float32(np.float32(1.0) + np.float32(np.float16(msg)))


def test_unrolled_prec32_forward_matches_binary32_decoder_and_gradient_is_close():
    code = I.irregular_code(256, 128, I.LAMBDA_NODE_FRACTIONS, seed=3)
    rng = np.random.default_rng(31)
    F, T = 3, 10
    bits = rng.integers(0, 2, (F, 256)).astype(np.uint8)
    llr = I.bpsk_llr(bits, 0.6, 32)
    s, _ = oracle.syndrome(code, bits)
    w = rng.uniform(0.6, 0.9, (T, code.n_types))
    u32 = oracle.nms_unrolled(code, llr, s, bits, w, prec32=True)
    d32 = oracle.decode(code, llr, s, algo=oracle.NMS, weights=w, max_iter=T, early_stop=False, prec32=True)
    np.testing.assert_array_equal(u32["post"], d32["post"])
    u64 = oracle.nms_unrolled(code, llr, s, bits, w)
    np.testing.assert_allclose(u32["dw"], u64["dw"], rtol=1e-4, atol=1e-9)


def test_scale_trace_is_channel_plus_message_magnitudes_on_a_hand_built_graph():
    """H = [[1 1 1 0], [0 1 0 1]], L = (1, -2, 3, 0.5), min-sum with alpha = 1,
    s = 0.  Iteration 1 (v2c = L_ch): row 0 sends (-2, +1, -1) to v0, v1, v2
    (sign product of the others times their smallest magnitude), row 1 sends
    (+0.5, -2) to v1, v3.  Scale |L_ch| + sum |c2v| = (3, 3.5, 4, 2.5) and
    L_post = (-1, -0.5, 2, -1.5).  Iteration 2: v2c of v1 to row 0 is
    -2 + 0.5 = -1.5 and to row 1 is -2 + 1 = -1; v0, v2, v3 send L_ch.  Row 0
    sends (-1.5, +1, -1), row 1 sends (+0.5, -1): L_post = (-0.5, -0.5, 2, -0.5)
    and scale (2.5, 3.5, 4, 1.5)."""
    H = np.array([[1, 1, 1, 0], [0, 1, 0, 1]], np.uint8)
    code = _csr_from_dense(H)
    L = np.array([[1.0, -2.0, 3.0, 0.5]])
    r = oracle.decode(code, L, None, algo=oracle.NMS, alpha=1.0, max_iter=2, early_stop=False, trace=True)
    np.testing.assert_array_equal(r["scale_trace"][0, 0], [1.0, 2.0, 3.0, 0.5])
    np.testing.assert_array_equal(r["post_trace"][0, 1], [-1.0, -0.5, 2.0, -1.5])
    np.testing.assert_array_equal(r["scale_trace"][0, 1], [3.0, 3.5, 4.0, 2.5])
    np.testing.assert_array_equal(r["post_trace"][0, 2], [-0.5, -0.5, 2.0, -0.5])
    np.testing.assert_array_equal(r["scale_trace"][0, 2], [2.5, 3.5, 4.0, 1.5])
