"""Pins of the oracle's quantiser/slicer and slice LLRs (Sec. III-B steps 1-4)
against brute force, high-precision integration, closed forms, symmetry and the
information identity -- nothing here re-uses the oracle's own formula."""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import ndtr

import oracle
from paper_2108_08418_amd import inputs as I

SNR = 3.0
SIG = math.sqrt(1.0 / SNR)
TH4 = I.equiprobable_thresholds(4, 1.0 + 1.0 / SNR)


def _gray(k):
    return k ^ (k >> 1)


def test_quantize_brute_force_including_exact_thresholds():
    rng = np.random.default_rng(1)
    y = np.concatenate([rng.normal(0, 1.3, 500), TH4, [-1e300, 1e300, 0.0, -0.0]])
    S = oracle.quantize(y, TH4, 4)
    for idx, yy in enumerate(y.tolist()):
        k = 0
        while k < len(TH4) and TH4[k] <= yy:      # first threshold above y
            k += 1
        g = _gray(k)
        for j in range(4):
            assert S[j, idx] == (g >> j) & 1
    # a value exactly on threshold i goes to interval i (the upper one)
    S_on = oracle.quantize(TH4, TH4, 4)
    for i in range(len(TH4)):
        g = _gray(i + 1)
        assert all(S_on[j, i] == (g >> j) & 1 for j in range(4))


def test_binary_labelling_is_plain_index():
    y = np.array([-5.0, 0.05, 5.0])
    S = oracle.quantize(y, TH4, 4, oracle.BINARY)
    ks = [0, 8, 15]
    for c, k in enumerate(ks):
        assert [S[j, c] for j in range(4)] == [(k >> j) & 1 for j in range(4)]


def test_gray_adjacent_intervals_differ_in_one_bit():
    mids = np.concatenate([[TH4[0] - 1], (TH4[:-1] + TH4[1:]) / 2, [TH4[-1] + 1]])
    S = oracle.quantize(mids, TH4, 4)
    for a in range(15):
        assert int((S[:, a] != S[:, a + 1]).sum()) == 1


def test_equiprobable_labels_chi_square():
    _, y = I.gaussian_pairs(1 << 18, SNR, 5)
    S = oracle.quantize(y, TH4, 4)
    lab = sum(S[j].astype(np.int64) << j for j in range(4))
    counts = np.bincount(lab, minlength=16)
    expect = len(y) / 16
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 50.0          # 15 dof: P(chi2 > 50) ~ 1e-5


def _mp_log_interval(x, lo, hi, sig, use_quad=False):
    """ln Pr(lo <= x + sig Z < hi) at 80 significant digits: the normal CDF
    difference (the definition), or -- for moderate arguments -- tanh-sinh
    quadrature of the density."""
    mp.mp.dps = 80
    a = -mp.inf if lo is None else mp.mpf(lo)
    b = mp.inf if hi is None else mp.mpf(hi)
    if use_quad:
        f = lambda u: mp.npdf(u, x, sig)
        pts = [a, mp.mpf(x), b] if a < x < b else [a, b]
        return mp.log(mp.quad(f, pts))
    return mp.log(mp.ncdf((b - x) / sig) - mp.ncdf((a - x) / sig))


def _mp_slice_llr(x, j, known_bits, sig, th, use_quad=False):
    t = [None] + list(th) + [None]
    num = mp.mpf(0)
    den = mp.mpf(0)
    for k in range(16):
        g = _gray(k)
        if any(((g >> i) & 1) != b for i, b in known_bits.items()):
            continue
        p = mp.e ** _mp_log_interval(x, t[k], t[k + 1], sig, use_quad)
        if (g >> j) & 1:
            den += p
        else:
            num += p
    return float(mp.log(num) - mp.log(den))


@pytest.mark.parametrize("j,mask", [(0, 0b0), (2, 0b11), (3, 0b111), (1, 0b1101)])
def test_slice_llr_matches_high_precision_integration(j, mask):
    rng = np.random.default_rng(10 + j)
    xs = np.concatenate([np.linspace(-8, 8, 9), rng.normal(0, 1.5, 4)])
    slices = rng.integers(0, 2, size=(4, len(xs))).astype(np.uint8)
    L = oracle.slice_llr(xs, SIG, TH4, 4, oracle.GRAY, j, mask, slices)
    for i, x in enumerate(xs.tolist()):
        known = {b: int(slices[b, i]) for b in range(4) if mask >> b & 1}
        ref = _mp_slice_llr(x, j, known, SIG, TH4)
        assert abs(L[i] - ref) <= 1e-12 * max(1.0, abs(ref)), (x, L[i], ref)
        if abs(x) <= 3:
            refq = _mp_slice_llr(x, j, known, SIG, TH4, use_quad=True)
            assert abs(L[i] - refq) <= 1e-12 * max(1.0, abs(refq)), (x, L[i], refq)


def test_one_bit_quantiser_closed_form():
    xs = np.linspace(-9, 9, 37)
    L = oracle.slice_llr(xs, 0.7, np.array([0.0]), 1, oracle.GRAY, 0, 0, np.zeros((1, len(xs)), np.uint8))
    mp.mp.dps = 40
    for x, l in zip(xs.tolist(), L.tolist()):
        ref = mp.log(mp.ncdf(-x / 0.7)) - mp.log(mp.ncdf(x / 0.7))
        assert abs(l - float(ref)) <= 1e-12 * max(1.0, abs(float(ref)))


def test_mirror_symmetry():
    xs = np.linspace(0.1, 6, 25)
    z = np.zeros((4, len(xs)), np.uint8)
    for j in range(4):
        Lp = oracle.slice_llr(xs, SIG, TH4, 4, oracle.GRAY, j, 0, z)
        Lm = oracle.slice_llr(-xs, SIG, TH4, 4, oracle.GRAY, j, 0, z)
        if j == 3:   # the MSB flips with the sign of y: odd in x
            np.testing.assert_allclose(Lp, -Lm, rtol=1e-12, atol=1e-12)
        else:        # reflected Gray bits below the MSB are even in x
            np.testing.assert_allclose(Lp, Lm, rtol=1e-12, atol=1e-12)


def _conditional_entropy_quadrature(j, snr=SNR, m=4, npts=300):
    """H(S_j | X, S_<j) by Gauss-Hermite quadrature over X ~ N(0, 1), with the
    interval probabilities from the linear-domain normal CDF."""
    sig = math.sqrt(1.0 / snr)
    th = I.equiprobable_thresholds(m, 1.0 + 1.0 / snr)
    u, w = np.polynomial.hermite_e.hermegauss(npts)
    w = w / w.sum()
    t = np.concatenate([[-np.inf], th, [np.inf]])
    P = ndtr((t[1:, None] - u[None, :]) / sig) - ndtr((t[:-1, None] - u[None, :]) / sig)  # [K, pts]
    labels = np.array([_gray(k) for k in range(2 ** m)])
    H = np.zeros(len(u))
    for prefix in range(2 ** j):
        sel = (labels & ((1 << j) - 1)) == prefix
        p0 = P[sel & (((labels >> j) & 1) == 0)].sum(0)
        p1 = P[sel & (((labels >> j) & 1) == 1)].sum(0)
        tot = p0 + p1
        with np.errstate(divide="ignore", invalid="ignore"):
            h = -(np.where(p0 > 0, p0 * np.log2(p0 / tot), 0) + np.where(p1 > 0, p1 * np.log2(p1 / tot), 0))
        H += h
    return float((w * H).sum())


def test_slice_capacities_match_quadrature_constants():
    # four-digit slice capacities at SNR 3, 16 equiprobable Gray intervals, computed beforehand
    # by an independent numerical integration
    caps = [1 - _conditional_entropy_quadrature(j) for j in range(4)]
    np.testing.assert_allclose(caps, [0.0228, 0.0747, 0.3153, 0.5469], atol=6e-4)


@pytest.mark.parametrize("j,mask", [(2, 0b11), (3, 0b111)])
def test_information_identity(j, mask):
    """1 - E[log2(1 + exp(-(1-2b) L))] estimates 1 - H(S_j | X, S_<j)."""
    x, y = I.gaussian_pairs(1 << 17, SNR, 77 + j)
    S = oracle.quantize(y, TH4, 4)
    L = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, j, mask, S)
    b = S[j].astype(np.float64)
    terms = np.logaddexp(0.0, -(1 - 2 * b) * L) / math.log(2.0)
    est = 1 - terms.mean()
    se = terms.std() / math.sqrt(len(terms))
    cap = 1 - _conditional_entropy_quadrature(j)
    assert abs(est - cap) < 5 * se + 1e-4


def test_log_domain_llr_is_finite_where_linear_domain_underflows():
    x, y = I.gaussian_pairs(1 << 18, SNR, 12345)
    S = oracle.quantize(y, TH4, 4)
    L3 = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, 3, 0b111, S)
    assert np.isfinite(L3).all()
    # far below zero the MSB (bit 3: y >= 0) has P(bit = 1 | x) = 1 - Phi(13)
    # ~ 6e-39, which the linear-domain difference rounds to exactly 0
    far = np.array([-7.5])
    p1_naive = ndtr(np.inf) - ndtr((0.0 - far[0]) / SIG)
    assert p1_naive == 0.0
    Lfar = oracle.slice_llr(far, SIG, TH4, 4, oracle.GRAY, 3, 0, np.zeros((4, 1), np.uint8))
    mp.mp.dps = 60
    ref = float(mp.log(mp.ncdf(-far[0] / SIG) - 0) - mp.log(1 - mp.ncdf(-far[0] / SIG)))
    assert np.isfinite(Lfar).all() and abs(Lfar[0] - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("j,code_rate", [(2, 0.1875), (3, 0.4921875)])
def test_slice_code_rates_respect_slepian_wolf(j, code_rate):
    """Syndrome bits per slice bit, 1 - R_j, must exceed H(S_j | X, S_<j)
    (Slepian-Wolf bound, Sec. III-B)."""
    q = I.slice_code_spec(j, 65536)
    assert abs((q.nb - q.mb) / q.nb - code_rate) < 1e-12
    assert 1 - code_rate >= _conditional_entropy_quadrature(j)


# ---------------------------------------------------------------------------
# soft priors from lower slices, and the binary-symmetric-channel hard LLR
# ---------------------------------------------------------------------------
def _mp_slice_llr_prior(x, j, known_bits, priors, sig, th):
    """80-digit enumeration of the 16 intervals: P_k(x) from the normal CDF,
    times Pr(S_i = b) = 1 / (1 + exp(-(1 - 2b) lambda_i)) for each prior slice."""
    mp.mp.dps = 80
    t = [None] + list(th) + [None]
    num = mp.mpf(0)
    den = mp.mpf(0)
    for k in range(16):
        g = _gray(k)
        if any(((g >> i) & 1) != b for i, b in known_bits.items()):
            continue
        p = mp.e ** _mp_log_interval(x, t[k], t[k + 1], sig)
        for i, lam in priors.items():
            s = 1 - 2 * ((g >> i) & 1)
            p *= 1 / (1 + mp.e ** (-s * mp.mpf(lam)))
        if (g >> j) & 1:
            den += p
        else:
            num += p
    return float(mp.log(num) - mp.log(den))


@pytest.mark.parametrize("j,known,prior", [(3, 0b11, 0b100), (2, 0b1, 0b10), (1, 0, 0b1101), (3, 0, 0b111)])
def test_slice_llr_prior_matches_high_precision_enumeration(j, known, prior):
    rng = np.random.default_rng(40 + j + known)
    xs = np.concatenate([np.linspace(-6, 6, 7), rng.normal(0, 1.5, 4)])
    slices = rng.integers(0, 2, size=(4, len(xs))).astype(np.uint8)
    lam = (rng.normal(0, 6, size=(4, len(xs)))).astype(np.float32)
    L = oracle.slice_llr_prior(xs, SIG, TH4, 4, oracle.GRAY, j, known, slices, prior, lam)
    for i, x in enumerate(xs.tolist()):
        kb = {b: int(slices[b, i]) for b in range(4) if known >> b & 1}
        pr = {b: float(lam[b, i]) for b in range(4) if prior >> b & 1}
        ref = _mp_slice_llr_prior(x, j, kb, pr, SIG, TH4)
        assert abs(L[i] - ref) <= 1e-12 * max(1.0, abs(ref)), (x, L[i], ref)


def test_hard_priors_equal_known_slices():
    """A prior of +inf (bit 0 certain) or -inf (bit 1 certain) is the same as
    holding that slice as a hard known bit."""
    rng = np.random.default_rng(7)
    xs = rng.normal(0, 1.2, 3000)
    slices = rng.integers(0, 2, size=(4, xs.size)).astype(np.uint8)
    lam = np.where(slices == 0, np.inf, -np.inf).astype(np.float32)
    for j, hard in [(2, 0b11), (3, 0b111), (1, 0b1)]:
        soft = 1 << (int(hard).bit_length() - 1)         # the highest known slice becomes a prior
        Lp = oracle.slice_llr_prior(xs, SIG, TH4, 4, oracle.GRAY, j, hard & ~soft, slices, soft, lam)
        Lk = oracle.slice_llr(xs, SIG, TH4, 4, oracle.GRAY, j, hard, slices)
        np.testing.assert_allclose(Lp, Lk, rtol=1e-14, atol=0)


def test_zero_priors_equal_unknown_slices():
    """lambda = 0 is no information: every label gets the same factor 1/2."""
    rng = np.random.default_rng(8)
    xs = rng.normal(0, 1.2, 3000)
    slices = rng.integers(0, 2, size=(4, xs.size)).astype(np.uint8)
    lam = np.zeros((4, xs.size), np.float32)
    Lp = oracle.slice_llr_prior(xs, SIG, TH4, 4, oracle.GRAY, 3, 0b1, slices, 0b110, lam)
    Lu = oracle.slice_llr(xs, SIG, TH4, 4, oracle.GRAY, 3, 0b1, slices)
    np.testing.assert_allclose(Lp, Lu, rtol=1e-12, atol=1e-12)


def test_bsc_llr_closed_forms():
    rng = np.random.default_rng(9)
    xs = rng.normal(0, 1.0, 5000)
    # sign: Alice's own quantised bit j (brute-force label below), magnitude ln((1-p)/p)
    k = np.array([sum(1 for t in TH4 if t <= v) for v in xs])
    for j in range(4):
        bit = (_gray(k) >> j) & 1
        for p in (0.03, 0.2, 0.45):
            L = oracle.slice_llr_bsc(xs, TH4, 4, oracle.GRAY, j, p)
            # d/dp of the binary entropy in nats is ln((1-p)/p): central difference
            h = 1e-6
            Hn = lambda q: -q * math.log(q) - (1 - q) * math.log(1 - q)
            mag = (Hn(p + h) - Hn(p - h)) / (2 * h)
            np.testing.assert_allclose(np.abs(L), mag, rtol=1e-8)
            np.testing.assert_array_equal(L < 0, bit == 1)
        np.testing.assert_array_equal(oracle.slice_llr_bsc(xs, TH4, 4, oracle.GRAY, j, 0.5), 0.0)
        np.testing.assert_allclose(oracle.slice_llr_bsc(xs, TH4, 4, oracle.GRAY, j, 0.9),
                                   -oracle.slice_llr_bsc(xs, TH4, 4, oracle.GRAY, j, 0.1), rtol=1e-15)
