"""TEST INFRASTRUCTURE -- fp64 oracle for Bob's quantiser/slicer and Alice's
slice LLRs (the first steps of slice reconciliation, Sec. III-B steps 1-4).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP library.
"""
from __future__ import annotations

import numpy as np
from scipy.special import log_ndtr, logsumexp

GRAY = 0
BINARY = 1


def label_of_index(k, labelling: int):
    """Interval index k -> m-bit label: binary-reflected Gray code g = k xor (k >> 1)
    (the Gray labelling of Sec. II Step 4) or the plain binary index."""
    k = np.asarray(k, dtype=np.int64)
    return k ^ (k >> 1) if labelling == GRAY else k


def quantize(y, thresholds, m_bits: int, labelling: int = GRAY):
    """Quantiser M(.) and slicing (Sec. III-B steps 1-2).

    k(y) = #{i : t_i <= y} (a value on a threshold goes to the upper interval),
    label = Gray(k), slice j = bit j of the label (j = 0 is the least
    significant bit, the paper's l_0).  Returns uint8 [m_bits, N].
    """
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(thresholds, dtype=np.float64)
    if t.shape != (2 ** m_bits - 1,):
        raise ValueError("need 2^m - 1 thresholds")
    k = np.zeros(y.shape, dtype=np.int64)
    for ti in t:                     # count thresholds at or below y
        k += (ti <= y)
    g = label_of_index(k, labelling)
    return np.stack([((g >> j) & 1).astype(np.uint8) for j in range(m_bits)])


def _log_interval_prob(lo, hi):
    """ln(Phi(hi) - Phi(lo)) for lo < hi (arrays), computed in the log domain.

    Above the mean (lo >= 0): Phi(hi) - Phi(lo) = Q(lo) - Q(hi) with Q(z) = Phi(-z);
    below (hi <= 0): Phi(hi) - Phi(lo); straddling: 1 - Phi(lo) - Q(hi).
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = np.empty(np.broadcast(lo, hi).shape)
    lo, hi = np.broadcast_arrays(lo, hi)
    up = lo >= 0
    dn = hi <= 0
    mid = ~(up | dn)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = log_ndtr(-lo[up])
        b = log_ndtr(-hi[up])
        out[up] = a + np.log1p(-np.exp(b - a))
        a = log_ndtr(hi[dn])
        b = log_ndtr(lo[dn])
        out[dn] = a + np.log1p(-np.exp(b - a))
        out[mid] = np.log1p(-(np.exp(log_ndtr(lo[mid])) + np.exp(log_ndtr(-hi[mid]))))
    return out


def log_interval_probs(x, sigma_n: float, thresholds):
    """ln P_k(x) = ln Pr(t_k <= Y < t_{k+1} | X = x), Y = x + N(0, sigma_n^2),
    for k = 0..2^m - 1 with t_0 = -inf and t_{2^m} = +inf.  Shape [2^m, N]."""
    x = np.asarray(x, dtype=np.float64)
    t = np.concatenate([[-np.inf], np.asarray(thresholds, dtype=np.float64), [np.inf]])
    lo = (t[:-1, None] - x[None, :]) / sigma_n
    hi = (t[1:, None] - x[None, :]) / sigma_n
    return _log_interval_prob(lo, hi)


def slice_llr(x, sigma_n: float, thresholds, m_bits: int, labelling: int, j: int,
              known_mask: int, slices):
    """Alice's LLR of Bob's slice j given her quadrature x and the slices listed
    in ``known_mask`` (Sec. III-B step 4, multistage decoding):

        L_j(x) = ln sum_{k in K_j^0} P_k(x) - ln sum_{k in K_j^1} P_k(x),

    K_j^b = intervals whose label has bit j = b and agrees with every known slice
    bit of this sample.  ``slices`` is uint8 [m_bits, N]; only rows in
    ``known_mask`` are read.  Returns fp64 [N].
    """
    if known_mask >> j & 1:
        raise ValueError("slice j is already known")
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    lp = log_interval_probs(x, sigma_n, thresholds)            # [K, N]
    labels = label_of_index(np.arange(2 ** m_bits), labelling)  # [K]
    consistent = np.ones((2 ** m_bits, N), dtype=bool)
    for i in range(m_bits):
        if known_mask >> i & 1:
            row = np.asarray(slices[i], dtype=np.int64) & 1
            consistent &= ((labels[:, None] >> i) & 1) == row[None, :]
    bitj = ((labels >> j) & 1)[:, None]
    with np.errstate(divide="ignore"):
        l0 = logsumexp(np.where(consistent & (bitj == 0), lp, -np.inf), axis=0)
        l1 = logsumexp(np.where(consistent & (bitj == 1), lp, -np.inf), axis=0)
    return l0 - l1


def slice_llr_prior(x, sigma_n: float, thresholds, m_bits: int, labelling: int, j: int,
                    known_mask: int, slices, prior_mask: int, prior_llr):
    """Alice's LLR of Bob's slice j when lower slices enter as soft priors
    (Sec. III-B step 4 read literally: the soft decoding output of a lower
    slice is a-priori information on the next):

        L_j(x) = ln sum_{k in K_j^0} P_k(x) W_k - ln sum_{k in K_j^1} P_k(x) W_k,
        W_k = prod_{i in prior_mask} Pr(S_i = bit i of label k),
        Pr(S_i = 0) = 1 / (1 + e^-lambda_i),  Pr(S_i = 1) = 1 / (1 + e^lambda_i),

    lambda_i = prior_llr[i] (an LLR ln P(0)/P(1)); K_j^b as in ``slice_llr``
    (labels agreeing with the hard slices in ``known_mask``).  ``prior_llr``
    is [m_bits, N]; only rows in ``prior_mask`` are read.  Returns fp64 [N].
    """
    if (known_mask | prior_mask) >> j & 1:
        raise ValueError("slice j is already known or has a prior")
    if known_mask & prior_mask:
        raise ValueError("a slice cannot be both known and a prior")
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    lp = log_interval_probs(x, sigma_n, thresholds)            # [K, N]
    labels = label_of_index(np.arange(2 ** m_bits), labelling)  # [K]
    consistent = np.ones((2 ** m_bits, N), dtype=bool)
    for i in range(m_bits):
        if known_mask >> i & 1:
            row = np.asarray(slices[i], dtype=np.int64) & 1
            consistent &= ((labels[:, None] >> i) & 1) == row[None, :]
        if prior_mask >> i & 1:
            lam = np.asarray(prior_llr[i], dtype=np.float64)[None, :]
            one = ((labels[:, None] >> i) & 1) == 1
            # ln Pr(S_i = b) = -ln(1 + e^{-lambda}) for b = 0, -ln(1 + e^{lambda}) for b = 1
            lp = lp - np.logaddexp(0.0, np.where(one, lam, -lam))
    bitj = ((labels >> j) & 1)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        l0 = logsumexp(np.where(consistent & (bitj == 0), lp, -np.inf), axis=0)
        l1 = logsumexp(np.where(consistent & (bitj == 1), lp, -np.inf), axis=0)
        return l0 - l1


def slice_llr_bsc(x, thresholds, m_bits: int, labelling: int, j: int, p: float):
    """Alice's hard LLR of Bob's slice j, her own quantised bit seen through a
    binary symmetric channel with crossover p (the bit error ratio p_j of
    Sec. II Step 4):  L_j = (1 - 2 a_j) ln((1 - p) / p),  a_j = bit j of the
    label of x under the same quantiser.  Returns fp64 [N]."""
    if not 0.0 < p < 1.0:
        raise ValueError("p must be in (0, 1)")
    a = quantize(x, thresholds, m_bits, labelling)[j].astype(np.float64)
    return (1.0 - 2.0 * a) * (np.log1p(-p) - np.log(p))
