"""Host-side (fp64) finite-length key-rate model and the sub-block length
optimiser (Sec. IV).

* C_Finite(N_R): the normal approximation of the coding rate at block length
  N_R and error probability eps_EC (Eq. for C_Finite):
      C_Finite = I_AB - (sqrt(N_R A) Q^-1(eps_EC) + (1/2) ln N_R) / N_R,
  with the channel dispersion A = (gamma / 2)(gamma + 2) / (gamma + 1)^2 (log2 e)^2
  (the printed (log eps_EC)^2 factor read as (log2 e)^2, the dispersion of
  the AWGN channel in bits^2).  The (1/2) ln N_R term keeps the paper's sign
  and natural logarithm: its printed derivative (Eq. for dK'/dN_R) follows
  from exactly this form.
* Delta_AEP (Eq. for Delta_AEP), B_1 and B_2 (Eqs. for B_1, B_2) and
  K'_Finite(N_R) = (N C_Finite - B_1) / (B_2 N_R) in bits per second
  (Eq. for the simplified optimisation).
* The optimal N_R: the root of the printed derivative on [1e5, N] (Brent),
  else the better end of the interval.
* K'_exp (Sec. V): the key rate from the code rates actually used and the
  measured reconciliation time, per sub-block length.

S_BE (the Holevo-bound estimate of the appendix) is an input here: its
derivation is not modelled.  Logarithms named log2 are base 2; ln is natural.
"""
from __future__ import annotations

import math

from scipy.optimize import brentq
from scipy.special import ndtri

LOG2E = 1.0 / math.log(2.0)


def q_inv(eps: float) -> float:
    """Inverse of the normal upper tail Q(z) = Pr(Z > z)."""
    return float(-ndtri(eps))


def capacity(gamma: float) -> float:
    """C(gamma) = (1/2) log2(1 + gamma), bits per channel use."""
    return 0.5 * math.log2(1.0 + gamma)


def dispersion(gamma: float) -> float:
    """A = (gamma / 2)(gamma + 2) / (gamma + 1)^2 (log2 e)^2."""
    return gamma / 2.0 * (gamma + 2.0) / (gamma + 1.0) ** 2 * LOG2E ** 2


def c_finite(N_R: float, I_AB: float, A: float, eps_ec: float) -> float:
    """I_AB - (sqrt(N_R A) Q^-1(eps_EC) + (1/2) ln N_R) / N_R."""
    return I_AB - (math.sqrt(N_R * A) * q_inv(eps_ec) + 0.5 * math.log(N_R)) / N_R


def delta_aep(m: int, N: float, eps_s: float, eps: float) -> float:
    """(m+1)^2 + 4(m+1) sqrt(log2(2 / eps_s^2)) + 2 log2(2 / (eps^2 eps_s))
    + 4 eps_s m / (eps sqrt(N)), eps the total failure probability."""
    return ((m + 1) ** 2 + 4.0 * (m + 1) * math.sqrt(math.log2(2.0 / eps_s ** 2))
            + 2.0 * math.log2(2.0 / (eps ** 2 * eps_s)) + 4.0 * eps_s * m / (eps * math.sqrt(N)))


def b1(N: float, S_BE: float, d_aep: float, eps_pa: float) -> float:
    """B_1 = N S_BE + sqrt(N) Delta_AEP + 2 log2(1 / (2 eps_PA))."""
    return N * S_BE + math.sqrt(N) * d_aep + 2.0 * math.log2(1.0 / (2.0 * eps_pa))


def b2(c_h: float, D: list[int], lam: list[dict]) -> float:
    """B_2 = c_h sum_j 7 D_j G_j / N_R: seconds per unit N_R of the whole
    decode.  G_j / N_R = 1 / sum_a(lambda_a / a), the edge count per bit
    (the printed m sum_b b rho_b equals it only for check-regular codes)."""
    return c_h * sum(7.0 * d / sum(f / a for a, f in l.items()) for d, l in zip(D, lam))


def efficiency(entropy_my: float, m: int, rates, I_AB: float) -> float:
    """The reconciliation efficiency beta of sliced reconciliation (Sec. III-B):
    (H(M(Y)) - m + sum_j R_j) / I_AB, with H(M(Y)) the entropy of Bob's m-bit
    labels per quadrature and R_j the rate of slice j's code (0 for a
    disclosed slice, 1 for one not sent)."""
    if len(rates) != m:
        raise ValueError("one rate per slice")
    return (entropy_my - m + float(sum(rates))) / I_AB


def quantiser_information(thresholds, snr: float) -> tuple[float, float]:
    """(H(M(Y)), I(M(Y); X)) in bits per quadrature for X ~ N(0, 1),
    Y = X + N(0, 1/snr) and the quantiser M with the given ascending
    thresholds: H from the interval probabilities of Y ~ N(0, 1 + 1/snr);
    I = H - H(M(Y) | X), the conditional entropy integrated over x by
    adaptive quadrature.  With rates R_j equal to the slice capacities,
    beta = I(M(Y); X) / I_AB (the slices' chain rule)."""
    import numpy as np
    from scipy.integrate import quad
    from scipy.special import ndtr
    t = np.concatenate([[-np.inf], np.asarray(thresholds, dtype=np.float64), [np.inf]])

    def ent(p):
        p = p[p > 0.0]
        return float(-(p * np.log2(p)).sum())

    H = ent(np.diff(ndtr(t / math.sqrt(1.0 + 1.0 / snr))))
    sn = math.sqrt(1.0 / snr)
    dens = lambda x: math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    Hc = quad(lambda x: ent(np.diff(ndtr((t - x) / sn))) * dens(x), -12.0, 12.0,
              points=[float(v) for v in t[1:-1]], limit=400, epsabs=1e-12, epsrel=1e-10)[0]
    return H, H - Hc


def k_exp(N: float, rate_sum: float, S_BE: float, d_aep: float, eps_pa: float, dt_exp: float) -> float:
    """K'_exp (Sec. V, the experimental key rate) in bits per second: the
    block's N quadratures reconciled with codes of summed rate sum_j R_j
    (0 for a disclosed slice) in the measured time dt_exp seconds,
        (N (sum_j R_j - S_BE) - sqrt(N) Delta_AEP - 2 log2(1 / (2 eps_PA))) / dt_exp,
    i.e. (N sum_j R_j - B_1) / dt_exp."""
    if dt_exp <= 0.0:
        raise ValueError("dt_exp must be positive")
    return (N * rate_sum - b1(N, S_BE, d_aep, eps_pa)) / dt_exp


def k_exp_curve(points: list[tuple[float, float, float]], N: float, S_BE: float, d_aep: float,
                eps_pa: float) -> tuple[list[float], float]:
    """K'_exp at each measured sub-block length: points are (N_R, sum_j R_j,
    dt_exp seconds for the N quadratures).  Returns the rates and the N_R of
    the largest."""
    k = [k_exp(N, r, S_BE, d_aep, eps_pa, dt) for _, r, dt in points]
    return k, points[int(max(range(len(k)), key=lambda i: k[i]))][0]


def k_prime(N_R: float, N: float, I_AB: float, A: float, eps_ec: float, B1: float, B2: float) -> float:
    """K'_Finite = (N C_Finite - B_1) / (B_2 N_R), bits per second."""
    return (N * c_finite(N_R, I_AB, A, eps_ec) - B1) / (B2 * N_R)


def dk_prime(N_R: float, N: float, I_AB: float, A: float, eps_ec: float, B1: float, B2: float) -> float:
    """dK'/dN_R in the paper's printed closed form."""
    q = q_inv(eps_ec)
    return (-N * I_AB / (B2 * N_R ** 2) - N / (2.0 * B2 * N_R ** 3)
            + 3.0 * N * math.sqrt(A) * q / (2.0 * B2 * N_R ** 2.5)
            + N * math.log(N_R) / (B2 * N_R ** 3) + B1 / (B2 * N_R ** 2))


def optimal_nr(N: float, I_AB: float, A: float, eps_ec: float, B1: float, B2: float,
               lo: float = 1e5, hi: float | None = None) -> tuple[float, float]:
    """(N_R*, K'_Finite(N_R*)) on lo <= N_R <= hi (default N): the root of the
    derivative when it changes sign there, else the better end."""
    hi = N if hi is None else hi
    f = lambda r: dk_prime(r, N, I_AB, A, eps_ec, B1, B2)
    if f(lo) > 0.0 > f(hi):
        r = brentq(f, lo, hi, xtol=1e-9 * lo, rtol=1e-14, maxiter=500)
    else:
        r = max((lo, hi), key=lambda x: k_prime(x, N, I_AB, A, eps_ec, B1, B2))
    return r, k_prime(r, N, I_AB, A, eps_ec, B1, B2)
