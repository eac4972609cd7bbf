"""Host-side (fp64) complexity model of slice reconciliation (Sec. III-C).

* E_j: arithmetic operations per BP iteration, 7 per edge (Eq. for E_j), with
  the edge count G = N_R / sum_a(lambda_a / a) of an edge-perspective variable
  degree distribution lambda.
* D_j: iterations to reach a target bit error ratio under density evolution
  with the Gaussian approximation (Eqs. for D_j, q_k, phi and its closed-form
  approximation, after Chung, Richardson and Urbanke).  The recursion tracks
  the mean u_k of the check-to-variable messages, starting from the mean m0 of
  the channel LLRs (2 / sigma^2 on a binary-input AWGN channel); the bit error
  ratio after k iterations is sum_a Lambda_a Q(sqrt((m0 + a u_k) / 2)) over
  the node-perspective variable degrees Lambda.
* Delta t = c_h sum_j E_j D_j (Eq. for Delta t).

Degree distributions are dicts {degree: fraction}, edge perspective unless
named otherwise.  Nothing here runs on the GPU.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.special import ndtr

# closed-form approximation of phi (Gaussian approximation), valid for 0 < v < 10
PHI_A, PHI_B, PHI_C = 0.4527, 0.86, 0.0218


_TABLE: tuple[CubicSpline, CubicSpline, float] | None = None
_V_MIN, _V_MAX = 1e-8, 300.0


def _phi_table():
    """ln phi on a log grid of v, phi(v) = E[2 / (1 + e^U)], U ~ N(v, 2v)
    (= 1 - E[tanh(U / 2)] without the cancellation).  Trapezoid rule in u
    over v +- (2v + 12 sd) with step min(0.05, sd / 30), the integrand taken
    in the log domain; the integrand is analytic in a strip of half-width pi,
    so the rule's error is far below fp64 rounding."""
    global _TABLE
    if _TABLE is None:
        lv = np.linspace(math.log(_V_MIN), math.log(_V_MAX), 3001)
        lp = np.empty_like(lv)
        for i, v in enumerate(np.exp(lv)):
            sd = math.sqrt(2.0 * v)
            h = min(0.05, sd / 30.0)
            u = np.arange(-v - 12.0 * sd, v + 12.0 * sd + h, h)
            lf = math.log(2.0) - np.logaddexp(0.0, u) - (u - v) ** 2 / (4.0 * v) - 0.5 * math.log(4.0 * math.pi * v)
            mx = lf.max()
            lp[i] = mx + math.log(np.trapezoid(np.exp(lf - mx), dx=h))
        # ln phi(ln v) and its inverse (ln phi is strictly decreasing), cubic
        _TABLE = (CubicSpline(lv, lp), CubicSpline(lp[::-1], lv[::-1]), float(lp[-1]))
    return _TABLE


def phi_exact(v: float) -> float:
    """phi(v) = 1 - E[tanh(U / 2)], U ~ N(v, 2v), phi(0) = 1; a cubic spline
    in (ln v, ln phi) through a quadrature table, clamped to 1e-8 <= v <= 300."""
    if v <= 0.0:
        return 1.0
    fwd, _, _ = _phi_table()
    return float(math.exp(fwd(math.log(min(max(v, _V_MIN), _V_MAX)))))


def phi_approx(v: float) -> float:
    """exp(-0.4527 v^0.86 + 0.0218) for v > 0, capped at 1 (the closed form
    exceeds 1 below v ~ 0.03); 1 at v = 0."""
    if v <= 0.0:
        return 1.0
    return min(1.0, math.exp(-PHI_A * v ** PHI_B + PHI_C))


def phi_inv_approx(w: float) -> float:
    """Inverse of the closed form: ((ln w - 0.0218) / -0.4527)^(1 / 0.86) for
    0 < w < 1, 0 at w >= 1, +inf at w <= 0."""
    if w >= 1.0:
        return 0.0
    if w <= 0.0:
        return math.inf
    return ((math.log(w) - PHI_C) / -PHI_A) ** (1.0 / PHI_B)


def phi_inv_exact(w: float) -> float:
    """Inverse of phi_exact (same table; ln phi is decreasing in ln v); values
    below phi(300) map to 300."""
    if w >= 1.0:
        return 0.0
    _, inv, lp_min = _phi_table()
    if w <= 0.0 or math.log(w) <= lp_min:
        return _V_MAX
    lw = math.log(w)
    v = math.exp(inv(lw))
    return float(min(max(v, _V_MIN), _V_MAX)) if lw < inv.x[-1] else _V_MIN


def node_fractions(lam: dict) -> dict:
    """Node-perspective variable degrees Lambda_a = (lambda_a / a) / sum(lambda_b / b)."""
    s = sum(f / a for a, f in lam.items())
    return {a: (f / a) / s for a, f in lam.items()}


def edges(n: int, lam: dict) -> float:
    """G = n / sum_a(lambda_a / a): edges of a length-n code with variable
    degree distribution lambda (exact for any rho)."""
    return n / sum(f / a for a, f in lam.items())


def ops_per_iteration(n: int, lam: dict) -> float:
    """E = 7 G: 3 operations per edge towards the checks and 4 back."""
    return 7.0 * edges(n, lam)


def ga_ber(m0: float, lam: dict, rho: dict, k_max: int, exact: bool = False) -> list[float]:
    """Bit error ratios after iterations 1..k_max (Gaussian approximation)."""
    phi = phi_exact if exact else phi_approx
    phi_inv = phi_inv_exact if exact else phi_inv_approx
    Lam = node_fractions(lam)
    u = 0.0
    out = []
    for _ in range(k_max):
        L = 1.0 - sum(f * phi(m0 + (a - 1) * u) for a, f in lam.items())
        u = sum(f * phi_inv(1.0 - L ** (b - 1)) for b, f in rho.items())
        if math.isinf(u):
            out.append(0.0)
            continue
        out.append(float(sum(f * ndtr(-math.sqrt((m0 + a * u) / 2.0)) for a, f in Lam.items())))
    return out


def iterations_to(target_ber: float, m0: float, lam: dict, rho: dict, k_max: int = 1000,
                  exact: bool = False) -> int | None:
    """D = min{k : BER_k <= target}, or None if not reached within k_max."""
    for k, p in enumerate(ga_ber(m0, lam, rho, k_max, exact), start=1):
        if p <= target_ber:
            return k
    return None


def threshold_sigma(lam: dict, rho: dict, exact: bool = False, target: float = 1e-12,
                    k_max: int = 3000, lo: float = 0.3, hi: float = 2.0, steps: int = 40) -> float:
    """Largest sigma of a binary-input AWGN channel (m0 = 2 / sigma^2) at which
    the recursion drives the bit error ratio below ``target`` (bisection)."""
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if iterations_to(target, 2.0 / mid ** 2, lam, rho, k_max, exact) is not None:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def biawgn_capacity(sigma2: float) -> float:
    """1 - E[log2(1 + e^-L)], L ~ N(2/sigma^2, 4/sigma^2): capacity of the
    binary-input AWGN channel (Gauss-Hermite, 200 nodes)."""
    m = 2.0 / sigma2
    t, w = np.polynomial.hermite.hermgauss(200)
    L = m + 2.0 * math.sqrt(m) * t
    return float(1.0 - (w * np.logaddexp(0.0, -L)).sum() / math.sqrt(math.pi) / math.log(2.0))


def biawgn_mean_for_capacity(C: float) -> float:
    """Channel LLR mean m0 = 2 / sigma^2 of the binary-input AWGN channel whose
    capacity is C (bisection on log sigma^2)."""
    lo, hi = 1e-4, 1e4
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if biawgn_capacity(mid) > C:
            lo = mid
        else:
            hi = mid
    return 2.0 / math.sqrt(lo * hi)


def degree_distributions(row_ptr, col_idx, n: int) -> tuple[dict, dict]:
    """Edge-perspective (lambda, rho) of a parity-check matrix in CSR form."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    E = col_idx.size
    dv = np.bincount(col_idx, minlength=n)
    dc = np.diff(row_ptr)
    lam = {int(a): float(a * c / E) for a, c in zip(*np.unique(dv[dv > 0], return_counts=True))}
    rho = {int(b): float(b * c / E) for b, c in zip(*np.unique(dc[dc > 0], return_counts=True))}
    return lam, rho


def decode_time(c_h: float, E: list[float], D: list[int]) -> float:
    """Delta t = c_h sum_j E_j D_j."""
    return c_h * sum(e * d for e, d in zip(E, D))
