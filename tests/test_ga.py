"""Pins of the host-side complexity model (Sec. III-C): the closed-form phi
against its integral definition (quadrature table and Monte Carlo), the
Gaussian-approximation threshold of the (3,6) ensemble against its published
value, edge counts of the paper's ensembles, binary-input AWGN capacity, and
the monotonicity of the predicted iteration count."""
import math

import numpy as np
import pytest

from paper_2108_08418_amd import ga

LAM_PAPER = {2: 0.25, 3: 0.3, 8: 0.45}        # lambda(x) = 0.25x + 0.3x^2 + 0.45x^7


def test_phi_table_matches_monte_carlo():
    """phi(v) = 1 - E[tanh(U/2)], U ~ N(v, 2v), sampled directly."""
    rng = np.random.default_rng(3)
    for v in (0.2, 1.0, 3.0, 7.0):
        u = rng.normal(v, math.sqrt(2 * v), 2_000_000)
        mc = 1.0 - np.tanh(u / 2).mean()
        assert abs(ga.phi_exact(v) - mc) < 2e-3, (v, ga.phi_exact(v), mc)


def test_phi_limits_and_monotonicity():
    assert ga.phi_exact(0.0) == 1.0 and ga.phi_approx(0.0) == 1.0
    vs = np.linspace(0.01, 50, 400)
    pe = [ga.phi_exact(v) for v in vs]
    assert all(a > b for a, b in zip(pe, pe[1:]))
    # adaptive quadrature of the definition, including the far tail where the
    # integrand's mass sits near u = 0 (about sqrt(v / 2) deviations out)
    from scipy.integrate import quad
    for v in (1e-3, 0.5, 5.0, 40.0, 120.0, 250.0):
        sd = math.sqrt(2 * v)
        f = lambda u: (1 - math.tanh(u / 2)) * math.exp(-(u - v) ** 2 / (4 * v)) / math.sqrt(4 * math.pi * v)
        ref, _ = quad(f, -v - 40 * sd, v + 40 * sd, points=[-v, 0.0, v], limit=2000, epsabs=0, epsrel=1e-10)
        assert abs(ga.phi_exact(v) / ref - 1) < 1e-8, (v, ga.phi_exact(v), ref)


def test_closed_form_phi_tracks_the_integral():
    """The closed form is within 1 % (relative) of the integral on 0.1 <= v <= 10."""
    vs = np.linspace(0.1, 10, 200)
    rel = max(abs(ga.phi_approx(v) - ga.phi_exact(v)) / ga.phi_exact(v) for v in vs)
    assert rel < 1e-2


@pytest.mark.parametrize("exact", [False, True])
def test_phi_inverse_round_trip(exact):
    phi = ga.phi_exact if exact else ga.phi_approx
    inv = ga.phi_inv_exact if exact else ga.phi_inv_approx
    for v in (0.05, 0.3, 1.0, 4.0, 9.0, 40.0):
        assert abs(inv(phi(v)) / v - 1) < 1e-6, (v, inv(phi(v)))
    assert inv(1.0) == 0.0


def test_ga_threshold_of_the_3_6_ensemble():
    """Chung, Richardson and Urbanke report sigma = 0.8747 for the (3,6)
    ensemble under the Gaussian approximation (exact density evolution:
    0.8809).  The closed-form phi reproduces it; the integral phi stays below
    the exact threshold."""
    s_cf = ga.threshold_sigma({3: 1.0}, {6: 1.0}, exact=False, steps=25, k_max=2000)
    assert abs(s_cf - 0.8747) < 5e-4, s_cf
    s_int = ga.threshold_sigma({3: 1.0}, {6: 1.0}, exact=True, steps=20, k_max=2000)
    assert 0.865 < s_int < 0.8809, s_int


def test_edge_counts_of_the_paper_ensembles():
    # lambda of the slice codes: sum(lambda_a / a) = 0.28125, E = 233,017 at n = 65536
    assert abs(ga.edges(65536, LAM_PAPER) - 65536 / 0.28125) < 1e-9
    assert round(ga.edges(65536, LAM_PAPER)) == 233017
    # (3,6) regular at n = 1024: 3072 edges; E = 7 G operations per iteration
    assert ga.edges(1024, {3: 1.0}) == 3072
    assert ga.ops_per_iteration(1024, {3: 1.0}) == 7 * 3072
    # node fractions of lambda: 4/9, 16/45, 1/5
    Lam = ga.node_fractions(LAM_PAPER)
    assert abs(Lam[2] - 4 / 9) < 1e-12 and abs(Lam[3] - 16 / 45) < 1e-12 and abs(Lam[8] - 0.2) < 1e-12


def test_degree_distributions_of_a_small_matrix():
    # 3 checks over 4 variables: rows {0,1,2}, {1,2,3}, {0,3}
    row_ptr, col_idx = [0, 3, 6, 8], [0, 1, 2, 1, 2, 3, 0, 3]
    lam, rho = ga.degree_distributions(row_ptr, col_idx, 4)
    assert lam == {2: 1.0}                       # every variable in two checks
    assert rho == {2: 2 / 8, 3: 6 / 8}


def test_biawgn_capacity_values():
    # SNR 0.16 (sigma^2 = 6.25): 0.1070 bits; noiseless limit 1; monotone in sigma^2
    assert abs(ga.biawgn_capacity(6.25) - 0.1070) < 2e-4
    assert ga.biawgn_capacity(1e-3) > 1 - 1e-9
    caps = [ga.biawgn_capacity(s) for s in (0.2, 0.5, 1.0, 2.0, 5.0)]
    assert all(a > b for a, b in zip(caps, caps[1:]))
    m0 = ga.biawgn_mean_for_capacity(0.5)
    assert abs(ga.biawgn_capacity(2.0 / m0) - 0.5) < 1e-9


def test_iteration_count_behaviour():
    lam, rho = {3: 1.0}, {6: 1.0}
    good = 2.0 / 0.80 ** 2                           # sigma 0.80, below the threshold
    bad = 2.0 / 0.95 ** 2                            # sigma 0.95, above it
    D = [ga.iterations_to(t, good, lam, rho) for t in (1e-3, 1e-6, 1e-9, 1e-12)]
    assert all(d is not None for d in D) and D == sorted(D) and D[0] < D[-1]
    assert ga.iterations_to(1e-6, bad, lam, rho, k_max=2000) is None
    ber = ga.ga_ber(good, lam, rho, 30)
    assert all(a >= b for a, b in zip(ber, ber[1:]))
    # Delta t = c_h sum E_j D_j; the paper's c_h = 3.2e-9 s gives 1 / (7 c_h) = 4.46e7 edge updates/s
    assert abs(ga.decode_time(3.2e-9, [7.0], [1]) * 4.464e7 - 1) < 1e-3


def test_slice_code_family_contains_the_chosen_codes():
    """The rate-selection candidates and the codes the pipeline uses are one family."""
    from paper_2108_08418_amd import inputs
    for j, mb in ((2, 104), (3, 65)):
        a = inputs.slice_code_spec(j, 4096)
        b = inputs.slice_code_at(j, 4096, mb)
        assert (a.shift == b.shift).all() and a.mb == b.mb == mb
    with pytest.raises(ValueError):
        inputs.slice_code_at(2, 4096, 128)
