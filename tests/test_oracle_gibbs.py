"""Pins for oracle.gibbs: each conditional draw against its closed form or brute force."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import gibbs, grid, model
from synth import CONFIGS, make_mock


@pytest.mark.parametrize("a", [0.7, 3.5, 50.0, 4000.0])
def test_gamma_marsaglia_tsang_ks(a):
    x = np.array([gibbs.gamma_mt(a, 9, 0, i, 3) for i in range(1500)])
    assert stats.kstest(x, stats.gamma(a).cdf).pvalue > 1e-3


def test_power_draw_is_inverse_gamma():
    """lambda_m ~ InvGamma(shape alpha - 1 + n_m/2, scale sigma_m/2) (eq. INVERSE_GAMMA)."""
    nm = np.array([26, 152])
    sigma = np.array([3.0, 40.0])
    for ap in (0.0, 1.0):
        draws = np.array([gibbs.draw_power(sigma, nm, [1.0, 1.0], ap, 4, 0, s) for s in range(1500)])
        for m in range(2):
            ig = stats.invgamma(a=ap - 1 + nm[m] / 2, scale=sigma[m] / 2)
            assert stats.kstest(draws[:, m], ig.cdf).pvalue > 1e-3
    # empty shells keep their value
    keep = gibbs.draw_power(np.array([1.0]), np.array([0]), [7.5], 1.0, 4, 0, 0)
    assert keep[0] == 7.5


def _gig_logpdf(p, A, B):
    return lambda x: (p - 1.0) * np.log(x) - 0.5 * (A * x + B / x)


def _gig_cdf_brute(p, A, B, xs):
    """Normalised CDF by quadrature of the unnormalised log density around its mode."""
    lp = _gig_logpdf(p, A, B)
    mode = ((p - 1) + math.sqrt((p - 1) ** 2 + A * B)) / A
    sd = 1.0 / math.sqrt((1 - p) / mode ** 2 + B / mode ** 3) if p < 1 else mode
    lo, hi = max(mode - 40 * sd, mode * 1e-6), mode + 40 * sd
    grid_x = np.linspace(lo, hi, 400001)
    logf = lp(grid_x) - lp(mode)
    f = np.exp(logf)
    c = integrate.cumulative_trapezoid(f, grid_x, initial=0.0)
    c /= c[-1]
    return np.interp(xs, grid_x, c), mode, grid_x[np.argmax(f)]


@pytest.mark.parametrize("p,A,B", [(-4591.0, 3700.0, 15000.0), (5.5, 2.0, 3.0),
                                   (-1.37e6, 1.1e6, 7.0e7), (-3.0, 40.0, 900.0)])
def test_gig_draw_ks_vs_quadrature(p, A, B):
    x = np.array([gibbs.gig(p, A, B, 5, 0, i, 1) for i in range(1200)])
    cdf = lambda v: _gig_cdf_brute(p, A, B, v)[0]
    assert stats.kstest(x, cdf).pvalue > 1e-3
    _, mode, argmax = _gig_cdf_brute(p, A, B, np.array([1.0]))
    assert abs(mode - argmax) < 1e-3 * mode


def test_bias_conditional_is_normal_with_corrected_moments():
    """Normalised exp(-chi^2/2) of eq. galaxybias_post on a b grid equals N(D/C, 1/C)."""
    mk = make_mock(CONFIGS["tiny8x2"])
    R, counts = mk["R"], mk["counts"]
    delta = mk["delta"]
    nbar = mk["nbar"]
    mom = gibbs.delta_moments(delta, R, counts)
    for l in range(2):
        S1, S2, T = mom[l]
        C = nbar[l] * S2
        D = T - nbar[l] * S1
        mu, sd = D / C, 1.0 / math.sqrt(C)
        bs = np.linspace(mu - 8 * sd, mu + 8 * sd, 20001)
        chi2 = np.array([model.psi_data_direct(delta, R[l:l + 1], counts[l:l + 1], [b], [nbar[l]])
                         for b in bs[::50]])
        logf = -(chi2 - chi2.min())
        f = np.exp(logf)
        f /= np.trapezoid(f, bs[::50])
        assert np.max(np.abs(f - stats.norm(mu, sd).pdf(bs[::50]))) < 1e-3 / sd


def test_bias_draws_and_fixed_mask():
    mk = make_mock(CONFIGS["tiny8x2"])
    mom = gibbs.delta_moments(mk["delta"], mk["R"], mk["counts"])
    S1, S2, T = mom[1]
    C = mk["nbar"][1] * S2
    D = T - mk["nbar"][1] * S1
    draws = np.array([gibbs.draw_bias(mom, mk["nbar"], mk["bias"], 1, 8, 0, s)[1]
                      for s in range(1500)])
    assert stats.kstest(draws, stats.norm(D / C, 1 / math.sqrt(C)).cdf).pvalue > 1e-3
    fixed = gibbs.draw_bias(mom, mk["nbar"], mk["bias"], 1, 8, 0, 0)
    assert fixed[0] == mk["bias"][0]


def test_nbar_moments_expand_A():
    mk = make_mock(CONFIGS["tiny8x2"])
    R, counts, delta = mk["R"], mk["counts"], mk["delta"]
    stat = gibbs.static_moments(R, counts)
    mom = gibbs.delta_moments(delta, R, counts)
    for l in range(2):
        b = mk["bias"][l]
        obs = R[l] > 0
        A_direct = float(np.sum(R[l][obs] * (1 + b * delta[obs]) ** 2))
        S0, B, nobs = stat[l]
        S1, S2, T = mom[l]
        assert math.isclose(S0 + 2 * b * S1 + b * b * S2, A_direct, rel_tol=1e-12)
        assert nobs == int(obs.sum())


def test_nbar_conditional_matches_likelihood_profile():
    """GIG(p = 1 - N_obs/2, A, B) is the Nbar profile of eq. nmean_post (flat prior)."""
    mk = make_mock(CONFIGS["tiny8x2"])
    R, counts, delta = mk["R"][:1], mk["counts"][:1], mk["delta"]
    b = mk["bias"][0]
    S0, B, nobs = gibbs.static_moments(R, counts)[0]
    S1, S2, T = gibbs.delta_moments(delta, R, counts)[0]
    A = S0 + 2 * b * S1 + b * b * S2
    xs = np.linspace(3.0, 7.0, 41)
    direct = np.array([-model.psi_data_direct(delta, R, counts, [b], [x]) - 0.5 * nobs * math.log(x)
                       for x in xs])
    gig = (1 - 0.5 * nobs - 1) * np.log(xs) - 0.5 * (A * xs + B / xs)
    assert np.ptp(direct - gig) < 1e-8 * np.max(np.abs(direct))


def test_degenerate_field_keeps_power_and_bias():
    """delta = 0 gives sigma_m = 0 and C = 0: both conditionals are improper, values kept."""
    lam = gibbs.draw_power(np.zeros(2), np.array([26, 152]), [3.0, 4.0], 1.0, 4, 0, 0)
    assert np.array_equal(lam, [3.0, 4.0])
    mom = [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0)]
    b = gibbs.draw_bias(mom, np.array([5.0, 1.0]), np.array([1.0, 1.4]), 0, 8, 0, 0)
    assert np.array_equal(b, [1.0, 1.4])
