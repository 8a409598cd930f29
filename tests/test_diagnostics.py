"""Pins for the chain diagnostics against processes with known answers."""
import numpy as np

from paper_1306_1821_amd import diagnostics as dg


def ar1(phi, n, m=1, seed=0):
    rng = np.random.default_rng(seed)
    x = np.zeros((m, n))
    e = rng.standard_normal((m, n)) * np.sqrt(1 - phi * phi)
    x[:, 0] = rng.standard_normal(m)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return x


def test_autocorr_of_ar1_is_geometric():
    x = ar1(0.8, 200000)[0]
    c = dg.autocorr(x, 10)
    assert np.allclose(c, 0.8 ** np.arange(11), atol=0.01)


def test_correlation_length_of_ar1():
    phi = 0.9
    x = ar1(phi, 400000)[0]
    want = int(np.ceil(np.log(0.1) / np.log(phi)))   # first n with phi^n < 0.1
    assert abs(dg.correlation_length(x) - want) <= 1


def test_ess_of_ar1_matches_integrated_time():
    phi = 0.7
    x = ar1(phi, 20000, m=4, seed=3)
    tau = (1 + phi) / (1 - phi)
    want = x.size / tau
    assert abs(dg.ess_bulk(x) / want - 1) < 0.15
    assert abs(dg.ess(x) / want - 1) < 0.15


def test_ess_of_iid_is_sample_size():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 5000))
    assert abs(dg.ess_bulk(x) / x.size - 1) < 0.1


def test_rhat_detects_disagreeing_chains():
    rng = np.random.default_rng(6)
    good = rng.standard_normal((4, 4000))
    assert dg.split_rhat(good) < 1.01
    bad = good + np.array([0.0, 0.0, 0.0, 1.0])[:, None]
    assert dg.split_rhat(bad) > 1.1
    trend = good + np.linspace(0, 3, 4000)[None, :]       # non-stationary within chains
    assert dg.split_rhat(trend) > 1.1


def test_burn_in_xi():
    assert np.allclose(dg.burn_in_xi([2.0, 1.0, 0.5], 1.0), [-1.0, 0.0, 0.5])
