"""The seeded input generator's magnitude-binned survey (the paper's own test
scenario on synthetic geometry): luminosity function, bias relation, selection."""
import numpy as np
from scipy import integrate

from synth import CONFIGS
from synth import mock as sm


def test_bias_relation_reference_point():
    # at M = M*_b the relation gives b* (a + b) = b* since a + b = 1
    assert abs(sm.lf_bias(sm.BIAS_MSTAR) - sm.BIAS_BSTAR) < 1e-12
    mc = sm.magnitude_bins(15)[1]
    b = sm.lf_bias(mc)
    assert np.all(np.diff(b) < 0)                       # brighter bins are more biased
    assert np.allclose(CONFIGS["paper15"].bias, b)


def test_luminosity_function_bin_integrals():
    edges = sm.magnitude_bins(15)[0]
    for lo, hi in zip(edges[:-1], edges[1:]):
        ref = integrate.quad(sm.schechter, lo, hi, epsabs=0, epsrel=1e-12)[0]
        assert abs(sm._lf_integral(lo, hi) - ref) < 1e-9 * ref
    vox = (750.0 / 128) ** 3
    nbar = np.array(CONFIGS["paper15"].nbar)
    assert np.allclose(nbar, [sm._lf_integral(a, b) * vox for a, b in zip(edges[:-1], edges[1:])])


def test_distance_modulus_low_redshift():
    # Hubble flow: D_L = r (1 + z) with z = r H0 / c to first order for small r (Mpc/h)
    r = np.array([1.0, 5.0, 10.0])
    z = r * 100.0 / 299792.458
    assert np.allclose(sm.distance_modulus(r), 5 * np.log10(r * (1 + z)) + 25, atol=1e-5)
    assert np.all(np.diff(sm.distance_modulus(np.linspace(1, 700, 50))) > 0)


def test_selection_fractions():
    r = np.linspace(1.0, 650.0, 300)
    f = sm.lf_selection(r, 15)
    assert np.all(f >= -1e-9) and np.all(f <= 1 + 1e-9)
    dm = sm.distance_modulus(r)
    edges = sm.magnitude_bins(15)[0]
    for l in range(15):
        whole = (sm.R_BRIGHT - dm <= edges[l]) & (sm.R_FAINT - dm >= edges[l + 1])
        none = (sm.R_FAINT - dm <= edges[l]) | (sm.R_BRIGHT - dm >= edges[l + 1])
        # away from the interpolation of the table the fractions are exactly 1 / 0
        assert np.all(f[l][whole & np.roll(whole, 1) & np.roll(whole, -1)] > 1 - 1e-3)
        assert np.all(f[l][none & np.roll(none, 1) & np.roll(none, -1)] < 1e-3)
