"""Chain diagnostics for sampler traces (host-side post-processing).

* autocorrelation C(omega)_n of Sec. "Testing burn-in and statistical
  efficiency" (eq. CORR_COEFF) and the correlation length: the first lag at
  which C drops below 0.1;
* burn-in deviation xi(omega_s) = 1 - omega_s / omega_0 (eq. BURN_IN);
* rank-normalised split R-hat and bulk effective sample size (Vehtari, Gelman,
  Simpson, Carpenter & Buerkner 2021), used for the ESS/s and equal-R-hat
  comparisons; ESS uses Geyer's initial monotone sequence on the combined
  autocorrelation of all chains.
"""
import numpy as np
from scipy import special


def autocorr(x, max_lag=None):
    """C_n = < (w_s - <w>)(w_{s+n} - <w>) > / Var(w), n = 0..max_lag."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    max_lag = n - 1 if max_lag is None else min(max_lag, n - 1)
    d = x - x.mean()
    f = np.fft.rfft(d, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[: max_lag + 1] / np.arange(n, n - max_lag - 1, -1)
    return ac / ac[0]


def correlation_length(x, threshold=0.1):
    """First lag n with C_n < threshold (len(x) if never)."""
    c = autocorr(x)
    below = np.nonzero(c < threshold)[0]
    return int(below[0]) if below.size else len(x)


def burn_in_xi(trace, truth):
    """xi = 1 - omega_s / omega_0 for every sample of a trace."""
    return 1.0 - np.asarray(trace, dtype=np.float64) / truth


def _split(chains):
    c = np.asarray(chains, dtype=np.float64)
    if c.ndim == 1:
        c = c[None, :]
    half = c.shape[1] // 2
    return np.concatenate([c[:, :half], c[:, half:2 * half]], axis=0)


def _rank_normal(c):
    flat = c.ravel()
    r = np.empty_like(flat)
    r[np.argsort(flat, kind="mergesort")] = np.arange(1, flat.size + 1)
    z = special.ndtri((r - 0.375) / (flat.size + 0.25))
    return z.reshape(c.shape)


def _rhat(c):
    m, n = c.shape
    means = c.mean(axis=1)
    B = n * means.var(ddof=1)
    W = c.var(axis=1, ddof=1).mean()
    var = (n - 1) / n * W + B / n
    return float(np.sqrt(var / W))


def split_rhat(chains):
    """Rank-normalised split R-hat: max of the bulk and folded versions."""
    c = _split(chains)
    bulk = _rhat(_rank_normal(c))
    folded = _rhat(_rank_normal(np.abs(c - np.median(c))))
    return max(bulk, folded)


def _ess(c):
    m, n = c.shape
    acov = np.array([autocorr(ch) * ch.var() for ch in c])       # m x n (biased var)
    chain_var = c.var(axis=1, ddof=1)
    W = chain_var.mean()
    var_plus = (n - 1) / n * W + c.mean(axis=1).var(ddof=1) if m > 1 else W
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer initial monotone sequence on paired sums
    tau = -1.0
    prev = np.inf
    for t in range(0, n - 1, 2):
        pair = rho[t] + rho[t + 1]
        if pair < 0:
            break
        pair = min(pair, prev)
        prev = pair
        tau += 2.0 * pair
    return float(m * n / max(tau, 1.0 / np.log10(m * n)))


def ess_bulk(chains):
    """Bulk effective sample size of one scalar over several chains (split, rank-normalised)."""
    return _ess(_rank_normal(_split(chains)))


def ess(chains):
    """Effective sample size without rank normalisation (split chains)."""
    return _ess(_split(chains))
