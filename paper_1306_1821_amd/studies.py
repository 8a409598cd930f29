"""Sampler studies beyond the headline benchmark.

joint_move_ablation: the P(k) correlation of the block sampler with and without
the joint (P, delta) move of row a10 (the paper's argument for it: without a
joint transition P and delta are strongly coupled and P(k) decorrelates over
very many sweeps; Sec. "Testing burn-in and statistical efficiency" measures it
with the autocorrelation of eq. CORR_COEFF and the correlation length).
"""
import numpy as np

from . import diagnostics
from .binding import Sampler
from .learned import chain_from_mock, data_dominated_shells, run_chains


def joint_move_ablation(mk, chains=4, burn=100, sweeps=3000, lags=(1, 10, 100, 1000), seed=31,
                        log=None):
    """Chains of the survey `mk` started at its truth field, the same eps and step
    count, with the joint move on and off.  Per mode: acceptance, ms per sweep and,
    per shell, the autocorrelation of ln P at `lags` (mean over chains), the
    correlation length (first lag below 0.1, per chain, then the median over chains)
    and the bulk ESS per sweep.  Returns {"joint": {...}, "no_joint": {...}}."""
    out = {}
    nb = mk["cfg"].nb
    for name, rj in (("joint", True), ("no_joint", False)):
        s = Sampler([chain_from_mock(mk, seed=seed, chain_id=i, rj=rj) for i in range(chains)])
        for i in range(chains):
            s.set_state(i, mk["delta"])
        s.use_graph(True)
        run_chains(s, burn)
        pk, acc, wall, _ = run_chains(s, sweeps, first_sweep=burn)
        s.close()
        lp = np.log(pk)                                  # [chains][sweeps][nb]
        max_lag = min(max(lags), sweeps - 1)
        ac = np.zeros((nb, len(lags)))
        corr_len = np.zeros(nb)
        for m in range(nb):
            acs = np.array([diagnostics.autocorr(lp[c, :, m], max_lag) for c in range(chains)])
            mean_ac = acs.mean(axis=0)
            ac[m] = [mean_ac[min(l, max_lag)] for l in lags]
            corr_len[m] = np.median([diagnostics.correlation_length(lp[c, :, m]) for c in range(chains)])
        ess = np.array([diagnostics.ess_bulk(lp[:, :, m]) for m in range(nb)])
        out[name] = dict(acceptance=float(acc.mean()), ms_per_sweep=1e3 * wall / sweeps,
                         autocorr=ac, corr_len=corr_len, ess_per_sweep=ess / (chains * sweeps),
                         ess_per_s=ess / wall, lags=list(lags), sweeps=sweeps, chains=chains)
        if log:
            dd = data_dominated_shells(mk)
            log(f"{name}: acceptance {acc.mean():.2f}, {1e3 * wall / sweeps:.2f} ms/sweep "
                f"({chains} chains); median over shells: correlation length "
                f"{np.median(corr_len):.0f} sweeps, C(lag) {dict(zip(lags, np.round(np.median(ac, 0), 3)))}; "
                f"data-dominated shells: correlation length {np.median(corr_len[dd]):.0f}, "
                f"ESS/s {np.median(out[name]['ess_per_s'][dd]):.3g}")
    return out
