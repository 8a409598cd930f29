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


def _corr(a, b):
    a = np.asarray(a, np.float64) - np.mean(a)
    b = np.asarray(b, np.float64) - np.mean(b)
    d = np.sqrt(np.sum(a * a) * np.sum(b * b))
    return float(np.sum(a * b) / d) if d > 0 else 0.0


def posterior_analysis(mk, chains=4, burn=100, sweeps=2000, seed=41, log=None):
    """Posterior structure of the block sampler on survey `mk` (Sec. "Results": the
    P-P correlation matrix, the bias-P and Nbar-P correlations, the ensemble mean
    and credible bands of P(k), mean and standard-deviation maps of the density):
    chains start at the truth field; after `burn` sweeps every sweep's P, b, Nbar
    are kept and every chain's density is folded into per-voxel running moments on
    the device (hmc_field_moments, pooled over chains)."""
    import torch
    cfg = mk["cfg"]
    n, nb, c = cfg.n, cfg.nb, cfg.nsub
    s = Sampler([chain_from_mock(mk, seed=seed, chain_id=i) for i in range(chains)])
    for i in range(chains):
        s.set_state(i, mk["delta"])
    sig, nmodes = s.shell_power(0)                       # the truth field's shell power
    p_truth = sig / np.maximum(nmodes, 1) * cfg.box ** 3 / n ** 3
    s.use_graph(True)
    run_chains(s, burn)
    dev = s.device
    mean = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    m2 = torch.zeros_like(mean)
    pk = np.zeros((chains, sweeps, nb))
    bias = np.zeros((chains, sweeps, c))
    nbar = np.zeros((chains, sweeps, c))
    count = 0
    for j in range(sweeps):
        st = s.sweep(burn + j)
        for i in range(chains):
            pk[i, j], bias[i, j], nbar[i, j] = st[i]["pk"], st[i]["bias"], st[i]["nbar"]
            count += 1
            s.field_moments(i, mean, m2, count)
    torch.cuda.synchronize(dev)
    mean_np = mean.cpu().numpy()
    sd_np = np.sqrt(m2.cpu().numpy() / max(1, count - 1))
    s.close()
    lp = np.log(pk).reshape(-1, nb)
    cpp = np.corrcoef(lp.T)
    off = cpp[~np.eye(nb, dtype=bool)]
    adj = np.array([cpp[m, m + 1] for m in range(nb - 1)])
    free = [l for l in range(c) if not ((cfg.fixed_mask >> l) & 1)]
    b_flat, nb_flat = bias.reshape(-1, c), nbar.reshape(-1, c)
    corr_bp = np.array([[_corr(b_flat[:, l], lp[:, m]) for m in range(nb)] for l in free])
    corr_np = np.array([[_corr(nb_flat[:, l], lp[:, m]) for m in range(nb)] for l in range(c)])
    corr_bn = np.array([_corr(b_flat[:, l], nb_flat[:, l]) for l in free])
    lo, med, hi = np.percentile(pk.reshape(-1, nb), [16, 50, 84], axis=0)
    covered = (lo <= p_truth) & (p_truth <= hi)
    obs = np.any(np.asarray(mk["R"]) > 0, axis=0)
    truth = np.asarray(mk["delta"], np.float64)
    out = dict(
        sweeps=sweeps, chains=chains,
        pp_max_abs_offdiag=float(np.max(np.abs(off))), pp_mean_abs_offdiag=float(np.mean(np.abs(off))),
        pp_adjacent_mean=float(np.mean(adj)),
        bias_p_corr_median=[float(np.median(r)) for r in corr_bp],
        nbar_p_corr_median=[float(np.median(r)) for r in corr_np],
        bias_nbar_corr=[float(x) for x in corr_bn],
        pk_mean=pk.reshape(-1, nb).mean(axis=0).tolist(), pk_band_16_84=[lo.tolist(), hi.tolist()],
        pk_truth=p_truth.tolist(), band_covers_truth=float(covered.mean()),
        mean_map_corr_observed=_corr(mean_np[obs], truth[obs]),
        mean_map_corr_unobserved=_corr(mean_np[~obs], truth[~obs]) if (~obs).any() else None,
        sd_map_mean_observed=float(sd_np[obs].mean()),
        sd_map_mean_unobserved=float(sd_np[~obs].mean()) if (~obs).any() else None,
        observed_fraction=float(obs.mean()))
    if log:
        log(f"P-P correlation: max |off-diagonal| {out['pp_max_abs_offdiag']:.3f}, mean "
            f"{out['pp_mean_abs_offdiag']:.3f}, adjacent shells {out['pp_adjacent_mean']:.3f}; "
            f"b-P median per free subsample {np.round(out['bias_p_corr_median'], 3)}; "
            f"Nbar-P {np.round(out['nbar_p_corr_median'], 3)}; b-Nbar {np.round(out['bias_nbar_corr'], 3)}; "
            f"68% band covers the truth shell power in {100 * out['band_covers_truth']:.0f}% of shells; "
            f"mean map vs truth: r = {out['mean_map_corr_observed']:.3f} observed, "
            f"{out['mean_map_corr_unobserved']} unobserved; sd map mean "
            f"{out['sd_map_mean_observed']:.3f} observed, {out['sd_map_mean_unobserved']} unobserved")
    return out
