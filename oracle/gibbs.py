"""Oracle: the Gibbs blocks around the density step (test infrastructure only).

* P(k) | delta (Sec. "Sample the power spectrum"): with a power-law prior
  P^-alpha the conditional is inverse-Gamma (eq. INVERSE_GAMMA); with
  x_m = sigma_m / P_m it is chi^2 with beta_m = 2(alpha + n_m/2 - 1) degrees of
  freedom (eq. XI_SQUARE) and P_m = sigma_m / x_m (eq. PS_sample).  Readings:
  n_m counts full-grid modes; sigma_m and P_m are in the unitary eigenvalue
  units lambda of ``model`` (P_phys = lambda V / N_vox); a chi^2_beta variate is
  drawn as 2 Gamma(beta/2) by Marsaglia & Tsang (2000) rather than as a sum of
  beta squared normals (same law, O(1) random numbers per shell); shells with
  n_m = 0 or sigma_m = 0 (an all-zero field, where the conditional is
  improper) keep their value.
* Nbar^l | delta, b (Sec. "The Nbar posterior distribution", Appendix A): GIG
  with p = 1 - N_obs/2, A = sum R (1 + b delta)^2, B = sum N^2 / R (eq. GIG_post).
  Readings: N_obs counts voxels with R^l > 0 (the main-text form; the appendix
  writes N_vox) and every sum runs over those voxels.  The draw uses the
  ratio-of-uniforms method with mode shift (Dagpunar 1989; Lehner 1989; the
  algorithm Hoermann & Leydold 2014 use for lambda > 1 or omega > 1), with the
  bounding rectangle found by bisection in float64.
* b^l | delta, Nbar (Sec. "The bias posterior distribution", Appendix B):
  normal with variance 1/C, mean D/C.  Completing the square of eq.
  galaxybias_post gives C = sum Nbar R delta^2 and D = sum (N - Nbar R) delta;
  the printed forms (sum Nbar R delta in the main-text variance, (N - Nbar) in
  D) are read as typos.  For delta = 0 on every observed voxel (C = 0) the
  conditional is improper and b is kept.  A mask holds chosen biases fixed: b, delta and P are
  degenerate under (k b, delta / k, P / k^2), and the paper's own test fixes
  one reference bias.
* Block order (eq. multiblock and the flowchart disagree): density HMC, P,
  joint (P, delta) move, Nbar, b, each using the latest values.
"""
import math

import numpy as np

from . import grid, hmc, model, philox

MAX_ATTEMPTS = 256


# --------------------------------------------------------------------------- chi^2
def gamma_mt(a, seed, chain, draw, sub):
    """Gamma(a, 1) by Marsaglia & Tsang; attempt j uses Philox block j of stream 5.

    Block words: (0,1) -> normal (Box-Muller cosine branch), 2 -> uniform for the
    acceptance test, 3 -> uniform for the a < 1 boost Gamma(a) = Gamma(a+1) U^(1/a).
    """
    boost = a < 1.0
    aa = a + 1.0 if boost else a
    d = aa - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)
    for j in range(MAX_ATTEMPTS):
        wd = philox.words(seed, chain, philox.STREAM_CHI2, draw, sub, [j])[0]
        u01 = philox.to_uniform(wd)
        x = math.sqrt(-2.0 * math.log(u01[0])) * math.cos(2.0 * math.pi * u01[1])
        t = 1.0 + c * x
        if t <= 0.0:
            continue
        v = t * t * t
        if math.log(u01[2]) < 0.5 * x * x + d - d * v + d * math.log(v):
            g = d * v
            if boost:
                g *= u01[3] ** (1.0 / a)
            return g
    raise RuntimeError("gamma_mt: no acceptance")


def draw_power(sigma, n_modes, lam_old, alpha_prior, seed, chain, sweep):
    """New lambda_m = sigma_m / x_m, x_m ~ chi^2(n_m + 2 alpha - 2); sub = m."""
    lam = np.array(lam_old, dtype=np.float64)
    for m in range(len(sigma)):
        if n_modes[m] == 0 or not sigma[m] > 0:   # improper conditional: keep P_m
            continue
        beta = n_modes[m] + 2.0 * alpha_prior - 2.0
        x = 2.0 * gamma_mt(0.5 * beta, seed, chain, sweep, m)
        lam[m] = sigma[m] / x
    return lam


# --------------------------------------------------------------------------- GIG
def _gig_bounds(lam, om):
    """Mode and ratio-of-uniforms rectangle for h(z) ~ z^(lam-1) exp(-om/2 (z + 1/z))."""
    m = ((lam - 1.0) + math.sqrt((lam - 1.0) ** 2 + om * om)) / om

    def lh(z):  # log h(z) - log h(m)
        d = z - m
        return (lam - 1.0) * math.log1p(d / m) - 0.5 * om * d * (1.0 - 1.0 / (z * m))

    def F(z):  # derivative of ln|z - m| + lh(z)/2
        return 1.0 / (z - m) + 0.5 * ((lam - 1.0) / z - 0.5 * om * (1.0 - 1.0 / (z * z)))

    def bisect(lo, hi):  # F(lo) > 0 > F(hi), F decreasing
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if F(mid) > 0.0:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    step = m
    while F(m + step) > 0.0:
        step *= 2.0
    zp = bisect(m, m + step)
    lo = 0.5 * m
    while F(lo) < 0.0:
        lo *= 0.5
    zm = bisect(lo, m)
    vp = (zp - m) * math.exp(0.5 * lh(zp))
    vm = (zm - m) * math.exp(0.5 * lh(zm))
    return m, vm, vp, lh


def gig(p, A, B, seed, chain, draw, sub):
    """One draw from density ~ x^(p-1) exp(-(A x + B / x)/2); Philox stream 6.

    With omega = sqrt(A B): for p >= 0, x = sqrt(B/A) z, z ~ h(lam = p);
    for p < 0, x = sqrt(B/A) / z, z ~ h(lam = -p) (1/x is GIG(-p, B, A)).
    Attempt j uses block j: word 0 -> u in (0, 1], word 1 -> v in [v-, v+].
    """
    lam = abs(p)
    om = math.sqrt(A * B)
    m, vm, vp, lh = _gig_bounds(lam, om)
    for j in range(MAX_ATTEMPTS):
        wd = philox.words(seed, chain, philox.STREAM_GIG, draw, sub, [j])[0]
        u01 = philox.to_uniform(wd)
        u = u01[0]
        v = vm + (vp - vm) * u01[1]
        z = v / u + m
        if z <= 0.0:
            continue
        if math.log(u) <= 0.5 * lh(z):
            s = math.sqrt(B / A)
            return s * z if p >= 0 else s / z
    raise RuntimeError("gig: no acceptance")


# --------------------------------------------------------------------------- moments
def static_moments(R, counts):
    """Per subsample: S0 = sum R, B = sum N^2/R, N_obs (all over R > 0)."""
    out = []
    for l in range(R.shape[0]):
        obs = R[l] > 0
        out.append((float(R[l][obs].sum()), float((counts[l][obs] ** 2 / R[l][obs]).sum()),
                    int(obs.sum())))
    return out


def delta_moments(delta, R, counts):
    """Per subsample: S1 = sum R delta, S2 = sum R delta^2, T = sum N delta (R > 0)."""
    out = []
    for l in range(R.shape[0]):
        obs = R[l] > 0
        r, d = R[l][obs], delta[obs]
        out.append((float((r * d).sum()), float((r * d * d).sum()), float((counts[l][obs] * d).sum())))
    return out


def draw_nbar(stat, mom, bias, seed, chain, sweep):
    """New Nbar^l for every subsample (sub = l)."""
    out = []
    for l, ((S0, B, nobs), (S1, S2, T)) in enumerate(zip(stat, mom)):
        A = S0 + 2.0 * bias[l] * S1 + bias[l] ** 2 * S2
        out.append(gig(1.0 - 0.5 * nobs, A, B, seed, chain, sweep, l))
    return np.array(out)


def draw_bias(mom, nbar, bias_old, fixed_mask, seed, chain, sweep):
    """New b^l ~ N(D/C, 1/C) for subsamples not held fixed (sub = l)."""
    out = np.array(bias_old, dtype=np.float64)
    for l, (S1, S2, T) in enumerate(mom):
        if (fixed_mask >> l) & 1 or not S2 > 0:  # S2 = 0 (delta = 0): improper, keep b
            continue
        C = nbar[l] * S2
        D = T - nbar[l] * S1
        z = philox.normals(seed, chain, philox.STREAM_BIAS, sweep, 1, sub=l)[0]
        out[l] = D / C + z / math.sqrt(C)
    return out


# --------------------------------------------------------------------------- sweep
def sweep(state, data, cfg, s):
    """One block sweep.  state: dict(dk, pk, bias, nbar); returns the new state.

    cfg: n, box, nb, eps, nsteps, alpha_prior, seed, chain, fixed_mask, rj (bool),
    and, if rj, lam_lo / lam_hi bounds of the joint move; optional tau_mode (the
    step count of the sweep's trajectory and joint move drawn by hmc.draw_steps
    from the Philox stream of chain tau_chain, default this chain).
    """
    from . import rj
    n, box, nb = cfg["n"], cfg["box"], cfg["nb"]
    R, counts = data["R"], data["counts"]
    dk, pk, bias, nbar = state["dk"], state["pk"], state["bias"], state["nbar"]
    growth = data.get("growth")                 # per-voxel D+ (eq. data_model), or None
    post = hmc.make_posterior(n, box, nb, pk, R, counts, bias, nbar, cfg.get("workers", 1), growth)
    if cfg.get("tau_mode", False):
        cfg = dict(cfg, nsteps=hmc.draw_steps(cfg["nsteps"], cfg["seed"],
                                              cfg.get("tau_chain", cfg["chain"]), s))
    tr = hmc.trajectory(dk, post, cfg["eps"], cfg["nsteps"], cfg["seed"], cfg["chain"], s)
    dk = tr["state"]
    n_modes = grid.mode_counts(n, nb)
    sigma = grid.shell_sums(dk, nb)
    lam = model.lambdas(pk, n, box)
    lam = draw_power(sigma, n_modes, lam, cfg["alpha_prior"], cfg["seed"], cfg["chain"], s)
    out = dict(dH=tr["dH"], accepted=tr["accepted"], log_u=tr["log_u"], sigma=sigma)
    if cfg.get("rj", False):
        jm = rj.joint_move(dk, lam, post, n_modes, cfg, s)
        dk, lam = jm["dk"], jm["lam"]
        out.update(rj_dH=jm["dH"], rj_accepted=jm["accepted"], rj_wall_hits=jm["wall_hits"],
                   rj_log_u=jm["log_u"])
    delta = grid.inv(dk, n)
    stat = static_moments(R, counts)
    mom = delta_moments(delta if growth is None else np.asarray(growth, np.float64) * delta, R, counts)
    nbar = draw_nbar(stat, mom, bias, cfg["seed"], cfg["chain"], s)
    bias = draw_bias(mom, nbar, bias, cfg["fixed_mask"], cfg["seed"], cfg["chain"], s)
    out.update(dk=dk, pk=lam * box ** 3 / n ** 3, bias=bias, nbar=nbar)
    return out
