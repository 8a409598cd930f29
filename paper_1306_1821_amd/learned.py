"""Learned warm start and mass for the density sampler.

The paper notes that the HMC mass only changes efficiency, not correctness
(text after eq. Mass_matrix), and that a start near the posterior shortens the
burn-in it studies (Sec. "Testing burn-in and statistical efficiency").  Here a
small 3-D CNN (include/cnn.h) predicts, per voxel, the posterior mean mu and
log-variance log v of the density from three survey fields: the data
combination beta of the force normalised by sum_l b_l^2 Nbar_l, the angular
mask and the radial selection.  mu becomes the starting state, log v the
real-space factor of the mass (hmc_set_mass); the Metropolis test still judges
every trajectory, so the chain's target is unchanged.

Training pairs come from the plain sampler itself: chains on seeded mocks,
started from each mock's truth field (drawn from the prior that the sampler
uses, so truth and data together are a draw from the joint distribution and
the truth is already a posterior draw), thinned, each sample paired with its
survey's input fields.  Training runs on the device with the library's own
forward/backward kernels and Adam.  All arrays stay on the GPU; this module
only orders the calls.
"""
import dataclasses
import time

import numpy as np

from . import diagnostics
from .binding import CNN_LAYERS, Sampler


def init_params(seed=0):
    """Initial network weights: uniform in +-sqrt(6 / fan_in), fan_in = 27 C_in
    (He et al. 2015, uniform form), zero biases; flat float32 in the layout of
    include/cnn.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        lim = np.sqrt(6.0 / (27 * ci))
        parts += [rng.uniform(-lim, lim, 27 * ci * co), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def beta_scale(bias, nbar):
    """1 / sum_l b_l^2 Nbar_l: beta times this is about R delta plus noise."""
    return 1.0 / float(np.sum(np.asarray(bias) ** 2 * np.asarray(nbar)))


def chain_from_mock(mk, **kw):
    cfg = mk["cfg"]
    spec = dict(n=cfg.n, box=cfg.box, nb=cfg.nb, R=mk["R"], counts=mk["counts"],
                bias=mk["bias"], nbar=mk["nbar"], pk=mk["pk_init"], fixed_mask=cfg.fixed_mask,
                nsteps=cfg.nsteps, eps=cfg.eps, rj=cfg.rj)
    spec.update(kw)
    return spec


def survey_inputs(net, sampler, chain, mk):
    """Network inputs of a survey from the sampler's beta (call before any sweep:
    sweeps redraw b and Nbar and with them beta)."""
    t = sampler.tensors(chain)
    return net.features(t["beta"], beta_scale(mk["bias"], mk["nbar"]), mk["mask"], mk["sel"])


def mock_series(cfg, seeds, dtype=np.float32):
    """Seeded mocks sharing one survey geometry."""
    from synth import make_mock, mask_and_selection
    geom = mask_and_selection(cfg)
    return [make_mock(dataclasses.replace(cfg, seed=int(s)), dtype=dtype, geometry=geom)
            for s in seeds]


def tune_step(sampler, eps0, target=0.8, rounds=5, trajs=8, first_index=3 << 30):
    """Common step size for all chains of `sampler` with acceptance near target.

    Runs bare trajectories (no Gibbs blocks) from the current states, with draw
    indices (32-bit) far from those of the sweeps, and rescales eps by the acceptance
    ratio.  Returns (eps, last acceptance rate)."""
    eps, idx, rate = float(eps0), int(first_index), 0.0
    for _ in range(rounds):
        sampler.set_step(None, eps)
        acc = []
        for _ in range(trajs):
            _, a = sampler.trajectory(idx)
            idx += 1
            acc.append(a)
        rate = float(np.mean(acc))
        eps *= float(np.clip(np.exp(1.5 * (rate - target)), 0.5, 1.5))
    sampler.set_step(None, eps)
    return eps, rate


def make_training_set(net, mocks, per_batch=8, burn=10, samples=31, thin=4, seed=7, eps=None,
                      log=None):
    """Plain-sampler draws on each mock: returns (inputs [n_mocks] device tensors,
    targets [n_samples] device tensors, owner index per target)."""
    inputs, targets, owner = [], [], []
    for b0 in range(0, len(mocks), per_batch):
        t0 = time.time()
        group = mocks[b0:b0 + per_batch]
        s = Sampler([chain_from_mock(mk, seed=seed, chain_id=b0 + i) for i, mk in enumerate(group)])
        for i, mk in enumerate(group):
            inputs.append(survey_inputs(net, s, i, mk))
            s.set_state(i, mk["delta"])
        if eps is not None:
            s.set_step(None, eps)
        s.use_graph(True)
        sweep, acc = 0, []
        for _ in range(burn):
            s.sweep(sweep)
            sweep += 1
        for _ in range(samples):
            for _ in range(thin):
                acc += [st["accepted"] for st in s.sweep(sweep)]
                sweep += 1
            for i in range(len(group)):
                targets.append(s.tensors(i)["delta_r"].clone())
                owner.append(b0 + i)
        s.close()
        if log:
            log(f"training draws: mocks {b0}..{b0 + len(group) - 1}, {sweep} sweeps, "
                f"acceptance {np.mean(acc):.2f}, {time.time() - t0:.1f} s")
    return inputs, targets, np.asarray(owner)


def train(net, inputs, targets, owner, steps, lr=2e-3, lr_min=1e-4, warmup=50, seed=0,
          log=None, log_every=200):
    """Adam on the per-voxel Gaussian loss, one (inputs, draw) pair per step,
    cosine learning-rate decay after a linear warm-up.  Returns the loss trace."""
    rng = np.random.default_rng(seed)
    order = np.concatenate([rng.permutation(len(targets)) for _ in range(steps // len(targets) + 1)])
    losses = np.empty(steps)
    t0 = time.time()
    for it in range(steps):
        j = order[it]
        if it < warmup:
            r = lr * (it + 1) / warmup
        else:
            r = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * (it - warmup) / max(1, steps - warmup)))
        losses[it] = net.train_step(inputs[owner[j]], targets[j], r)
        if log and (it + 1) % log_every == 0:
            log(f"train step {it + 1}/{steps}: loss {losses[max(0, it - log_every + 1):it + 1].mean():.4f}"
                f" ({time.time() - t0:.1f} s)")
    return losses


def held_out_loss(net, inputs, targets, owner):
    """Mean loss over (inputs, draw) pairs without updating the network."""
    return float(np.mean([net.gradient(inputs[owner[j]], targets[j])[1] for j in range(len(targets))]))


def burn_in_length(trace, lo, hi, hold=10):
    """First index after which `trace` stays inside [lo, hi] for `hold` samples."""
    inside = (np.asarray(trace) >= lo) & (np.asarray(trace) <= hi)
    for s in range(len(inside) - hold + 1):
        if inside[s:s + hold].all():
            return s
    return len(inside)


def pk_log_bias(pk_trace, pk_true):
    """Mean over shells of ln(P_s / P_true) per sample (a scalar burn-in statistic,
    the logarithmic form of xi of eq. BURN_IN averaged over shells)."""
    return np.mean(np.log(np.asarray(pk_trace) / np.asarray(pk_true)[None, :]), axis=1)


def run_chains(sampler, sweeps, first_sweep=0, energies=False):
    """Gibbs sweeps; returns P traces [chains][sweeps][nb], acceptance, wall seconds
    and (optionally) the potential prior + data per sweep [chains][sweeps]."""
    k = len(sampler.chains)
    pk = [[] for _ in range(k)]
    pot = [[] for _ in range(k)]
    acc = []
    t0 = time.time()
    for s in range(first_sweep, first_sweep + sweeps):
        st = sampler.sweep(s)
        acc.append([x["accepted"] for x in st])
        for i in range(k):
            pk[i].append(st[i]["pk"])
            if energies:
                e = sampler.hamiltonian(i)
                pot[i].append(e[1] + e[2])
    wall = time.time() - t0
    return np.asarray(pk), np.asarray(acc, dtype=float), wall, np.asarray(pot)


def pk_ess_summary(pk, wall):
    """Per-shell bulk ESS, ESS/s and split R-hat of the P traces [chains][sweeps][nb]."""
    nb = pk.shape[2]
    ess = np.array([diagnostics.ess_bulk(np.log(pk[:, :, m])) for m in range(nb)])
    rhat = np.array([diagnostics.split_rhat(np.log(pk[:, :, m])) for m in range(nb)])
    return dict(ess=ess, ess_per_s=ess / wall, rhat=rhat, wall=wall)


def ess_table(r, shells=None):
    """Median / min ESS/s and max split R-hat over the given shells (all if None)."""
    sel = np.arange(len(r["ess"])) if shells is None else np.asarray(shells)
    return dict(median_ess_per_s=float(np.median(r["ess_per_s"][sel])),
                min_ess_per_s=float(r["ess_per_s"][sel].min()),
                max_rhat=float(r["rhat"][sel].max()),
                shells_rhat_below_1_01=int((r["rhat"][sel] < 1.01).sum()), shells=int(sel.size))


def warm_up(sampler, trajs, first_index=2 << 30):
    """Bare trajectories under the starting P, b and Nbar before the first sweep:
    the density settles given the spectrum before P is first redrawn from it
    (a start with too little power, such as a posterior mean, would otherwise
    pull the first P draws far down)."""
    for i in range(trajs):
        sampler.trajectory(first_index + i)


def start_chains(mk, n_chains, start=None, mu=None, lv=None, mass=None, eps=None, seed=11,
                 graph=True, mass_kind="learned"):
    """A sampler with n_chains chains on mock mk (chain ids 0..n-1, shared seed).

    start: None (delta = 0), "mean" (delta = mu) or "draw" (hmc_warm_start from
    mu and lv, draw index = chain id, so chains start apart); mass: log-variance
    field of the learned mass for every chain (None: the plain mass); mass_kind:
    "learned" or "diagonal" (the real-space diagonal variant)."""
    s = Sampler([chain_from_mock(mk, seed=seed, chain_id=i, **({} if eps is None else dict(eps=eps)))
                 for i in range(n_chains)])
    for i in range(n_chains):
        if start == "mean":
            s.set_state(i, mu)
        elif start == "draw":
            s.warm_start(i, mu, lv, draw_index=i)
    if mass is not None:
        s.set_mass(None, mass, kind=mass_kind)
    s.use_graph(graph)
    return s


BURN_RUNS = [("truth", "truth", False), ("zero", None, False), ("mean", "mean", False),
             ("warm", "draw", False), ("warm+mass", "draw", True)]


def data_dominated_shells(mk):
    """Shells whose prior variance times the mean data precision exceeds one
    (lambda_m mean(alpha) > 1: on average the data, not the prior, fix those
    modes, so their P is constrained; P of the others can drift far under the
    1/P prior)."""
    cfg = mk["cfg"]
    R = np.asarray(mk["R"], np.float64)
    abar = float(np.mean(sum(b * b * nb * (R[l] > 0) * R[l]
                             for l, (b, nb) in enumerate(zip(mk["bias"], mk["nbar"])))))
    lam = np.asarray(mk["pk_init"]) * cfg.n ** 3 / cfg.box ** 3
    return np.nonzero(lam * abar > 1.0)[0]


def burn_in_study(mk, mu, lv, sweeps=300, warm_trajs=0, eps=(None, None), seed=11,
                  runs=BURN_RUNS, log=None):
    """One chain per start on the same random numbers.  The reference run starts
    at the mock's truth field, itself a posterior draw (the truth was drawn from
    the prior the sampler uses), so its trace is stationary from the first
    sweep; the others start at delta = 0 (the paper's method), delta = mu, the
    warm start from (mu, lv), and the warm start with the learned mass.

    Statistics per sweep: the potential (prior + data) and the mean ln(P / P0)
    over the data-dominated shells.  Burn-in of a run: the first sweep after
    which its trace stays 10 sweeps in the reference's mean +- 3 sd."""
    shells = data_dominated_shells(mk)
    if shells.size == 0:
        shells = np.arange(mk["cfg"].nb)
    out = {}
    for name, start, learned_mass in runs:
        if start == "truth":
            s = start_chains(mk, 1, "mean", mk["delta"], None, None, eps[0], seed)
        else:
            s = start_chains(mk, 1, start, mu, lv, lv if learned_mass else None,
                             eps[1] if learned_mass else eps[0], seed)
        e0 = s.hamiltonian(0)
        warm_up(s, warm_trajs)
        pk, acc, wall, pot = run_chains(s, sweeps, energies=True)
        s.close()
        first = np.nonzero(acc[:, 0] > 0)[0]
        out[name] = dict(pot=pot[0], logbias=pk_log_bias(pk[0][:, shells], mk["pk_init"][shells]),
                         start_potential=e0[1] + e0[2], acceptance=float(acc.mean()), wall=wall,
                         first_accept=int(first[0]) if first.size else sweeps)
    ref = out.get("truth")
    for key in ("pot", "logbias"):
        base = ref[key] if ref is not None else np.concatenate([r[key][sweeps // 2:] for r in out.values()])
        lo, hi = base.mean() - 3 * base.std(), base.mean() + 3 * base.std()
        for name, r in out.items():
            r["burn_" + key] = burn_in_length(r[key], lo, hi)
    if log:
        log(f"burn-in statistics over {shells.size} data-dominated shells")
        for name, r in out.items():
            log(f"burn-in {name}: potential {r['burn_pot']} sweeps, ln P bias {r['burn_logbias']} "
                f"sweeps, first accepted trajectory {r['first_accept']}; start potential "
                f"{r['start_potential']:.6g}, first {np.round(r['pot'][:3], 0)}, tail "
                f"{r['pot'][sweeps // 2:].mean():.6g}; ln P bias first {np.round(r['logbias'][:3], 3)} "
                f"tail {r['logbias'][sweeps // 2:].mean():.3f}; acceptance {r['acceptance']:.2f}")
    return out


def ess_study(mk, mu, lv, chains=4, burn=100, sweeps=600, target=0.8, eps0=None, seed=21,
              log=None):
    """P(k) efficiency of the plain mass, the learned mass and its real-space diagonal
    variant: `chains` chains each,
    warm-started from (mu, lv) with different draws, step size tuned to the
    same acceptance, `burn` sweeps dropped, then ESS, ESS/s and split R-hat of
    ln P per shell."""
    out = {}
    for name, mass, kind in [("plain", None, "learned"), ("learned", lv, "learned"),
                             ("diagonal", lv, "diagonal")]:
        s = start_chains(mk, chains, "draw", mu, lv, mass, eps0, seed, mass_kind=kind)
        # the diagonal variant lacks the Fourier preconditioning: its step can be far
        # smaller, so it gets more tuning rounds (each moves eps by at most 2x)
        eps, rate = tune_step(s, eps0 if eps0 is not None else mk["cfg"].eps, target=target,
                              rounds=10 if kind == "diagonal" else 5)
        for i in range(chains):          # tuning moved the states: start again
            s.warm_start(i, mu, lv, draw_index=i)
        run_chains(s, burn)
        pk, acc, wall, _ = run_chains(s, sweeps, first_sweep=burn)
        s.close()
        r = pk_ess_summary(pk, wall)
        r.update(eps=eps, tune_acceptance=rate, acceptance=float(acc.mean()),
                 ms_per_sweep=1e3 * wall / sweeps)
        out[name] = r
        if log:
            dd = ess_table(r, data_dominated_shells(mk))
            log(f"ESS {name}: eps {eps:.4f}, acceptance {r['acceptance']:.2f}, {r['ms_per_sweep']:.1f} "
                f"ms/sweep; ESS/s median {np.median(r['ess_per_s']):.3g} min {r['ess_per_s'].min():.3g}; "
                f"R-hat max {r['rhat'].max():.3f}, shells with R-hat < 1.01: "
                f"{int((r['rhat'] < 1.01).sum())}/{len(r['rhat'])}; data-dominated shells: {dd}")
    return out



def equal_rhat_study(mk, mu, lv, shells, chains=4, burn=200, block=500, max_seconds=600.0,
                     rhat_target=1.01, target=0.8, eps0=None, seed=21, log=None,
                     arms=(("plain", False), ("learned", True))):
    """P(k) efficiency of the plain and the learned mass at equal convergence.

    Each arm: `chains` chains warm-started from (mu, lv) with different draws, eps
    tuned to the same acceptance, `burn` sweeps dropped, then blocks of `block`
    sweeps until the rank-normalised split R-hat of ln P is below `rhat_target` on
    every shell in `shells` over the whole window after burn-in, or `max_seconds`
    of sampling have passed.  ESS/s is the bulk ESS of that window over its wall
    time (Sec. "Testing burn-in and statistical efficiency" measures efficiency by
    the autocorrelation of eq. CORR_COEFF; the bulk ESS sums it).  An arm that
    does not reach the target reports the R-hat it reached and the sweeps the
    target would take, from R-hat - 1 falling as 1 / ESS, i.e. as 1 / sweeps."""
    shells = np.asarray(shells)
    out = {}
    for name, learned_mass in arms:
        s = start_chains(mk, chains, "draw", mu, lv, lv if learned_mass else None, eps0, seed)
        # ten rounds of 16 trajectories: both arms end near the target acceptance
        eps, rate = tune_step(s, eps0 if eps0 is not None else mk["cfg"].eps, target=target,
                              rounds=10, trajs=16)
        for i in range(chains):
            s.warm_start(i, mu, lv, draw_index=i)
        run_chains(s, burn)
        parts, accs, wall, sweeps, history = [], [], 0.0, 0, []
        while True:
            pk, acc, w, _ = run_chains(s, block, first_sweep=burn + sweeps)
            parts.append(pk)
            accs.append(acc)
            wall += w
            sweeps += block
            trace = np.concatenate(parts, axis=1)
            rh = np.array([diagnostics.split_rhat(np.log(trace[:, :, m])) for m in shells])
            history.append((sweeps, float(rh.max())))
            if log:
                log(f"{name}: {sweeps} sweeps, {wall:.0f} s, max split R-hat {rh.max():.4f}")
            if rh.max() < rhat_target or wall > max_seconds:
                break
        s.close()
        r = pk_ess_summary(trace, wall)
        reached = bool(rh.max() < rhat_target)
        need = sweeps if reached else int(np.ceil(sweeps * (rh.max() - 1.0) / (rhat_target - 1.0)))
        r.update(eps=eps, tune_acceptance=rate, acceptance=float(np.concatenate(accs).mean()),
                 ms_per_sweep=1e3 * wall / sweeps, sweeps=sweeps, reached=reached,
                 max_rhat=float(rh.max()), sweeps_to_target=need,
                 seconds_to_target=need * wall / sweeps, history=history)
        out[name] = r
        if log:
            t = ess_table(r, shells)
            log(f"{name}: eps {eps:.4f}, acceptance {r['acceptance']:.2f}, {r['ms_per_sweep']:.1f} ms/sweep, "
                f"R-hat {r['max_rhat']:.4f} after {sweeps} sweeps ({'reached' if reached else 'not reached'}; "
                f"target at ~{need} sweeps), ESS/s median {t['median_ess_per_s']:.3g} min {t['min_ess_per_s']:.3g}")
    return out
