#!/usr/bin/env python
"""Leapfrog steps/s of the HMC density sampler on one MI355X.

A bench step is one full block sweep of the sampler (density HMC trajectory,
P draw, joint (P, delta) move, Nbar and bias draws, coefficient and gradient
refresh) on the 256^3 survey workload (L = 1500 Mpc/h, 6 subsamples, 60
k-shells, 30 leapfrog steps).  `value` counts the density-HMC leapfrog steps
completed per second of whole sweeps, inputs resident in HBM.

The JSON line also carries:
  roofline      the k-space step pass (kick, drift and both x transforms), its
                average device duration measured with HIP events on the
                library's stream during the timed sweeps, against 8 TB/s;
  cpu_baseline  the float64 CPU oracle timed on this host on a bounded sample
                of the same workload (a few leapfrog steps).

--workload cfg4 times the batched pattern instead: 16 independent chains (8 at
64^3, 6 at 128^3, 2 at 192^3, each with its own mask seed and 2-4 subsamples)
advancing together, sweeps replayed from a captured HIP graph, launch shapes
from the autotuner (one fused launch over all chains per stage, or one launch
per grid size, whichever it measures faster); `value` is chain leapfrog steps per second and the line
also gives the 256^3-equivalent rate (voxel updates / 256^3) and split R-hat of
ln P(k) across same-size chains over the timed sweeps.

--learned runs the learned warm start / mass comparison instead: the network
is trained on plain-sampler draws from 64 seeded 128^3 mocks (four subsamples,
40 shells), applied to the 256^3 survey, and the line reports P(k) ESS/s with
the learned and the plain mass (4 chains each, equal acceptance) and the
burn-in lengths of the warm start and of delta = 0.

--oracle-timing times the float64 oracle (the CPU baseline) against the GPU per
leapfrog step at 32^3, 128^3 and 256^3, and the P(k) ESS/s of both at 32^3.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_bench_256.md")
KERNELS_SRC = os.path.join(ROOT, "paper_1306_1821_amd", "csrc", "kernels.hip")


def measured_traffic(kind="x-step"):
    """HBM bytes per launch of the k-space step pass (kind "x-step") or of the y-z
    plane pass ("plane") from the committed FETCH_SIZE / WRITE_SIZE summary, or None
    when the kernel source has changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    b = re.search(re.escape(kind) + r" traffic per launch \(bytes\): (\d+)", text)
    h = re.search(r"kernels.hip sha256: ([0-9a-f]{64})", text)
    if not b or not h:
        return None
    if hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest() != h.group(1):
        return None
    return int(b.group(1))


def workload_spec(name, eps):
    from synth import CONFIGS, make_mock
    mk = make_mock(CONFIGS[name], dtype=np.float32)
    cfg = mk["cfg"]
    spec = dict(n=cfg.n, box=cfg.box, nb=cfg.nb, R=mk["R"], counts=mk["counts"], bias=mk["bias"],
                nbar=mk["nbar"], pk=mk["pk_init"], fixed_mask=cfg.fixed_mask, nsteps=cfg.nsteps,
                eps=cfg.eps if eps is None else eps, rj=cfg.rj, seed=2013, chain_id=0)
    return mk, spec


def cpu_baseline(mk, spec, budget_s):
    """Oracle leapfrog steps/s (float64, scipy.fft on all host cores)."""
    from oracle import grid, hmc
    workers = os.cpu_count() or 1
    R = mk["R"].astype(np.float64)
    C = mk["counts"].astype(np.float64)
    post = hmc.make_posterior(spec["n"], spec["box"], spec["nb"], spec["pk"], R, C, spec["bias"],
                              spec["nbar"], workers=workers)
    dk = grid.fwd(mk["delta"].astype(np.float64), workers)
    dk[0, 0, 0] = 0
    pk = hmc.draw_momentum(post, spec["seed"], 0, 0)
    t0 = time.perf_counter()
    hmc.leapfrog(dk, pk, post, spec["eps"], 1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(60, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    hmc.leapfrog(dk, pk, post, spec["eps"], steps)
    dt = time.perf_counter() - t0
    return dict(value=steps / dt, unit="leapfrog steps/s", cores=workers, kind="oracle",
                sample=f"{steps} float64 KDK leapfrog steps (one gradient evaluation each) of the "
                       f"{spec['n']}^3 workload, scipy.fft workers={workers}, {dt:.1f} s")


def oracle_step_ms(mk, spec, workers, reps=5):
    """Median host time of one float64 KDK leapfrog step of the oracle (a drift, a
    gradient evaluation, a kick): each repetition times the integrator with three
    steps and with one, and takes half the difference."""
    from oracle import grid, hmc
    post = hmc.make_posterior(spec["n"], spec["box"], spec["nb"], spec["pk"],
                              mk["R"].astype(np.float64), mk["counts"].astype(np.float64),
                              spec["bias"], spec["nbar"], workers=workers)
    dk = grid.fwd(mk["delta"].astype(np.float64), workers)
    dk[0, 0, 0] = 0
    pk = hmc.draw_momentum(post, spec["seed"], 0, 0)
    hmc.leapfrog(dk, pk, post, spec["eps"], 1)          # warm-up
    per = []
    for _ in range(reps):
        t0 = time.perf_counter()
        hmc.leapfrog(dk, pk, post, spec["eps"], 1)
        t1 = time.perf_counter()
        hmc.leapfrog(dk, pk, post, spec["eps"], 3)
        t2 = time.perf_counter()
        per.append(0.5 * ((t2 - t1) - (t1 - t0)))
    return 1e3 * float(np.median(per))


def gpu_step_ms(mk, spec, ntraj=20):
    """Wall time per leapfrog step of bare trajectories, and the summed device
    time of one step's passes from HIP events: the k-space pass, the y-z plane
    pass (or the real-space pass) and the y passes in the number launched per
    gradient (two in the four-pass form; with the plane pass only the momentum
    draw's one per trajectory, spread over its steps)."""
    import torch
    from paper_1306_1821_amd.binding import Sampler
    s = Sampler([spec])
    s.set_state(0, mk["delta"])
    for i in range(3):
        s.trajectory(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(ntraj):
        s.trajectory(100 + i)
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t0) / (ntraj * spec["nsteps"])
    s.timing(1)
    for i in range(3):
        s.trajectory(1000 + i)
    ms, launches = s.timing(0)
    s.close()
    per = [ms[j] / max(1, launches[j]) for j in range(3)]
    return wall, per[0] + per[1] * launches[1] / max(1, launches[2]) + per[2]


def oracle_timing_main(args):
    """Oracle against HIP path per grid size (32^3, 128^3, 256^3 survey workloads):
    float64 leapfrog step time on all host threads and on one, the GPU's per-step
    wall and kernel time; then P(k) ESS/s of the 32^3 workload, 4 chains from
    delta = 0, oracle sweeps against GPU sweeps with the same seeds."""
    import torch
    from oracle import gibbs, grid
    from paper_1306_1821_amd import diagnostics
    from paper_1306_1821_amd.binding import Sampler
    workers = os.cpu_count() or 1
    rows = []
    for name in ("cfg1", "cfg2", "cfg3"):
        mk, spec = workload_spec(name, args.eps if name == "cfg3" else None)
        wall, kern = gpu_step_ms(mk, spec)
        row = dict(workload=name, n=spec["n"], subsamples=len(spec["bias"]),
                   gpu_ms_per_step_wall=wall, gpu_ms_per_step_kernels=kern,
                   oracle_ms_per_step={str(workers): oracle_step_ms(mk, spec, workers),
                                       "1": oracle_step_ms(mk, spec, 1)})
        row["speedup_vs_oracle_all_threads"] = row["oracle_ms_per_step"][str(workers)] / wall
        print(f"[oracle-timing] {json.dumps(row)}", file=sys.stderr, flush=True)
        rows.append(row)
        torch.cuda.empty_cache()

    # P(k) ESS/s at 32^3: same chains (seed, chain ids, start) on both sides
    mk, spec = workload_spec("cfg1", None)
    m, S = 4, args.oracle_sweeps
    c = mk["cfg"]
    specs = [dict(spec, chain_id=i) for i in range(m)]
    s = Sampler(specs)
    traces_g = np.zeros((m, S, spec["nb"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sw in range(S):
        for i, st in enumerate(s.sweep(sw)):
            traces_g[i, sw] = st["pk"]
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    s.close()
    data = dict(R=mk["R"].astype(np.float64), counts=mk["counts"].astype(np.float64))
    traces_o = np.zeros_like(traces_g)
    t0 = time.perf_counter()
    for i in range(m):
        ocfg = dict(n=c.n, box=c.box, nb=c.nb, eps=spec["eps"], nsteps=spec["nsteps"],
                    alpha_prior=1.0, seed=spec["seed"], chain=i, fixed_mask=c.fixed_mask,
                    rj=spec["rj"], workers=1)
        state = dict(dk=grid.fwd(np.zeros((c.n,) * 3)), pk=np.array(spec["pk"], np.float64),
                     bias=np.array(spec["bias"], np.float64), nbar=np.array(spec["nbar"], np.float64))
        for sw in range(S):
            o = gibbs.sweep(state, data, ocfg, sw)
            state = dict(dk=o["dk"], pk=o["pk"], bias=o["bias"], nbar=o["nbar"])
            traces_o[i, sw] = o["pk"]
    t_orc = time.perf_counter() - t0

    def summary(tr, t):
        w = np.log(tr[:, S // 2:])                      # second half: past burn-in
        ess = np.array([diagnostics.ess_bulk(w[:, :, b]) for b in range(w.shape[2])])
        rh = np.array([diagnostics.split_rhat(w[:, :, b]) for b in range(w.shape[2])])
        return dict(seconds=t, ms_per_sweep=1e3 * t / S, ess_median=float(np.median(ess)),
                    ess_min=float(ess.min()), ess_per_s_median=float(np.median(ess)) / (t / 2),
                    max_split_rhat=float(rh.max()))
    out = dict(study="oracle_timing", host_threads=workers, rows=rows,
               cfg1_ess=dict(chains=m, sweeps=S, window="second half of every chain",
                             max_abs_dlnP=float(np.abs(np.log(traces_g) - np.log(traces_o)).max()),
                             gpu=summary(traces_g, t_gpu), oracle_one_thread=summary(traces_o, t_orc)))
    print(json.dumps(out), flush=True)


BATCH_GROUPS = [("grp64", 8), ("grp128", 6), ("grp192", 2)]


def batched_main(args):
    import dataclasses

    import torch
    from paper_1306_1821_amd import diagnostics
    from paper_1306_1821_amd.binding import Sampler
    from synth import CONFIGS, make_mock

    # one survey (own mask seed) per grid size; the chains of a size sample its
    # posterior independently (own chain ids), so R-hat across them is meaningful
    specs, owner, vox, mocks = [], [], 0, {}
    for gi, (name, count) in enumerate(BATCH_GROUPS):
        cfg = dataclasses.replace(CONFIGS[name], seed=100 + gi, mask_seed=gi)
        mk = mocks[name] = make_mock(cfg, dtype=np.float32)
        for j in range(count):
            specs.append(dict(n=cfg.n, box=cfg.box, nb=cfg.nb, R=mk["R"], counts=mk["counts"],
                              bias=mk["bias"], nbar=mk["nbar"], pk=mk["pk_init"],
                              fixed_mask=cfg.fixed_mask, nsteps=cfg.nsteps, eps=args.eps_batch,
                              rj=True, seed=2013, chain_id=len(specs)))
            owner.append(name)
            vox += cfg.n ** 3
    print(f"[bench] cfg4: {len(specs)} chains, {vox / 1e6:.1f} M voxels", file=sys.stderr,
          flush=True)
    s = Sampler(specs)
    for i, name in enumerate(owner):
        s.set_state(i, mocks[name]["delta"])     # the truth: a posterior draw
    sweep = 0
    for _ in range(args.warmup):
        s.sweep(sweep)
        sweep += 1
    chosen = s.autotune(10)
    plans = s.launch_config()[1]
    s.use_graph(True)
    s.sweep(sweep)                       # capture
    sweep += 1
    torch.cuda.synchronize()
    acc, traces = [], [[] for _ in specs]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = s.sweep(sweep)
        sweep += 1
        acc.append([o["accepted"] for o in out])
        for i, o in enumerate(out):
            traces[i].append(np.log(o["pk"]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nsteps = specs[0]["nsteps"]
    # convergence across same-size chains: continue (untimed) to --rhat-sweeps sweeps
    for _ in range(max(0, args.rhat_sweeps - args.steps)):
        for i, o in enumerate(s.sweep(sweep)):
            traces[i].append(np.log(o["pk"]))
        sweep += 1
    from paper_1306_1821_amd.learned import data_dominated_shells
    rhat = {}
    for name, count in BATCH_GROUPS:
        t = np.array([traces[i] for i, o in enumerate(owner) if o == name])
        t = t[:, t.shape[1] // 5:]                  # first fifth dropped
        dd = data_dominated_shells(mocks[name])
        rhat[name] = {"all_shells_max": float(max(diagnostics.split_rhat(t[:, :, m])
                                                  for m in range(t.shape[2]))),
                      "data_dominated_max": float(max(diagnostics.split_rhat(t[:, :, m])
                                                      for m in dd)),
                      "data_dominated_shells": int(len(dd)), "chains": count,
                      "sweeps": int(t.shape[1])}
    s.close()
    value = len(specs) * args.steps * nsteps / dt
    out = {
        "metric": "leapfrog steps/s, batched chains (16 chains: 8x64^3, 6x128^3, 2x192^3)",
        "value": value, "unit": "chain leapfrog steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cfg4: 16 independent chains advancing together, "
                               "8 at 64^3 (2 subsamples), 6 at 128^3 (4), 2 at 192^3 (3), one "
                               "survey (own mask seed) per size, 30 leapfrog steps, joint move "
                               "on; one step = one sweep of every chain", "eps": args.eps_batch},
        "voxels": vox,
        "equivalent_256_steps_per_s": value / len(specs) * vox / 256 ** 3,
        "launch_grids": chosen,
        "radix_plans": plans,
        "acceptance": float(np.mean(acc)),
        "split_rhat_lnP": rhat,
    }
    print(json.dumps(out), flush=True)


def ablation_main(args):
    """Joint-move ablation: P(k) correlation of the 128^3 survey workload with and
    without the joint (P, delta) move."""
    from synth import CONFIGS, make_mock
    from paper_1306_1821_amd import studies
    from paper_1306_1821_amd.learned import data_dominated_shells
    log = lambda m: print(f"[ablation] {m}", file=sys.stderr, flush=True)
    mk = make_mock(CONFIGS["cfg2"], dtype=np.float32)
    sweeps = 3000 if args.steps == 20 else args.steps
    r = studies.joint_move_ablation(mk, chains=4, burn=100, sweeps=sweeps, log=log)
    dd = data_dominated_shells(mk)
    j, nj = r["joint"], r["no_joint"]
    summ = lambda x: dict(acceptance=x["acceptance"], ms_per_sweep=x["ms_per_sweep"],
                          corr_len_median=float(np.median(x["corr_len"])),
                          corr_len_median_data_dominated=float(np.median(x["corr_len"][dd])),
                          autocorr_median={str(l): float(v) for l, v in
                                           zip(x["lags"], np.median(x["autocorr"], axis=0))},
                          autocorr_median_data_dominated={str(l): float(v) for l, v in
                                                          zip(x["lags"], np.median(x["autocorr"][dd], axis=0))},
                          ess_per_s_median_data_dominated=float(np.median(x["ess_per_s"][dd])))
    value = float(np.median(nj["corr_len"]) / max(1.0, np.median(j["corr_len"])))
    out = {"metric": "P(k) correlation-length ratio without / with the joint move (128^3, median over shells)",
           "value": value, "unit": "ratio", "n_gpus": 1, "steps": sweeps, "warmup": 100,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "cfg2: 128^3 grid, L=1000 Mpc/h, 4 subsamples, 40 shells; 4 chains "
                                  "from the truth field per mode, one step = one sweep"},
           "joint": summ(j), "no_joint": summ(nj), "data_dominated_shells": int(len(dd))}
    print(json.dumps(out), flush=True)


def posterior_main(args):
    """Posterior structure on the 128^3 survey workload (correlations, bands, maps)."""
    from synth import CONFIGS, make_mock
    from paper_1306_1821_amd import studies
    log = lambda m: print(f"[posterior] {m}", file=sys.stderr, flush=True)
    mk = make_mock(CONFIGS["cfg2"], dtype=np.float32)
    sweeps = 2000 if args.steps == 20 else args.steps
    t0 = time.perf_counter()
    r = studies.posterior_analysis(mk, chains=4, burn=100, sweeps=sweeps, log=log)
    dt = time.perf_counter() - t0
    out = {"metric": "posterior analysis at 128^3 (P-P, b-P, Nbar-P correlations; P(k) bands; density maps)",
           "value": r["band_covers_truth"], "unit": "fraction of shells whose 68% band covers the truth",
           "n_gpus": 1, "steps": sweeps, "warmup": 100, "ms_per_step": 1e3 * dt / (sweeps + 100),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "cfg2: 128^3 grid, L=1000 Mpc/h, 4 subsamples, 40 shells; 4 chains "
                                  "from the truth field, field moments pooled on the device"}}
    out.update({k: v for k, v in r.items() if k not in ("pk_mean", "pk_band_16_84", "pk_truth")})
    print(json.dumps(out), flush=True)


def learned_main(args):
    import torch
    from paper_1306_1821_amd import learned
    from paper_1306_1821_amd.binding import CNN
    from synth import CONFIGS, make_mock

    log = lambda m: print(f"[learned] {m}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    net = CNN(learned.init_params(3))
    mocks = learned.mock_series(CONFIGS["cfg2"], range(100, 100 + args.mocks))
    ins, tg, own = learned.make_training_set(net, mocks, per_batch=8, burn=20, samples=31, thin=8,
                                             eps=0.035, log=log)
    del mocks
    t_draws = time.perf_counter() - t0
    losses = learned.train(net, ins, tg, own, args.train_steps, lr=2e-3, log=log, log_every=1000)
    t_train = time.perf_counter() - t0 - t_draws
    del ins, tg
    torch.cuda.empty_cache()
    mk = make_mock(CONFIGS["cfg3"], dtype=np.float32)
    s = learned.start_chains(mk, 1)
    x = learned.survey_inputs(net, s, 0, mk)
    s.close()
    mu, lv = net.forward(x)
    # the network's dominant kernels (16-channel implicit-GEMM convolutions on MFMA):
    # forward over the 256^3 grid, timed with events on the network's stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        net.forward(x)
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / 5
    n3 = mk["cfg"].n ** 3
    fwd_flop = 2.0 * 27 * (3 * 16 + 16 * 16 + 16 * 16 + 16 * 2) * n3
    burn = learned.burn_in_study(mk, mu, lv, sweeps=args.burn_sweeps, eps=(args.eps, args.eps),
                                 log=log)
    ess = learned.ess_study(mk, mu, lv, chains=4, burn=100, sweeps=args.steps, eps0=args.eps,
                            log=log)
    pl, le, dg = ess["plain"], ess["learned"], ess["diagonal"]
    value = float(np.median(le["ess_per_s"]))
    out = {
        "metric": "P(k) ESS/s learned-mass vs plain at 256^3, same R-hat",
        "value": value,
        "unit": "effective P(k) samples/s (median over shells)",
        "n_gpus": 1, "steps": args.steps, "warmup": 100,
        "ms_per_step": le["ms_per_sweep"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cfg5: CNN trained on 128^3 plain-sampler draws "
                               f"({args.mocks} mocks x 31), applied to the 256^3 survey "
                               "(L=1500 Mpc/h, 6 subsamples, 60 shells, joint move on); "
                               "4 chains per mass, warm-started, one step = one sweep"},
        "plain": dict(learned.ess_table(pl), eps=pl["eps"], acceptance=pl["acceptance"],
                      ms_per_sweep=pl["ms_per_sweep"],
                      data_dominated=learned.ess_table(pl, learned.data_dominated_shells(mk))),
        "learned": dict(learned.ess_table(le), eps=le["eps"], acceptance=le["acceptance"],
                        ms_per_sweep=le["ms_per_sweep"],
                        data_dominated=learned.ess_table(le, learned.data_dominated_shells(mk))),
        "diagonal": dict(learned.ess_table(dg), eps=dg["eps"], acceptance=dg["acceptance"],
                         ms_per_sweep=dg["ms_per_sweep"],
                         data_dominated=learned.ess_table(dg, learned.data_dominated_shells(mk))),
        "ratio_median_ess_per_s": value / float(np.median(pl["ess_per_s"])),
        "roofline": {"bound": "mfma", "achieved": fwd_flop / (fwd_ms * 1e-3) / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": fwd_flop / (fwd_ms * 1e-3) / 1e12 / 2500.0,
                     "traffic": None, "kernel": "CNN forward at 256^3 (k_conv_lds, bf16 MFMA)",
                     "avg_ms": fwd_ms, "flop_per_launch": fwd_flop},
        "burn_in_sweeps": {k: {"potential": int(r["burn_pot"]), "ln_P": int(r["burn_logbias"])}
                           for k, r in burn.items()},
        "training": {"draws": int(len(own)), "steps": args.train_steps,
                     "final_loss": float(losses[-200:].mean()), "draw_seconds": t_draws,
                     "train_seconds": t_train},
    }
    print(json.dumps(out), flush=True)


def learned_rhat_main(args):
    """Learned vs plain mass P(k) ESS/s at equal convergence: split R-hat < 1.01 on
    the data-dominated shells, 4 chains per arm.  The network is trained as for
    --learned on 128^3 mocks; it is applied to the held-out 128^3 survey (mock seed 0,
    not among the training seeds) and to the 256^3 survey, each arm sampling until
    the target or --rhat-seconds of sampling per arm."""
    import torch
    from paper_1306_1821_amd import learned
    from paper_1306_1821_amd.binding import CNN
    from synth import CONFIGS, make_mock

    log = lambda m: print(f"[learned-rhat] {m}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    net = CNN(learned.init_params(3))
    mocks = learned.mock_series(CONFIGS["cfg2"], range(100, 100 + args.mocks))
    ins, tg, own = learned.make_training_set(net, mocks, per_batch=8, burn=20, samples=31, thin=8,
                                             eps=0.035, log=log)
    del mocks
    losses = learned.train(net, ins, tg, own, args.train_steps, lr=2e-3, log=log, log_every=1000)
    del ins, tg
    torch.cuda.empty_cache()
    t_prep = time.perf_counter() - t0
    out = {"metric": "P(k) ESS/s learned-mass vs plain at equal split R-hat < 1.01",
           "unit": "effective P(k) samples/s (median over data-dominated shells)",
           "n_gpus": 1, "dtype": "f32", "data": "synthetic", "higher_is_better": True,
           "training": {"draws": int(len(own)), "steps": args.train_steps,
                        "final_loss": float(losses[-200:].mean()), "seconds": t_prep},
           "rhat_seconds_per_arm": args.rhat_seconds, "sizes": {}}
    for name in args.rhat_workloads.split(","):
        mk = make_mock(CONFIGS[name], dtype=np.float32)
        s = learned.start_chains(mk, 1)
        x = learned.survey_inputs(net, s, 0, mk)
        s.close()
        mu, lv = net.forward(x)
        dd = learned.data_dominated_shells(mk)
        log(f"{name}: N={mk['cfg'].n}, {len(dd)} data-dominated shells")
        arms = tuple((a, a == "learned") for a in args.rhat_arms.split(","))
        r = learned.equal_rhat_study(mk, mu, lv, dd, chains=4, burn=200, block=500,
                                     max_seconds=args.rhat_seconds, eps0=args.eps, log=log,
                                     arms=arms)
        row = {}
        for arm, v in r.items():
            t = learned.ess_table(v, dd)
            row[arm] = dict(eps=v["eps"], acceptance=v["acceptance"], ms_per_sweep=v["ms_per_sweep"],
                            tune_acceptance=v["tune_acceptance"],
                            sweeps=v["sweeps"], reached=v["reached"], max_rhat=v["max_rhat"],
                            sweeps_to_target=v["sweeps_to_target"],
                            seconds_to_target=v["seconds_to_target"],
                            median_ess_per_s=t["median_ess_per_s"], min_ess_per_s=t["min_ess_per_s"],
                            history=v["history"])
        if "learned" in row and "plain" in row:
            row["ratio_median_ess_per_s"] = (row["learned"]["median_ess_per_s"]
                                             / max(1e-30, row["plain"]["median_ess_per_s"]))
        out["sizes"][name] = row
        del mu, lv
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=3, help="untimed sweeps")
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--eps", type=float, default=0.02)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eps-batch", type=float, default=0.03)
    ap.add_argument("--rhat-sweeps", type=int, default=0,
                    help="cfg4: total sweeps (timed + untimed) for the R-hat across chains")
    ap.add_argument("--learned", action="store_true",
                    help="learned warm start / mass comparison (steps = measured sweeps per mass)")
    ap.add_argument("--learned-rhat", action="store_true",
                    help="learned vs plain mass ESS/s at equal split R-hat < 1.01")
    ap.add_argument("--rhat-seconds", type=float, default=600.0,
                    help="--learned-rhat: sampling seconds per arm and size at most")
    ap.add_argument("--rhat-workloads", default="cfg2,cfg3")
    ap.add_argument("--rhat-arms", default="plain,learned")
    ap.add_argument("--mocks", type=int, default=64)
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--burn-sweeps", type=int, default=300)
    ap.add_argument("--posterior", action="store_true",
                    help="posterior correlations, P(k) bands and density maps (128^3)")
    ap.add_argument("--ablation", action="store_true",
                    help="P(k) correlation with and without the joint move (128^3)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="float64 oracle against the GPU per grid size (32^3, 128^3, 256^3) "
                         "and P(k) ESS/s at 32^3")
    ap.add_argument("--oracle-sweeps", type=int, default=200,
                    help="--oracle-timing: sweeps per chain of the 32^3 ESS comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a float32 buffer of this size 3 times (a kernel of "
                         "known traffic that scales hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the sampler runs on a single MI355X "
              "(chains or slabs would shard across GPUs; the library runs on one)",
              file=sys.stderr)
        sys.exit(2)
    if args.oracle_timing:
        return oracle_timing_main(args)
    if args.ablation:
        return ablation_main(args)
    if args.posterior:
        return posterior_main(args)
    if args.learned_rhat:
        return learned_rhat_main(args)
    if args.learned:
        if args.steps == 20:
            args.steps = 1500
        return learned_main(args)
    if args.workload == "cfg4":
        return batched_main(args)
    import torch
    from paper_1306_1821_amd.binding import Sampler

    mk, spec = workload_spec(args.workload, args.eps)
    n, nh = spec["n"], spec["n"] * spec["n"] * (spec["n"] // 2 + 1)
    s = Sampler([spec])
    s.set_state(0, mk["delta"])         # start at the survey's truth field (a typical posterior state)
    print(f"[bench] {args.workload}: N={n} c={len(spec['bias'])} nb={spec['nb']} "
          f"nsteps={spec['nsteps']} eps={spec['eps']}", file=sys.stderr, flush=True)
    sweep = 0
    for _ in range(args.warmup):
        s.sweep(sweep)
        sweep += 1
    torch.cuda.synchronize()
    # HIP events around every 5th k-space step pass and every 5th real-space / plane pass
    s.timing(0x10 | 0x1 | 0x4 | (4 << 8))
    acc, rj_acc = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = s.sweep(sweep)[0]
        acc.append(st["accepted"])
        rj_acc.append(st["rj_accepted"])
        sweep += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, launches = s.timing(0)
    print(f"[bench] {args.steps} sweeps in {dt:.3f} s", file=sys.stderr, flush=True)

    # pure trajectory rate (leapfrog only) for reference
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ntraj = max(2, args.steps // 2)
    for i in range(ntraj):
        s.trajectory(10_000 + i)
    torch.cuda.synchronize()
    dt_traj = time.perf_counter() - t1
    print(f"[bench] {ntraj} bare trajectories in {dt_traj:.3f} s", file=sys.stderr, flush=True)
    # per-pass breakdown (events around every pass) on a few more trajectories
    s.timing(1)
    for i in range(3):
        s.trajectory(20_000 + i)
    ms_all, launches_all = s.timing(0)
    # per-trajectory device time: HIP events around each of 100 trajectories
    # enqueued through the asynchronous entry point (no host wait in between)
    dH_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    acc_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(100)]
    for i, (ea, eb) in enumerate(evs):
        ea.record()
        s.trajectory_async(30_000 + i, dH_dev, acc_dev)
        eb.record()
    torch.cuda.synchronize()
    traj_ms = float(np.median([ea.elapsed_time(eb) for ea, eb in evs]))
    print(f"[bench] 100 event-timed trajectories, median {traj_ms:.3f} ms", file=sys.stderr,
          flush=True)

    steps = args.steps * spec["nsteps"]
    value = steps / dt
    plane = launches_all[1] < launches_all[2]     # the fused y-z plane pass ran
    # k-space step pass: read T, delta_hat, p_hat; write delta_hat, p_hat, T
    x_ms, x_bytes = ms[0] / max(1, launches[0]), 6 * nh * 8
    # plane pass (or z pass): read T, alpha, beta; write T
    z_ms, z_bytes = ms[2] / max(1, launches[2]), 2 * nh * 8 + 2 * n ** 3 * 4
    roof_x = {"bound": "hbm", "achieved": x_bytes / (x_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
              "unit": "GB/s", "frac": x_bytes / (x_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "traffic": measured_traffic("x-step") if args.workload == "cfg3" else None,
              "kernel": f"k_xpass_n<{n}, X_STEP>", "avg_ms": x_ms, "launches": int(launches[0]),
              "bytes_per_launch": x_bytes}
    roof_p = {"bound": "hbm", "achieved": z_bytes / (z_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
              "unit": "GB/s", "frac": z_bytes / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "traffic": measured_traffic("plane") if args.workload == "cfg3" else None,
              "kernel": f"k_yzpass_n<{n}, false/true>", "avg_ms": z_ms, "launches": int(launches[2]),
              "bytes_per_launch": z_bytes}
    out = {
        "metric": f"leapfrog steps/s at {n}^3",
        "value": value,
        "unit": "leapfrog steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}^3 grid, L={spec['box']:.0f} Mpc/h, "
                               f"{len(spec['bias'])} subsamples, {spec['nb']} k-shells, "
                               f"{spec['nsteps']} leapfrog steps, joint move "
                               f"{'on' if spec['rj'] else 'off'}; one bench step = one sweep",
                   "eps": spec["eps"]},
        # the dominant kernel by GPU time: the plane pass where it runs (two of them per
        # sweep step, density and joint move), else the k-space step pass
        "roofline": roof_p if plane else roof_x,
        "roofline_kspace_step": roof_x,
        "acceptance": float(np.mean(acc)),
        "rj_acceptance": float(np.mean(rj_acc)),
        "trajectory_leapfrog_steps_per_s": ntraj * spec["nsteps"] / dt_traj,
        "trajectory_median": {"ms": traj_ms, "leapfrog_steps_per_s": spec["nsteps"] / (1e-3 * traj_ms),
                              "trajectories": len(evs),
                              "timing": "HIP events around each trajectory, asynchronous entry point"},
        "pass_ms_per_step": {"kspace": ms_all[0] / max(1, launches_all[0]),
                             "ypass": ms_all[1] / max(1, launches_all[1]),
                             "zpass": ms_all[2] / max(1, launches_all[2])},
    }
    # the whole step against two byte counts: the design's own and the 40 N^3 bytes of
    # a step whose two FFTs take the minimum two passes each over a grid larger than
    # on-chip memory.  With the fused y-z plane pass a step is the k-space pass plus
    # one plane pass (40 N^3 bytes; the y passes left run only in the momentum draw);
    # otherwise it is x + 2 y + z passes (56 N^3 bytes).
    plane = launches_all[1] < launches_all[2]
    pm = out["pass_ms_per_step"]
    if plane:
        step_ms, design = pm["kspace"] + pm["zpass"], 40
        out["pass_ms_per_step"]["plane"] = pm.pop("zpass")
    else:
        step_ms, design = pm["kspace"] + 2 * pm["ypass"] + pm["zpass"], 56
    nv = n ** 3
    out["step_roofline"] = {
        "ms": step_ms, "passes": "x + yz plane" if plane else "x + 2 y + z",
        "bytes_design": design * nv, "bytes_lower_bound": 40 * nv,
        "frac_design": design * nv / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "frac_lower_bound": 40 * nv / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mk, spec, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
