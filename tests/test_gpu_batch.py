"""Batched chains and graph replay on the GPU."""
import numpy as np
import pytest

from gpu_common import chain_spec, mock, start_state
from paper_1306_1821_amd import diagnostics as dg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1821_amd.binding import Sampler  # noqa: E402


def test_graph_replays_equal_direct_launches():
    """Every replay of the captured sweep / trajectory equals the directly launched one."""
    mks = [mock("small16"), mock("cfg1")]
    specs = [chain_spec(m, eps=0.05, nsteps=8, seed=37, chain_id=i, rj=True)
             for i, m in enumerate(mks)]
    runs = []
    for graph in (False, True):
        s = Sampler(specs)
        for i, m in enumerate(mks):
            s.set_state(i, start_state(m)[0])
        if graph:
            s.use_graph(True)
        trace = []
        for sw in range(4):
            trace.append(s.sweep(sw))
            trace.append(s.trajectory(100 + sw))
            _ = s.state(0)["delta_k"].sum()          # eager work between replays
        trace.append([s.state(i)["delta_k"] for i in range(2)])
        runs.append(trace)
        s.close()
    for a, b in zip(runs[0][:-1], runs[1][:-1]):
        if isinstance(a, tuple):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        else:
            for x, y in zip(a, b):
                assert x["dH"] == y["dH"] and np.array_equal(x["pk"], y["pk"])
                assert np.array_equal(x["nbar"], y["nbar"]) and np.array_equal(x["bias"], y["bias"])
    for x, y in zip(runs[0][-1], runs[1][-1]):
        assert np.array_equal(x, y)


@pytest.mark.timeout(300)
def test_batched_chains_converge_together():
    """Same-size chains in one batch sample the same P(k) posterior: rank-normalised
    split R-hat below 1.01 on every data-informed shell, four chains per size.

    The slowest shell is the first 32^3 shell (26 modes): with eps = 0.12 and 16
    steps its bulk ESS grows by about 90 per 4000 sweeps over four chains (measured),
    so 48000 sweeps put R-hat near 1.006; the 16^3 chains pass 1.01 by about 8000."""
    groups = [("small16", 4, 0.08, 10, 16000), ("cfg1", 4, 0.12, 16, 48000)]
    burn = 4000
    for name, k, eps, nst, nsweep in groups:
        m = mock(name)
        specs = [chain_spec(m, eps=eps, nsteps=nst, seed=41, chain_id=c, rj=True) for c in range(k)]
        s = Sampler(specs)
        for i in range(k):
            s.set_state(i, start_state(m)[0])
        s.use_graph(True)
        traces = [[] for _ in specs]
        acc = []
        for sw in range(nsweep):
            out = s.sweep(sw)
            acc.append([o["accepted"] for o in out])
            for i, o in enumerate(out):
                traces[i].append(np.log(o["pk"]))
        s.close()
        assert np.mean(acc) > 0.5
        t = np.array([tr[burn:] for tr in traces])          # chains x samples x shells
        nb = t.shape[2]
        # shells the data inform: centres below 0.7 of the Nyquist frequency
        # (k_corner = sqrt(3) k_Nyquist); the rest follow the flat Jeffreys tail
        head = [mm for mm in range(nb) if (mm + 0.5) / nb * np.sqrt(3.0) <= 0.7]
        rh = [dg.split_rhat(t[:, :, mm]) for mm in head]
        print(name, "split R-hat per shell", np.round(rh, 4), "min bulk ESS",
              min(dg.ess_bulk(t[:, :, mm]) for mm in head), flush=True)
        assert max(rh) < 1.01, (name, rh)


@pytest.mark.parametrize("names", [("cfg1",), ("small16", "cfg1", "tiny8x2")])
def test_launch_shapes_do_not_change_results(names):
    """Persistent grids (XCD-aware tile walk), one launch per size group and the
    autotuner's choice give bit-identical sweeps; the autotuner leaves the state
    unchanged."""
    mks = [mock(n) for n in names]
    specs = [chain_spec(m, eps=0.05, nsteps=8, seed=41, chain_id=i, rj=True)
             for i, m in enumerate(mks)]
    finals = []
    for shape in ("default", 16, 20, 40, -1, "auto"):
        s = Sampler(specs)
        for i, m in enumerate(mks):
            s.set_state(i, start_state(m)[0])
        if shape == "auto":
            before = [s.state(i)["delta_k"] for i in range(len(mks))]
            chosen = s.autotune(3)
            assert len(chosen) == 3 and all(g >= -1 for g in chosen)
            for i in range(len(mks)):
                assert np.array_equal(s.state(i)["delta_k"], before[i])
        elif shape != "default":
            for cls in range(3):
                s.set_launch(cls, shape)
        stats = [s.sweep(sw) for sw in range(3)]
        finals.append(([s.state(i)["delta_k"] for i in range(len(mks))],
                       [[x["pk"] for x in st] for st in stats]))
        s.close()
    for dk, pk in finals[1:]:
        for a, b in zip(dk, finals[0][0]):
            assert np.array_equal(a, b)
        for sw_a, sw_b in zip(pk, finals[0][1]):
            for a, b in zip(sw_a, sw_b):
                assert np.array_equal(a, b)


def test_set_step_equals_configured_step():
    """hmc_set_step gives the same trajectories as a context configured with that eps."""
    m = mock("cfg1")
    a = Sampler([chain_spec(m, eps=0.03, nsteps=8, seed=3)])
    b = Sampler([chain_spec(m, eps=0.07, nsteps=8, seed=3)])
    for s in (a, b):
        s.set_state(0, start_state(m)[0])
    b.set_step(0, 0.03)
    for i in range(3):
        ra, rb = a.trajectory(i), b.trajectory(i)
        assert ra[0][0] == rb[0][0] and ra[1][0] == rb[1][0]
    assert np.array_equal(a.state(0)["delta_k"], b.state(0)["delta_k"])
    with pytest.raises(Exception):
        b.set_step(0, -1.0)
    a.close()
    b.close()


def test_drawn_step_counts_with_graphs():
    """With tau_mode the step count varies per trajectory; graph replay (one graph per
    step count) equals direct launches, and a batch of chains shares the draw."""
    mks = [mock("small16"), mock("cfg1")]
    specs = [chain_spec(m, eps=0.05, nsteps=12, seed=29, chain_id=i, rj=True, tau_mode=True)
             for i, m in enumerate(mks)]
    runs = []
    for graph in (False, True):
        s = Sampler(specs)
        for i, m in enumerate(mks):
            s.set_state(i, start_state(m)[0])
        s.use_graph(graph)
        out = [s.trajectory(100 + t) for t in range(4)] + [s.sweep(t) for t in range(4)]
        runs.append((out, [s.state(i)["delta_k"] for i in range(2)]))
        s.close()
    for a, b in zip(runs[0][0], runs[1][0]):
        if isinstance(a, tuple):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        else:
            for x, y in zip(a, b):
                assert x["dH"] == y["dH"] and np.array_equal(x["pk"], y["pk"])
    for x, y in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(x, y)


def test_async_calls_equal_synchronous_ones():
    """Queued trajectories / sweeps writing their results to device buffers give the
    same results and states as the synchronous calls."""
    mks = [mock("small16"), mock("cfg1")]
    specs = [chain_spec(m, eps=0.05, nsteps=8, seed=31, chain_id=i, rj=True)
             for i, m in enumerate(mks)]
    a, b = Sampler(specs), Sampler(specs)
    for s in (a, b):
        for i, m in enumerate(mks):
            s.set_state(i, start_state(m)[0])
    ref_t = [a.trajectory(200 + t) for t in range(3)]
    ref_s = [a.sweep(t) for t in range(3)]
    dH = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    acc = torch.zeros((3, 2), dtype=torch.int32, device="cuda")
    rec = torch.zeros((3, b.sweep_record_size()), dtype=torch.float64, device="cuda")
    for t in range(3):
        b.trajectory_async(200 + t, dH[t], acc[t])
    for t in range(3):
        b.sweep_async(t, rec[t])
    torch.cuda.synchronize()
    dH, acc, rec = dH.cpu().numpy(), acc.cpu().numpy(), rec.cpu().numpy()
    for t in range(3):
        assert np.array_equal(dH[t], ref_t[t][0]) and np.array_equal(acc[t].astype(bool), ref_t[t][1])
        off = 0
        for i, st in enumerate(ref_s[t]):
            r = rec[t, off:]
            nb, c = len(st["pk"]), len(st["bias"])
            assert r[0] == st["dH"] and bool(r[1]) == st["accepted"]
            assert r[2] == st["rj_dH"] and bool(r[3]) == st["rj_accepted"] and r[4] == 0
            assert r[5] == st["rj_wall_hits"]
            h = 6
            assert np.array_equal(r[h:h + nb], st["pk"])
            assert np.array_equal(r[h + nb:h + nb + c], st["bias"])
            assert np.array_equal(r[h + nb + c:h + nb + 2 * c], st["nbar"])
            off += h + nb + 2 * c
    for i in range(2):
        assert np.array_equal(a.state(i)["delta_k"], b.state(i)["delta_k"])
    a.close()
    b.close()


def test_pass_timing_classes_and_sampling():
    """Pass timing counts launches per class; a class mask records only those
    classes and a sampling stride every stride-th launch of each; timing does
    not change results."""
    m = mock("cfg1")
    nsteps = 8
    runs = {}
    for enable in (0, 1, 0x11, 0x411):
        s = Sampler([chain_spec(m, eps=0.05, nsteps=nsteps, seed=5)])
        s.set_state(0, start_state(m)[0])
        if enable:
            s.timing(enable)
        res = [s.trajectory(i) for i in range(3)]
        ms, n = s.timing(0)
        runs[enable] = (res, n, ms, s.state(0)["delta_k"])
        s.close()
    interior = runs[1][1][0]
    assert interior > 0 and runs[1][1][1] > 0 and runs[1][1][2] > 0
    assert np.all(runs[1][2][runs[1][1] > 0] > 0)
    assert runs[0x11][1][0] == interior and np.all(runs[0x11][1][1:] == 0)
    assert runs[0x411][1][0] == (interior + 4) // 5 and np.all(runs[0x411][1][1:] == 0)
    for enable in (1, 0x11, 0x411):
        assert np.array_equal(runs[enable][3], runs[0][3])
        for a, b in zip(runs[enable][0], runs[0][0]):
            assert a[0][0] == b[0][0] and a[1][0] == b[1][0]


def test_joint_move_shortens_pk_correlation():
    """Ablation of the joint (P, delta) move at 32^3: with it the median correlation
    length of ln P over shells is shorter than without (same chains, eps, steps)."""
    from paper_1306_1821_amd import studies
    from synth import CONFIGS, make_mock
    mk = make_mock(CONFIGS["cfg1"], dtype=np.float32)
    r = studies.joint_move_ablation(mk, chains=4, burn=50, sweeps=1500, lags=(1, 10, 100))
    j, nj = np.median(r["joint"]["corr_len"]), np.median(r["no_joint"]["corr_len"])
    print("median correlation length with / without the joint move:", j, nj)
    assert j < nj


@pytest.mark.timeout(400)
def test_joint_move_leaves_power_posterior_invariant():
    """The device counterpart of the oracle's stationarity pin (Appendix C,
    eq. spec_posterior_MIXING_1; eq. INVERSE_GAMMA): with the proper prior
    alpha = 0, sweeps of {density HMC, P draw, Nbar and b draws} with and without
    the joint (P, delta) move leave the same posterior invariant, so the mean of
    ln P per shell agrees within 4 standard errors (bulk ESS of four 8^3 chains per
    arm, 6000 sweeps each).  A joint move whose HMC mass followed theta moved the
    first shell's mean by half a posterior standard deviation in the oracle."""
    m = mock("tiny8x2")
    res = {}
    for rj in (False, True):
        specs = [chain_spec(m, eps=0.15, nsteps=8, seed=71, chain_id=c, rj=rj, alpha_prior=0.0)
                 for c in range(4)]
        s = Sampler(specs)
        for i in range(4):
            s.set_state(i, start_state(m)[0])
        s.use_graph(True)
        traces = [[] for _ in specs]
        for sw in range(6000):
            for i, o in enumerate(s.sweep(sw)):
                traces[i].append(np.log(o["pk"]))
        s.close()
        res[rj] = np.array([t[200:] for t in traces])          # chains x samples x shells
    a, b = res[False], res[True]
    for mm in range(a.shape[2]):
        ea, eb = dg.ess_bulk(a[:, :, mm]), dg.ess_bulk(b[:, :, mm])
        se = np.sqrt(a[:, :, mm].var() / ea + b[:, :, mm].var() / eb)
        d = b[:, :, mm].mean() - a[:, :, mm].mean()
        print(f"shell {mm}: mean ln P without {a[:, :, mm].mean():.4f}, with {b[:, :, mm].mean():.4f}, "
              f"difference {d / se:+.2f} SE (bulk ESS {ea:.0f}, {eb:.0f})", flush=True)
        assert abs(d) < 4 * se, (mm, d / se)


def test_field_moments_match_numpy():
    """hmc_field_moments: the running float64 mean and sum of squared deviations of
    delta_r over sweeps of two chains (pooled) equal numpy's on the stored states."""
    mks = [mock("small16"), mock("small16")]
    s = Sampler([chain_spec(m, eps=0.08, nsteps=8, seed=61, chain_id=i, rj=True)
                 for i, m in enumerate(mks)])
    for i, m in enumerate(mks):
        s.set_state(i, start_state(m)[0])
    n = mks[0]["cfg"].n
    mean = torch.zeros((n, n, n), dtype=torch.float64, device=s.device)
    m2 = torch.zeros_like(mean)
    states, count = [], 0
    for sw in range(6):
        s.sweep(sw)
        for i in range(2):
            count += 1
            s.field_moments(i, mean, m2, count)
            states.append(s.state(i)["delta_r"].astype(np.float64))
    x = np.array(states)
    mu = x.mean(axis=0)
    var = x.var(axis=0, ddof=1)
    assert np.max(np.abs(mean.cpu().numpy() - mu)) < 1e-12 * np.max(np.abs(mu))
    assert np.max(np.abs(m2.cpu().numpy() / (count - 1) - var)) < 1e-10 * np.max(var)
    with pytest.raises(Exception):
        s.field_moments(0, mean, m2, 0)
    s.close()


def test_mixed_size_batch_sweeps_match_single_chains():
    """Chains of 8^3, 16^3, 32^3 and 64^3 (each with its own survey support mask,
    tiles and partial sums inside the shared launches) sweep, joint move on, as the
    same chains do alone: the sweep records agree to float32 rounding."""
    mks = [mock("tiny8x2"), mock("small16"), mock("cfg1"), mock("paper15s")]
    specs = [chain_spec(m, eps=0.04, nsteps=8, seed=37, chain_id=i, rj=True)
             for i, m in enumerate(mks)]
    batch = Sampler(specs)
    for i, m in enumerate(mks):
        batch.set_state(i, start_state(m)[0])
    got = [batch.sweep(t) for t in range(3)]
    batch.close()
    for i, m in enumerate(mks):
        solo = Sampler([specs[i]])
        solo.set_state(0, start_state(m)[0])
        for t in range(3):
            ref = solo.sweep(t)[0]
            g = got[t][i]
            print(f"chain {i} sweep {t}: dH {g['dH']:.5e}/{ref['dH']:.5e} "
                  f"rj_dH {g['rj_dH']:.4e}/{ref['rj_dH']:.4e}")
            assert g["accepted"] == ref["accepted"] and g["rj_accepted"] == ref["rj_accepted"]
            assert abs(g["dH"] - ref["dH"]) < 1e-3 * max(1.0, abs(ref["dH"]))
            np.testing.assert_allclose(g["pk"], ref["pk"], rtol=1e-4)
            np.testing.assert_allclose(g["nbar"], ref["nbar"], rtol=1e-5)
            np.testing.assert_allclose(g["bias"], ref["bias"], rtol=1e-4)
        solo.close()
