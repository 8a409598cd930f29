"""GPU parity: libhmc kernels (through the C-ABI) against the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import (chain_spec, coefficients32, dh_tol, mock, oracle_posterior, plain_mock,
                        rel_l2, start_state)
from oracle import grid, hmc, model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1821_amd.binding import Sampler  # noqa: E402

SIZES = [(8, 500.0, 4), (16, 500.0, 8), (32, 500.0, 16), (64, 500.0, 20), (128, 1000.0, 40),
         (192, 1500.0, 60), (256, 1500.0, 60)]


def sampler_for(mk, **kw):
    return Sampler([chain_spec(mk, **kw)])


@pytest.mark.parametrize("n,box,nb", SIZES + [(128, 1000.0, 110), (256, 1500.0, 128)])
def test_shell_index_and_counts_bit_exact(n, box, nb):       # incl. the most shells a grid fills
    mk = plain_mock(n, box, nb)
    s = sampler_for(mk)
    assert np.array_equal(s.shell_index(0).astype(np.int64), grid.half_shells(n, nb))
    _, nm = s.shell_power(0)
    assert np.array_equal(nm, grid.mode_counts(n, nb))
    s.close()


@pytest.mark.parametrize("n,box,nb", SIZES)
def test_shell_power_on_uploaded_state(n, box, nb):
    mk = plain_mock(n, box, nb)
    s = sampler_for(mk)
    rng = np.random.default_rng(n)
    dk = (rng.standard_normal((n, n, n // 2 + 1)) + 1j * rng.standard_normal((n, n, n // 2 + 1)))
    dk = dk.astype(np.complex64)
    s.tensors(0)["delta_k"].copy_(torch.as_tensor(dk))
    sig, _ = s.shell_power(0)
    ref = grid.shell_sums(dk.astype(np.complex128), nb)
    np.testing.assert_allclose(sig, ref, rtol=1e-12)
    s.close()


@pytest.mark.parametrize("n,box,nb", SIZES)
def test_gradient_and_transforms(n, box, nb):
    """set_state: delta_hat = F delta, delta_r = F^-1 delta_hat, grad = F(alpha delta - beta)."""
    mk = plain_mock(n, box, nb, nsub=2)
    a32, b32 = coefficients32(mk)
    s = sampler_for(mk)
    s.set_coefficients(0, a32, b32)
    d32, dk = start_state(mk)
    s.set_state(0, d32)
    st = s.state(0)
    post = oracle_posterior(mk, a32, b32)
    f, gk, delta = model.force_k(dk, post.lam_k, post.alpha, post.beta)
    assert rel_l2(st["delta_k"], dk) < 2e-6
    assert rel_l2(st["delta_r"], delta) < 2e-6
    gk_ref = gk.copy()
    gk_ref[0, 0, 0] = 0.0
    err = rel_l2(st["grad_k"], gk_ref)
    print(f"N={n}: gradient rel-L2 {err:.2e}")
    assert err < 1e-5
    s.close()


@pytest.mark.parametrize("n,box,nb", SIZES)
def test_hamiltonian_on_identical_arrays(n, box, nb):
    mk = plain_mock(n, box, nb, nsub=2)
    a32, b32 = coefficients32(mk)
    s = sampler_for(mk)
    s.set_coefficients(0, a32, b32)
    rng = np.random.default_rng(7 + n)
    h = n // 2 + 1
    dk = (0.3 * (rng.standard_normal((n, n, h)) + 1j * rng.standard_normal((n, n, h)))).astype(np.complex64)
    pk = (rng.standard_normal((n, n, h)) + 1j * rng.standard_normal((n, n, h))).astype(np.complex64)
    dr = (0.5 * rng.standard_normal((n, n, n))).astype(np.float32)
    t = s.tensors(0)
    t["delta_k"].copy_(torch.as_tensor(dk))
    t["mom_k"].copy_(torch.as_tensor(pk))
    t["delta_r"].copy_(torch.as_tensor(dr))
    got = s.hamiltonian(0)
    post = oracle_posterior(mk, a32, b32)
    ref = hmc.energies(dk.astype(np.complex128), pk.astype(np.complex128), dr.astype(np.float64), post)
    print(f"N={n}: energies {got} vs {ref}")
    for g, r in zip(got, ref):
        assert abs(g - r) < max(1e-6, 1e-13 * abs(r))
    s.close()


TRAJ_CASES = [("tiny8x2", 0.1, 10), ("small16", 0.1, 10), ("cfg1", 0.05, 20), (64, 0.05, 10),
              (128, 0.04, 8), (192, 0.03, 8),     # 192^3: radix-3/12 transforms
              ("cfg3", 0.02, 4)]                  # cfg3: the 256^3 bench workload
PLAIN_GEOMETRY = {64: (500.0, 20), 128: (1000.0, 40), 192: (1500.0, 60)}


def traj_mock(case):
    if isinstance(case, str):
        return mock(case)
    box, nb = PLAIN_GEOMETRY[case]
    return plain_mock(case, box, nb, nsub=2)


@pytest.mark.parametrize("case,eps,nsteps", TRAJ_CASES)
def test_trajectory_matches_oracle(case, eps, nsteps):
    mk = traj_mock(case)
    n = mk["cfg"].n
    a32, b32 = coefficients32(mk)
    s = sampler_for(mk, eps=eps, nsteps=nsteps, seed=17)
    s.set_coefficients(0, a32, b32)
    d32, dk = start_state(mk)
    s.set_state(0, d32)
    post = oracle_posterior(mk, a32, b32, workers=8)
    for traj in range(2):
        before = s.state(0)
        dH, acc = s.trajectory(traj)
        st = s.state(0)
        ref = hmc.trajectory(before["delta_k"].astype(np.complex128), post, eps, nsteps, 17, 0, traj)
        e_p = rel_l2(st["mom_k"], ref["p1"])
        margin = abs(ref["log_u"] + ref["dH"])
        print(f"N={n} traj {traj}: dH gpu {dH[0]:.6e} oracle {ref['dH']:.6e} "
              f"|diff| {abs(dH[0] - ref['dH']):.2e}; p rel-L2 {e_p:.2e}; acc {acc[0]} {ref['accepted']}")
        assert e_p < 1e-4
        assert abs(dH[0] - ref["dH"]) < dh_tol(n)   # end to end, float32 state
        if margin > dh_tol(n):
            assert bool(acc[0]) == ref["accepted"]
        if acc[0] and ref["accepted"]:
            assert rel_l2(st["delta_k"], ref["proposal"]) < 1e-4
            assert rel_l2(st["grad_k"], np.where(post.shells >= 0, ref["grad1"], 0)) < 1e-4
        if not acc[0]:
            assert np.array_equal(st["delta_k"], before["delta_k"])
            assert np.array_equal(st["delta_r"], before["delta_r"])
    s.close()


def test_trajectories_from_zero_match_oracle():
    """The end-to-end case of the float32-state analysis: 8^3, eps 0.05, 20 steps,
    every trajectory started at delta = 0 with its own momentum draw."""
    mk = mock("tiny8x2")
    n = mk["cfg"].n
    a32, b32 = coefficients32(mk)
    s = sampler_for(mk, eps=0.05, nsteps=20, seed=17)
    s.set_coefficients(0, a32, b32)
    post = oracle_posterior(mk, a32, b32, workers=4)
    diffs = []
    for traj in range(16):
        s.set_state(0, np.zeros((n, n, n), np.float32))
        before = s.state(0)
        assert not before["delta_k"].any()
        dH, acc = s.trajectory(traj)
        ref = hmc.trajectory(before["delta_k"].astype(np.complex128), post, 0.05, 20, 17, 0, traj)
        diffs.append(abs(dH[0] - ref["dH"]))
        if abs(ref["log_u"] + ref["dH"]) > dh_tol(n):
            assert bool(acc[0]) == ref["accepted"]
    print(f"|dH diff| from delta = 0: median {np.median(diffs):.2e}, max {max(diffs):.2e}")
    assert max(diffs) < dh_tol(n)
    s.close()


@pytest.mark.timeout(300)
def test_chain_matches_dense_wiener_posterior():
    """Fixed P, b, Nbar at 8^3: the device's HMC draws have the closed-form Wiener
    mean and covariance (eqs. Wiener_Posterior_psi, Wiener_Posterior_force; the dense
    solve of tests/dense.py on the zero-mean subspace).  Draws whitened by that
    covariance have zero mean and unit variance within their ESS-based errors."""
    import dense
    from test_oracle_hmc import _ess
    mk = mock("tiny8x2")
    cfg = mk["cfg"]
    n = cfg.n
    a32, b32 = coefficients32(mk)
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    mu, cov, Q, U = dense.wiener(n, lam_m, cfg.nb, a32.astype(np.float64), b32.astype(np.float64))
    evals, evecs = np.linalg.eigh(U.T @ cov @ U)
    T = (U @ evecs) / np.sqrt(evals)            # whitening map on the subspace
    s = sampler_for(mk, eps=0.2, nsteps=12, seed=11, tau_mode=True)   # drawn lengths
    s.set_coefficients(0, a32, b32)
    # start at an exact draw of the posterior, so that the chain is stationary from the
    # first trajectory (from the mean itself a slowly mixing mass needs thousands of
    # trajectories to reach the posterior's spread)
    z0 = np.random.default_rng(3).standard_normal(len(evals))
    start = mu + (U @ evecs) @ (np.sqrt(evals) * z0)
    s.set_state(0, start.reshape(n, n, n).astype(np.float32))
    samples, acc, nsamp = [], 0, 3000
    for t in range(nsamp):
        dH, a = s.trajectory(t)
        acc += int(a[0])
        samples.append(s.state(0)["delta_r"].reshape(-1).astype(np.float64))
    s.close()
    y = (np.array(samples) - mu) @ T                # iid N(0, 1) per column if exact
    ess = np.array([_ess(y[:, j]) for j in range(y.shape[1])])
    zmean = y.mean(axis=0) * np.sqrt(ess)
    var = y.var(axis=0)
    print(f"acceptance {acc / nsamp:.2f}, median ESS {np.median(ess):.0f}, max |z-mean| "
          f"{np.max(np.abs(zmean)):.2f}, mean z^2 {np.mean(zmean ** 2):.2f}, mean variance {var.mean():.4f}")
    assert acc / nsamp > 0.6
    assert np.max(np.abs(zmean)) < 5.0
    assert abs(np.mean(zmean ** 2) - 1.0) < 0.3
    assert np.max(np.abs(var - 1.0) * np.sqrt(ess / 2.0)) < 6.0
    assert abs(var.mean() - 1.0) < 0.03


@pytest.mark.parametrize("eps,accepted", [(0.02, True), (0.8, False)])
def test_gradient_cache_after_trajectory(eps, accepted):
    """After a trajectory, accepted (small step) or rejected (eps = 0.8: dH of 50-70 in
    the oracle), grad_k holds F(alpha delta - beta) of the state's delta_hat: the next
    trajectory's first kick and the joint move's start read it from there."""
    mk = mock("small16")
    a32, b32 = coefficients32(mk)
    s = sampler_for(mk, eps=eps, nsteps=10, seed=31)
    s.set_coefficients(0, a32, b32)
    d32, _ = start_state(mk)
    s.set_state(0, d32)
    post = oracle_posterior(mk, a32, b32)
    for traj in range(2):
        dH, acc = s.trajectory(traj)
        assert bool(acc[0]) == accepted, (traj, dH[0])
        st = s.state(0)
        _, gk, _ = model.force_k(st["delta_k"].astype(np.complex128), post.lam_k, post.alpha,
                                 post.beta)
        err = rel_l2(st["grad_k"], np.where(post.shells >= 0, gk, 0))
        print(f"eps {eps} traj {traj}: dH {dH[0]:.4e} accepted {acc[0]}, grad_k rel-L2 {err:.2e}")
        assert err < 1e-5
    s.close()


def test_batched_mixed_sizes_match_oracle():
    """Chains of 8^3, 16^3 and 32^3 advance in the same launches; each matches the oracle."""
    names = ["tiny8x2", "small16", "cfg1"]
    mks = [mock(x) for x in names]
    specs = [chain_spec(m, eps=0.05, nsteps=10, seed=5, chain_id=i) for i, m in enumerate(mks)]
    s = Sampler(specs)
    posts = []
    for i, m in enumerate(mks):
        a32, b32 = coefficients32(m)
        s.set_coefficients(i, a32, b32)
        d32, _ = start_state(m)
        s.set_state(i, d32)
        posts.append(oracle_posterior(m, a32, b32))
    befores = [s.state(i)["delta_k"] for i in range(3)]
    dH, acc = s.trajectory(3)
    for i in range(3):
        ref = hmc.trajectory(befores[i].astype(np.complex128), posts[i], 0.05, 10, 5, i, 3)
        st = s.state(i)
        assert rel_l2(st["mom_k"], ref["p1"]) < 1e-4, i
        assert abs(dH[i] - ref["dH"]) < dh_tol(mks[i]["cfg"].n), i
    s.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case,eps,nsteps", [("cfg3", 0.02, 4), (192, 0.03, 8), ("cfg2", 0.04, 8),
                                             (64, 0.05, 10)])
def test_plane_pass_matches_separate_passes_and_oracle(case, eps, nsteps):
    """From 64^3 to 256^3 the gradient evaluations run the fused y-z plane pass
    (inverse y, C2R z, data force, R2C z, forward y with the plane on chip; the
    kz = 0 and kz = N/2 columns travel as one complex column).  Against the
    separate y, z, y passes and against the oracle: the gradient of set_state, the
    data energy, the real field, and a trajectory's end point and dH."""
    mk = traj_mock(case)
    n = mk["cfg"].n
    a32, b32 = coefficients32(mk)
    d32, dk = start_state(mk)
    post = oracle_posterior(mk, a32, b32, workers=16)
    f, gk, delta = model.force_k(dk, post.lam_k, post.alpha, post.beta)
    gk[0, 0, 0] = 0.0
    got = {}
    for fused in (True, False):
        s = sampler_for(mk, eps=eps, nsteps=nsteps, seed=19)
        s.set_plane_pass(fused)
        s.set_coefficients(0, a32, b32)
        s.set_state(0, d32)
        st = s.state(0)
        h = s.hamiltonian(0)
        dH, acc = s.trajectory(0)
        got[fused] = dict(st=st, data=h[2], dH=dH[0], after=s.state(0))
        e_g = rel_l2(st["grad_k"], gk)
        e_d = rel_l2(st["delta_r"], delta)
        print(f"fused={fused}: gradient rel-L2 {e_g:.2e}, delta rel-L2 {e_d:.2e}, data energy "
              f"{h[2]:.9e}, dH {dH[0]:.6e}", flush=True)
        assert e_g < 1e-5 and e_d < 2e-6
        s.close()
    a, b = got[True], got[False]
    assert rel_l2(a["st"]["grad_k"], b["st"]["grad_k"]) < 2e-6
    assert abs(a["data"] - b["data"]) < 1e-9 * abs(b["data"]) + 1e-6
    ref = hmc.trajectory(a["st"]["delta_k"].astype(np.complex128), post, eps, nsteps, 19, 0, 0)
    for k in (True, False):
        assert abs(got[k]["dH"] - ref["dH"]) < dh_tol(n)
    assert rel_l2(a["after"]["mom_k"], b["after"]["mom_k"]) < 2e-6


@pytest.mark.timeout(300)
@pytest.mark.parametrize("launch", [0, -1])
def test_batched_64_128_192_match_oracle(launch):
    """The batched workload's grid sizes (64^3, 128^3, 192^3, each with its own
    survey) advance in the same launches, either one launch per stage over all
    chains (launch 0: the mixed-size kernels) or one launch per grid size
    (launch -1); every chain matches its own oracle trajectory."""
    names = ["grp64", "grp128", "grp192"]
    mks = [mock(x) for x in names]
    eps, nsteps = 0.03, 6
    specs = [chain_spec(m, eps=eps, nsteps=nsteps, seed=9, chain_id=i) for i, m in enumerate(mks)]
    s = Sampler(specs)
    for cls in range(3):
        s.set_launch(cls, launch)
    posts = []
    for i, m in enumerate(mks):
        a32, b32 = coefficients32(m)
        s.set_coefficients(i, a32, b32)
        s.set_state(i, start_state(m)[0])
        posts.append(oracle_posterior(m, a32, b32, workers=16))
    for traj in range(2):
        befores = [s.state(i)["delta_k"] for i in range(3)]
        dH, acc = s.trajectory(traj)
        for i in range(3):
            ref = hmc.trajectory(befores[i].astype(np.complex128), posts[i], eps, nsteps, 9, i, traj)
            st = s.state(i)
            e_p = rel_l2(st["mom_k"], ref["p1"])
            print(f"launch {launch} {names[i]} traj {traj}: dH {dH[i]:.6e}/{ref['dH']:.6e} "
                  f"p rel-L2 {e_p:.2e} acc {acc[i]}/{ref['accepted']}", flush=True)
            assert e_p < 1e-4, i
            tol = dh_tol(mks[i]["cfg"].n)
            assert abs(dH[i] - ref["dH"]) < tol, i
            if abs(ref["log_u"] + ref["dH"]) > tol:
                assert bool(acc[i]) == ref["accepted"], i
            if acc[i] and ref["accepted"]:
                assert rel_l2(st["delta_k"], ref["proposal"]) < 1e-4, i
    s.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("plan", [1, 2, 3])
@pytest.mark.parametrize("n,box,nb", [s for s in SIZES if s[0] >= 64])
def test_radix_plans_match_oracle(n, box, nb, plan):
    """The alternative radix plans and tile shape (plan 3: twice the threads per
    pencil) of the step, y and force passes, with the separate y and real-space
    passes: the gradient of set_state (y passes, force pass) and a trajectory (step
    pass) against the oracle; a plan's results are reproducible."""
    mk = plain_mock(n, box, nb, nsub=2)
    a32, b32 = coefficients32(mk)
    post = oracle_posterior(mk, a32, b32, workers=8)
    d32, dk = start_state(mk)
    f, gk, delta = model.force_k(dk, post.lam_k, post.alpha, post.beta)
    gk[0, 0, 0] = 0.0
    finals = []
    for rep in range(2):
        s = sampler_for(mk, eps=0.05, nsteps=6, seed=23)
        s.set_plane_pass(False)
        for cls in range(3):
            s.set_plan(cls, plan)
        assert s.launch_config()[1] == [plan] * 3
        s.set_coefficients(0, a32, b32)
        s.set_state(0, d32)
        st = s.state(0)
        err = rel_l2(st["grad_k"], gk)
        print(f"N={n} plan {plan}: gradient rel-L2 {err:.2e}")
        assert err < 1e-5
        if n <= 128 or plan == 3:
            before = s.state(0)
            dH, acc = s.trajectory(0)
            ref = hmc.trajectory(before["delta_k"].astype(np.complex128), post, 0.05, 6, 23, 0, 0)
            e_p = rel_l2(s.state(0)["mom_k"], ref["p1"])
            print(f"N={n} plan {plan}: dH {dH[0]:.6e} oracle {ref['dH']:.6e}, p rel-L2 {e_p:.2e}")
            assert e_p < 1e-4
            finals.append((dH[0], s.state(0)["delta_k"]))
        s.close()
    if finals:
        assert finals[0][0] == finals[1][0] and np.array_equal(finals[0][1], finals[1][1])


def test_init_rejects_unobserved_subsample_and_empty_shells():
    """Degenerate inputs the method cannot sample: a subsample without any voxel
    with R > 0 (the Nbar conditional is improper) and more shells than the grid
    fills; both fail at init with HMC_EINVAL and a message."""
    from paper_1306_1821_amd.binding import HmcError
    mk = plain_mock(16, 500.0, 8, nsub=2)
    R = np.array(mk["R"])
    R[1] = 0.0
    counts = np.array(mk["counts"])
    counts[1] = 0.0
    spec = chain_spec(mk, R=R, counts=counts)
    with pytest.raises(HmcError, match="no voxel with R > 0"):
        Sampler([spec])
    with pytest.raises(HmcError, match="no modes"):
        Sampler([chain_spec(plain_mock(8, 500.0, 4), nb=64, pk=np.full(64, 1e4))])
