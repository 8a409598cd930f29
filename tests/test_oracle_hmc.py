"""Pins for oracle.hmc: integrator properties and exactness against the dense Wiener posterior."""
import numpy as np
import pytest

import dense
from oracle import grid, hmc, model
from synth import CONFIGS, make_mock


def posterior(name="tiny8x2", delta_start=True):
    mk = make_mock(CONFIGS[name])
    cfg = mk["cfg"]
    post = hmc.make_posterior(cfg.n, cfg.box, cfg.nb, mk["pk_init"], mk["R"], mk["counts"],
                              mk["bias"], mk["nbar"])
    dk = grid.fwd(mk["delta"]) if delta_start else np.zeros((cfg.n, cfg.n, cfg.n // 2 + 1), complex)
    dk[0, 0, 0] = 0
    return mk, cfg, post, dk


def test_reversibility():
    mk, cfg, post, dk = posterior()
    p = hmc.draw_momentum(post, 3, 0, 0)
    d1, p1, _, _ = hmc.leapfrog(dk, p, post, 0.1, 15)
    d2, p2, _, _ = hmc.leapfrog(d1, -p1, post, 0.1, 15)
    assert np.max(np.abs(d2 - dk)) < 1e-11 * np.max(np.abs(dk))
    assert np.max(np.abs(p2 + p)) < 1e-11 * np.max(np.abs(p))


def test_energy_error_is_second_order():
    mk, cfg, post, dk = posterior()
    p = hmc.draw_momentum(post, 4, 0, 0)
    d0 = grid.inv(dk, cfg.n)
    H0 = sum(hmc.energies(dk, p, d0, post))
    errs = []
    for eps, n in [(0.1, 10), (0.05, 20), (0.025, 40), (0.0125, 80)]:
        d1, p1, _, x1 = hmc.leapfrog(dk, p, post, eps, n)
        errs.append(abs(sum(hmc.energies(d1, p1, x1, post)) - H0))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.1), slopes


def test_leapfrog_equals_dense_affine_map():
    """The FFT leapfrog equals iterating the dense affine KDK map in real space."""
    mk, cfg, post, dk = posterior()
    n = cfg.n
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    _, _, Q, U = dense.wiener(n, lam_m, cfg.nb, post.alpha, post.beta)
    sh = dense.shell_full(n, cfg.nb)
    inv_m = np.where(sh >= 0, 1.0 / model.mass_table(lam_m, post.abar)[np.maximum(sh, 0)], 0.0)
    Minv = dense.fourier_diag_operator(n, inv_m)
    P = U @ U.T
    b = P @ post.beta.reshape(-1)
    pk = hmc.draw_momentum(post, 5, 0, 0)
    eps, steps = 0.12, 9
    d = grid.inv(dk, n).reshape(-1)
    p = grid.inv(pk, n).reshape(-1)
    f = lambda x: P @ (Q @ x) - b
    p = p - 0.5 * eps * f(d)
    for s in range(steps):
        d = d + eps * Minv @ p
        p = p - (eps if s < steps - 1 else 0.5 * eps) * f(d)
    d1, p1, _, _ = hmc.leapfrog(dk, pk, post, eps, steps)
    assert np.max(np.abs(grid.inv(d1, n).reshape(-1) - d)) < 1e-11 * np.max(np.abs(d))
    assert np.max(np.abs(grid.inv(p1, n).reshape(-1) - p)) < 1e-11 * np.max(np.abs(p))
    # volume preservation: the linear part of one step has unit determinant on the subspace
    I = np.eye(n ** 3)
    A11 = I - eps * eps / 2 * Minv @ P @ Q
    lin = np.block([[A11, eps * Minv],
                    [-eps * P @ Q + eps ** 3 / 4 * P @ Q @ Minv @ P @ Q, I - eps * eps / 2 * P @ Q @ Minv]])
    W = np.block([[U, np.zeros_like(U)], [np.zeros_like(U), U]])
    sign, logdet = np.linalg.slogdet(W.T @ lin @ W)
    assert sign > 0 and abs(logdet) < 1e-8


def _ess(x):
    """Effective sample size by Geyer's initial positive sequence (plain numpy)."""
    x = np.asarray(x) - np.mean(x)
    n = len(x)
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n] / (np.arange(n, 0, -1))
    ac /= ac[0]
    s = 0.0
    for t in range(1, n // 2):
        pair = ac[2 * t - 1] + ac[2 * t]
        if pair < 0:
            break
        s += pair
    return n / max(1.0, 1.0 + 2.0 * (s + 0.0))


@pytest.mark.slow
def test_chain_matches_dense_wiener_posterior():
    """Fixed P, b, Nbar at 8^3: HMC draws have the closed-form Wiener mean and covariance."""
    mk, cfg, post, dk = posterior()
    n = cfg.n
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    mu, cov, Q, U = dense.wiener(n, lam_m, cfg.nb, post.alpha, post.beta)
    evals, evecs = np.linalg.eigh(U.T @ cov @ U)
    T = (U @ evecs) / np.sqrt(evals)            # whitening map on the subspace
    dk = grid.fwd(mu.reshape(n, n, n))
    samples = []
    acc = 0
    nsamp = 3000
    for t in range(nsamp):
        steps = 6 + (t % 7)                      # varied lengths avoid resonant trajectories
        tr = hmc.trajectory(dk, post, 0.2, steps, 11, 0, t)
        dk = tr["state"]
        acc += tr["accepted"]
        samples.append(grid.inv(dk, n).reshape(-1))
    S = np.array(samples)
    y = (S - mu) @ T                              # should be iid N(0, 1) per column
    assert acc / nsamp > 0.6
    ess = np.array([_ess(y[:, j]) for j in range(y.shape[1])])
    zmean = y.mean(axis=0) * np.sqrt(ess)
    assert np.max(np.abs(zmean)) < 5.0
    assert abs(np.mean(zmean ** 2) - 1.0) < 0.3
    var = y.var(axis=0)
    assert np.max(np.abs(var - 1.0) * np.sqrt(ess / 2.0)) < 6.0
    assert abs(var.mean() - 1.0) < 0.03


def test_learned_mass_with_unit_D_is_plain_leapfrog():
    mk, cfg, post, dk = posterior()
    p = hmc.draw_momentum(post, 6, 0, 0)
    one = np.ones((cfg.n,) * 3)
    d1, p1, _, _ = hmc.leapfrog(dk, p, post, 0.1, 7)
    d2, p2, _ = hmc.leapfrog_learned(dk, p, post, one, 0.1, 7)
    assert np.max(np.abs(d1 - d2)) < 1e-11 * np.max(np.abs(d1))
    assert np.max(np.abs(p1 - p2)) < 1e-11 * np.max(np.abs(p1))


def test_learned_mass_leapfrog_is_dense_affine_map():
    """In the variables (delta, pi) with pi = F^-1(p_hat / sqrt(m)) the learned leapfrog is
    delta' = T pi, pi' = -T^T (Q delta - beta), T = P S C, S = diag(D^(1/2)),
    C = F^-1 diag(m^-1/2) F: checked against those dense matrices at 8^3."""
    mk, cfg, post, dk = posterior()
    n = cfg.n
    rng = np.random.default_rng(12)
    sqrtD = hmc.mass_factor(0.5 * rng.standard_normal((n, n, n)))
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    _, _, Q, U = dense.wiener(n, lam_m, cfg.nb, post.alpha, post.beta)
    sh = dense.shell_full(n, cfg.nb)
    isq = np.where(sh >= 0, 1.0 / np.sqrt(model.mass_table(lam_m, post.abar)[np.maximum(sh, 0)]), 0.0)
    C = dense.fourier_diag_operator(n, isq)
    P = U @ U.T
    T = P @ (sqrtD.reshape(-1)[:, None] * C)
    beta = post.beta.reshape(-1)
    pk = hmc.draw_momentum(post, 8, 0, 0)
    sel = post.shells >= 0
    eps, steps = 0.1, 6
    d = grid.inv(dk, n).reshape(-1)
    pi = grid.inv(np.where(sel, pk / np.sqrt(np.where(sel, post.mass_k, 1.0)), 0.0), n).reshape(-1)
    pi = pi - 0.5 * eps * T.T @ (Q @ d - beta)
    for i in range(steps):
        d = d + eps * T @ pi
        pi = pi - (eps if i < steps - 1 else 0.5 * eps) * T.T @ (Q @ d - beta)
    d1, p1, _ = hmc.leapfrog_learned(dk, pk, post, sqrtD, eps, steps)
    pi1 = grid.inv(np.where(sel, p1 / np.sqrt(np.where(sel, post.mass_k, 1.0)), 0.0), n).reshape(-1)
    assert np.max(np.abs(grid.inv(d1, n).reshape(-1) - d)) < 1e-10 * np.max(np.abs(d))
    assert np.max(np.abs(pi1 - pi)) < 1e-10 * np.max(np.abs(pi))


@pytest.mark.slow
def test_learned_mass_chain_matches_dense_wiener_posterior():
    """The learned-mass HMC targets the same Wiener posterior (8^3, fixed P, b, Nbar)."""
    mk, cfg, post, dk = posterior()
    n = cfg.n
    rng = np.random.default_rng(14)
    sqrtD = hmc.mass_factor(0.5 * rng.standard_normal((n, n, n)))
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    mu, cov, Q, U = dense.wiener(n, lam_m, cfg.nb, post.alpha, post.beta)
    evals, evecs = np.linalg.eigh(U.T @ cov @ U)
    W = (U @ evecs) / np.sqrt(evals)
    dk = grid.fwd(mu.reshape(n, n, n))
    S, acc = [], 0
    for t in range(2500):
        tr = hmc.trajectory_learned(dk, post, sqrtD, 0.15, 6 + (t % 7), 19, 0, t)
        dk = tr["state"]
        acc += tr["accepted"]
        S.append(grid.inv(dk, n).reshape(-1))
    y = (np.array(S) - mu) @ W
    assert acc / 2500 > 0.5
    ess = np.array([_ess(y[:, j]) for j in range(y.shape[1])])
    zmean = y.mean(axis=0) * np.sqrt(ess)
    assert np.max(np.abs(zmean)) < 5.0
    assert abs(np.mean(zmean ** 2) - 1.0) < 0.3
    assert abs(y.var(axis=0).mean() - 1.0) < 0.04


def test_learned_mass_reversible_and_second_order():
    mk, cfg, post, dk = posterior()
    rng = np.random.default_rng(13)
    sqrtD = hmc.mass_factor(0.4 * rng.standard_normal((cfg.n,) * 3))
    p = hmc.draw_momentum(post, 9, 0, 0)
    d1, p1, _ = hmc.leapfrog_learned(dk, p, post, sqrtD, 0.1, 10)
    d2, p2, _ = hmc.leapfrog_learned(d1, -p1, post, sqrtD, 0.1, 10)
    assert np.max(np.abs(d2 - dk)) < 1e-10 * np.max(np.abs(dk))
    d0 = grid.inv(dk, cfg.n)
    H0 = sum(hmc.energies(dk, p, d0, post))
    errs = []
    for eps, n in [(0.1, 10), (0.05, 20), (0.025, 40)]:
        a, b, x = hmc.leapfrog_learned(dk, p, post, sqrtD, eps, n)
        errs.append(abs(sum(hmc.energies(a, b, x, post)) - H0))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.15), slopes


def test_diagonal_mass_drift_is_p_diag_v_p_minus_rank_one():
    """Real-space diagonal variant (reading of the mass freedom after eq.
    Mass_matrix): a real-space momentum r (zero mean) enters as p_hat =
    F(D^(1/2) r) with its k = 0 entry zeroed (the whitened mean stays frozen), and
    the drift velocity is the inverse mass applied to r,
        P diag(v) r - mean(v) (s . r / N^3) P s,   s = D^(1/2) = sqrt(v / mean(v)):
    P diag(v) P up to one rank-one term, positive on the zero-mean fields.  Checked
    against that expanded form with numpy's FFT, and the kinetic energy against
    1/2 mean(v) |s r - mean(s r)|^2."""
    mk, cfg, post, dk = posterior()
    n = cfg.n
    rng = np.random.default_rng(31)
    lv = 0.7 * rng.standard_normal((n, n, n)) - 1.5
    post_d, sqrtD = hmc.diagonal_mass(post, lv)
    v = np.exp(lv)
    mv = v.mean()
    r = rng.standard_normal((n, n, n))
    r -= r.mean()
    pk = np.fft.rfftn(sqrtD * r, norm="ortho")
    pk[0, 0, 0] = 0.0
    got = hmc.learned_velocity(pk, post_d, sqrtD)
    s = np.sqrt(v / mv)
    w = v * r
    y = (w - w.mean()) - mv * np.mean(s * r) * (s - s.mean())
    want = np.fft.rfftn(y, norm="ortho")
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    kin = hmc.energies(dk, pk, grid.inv(dk, n), post_d)[0]
    q = s * r - np.mean(s * r)
    assert abs(kin - 0.5 * mv * np.sum(q * q)) < 1e-10 * kin


def test_diagonal_mass_reversible_and_second_order():
    mk, cfg, post, dk = posterior()
    rng = np.random.default_rng(17)
    post_d, sqrtD = hmc.diagonal_mass(post, 0.6 * rng.standard_normal((cfg.n,) * 3) - 2.0)
    p = hmc.draw_momentum(post_d, 5, 0, 0)
    d1, p1, _ = hmc.leapfrog_learned(dk, p, post_d, sqrtD, 0.05, 10)
    d2, p2, _ = hmc.leapfrog_learned(d1, -p1, post_d, sqrtD, 0.05, 10)
    assert np.max(np.abs(d2 - dk)) < 1e-10 * np.max(np.abs(dk))
    H0 = sum(hmc.energies(dk, p, grid.inv(dk, cfg.n), post_d))
    errs = []
    for eps, k in [(0.02, 10), (0.01, 20), (0.005, 40)]:
        a, b, x = hmc.leapfrog_learned(dk, p, post_d, sqrtD, eps, k)
        errs.append(abs(sum(hmc.energies(a, b, x, post_d)) - H0))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.15), (errs, slopes)


def _lam_full(post, n, nb):
    sh = dense.shell_full(n, nb)
    lam_m = np.zeros(nb)
    for m in range(nb):
        lam_m[m] = post.lam_k[post.shells == m][0]
    return np.where(sh >= 0, lam_m[np.maximum(sh, 0)], 0.0)


def test_prior_draw_covariance_matches_dense_prior():
    """xi = F^-1(sqrt(lambda) F w) has covariance S = F^H diag(lambda) F (dense)."""
    mk, cfg, post, _ = posterior("tiny8")
    n = cfg.n
    S = dense.fourier_diag_operator(n, _lam_full(post, n, cfg.nb))
    K = 800
    X = np.stack([hmc.prior_draw(post, 5, 0, d).reshape(-1) for d in range(K)])
    C = X.T @ X / K
    rng = np.random.default_rng(3)
    x = np.arange(n)
    wave = np.cos(2 * np.pi * x / n)[:, None, None] * np.ones((n, n, n))
    e0 = np.zeros(n ** 3)
    e0[0] = 1.0
    pair = e0.copy()
    pair[1] = 1.0
    for u in [e0, pair, wave.reshape(-1), rng.standard_normal(n ** 3)]:
        ref = u @ S @ u
        assert abs(u @ C @ u / ref - 1.0) < 0.2, (u @ C @ u, ref)
    # per-voxel variance: N^-3 sum_k lambda_k
    assert abs(np.mean(np.diag(C)) / (np.sum(_lam_full(post, n, cfg.nb)) / n ** 3) - 1) < 0.05


def test_warm_start_mean_and_variance():
    """Over draws, delta has mean mu - mean(mu) and per-voxel variance exp(s)."""
    mk, cfg, post, _ = posterior("tiny8")
    n = cfg.n
    rng = np.random.default_rng(4)
    mu = 0.3 * rng.standard_normal((n, n, n))
    lv = np.log(0.05) + 0.6 * rng.standard_normal((n, n, n))
    K = 800
    D = np.stack([grid.inv(hmc.warm_start(mu, lv, post, 9, 1, d), n) for d in range(K)])
    v = np.exp(lv)
    z = (D.mean(axis=0) - (mu - mu.mean())) / np.sqrt(v / K)
    assert np.max(np.abs(z)) < 5.0
    ratio = D.var(axis=0) / v
    assert abs(ratio.mean() - 1.0) < 0.05
    assert np.corrcoef(D.var(axis=0).ravel(), v.ravel())[0, 1] > 0.9


def test_drawn_step_counts_are_uniform():
    """n = 1 + floor(u n_max) covers 1..n_max with equal frequency (chi-square)."""
    from scipy import stats
    n_max, K = 12, 6000
    draws = np.array([hmc.draw_steps(n_max, 7, 3, t) for t in range(K)])
    assert draws.min() == 1 and draws.max() == n_max
    counts = np.bincount(draws, minlength=n_max + 1)[1:]
    assert stats.chisquare(counts).pvalue > 1e-3
    # different chains and streams give different sequences
    other = np.array([hmc.draw_steps(n_max, 7, 4, t) for t in range(200)])
    assert np.mean(other != draws[:200]) > 0.8
