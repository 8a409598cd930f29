"""Pins for oracle.model: potential and force against their definitions."""
import numpy as np

import dense
from oracle import grid, model
from synth import CONFIGS, make_mock


def setup(name="tiny8x2"):
    mk = make_mock(CONFIGS[name])
    cfg = mk["cfg"]
    n, nb = cfg.n, cfg.nb
    alpha, beta, abar = model.coefficients(mk["R"], mk["counts"], mk["bias"], mk["nbar"])
    shells = grid.half_shells(n, nb)
    lam_k = model.per_mode(model.lambdas(mk["pk_init"], n, cfg.box), shells)
    return mk, cfg, alpha, beta, abar, shells, lam_k


def test_expanded_data_term_differs_by_constant():
    mk, cfg, alpha, beta, *_ = setup()
    rng = np.random.default_rng(5)
    vals = []
    for _ in range(4):
        d = 0.5 * rng.standard_normal(alpha.shape)
        vals.append(model.psi_data_direct(d, mk["R"], mk["counts"], mk["bias"], mk["nbar"])
                    - model.psi_data(d, alpha, beta))
    assert np.ptp(vals) < 1e-9 * abs(vals[0])


def test_alpha_beta_zero_where_unobserved():
    mk, cfg, alpha, beta, *_ = setup()
    obs = (mk["R"] > 0).any(axis=0)
    assert np.all(alpha[~obs] == 0) and np.all(beta[~obs] == 0)
    assert np.all(alpha[obs] > 0)


def test_gradient_finite_differences():
    mk, cfg, alpha, beta, abar, shells, lam_k = setup()
    w = grid.half_weights(cfg.n)
    rng = np.random.default_rng(6)
    d = grid.inv(grid.fwd(0.5 * rng.standard_normal(alpha.shape)), cfg.n)
    g = model.grad_real(d, lam_k, alpha, beta)
    for _ in range(5):
        v = rng.standard_normal(d.shape)
        h = 1e-5
        fd = (model.psi_total(d + h * v, lam_k, w, alpha, beta)
              - model.psi_total(d - h * v, lam_k, w, alpha, beta)) / (2 * h)
        assert abs(fd - np.sum(g * v)) < 1e-7 * max(1.0, abs(fd))


def test_force_matches_dense_precision():
    """F^-1 of force_k equals P (Q delta - beta), Q = S^-1 + diag(alpha), P the mean projector."""
    mk, cfg, alpha, beta, abar, shells, lam_k = setup()
    n = cfg.n
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    mu, cov, Q, U = dense.wiener(n, lam_m, cfg.nb, alpha, beta)
    rng = np.random.default_rng(7)
    d = rng.standard_normal(n ** 3)
    d -= d.mean()
    f, gk, delta = model.force_k(grid.fwd(d.reshape(n, n, n)), lam_k, alpha, beta)
    ref = Q @ d - beta.reshape(-1)
    ref -= ref.mean()
    got = grid.inv(f, n).reshape(-1)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def test_mass_is_fourier_diagonal_of_precision():
    """m_k = 1/lambda + mean(alpha) is the diagonal of F Q F^H (eq. Mass_matrix)."""
    mk, cfg, alpha, beta, abar, shells, lam_k = setup()
    n = cfg.n
    lam_m = model.lambdas(mk["pk_init"], n, cfg.box)
    _, _, Q, _ = dense.wiener(n, lam_m, cfg.nb, alpha, beta)
    F = dense.dft_matrix(n)
    diag = np.real(np.einsum("ij,jk,ik->i", F, Q, F.conj()))
    sh = dense.shell_full(n, cfg.nb)
    want = model.mass_table(lam_m, abar)[np.maximum(sh, 0)]
    sel = sh >= 0
    assert np.allclose(diag[sel], want[sel], rtol=1e-10)


def _growth(mk):
    n, box = mk["cfg"].n, mk["cfg"].box
    c = (np.arange(n) + 0.5) * box / n - 0.5 * box
    r = np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)
    return 1.0 / (1.0 + r / 400.0)


def test_growth_factor_data_term_differs_by_constant():
    """Per-voxel growth factor (a variant the paper's data model allows): psi_data with
    the coefficients of D+ equals the likelihood written straight from eq. data_model,
    mean counts Nbar R (1 + b D+ delta), up to a constant."""
    mk = make_mock(CONFIGS["tiny8x2"])
    g = _growth(mk)
    alpha, beta, _ = model.coefficients(mk["R"], mk["counts"], mk["bias"], mk["nbar"], g)
    rng = np.random.default_rng(15)
    vals = []
    for _ in range(4):
        d = 0.5 * rng.standard_normal(alpha.shape)
        direct = 0.0
        for l in range(mk["R"].shape[0]):
            obs = mk["R"][l] > 0
            r = mk["R"][l][obs]
            res = mk["counts"][l][obs] - mk["nbar"][l] * r * (1 + mk["bias"][l] * g[obs] * d[obs])
            direct += 0.5 * np.sum(res ** 2 / (mk["nbar"][l] * r))
        vals.append(direct - model.psi_data(d, alpha, beta))
    assert np.ptp(vals) < 1e-9 * abs(vals[0])


def test_growth_factor_bias_conditional_mean():
    """With D+ the bias conditional's mean D/C from the moments of D+ delta is the
    minimiser over b of the data-model likelihood (a parabola in b)."""
    from oracle import gibbs
    mk = make_mock(CONFIGS["tiny8x2"])
    g = _growth(mk)
    rng = np.random.default_rng(16)
    d = 0.5 * rng.standard_normal(g.shape)
    mom = gibbs.delta_moments(g * d, mk["R"], mk["counts"])
    for l in range(mk["R"].shape[0]):
        obs = mk["R"][l] > 0
        r, nb = mk["R"][l][obs], mk["nbar"][l]

        def psi(b):
            res = mk["counts"][l][obs] - nb * r * (1 + b * g[obs] * d[obs])
            return 0.5 * np.sum(res ** 2 / (nb * r))
        b0, h = 1.0, 0.5
        f0, fp, fm = psi(b0), psi(b0 + h), psi(b0 - h)
        b_min = b0 - h * (fp - fm) / (2 * (fp - 2 * f0 + fm))
        S1, S2, T = mom[l]
        assert abs((T - nb * S1) / (nb * S2) - b_min) < 1e-9 * max(1.0, abs(b_min))
