"""Pins for oracle.rj: the joint (P, delta) move."""
import numpy as np
import pytest

from oracle import gibbs, grid, hmc, model, rj
from synth import CONFIGS, make_mock


def setup(alpha_prior=1.0):
    mk = make_mock(CONFIGS["tiny8x2"])
    cfg = mk["cfg"]
    post = hmc.make_posterior(cfg.n, cfg.box, cfg.nb, mk["pk_init"], mk["R"], mk["counts"],
                              mk["bias"], mk["nbar"])
    lam = model.lambdas(mk["pk_init"], cfg.n, cfg.box)
    dk = grid.fwd(mk["delta"])
    dk[0, 0, 0] = 0
    rcfg = dict(eps=0.1, nsteps=10, alpha_prior=alpha_prior, seed=21, chain=0,
                lam_lo=lam * np.exp(-10), lam_hi=lam * np.exp(10))
    return mk, cfg, post, lam, dk, rcfg


def test_theta_gradient_finite_differences():
    mk, cfg, post, lam, dk, rcfg = setup()
    th0 = np.log(lam)
    rng = np.random.default_rng(3)
    th = th0 + 0.3 * rng.standard_normal(th0.shape)
    U, dU, *_ = rj.potential(th, th0, dk, post, 1.0)
    for m in range(len(th)):
        e = np.zeros_like(th)
        e[m] = 1e-6
        fd = (rj.potential(th + e, th0, dk, post, 1.0)[0]
              - rj.potential(th - e, th0, dk, post, 1.0)[0]) / 2e-6
        assert abs(fd - dU[m]) < 1e-6 * max(1.0, abs(fd))


def test_potential_is_likelihood_of_rescaled_field():
    """U(theta) - (alpha-1) sum theta equals psi_data at delta_hat sqrt(lambda'/lambda)."""
    mk, cfg, post, lam, dk, rcfg = setup()
    th0 = np.log(lam)
    th = th0 + np.array([0.2, -0.1, 0.05, 0.3])
    U, _, dkt, delta, _ = rj.potential(th, th0, dk, post, 0.0)
    scale = np.sqrt(np.exp(th) / lam)[np.maximum(post.shells, 0)]
    want = grid.inv(np.where(post.shells >= 0, dk * scale, 0), cfg.n)
    assert np.max(np.abs(delta - want)) < 1e-12
    assert abs(U + th.sum() - model.psi_data(want, post.alpha, post.beta)) < 1e-9 * abs(U)


def test_reflection_keeps_bounds_and_flips_momentum():
    th, rho = rj._reflect(np.array([0.5, 2.5, -1.7]), np.array([1.0, 1.0, -1.0]), -1.0, 2.0)
    assert np.allclose(th, [0.5, 1.5, -0.3]) and np.allclose(rho, [1.0, -1.0, 1.0])


def test_joint_move_runs_backwards_to_its_start():
    """Detailed balance needs a reversible map: from the proposal's end point with
    the momentum negated, the move (same mass, same integrator) returns to the
    start, and its energy error is the negative of the forward one."""
    mk, cfg, post, lam, dk, rcfg = setup()
    nm = grid.mode_counts(cfg.n, cfg.nb)
    r = dict(rcfg, eps=0.15, nsteps=12)
    fwd = rj.joint_move(dk, lam, post, nm, r, 3)
    assert np.max(np.abs(fwd["theta"] - np.log(lam))) > 0.05      # the move went somewhere
    back = rj.joint_move(fwd["dk_prop"], np.exp(fwd["theta"]), post, nm, r, 3, rho0=-fwd["rho"])
    assert np.allclose(back["mass"], fwd["mass"], rtol=0, atol=0)
    assert np.max(np.abs(back["theta"] - np.log(lam))) < 1e-10
    assert abs(back["dH"] + fwd["dH"]) < 1e-8 * max(1.0, abs(fwd["H0"]))
    dkb = back["dk_prop"]
    assert np.max(np.abs(dkb - dk)) < 1e-10 * np.max(np.abs(dk))


def test_joint_move_reports_wall_hits():
    """Walls one step away are hit and counted; distant walls are not."""
    mk, cfg, post, lam, dk, rcfg = setup()
    nm = grid.mode_counts(cfg.n, cfg.nb)
    far = rj.joint_move(dk, lam, post, nm, rcfg, 5)
    assert far["wall_hits"] == 0
    near = rj.joint_move(dk, lam, post, nm, dict(rcfg, lam_lo=lam * np.exp(-0.05),
                                                 lam_hi=lam * np.exp(0.05)), 5)
    assert near["wall_hits"] > 0
    assert np.all(np.abs(near["theta"] - np.log(lam)) <= 0.05 + 1e-12)


def test_joint_move_energy_error_second_order():
    mk, cfg, post, lam, dk, rcfg = setup()
    nm = grid.mode_counts(cfg.n, cfg.nb)
    errs = []
    for eps, n in [(0.1, 10), (0.05, 20), (0.025, 40)]:
        r = dict(rcfg, eps=eps, nsteps=n)
        errs.append(abs(rj.joint_move(dk, lam, post, nm, r, 0)["dH"]))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.15), slopes


@pytest.mark.slow
def test_joint_move_preserves_power_posterior():
    """Chains {delta-HMC + inverse-Gamma P} and {delta-HMC + joint move} agree on P.

    With a proper prior (alpha = 0) both kernels leave the joint posterior of
    (delta, P) invariant (eq. INVERSE_GAMMA and Appendix C's
    eq. spec_posterior_MIXING_1), so the marginal of ln P per shell must be the
    same.  6000 sweeps per arm: a joint move whose HMC mass follows theta, the
    variable it moves, shifts the mean of ln P on the first shell by half a
    posterior standard deviation (about 6.7 ESS-based standard errors here),
    which the 4-standard-error window catches.  The variance ratio is checked on
    the two data-dominated shells only: the noise-dominated ones have rare long
    excursions into low P that make their variance estimate unreliable at this
    length (their means are still compared).
    """
    mk, cfg, post0, lam0, dk0, rcfg = setup(alpha_prior=0.0)
    nm = grid.mode_counts(cfg.n, cfg.nb)
    n, box, nb = cfg.n, cfg.box, cfg.nb

    def run(use_rj, nsweep=6000):
        dk, lam = dk0.copy(), lam0.copy()
        out = []
        for s in range(nsweep):
            post = hmc.make_posterior(n, box, nb, lam * box ** 3 / n ** 3, mk["R"], mk["counts"],
                                      mk["bias"], mk["nbar"])
            dk = hmc.trajectory(dk, post, 0.2, 6 + s % 5, 31 + use_rj, 0, s)["state"]
            if use_rj:
                jm = rj.joint_move(dk, lam, post, nm, dict(rcfg, seed=41, eps=0.15, nsteps=8), s)
                dk, lam = jm["dk"], jm["lam"]
            else:
                lam = gibbs.draw_power(grid.shell_sums(dk, nb), nm, lam, 0.0, 51, 0, s)
            out.append(np.log(lam))
        return np.array(out[200:])

    a = run(False)
    b = run(True)
    from test_oracle_hmc import _ess
    for m in range(nb):
        ea, eb = _ess(a[:, m]), _ess(b[:, m])
        se = np.sqrt(a[:, m].var() / ea + b[:, m].var() / eb)
        assert abs(a[:, m].mean() - b[:, m].mean()) < 4 * se, (m, (b[:, m].mean() - a[:, m].mean()) / se)
    for m in (0, 1):
        assert 0.75 < b[:, m].var() / a[:, m].var() < 1.33, m
