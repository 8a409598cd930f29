"""Oracle: the joint (P, delta) move (test infrastructure only).

Sec. "Exploring the low signal to noise regime" and Appendix C: following Jewell
et al. (2009) the density is moved deterministically with the power spectrum,
delta_hat' = sqrt(P'/P) delta_hat (eq. det_trans), and P' is drawn from
P(P' | u, d) ~ P(P') prod_l exp(-chi^2_l(delta(P', u)) / 2)
(eq. spec_posterior_MIXING_1) with HMC, as the paper prescribes, instead of a
plain Metropolis step.

Readings:
* the whitened field is u_k = delta_hat_k / sqrt(lambda_k) (the paper's
  delta_hat / P is inconsistent with delta_hat' = sqrt(P') u); the Jacobian
  prod sqrt(P'/P) of the transition cancels the det S ratio of the prior, so
  the target in P given u is the P prior times the likelihood only;
* HMC runs in theta_m = ln lambda_m, so the power-law prior P^-alpha becomes
  the potential (alpha - 1) theta_m; the potential is
  U(theta) = psi_data(F^-1(e^(theta/2) u)) + (alpha - 1) sum_m theta_m with
  dU/dtheta_m = 1/2 sum_{k in m} w_k Re(conj(delta_hat_k) g_hat_k) + (alpha - 1),
  g_hat = F(alpha_i delta_i - beta_i);
* mass M_m = max(1, n_m lambda_ref,m mean(alpha) / 4) (a Gauss-Newton estimate of
  the curvature) with lambda_ref the fixed reference at the centre of the walls
  below (the lambda the chain started from), the same eps and step count as the
  density HMC, KDK.  The mass may depend on anything the move holds fixed (u, b,
  Nbar, hence mean(alpha)) but not on theta: with a mass taken at the current
  theta the reverse move from theta' would run another leapfrog map and the
  Metropolis test would no longer give detailed balance;
* theta is confined to [ln lambda_lo, ln lambda_hi] by reflection (position
  mirrored, momentum negated), which keeps the integrator reversible and
  volume preserving; with the Jeffreys prior the target is flat as theta -> -inf
  for shells the data barely inform, so a bound is needed; every reflection
  is counted and reported;
* momenta from Philox stream 8 (element m), accept uniform from stream 9.
"""
import numpy as np

from . import grid, model, philox


def _reflect(theta, rho, lo, hi, hits=None):
    """Mirror theta into [lo, hi], negating rho once per reflection; hits[m] counts them."""
    theta = theta.copy()
    rho = rho.copy()
    for _ in range(64):
        over = theta > hi
        under = theta < lo
        if not (over.any() or under.any()):
            break
        theta = np.where(over, 2.0 * hi - theta, theta)
        theta = np.where(under, 2.0 * lo - theta, theta)
        rho = np.where(over | under, -rho, rho)
        if hits is not None:
            hits += (over | under)
    return theta, rho


def potential(theta, theta0, dk0, post, alpha_prior):
    """U(theta), dU/dtheta and the field at theta (delta_hat, delta, grad_hat)."""
    nb = post.nb
    scale = np.exp(0.5 * (theta - theta0))
    sel = post.shells >= 0
    dk = np.where(sel, dk0 * scale[np.where(sel, post.shells, 0)], 0.0)
    delta = grid.inv(dk, post.n, post.workers)
    g = post.alpha * delta - post.beta
    gk = grid.fwd(g, post.workers)
    dots = np.bincount(post.shells[sel], weights=(post.w * np.real(np.conj(dk) * gk))[sel],
                       minlength=nb)
    U = model.psi_data(delta, post.alpha, post.beta) + (alpha_prior - 1.0) * float(theta.sum())
    dU = 0.5 * dots + (alpha_prior - 1.0)
    return U, dU, dk, delta, gk


def joint_move(dk, lam, post, n_modes, cfg, s, rho0=None):
    """One HMC proposal in theta = ln lambda at fixed u; returns the new (dk, lam).

    rho0 replaces the Philox momentum draw when given (used to run a move
    backwards from a proposal's end point).
    """
    eps, nsteps, ap = cfg["eps"], cfg["nsteps"], cfg["alpha_prior"]
    seed, chain = cfg["seed"], cfg["chain"]
    lo = np.log(cfg["lam_lo"])
    hi = np.log(cfg["lam_hi"])
    theta0 = np.log(np.asarray(lam, dtype=np.float64))
    lam_ref = np.sqrt(np.asarray(cfg["lam_lo"], float) * np.asarray(cfg["lam_hi"], float))
    mass = np.maximum(1.0, 0.25 * n_modes * lam_ref * post.abar)
    if rho0 is None:
        rho0 = np.sqrt(mass) * philox.normals(seed, chain, philox.STREAM_RJ_MOMENTA, s, len(lam))
    rho0 = np.asarray(rho0, dtype=np.float64)
    U0, dU, _, _, _ = potential(theta0, theta0, dk, post, ap)
    H0 = 0.5 * float(np.sum(rho0 * rho0 / mass)) + U0
    theta, rho = theta0.copy(), rho0 - 0.5 * eps * dU
    hits = np.zeros(len(lam), dtype=np.int64)
    for i in range(nsteps):
        theta = theta + eps * rho / mass
        theta, rho = _reflect(theta, rho, lo, hi, hits)
        U1, dU, dk1, delta1, gk1 = potential(theta, theta0, dk, post, ap)
        rho = rho - (eps if i < nsteps - 1 else 0.5 * eps) * dU
    H1 = 0.5 * float(np.sum(rho * rho / mass)) + U1
    dH = H1 - H0
    u = philox.uniform(seed, chain, philox.STREAM_RJ_ACCEPT, s)
    acc = bool(np.log(u) < -dH)
    return dict(dH=dH, accepted=acc, log_u=float(np.log(u)), theta=theta, rho=rho, H0=H0, H1=H1,
                mass=mass,
                wall_hits=int(hits.sum()), dk_prop=dk1,
                dk=dk1 if acc else dk, lam=np.exp(theta) if acc else np.asarray(lam, float),
                grad=gk1 if acc else None)
