"""Oracle: the HMC density step (test infrastructure only).

Sec. "The HMC algorithm": with potential psi = -ln P (eq. Potential), momenta p
and mass M, H = 1/2 p^T M^-1 p + psi (eq. Hamiltonian).  A trajectory draws
p ~ N(0, M), integrates Hamilton's equations (eqs. HAMILTON1_a, HAMILTON2_a) with
a leapfrog scheme and accepts with probability min(1, exp(-dH))
(eq. acceptance_rule).

Readings (the paper leaves these open):
* the sign of eq. HAMILTON2: dp/dt = -d psi/dx, as used in eq. HAMILTON2_a;
* leapfrog ordering kick-drift-kick (half kick, n x [drift, kick], last kick
  halved), fixed step eps and step count n;
* the mass is diagonal in Fourier space (m_k of ``model.mass_table``), so the
  kinetic term is K = 1/2 sum_k |p_hat_k|^2 / m_k and p ~ N(0, M) is drawn as
  p_hat = sqrt(m_k) F w with w real white noise (Philox stream 3);
* the mean mode k = 0 is frozen: delta_hat_0 = p_hat_0 = 0 throughout;
* accept iff ln u < -dH with u from Philox stream 4 (strict inequality).

State variables are delta_hat (half grid) and p_hat; sums over the stored
half grid carry the full-grid weight w_k (``grid.half_weights``).
"""
from dataclasses import dataclass, replace

import numpy as np

from . import grid, model, philox


@dataclass
class Posterior:
    """Everything the density step holds fixed during one trajectory."""
    n: int
    box: float
    nb: int
    shells: np.ndarray
    w: np.ndarray
    lam_k: np.ndarray
    mass_k: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    abar: float
    workers: int = 1


def make_posterior(n, box, nb, pk, R, counts, bias, nbar, workers=1, growth=None):
    shells = grid.half_shells(n, nb)
    alpha, beta, abar = model.coefficients(R, counts, bias, nbar, growth)
    lam = model.lambdas(pk, n, box)
    return Posterior(n, box, nb, shells, grid.half_weights(n), model.per_mode(lam, shells),
                     model.per_mode(model.mass_table(lam, abar), shells), alpha, beta, abar,
                     workers)


def draw_momentum(post, seed, chain, traj):
    """p_hat = sqrt(m_k) F w, w ~ N(0, 1) per voxel from Philox stream 3."""
    n = post.n
    wn = philox.normals(seed, chain, philox.STREAM_MOMENTA, traj, n ** 3).reshape(n, n, n)
    wk = grid.fwd(wn, post.workers)
    return np.where(post.shells >= 0, np.sqrt(np.where(post.shells >= 0, post.mass_k, 1.0)) * wk,
                    0.0)


def energies(dk, pk, delta, post):
    """(kinetic, prior, data) parts of H for a given state."""
    sel = post.shells >= 0
    kin = 0.5 * np.sum((post.w * np.abs(pk) ** 2)[sel] / post.mass_k[sel])
    pri = 0.5 * np.sum((post.w * np.abs(dk) ** 2)[sel] / post.lam_k[sel])
    dat = model.psi_data(delta, post.alpha, post.beta)
    return float(kin), float(pri), float(dat)


def leapfrog(dk, pk, post, eps, nsteps):
    """KDK integration; returns (delta_hat, p_hat, grad_hat, delta) at the end."""
    f, gk, delta = model.force_k(dk, post.lam_k, post.alpha, post.beta, post.workers)
    inv_m = np.where(post.shells >= 0, 1.0 / np.where(post.shells >= 0, post.mass_k, 1.0), 0.0)
    pk = pk - 0.5 * eps * f
    for s in range(nsteps):
        dk = dk + eps * pk * inv_m
        f, gk, delta = model.force_k(dk, post.lam_k, post.alpha, post.beta, post.workers)
        pk = pk - (eps if s < nsteps - 1 else 0.5 * eps) * f
    return dk, pk, gk, delta


def draw_steps(n_max, seed, chain, traj):
    """Uniformly drawn pseudo-time (text after eq. HAMILTON2_a: tau is drawn from a
    uniform distribution): n = 1 + floor(u n_max), u from Philox stream 10, so that
    tau = n eps is uniform on {eps, 2 eps, ..., n_max eps}."""
    u = philox.uniform(seed, chain, philox.STREAM_TAU, traj)
    return min(n_max, 1 + int(u * n_max))


def trajectory(dk, post, eps, nsteps, seed, chain, traj):
    """One HMC proposal + accept.  Returns a dict with the new state and dH."""
    pk0 = draw_momentum(post, seed, chain, traj)
    delta0 = grid.inv(dk, post.n, post.workers)
    e0 = energies(dk, pk0, delta0, post)
    dk1, pk1, gk1, delta1 = leapfrog(dk, pk0, post, eps, nsteps)
    e1 = energies(dk1, pk1, delta1, post)
    dH = sum(e1) - sum(e0)
    u = philox.uniform(seed, chain, philox.STREAM_ACCEPT, traj)
    acc = bool(np.log(u) < -dH)
    return dict(p0=pk0, e0=e0, e1=e1, dH=dH, accepted=acc, log_u=float(np.log(u)),
                proposal=dk1, p1=pk1, grad1=gk1, delta1=delta1,
                state=dk1 if acc else dk)


# --------------------------------------------------------------------------- learned mass
# The mass only affects efficiency (text after eq. Mass_matrix).  The learned
# variant keeps the Fourier diagonal m_k and adds a real-space diagonal D from
# the network's variance.  Because the mean mode is frozen, the field is written
# delta = T z with T = P D^(1/2) F^-1 diag(m_k^-1/2) (P removes the mean) and z
# moves with unit mass, so the inverse mass on delta is T T^T =
# P D^(1/2) F^-1 diag(1/m_k) F D^(1/2) P (symmetric on the zero-mean subspace).
# Carrying the momentum as p_hat = sqrt(m_k) pi_hat (pi conjugate to z):
#   p ~ N(0, M)  is  p_hat = sqrt(m_k) F w (as for the plain mass),
#   kinetic      1/2 sum_k |p_hat|^2 / m_k,
#   kick         p_hat -= eps F(D^(1/2) P grad psi),
#   drift        delta_hat += eps [F(D^(1/2) F^-1(p_hat / m_k))]_{k != 0},
# grad psi = F^-1(delta_hat / lambda) + alpha delta - beta.  D = 1 gives the
# plain leapfrog.

def learned_force(dk, post, sqrtD):
    """F(D^(1/2) P grad psi) with the k = 0 entry zeroed; also returns delta."""
    n = post.n
    sel = post.shells >= 0
    delta = grid.inv(dk, n, post.workers)
    prior = grid.inv(np.where(sel, dk / np.where(sel, post.lam_k, 1.0), 0.0), n, post.workers)
    g = prior + post.alpha * delta - post.beta
    g = g - g.mean()                                   # P grad psi
    f = grid.fwd(sqrtD * g, post.workers)
    f[0, 0, 0] = 0.0
    return f, delta


def learned_velocity(pk, post, sqrtD):
    """F(D^(1/2) F^-1(p_hat' / m_k)) with the k = 0 entry zeroed."""
    n = post.n
    sel = post.shells >= 0
    q = grid.inv(np.where(sel, pk / np.where(sel, post.mass_k, 1.0), 0.0), n, post.workers)
    u = grid.fwd(sqrtD * q, post.workers)
    u[0, 0, 0] = 0.0
    return u


def leapfrog_learned(dk, pk, post, sqrtD, eps, nsteps):
    """KDK with the learned mass; returns (delta_hat, p_hat', delta) at the end."""
    f, delta = learned_force(dk, post, sqrtD)
    pk = pk - 0.5 * eps * f
    for s in range(nsteps):
        dk = dk + eps * learned_velocity(pk, post, sqrtD)
        f, delta = learned_force(dk, post, sqrtD)
        pk = pk - (eps if s < nsteps - 1 else 0.5 * eps) * f
    return dk, pk, delta


def mass_factor(logvar):
    """D^(1/2) with D = v / mean(v), v = exp(logvar)."""
    v = np.exp(np.asarray(logvar, dtype=np.float64))
    return np.sqrt(v / v.mean())


def diagonal_mass(post, logvar):
    """The real-space diagonal variant of the mass from the same field v = exp(logvar),
    written in the learned form above with D = v/mean(v) and the Fourier diagonal
    replaced by the constant m_k = 1/mean(v).  As the k = 0 entry of the whitened
    momentum stays frozen, the inverse mass is P D^(1/2) (I - Pi_0) D^(1/2) P mean(v)
    (Pi_0 the projection on constant fields): P diag(v) P less one rank-one term,
    positive definite on the zero-mean fields.  Returns (posterior with that m_k,
    D^(1/2)) for trajectory_learned."""
    v = np.exp(np.asarray(logvar, dtype=np.float64))
    return replace(post, mass_k=np.full_like(post.mass_k, 1.0 / v.mean())), np.sqrt(v / v.mean())


def trajectory_learned(dk, post, sqrtD, eps, nsteps, seed, chain, traj):
    pk0 = draw_momentum(post, seed, chain, traj)
    delta0 = grid.inv(dk, post.n, post.workers)
    e0 = energies(dk, pk0, delta0, post)
    dk1, pk1, delta1 = leapfrog_learned(dk, pk0, post, sqrtD, eps, nsteps)
    e1 = energies(dk1, pk1, delta1, post)
    dH = sum(e1) - sum(e0)
    u = philox.uniform(seed, chain, philox.STREAM_ACCEPT, traj)
    acc = bool(np.log(u) < -dH)
    return dict(p0=pk0, e0=e0, e1=e1, dH=dH, accepted=acc, log_u=float(np.log(u)),
                proposal=dk1, p1=pk1, delta1=delta1, state=dk1 if acc else dk)


def prior_draw(post, seed, chain, draw):
    """xi = F^-1(sqrt(lambda_k) F w), w ~ N(0, 1) per voxel from Philox stream 11:
    a draw from the Gaussian prior S (eq. Wiener_Posterior_psi's first term)."""
    n = post.n
    sel = post.shells >= 0
    w = philox.normals(seed, chain, philox.STREAM_WARM, draw, n ** 3).reshape(n, n, n)
    wk = grid.fwd(w, post.workers)
    return grid.inv(np.where(sel, np.sqrt(np.where(sel, post.lam_k, 0.0)) * wk, 0.0), n,
                    post.workers)


def warm_start(mu, logvar, post, seed, chain, draw):
    """Start state from a predicted posterior mean mu and log-variance s: a prior
    draw rescaled from the prior variance per voxel sigma^2 = N^-3 sum_{k!=0}
    lambda_k to exp(s) and shifted by mu.  Returns delta_hat (k = 0 zeroed)."""
    sel = post.shells >= 0
    sigma2 = float(np.sum((post.w * np.where(sel, post.lam_k, 0.0))[sel])) / post.n ** 3
    xi = prior_draw(post, seed, chain, draw)
    delta = np.asarray(mu, np.float64) + np.sqrt(np.exp(np.asarray(logvar, np.float64)) / sigma2) * xi
    dk = grid.fwd(delta, post.workers)
    dk[0, 0, 0] = 0.0
    return dk

