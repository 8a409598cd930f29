"""Oracle: data model, Wiener potential, force and mass (test infrastructure only).

Data model (eq. data_model, with R = C F): N^l_i = Nbar^l R^l_i (1 + b^l delta_i)
+ eps, eps Gaussian with variance Nbar^l R^l_i (eq. cov_mat_noise).  Readings:
* the growth factor D+ of eq. data_model does not reappear in the likelihood
  (eq. LH_per_dataset) or anything after it; it is taken as 1;
* the likelihood divides by Nbar R, so every data sum runs over voxels with
  R^l_i > 0 only (unobserved voxels carry no data).

Potential (eq. Wiener_Posterior_psi, constants dropped):
  psi = 1/2 delta^T S^-1 delta
        + 1/2 sum_l sum_{i: R>0} (N - Nbar R (1 + b delta))^2 / (Nbar R)
Expanding the square, the data part equals (up to a delta-independent constant)
  sum_i (1/2 alpha_i delta_i^2 - beta_i delta_i),
  alpha_i = sum_l b_l^2 Nbar_l R^l_i,  beta_i = sum_l b_l (N^l_i - Nbar_l R^l_i),
which are exactly the diagonal and constant terms of the force of eq.
Wiener_Posterior_force.

S is diagonal in Fourier space with eigenvalue lambda_k = P(k) N_vox / V in the
unitary convention of ``grid`` (P in (Mpc/h)^3, V = L^3), P binned in shells.
The mean mode k = 0 is held at zero (its prior variance P(0) = 0).

Mass (text after eq. Mass_matrix): the diagonal of S^-1 + diag(alpha) in its
Fourier representation, m_k = 1/lambda_k + mean_i(alpha_i), because the Fourier
diagonal of a real-space diagonal matrix is its mean.
"""
import numpy as np

from . import grid


def coefficients(R, counts, bias, nbar, growth=None):
    """alpha, beta of the force (float64 [N][N][N]) and the mean of alpha.  growth:
    per-voxel linear growth factor D+ of eq. data_model (None: D+ = 1); the mean
    counts are Nbar R (1 + b D+ delta), so alpha carries D+^2 and beta D+."""
    R = np.asarray(R, dtype=np.float64)
    counts = np.asarray(counts, dtype=np.float64)
    alpha = np.zeros(R.shape[1:])
    beta = np.zeros(R.shape[1:])
    for l in range(R.shape[0]):
        obs = R[l] > 0
        alpha += np.where(obs, bias[l] ** 2 * nbar[l] * R[l], 0.0)
        beta += np.where(obs, bias[l] * (counts[l] - nbar[l] * R[l]), 0.0)
    if growth is not None:
        g = np.asarray(growth, dtype=np.float64)
        alpha *= g * g
        beta *= g
    return alpha, beta, float(alpha.mean())


def lambdas(pk, n, box):
    """Unitary prior eigenvalue per shell, lambda_m = P_m N_vox / V."""
    return np.asarray(pk, dtype=np.float64) * n ** 3 / box ** 3


def mass_table(lam, abar):
    """m_m = 1/lambda_m + mean(alpha) for each shell."""
    return 1.0 / np.asarray(lam, dtype=np.float64) + abar


def per_mode(table, shells):
    """Expand a per-shell table to the half grid; k = 0 gets +inf (frozen)."""
    out = np.full(shells.shape, np.inf)
    sel = shells >= 0
    out[sel] = np.asarray(table, dtype=np.float64)[shells[sel]]
    return out


def psi_data_direct(delta, R, counts, bias, nbar):
    """Data part of psi straight from eq. Wiener_Posterior_psi (no expansion)."""
    tot = 0.0
    for l in range(R.shape[0]):
        obs = R[l] > 0
        r = R[l][obs]
        resid = counts[l][obs] - nbar[l] * r * (1.0 + bias[l] * delta[obs])
        tot += 0.5 * np.sum(resid ** 2 / (nbar[l] * r))
    return tot


def psi_data(delta, alpha, beta):
    """sum_i (1/2 alpha delta^2 - beta delta): psi_data_direct minus a constant."""
    return float(np.sum(0.5 * alpha * delta * delta - beta * delta))


def psi_prior(dk, lam_k, w):
    """1/2 delta^T S^-1 delta = 1/2 sum_k w |delta_hat|^2 / lambda_k (k = 0 excluded)."""
    return float(0.5 * np.sum(w * np.abs(dk) ** 2 / lam_k))


def force_k(dk, lam_k, alpha, beta, workers=1):
    """Fourier transform of grad psi: delta_hat/lambda + F(alpha delta - beta).

    Returns (force_hat, grad_hat, delta) with the k = 0 entry of force_hat
    zeroed (the mean mode is frozen).
    """
    n = dk.shape[0]
    delta = grid.inv(dk, n, workers)
    g = alpha * delta - beta
    gk = grid.fwd(g, workers)
    f = dk / lam_k + gk
    f[0, 0, 0] = 0.0
    return f, gk, delta


def grad_real(delta, lam_k, alpha, beta):
    """Real-space grad psi (including the data force on the mean mode)."""
    n = delta.shape[0]
    dk = grid.fwd(delta)
    prior = np.where(np.isfinite(lam_k), dk / lam_k, 0.0)
    return grid.inv(prior, n) + alpha * delta - beta


def psi_total(delta, lam_k, w, alpha, beta):
    dk = grid.fwd(delta)
    prior = 0.5 * np.sum(np.where(np.isfinite(lam_k), w * np.abs(dk) ** 2 / lam_k, 0.0))
    return float(prior) + psi_data(delta, alpha, beta)
