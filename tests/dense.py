"""Dense-matrix forms of the 8^3 posterior, built from plain linear algebra.

Used as pins for the oracle: nothing here calls oracle code.  The unitary DFT
matrix is kron(E, E, E) / N^1.5 with E[k, j] = exp(-2 pi i j k / N); the prior
precision S^-1 and the inverse mass are F^H diag(.) F with per-mode values that
depend on |k| only (so both are real symmetric).
"""
import numpy as np


def dft_matrix(n):
    j = np.arange(n)
    E = np.exp(-2j * np.pi * np.outer(j, j) / n)
    return np.kron(np.kron(E, E), E) / n ** 1.5


def full_q(n):
    f = np.array([k if k <= n // 2 else k - n for k in range(n)])
    return (f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2).reshape(-1)


def shell_full(n, nb):
    """Full-grid shell index by the integer rule, written independently."""
    q = full_q(n)
    qmax = 3 * (n // 2) ** 2
    out = np.empty(q.shape, dtype=np.int64)
    for i, qq in enumerate(q):
        if qq == 0:
            out[i] = -1
            continue
        t = 1
        while t * t * qmax < nb * nb * qq:
            t += 1
        out[i] = t - 1
    return out


def fourier_diag_operator(n, per_mode_inv):
    """Real matrix F^H diag(per_mode_inv) F (per_mode_inv on the full grid)."""
    F = dft_matrix(n)
    A = F.conj().T @ (per_mode_inv[:, None] * F)
    assert np.max(np.abs(A.imag)) < 1e-10
    return A.real


def subspace_basis(nv):
    """Orthonormal basis of the zero-mean subspace (nv x (nv-1))."""
    M = np.eye(nv) - 1.0 / nv
    u, s, _ = np.linalg.svd(M)
    return u[:, : nv - 1]


def wiener(n, lam_m, nb, alpha, beta):
    """Mean and covariance of exp(-1/2 d^T Q d + beta^T d) on the zero-mean subspace."""
    sh = shell_full(n, nb)
    inv_lam = np.where(sh >= 0, 1.0 / np.asarray(lam_m)[np.maximum(sh, 0)], 0.0)
    Q = fourier_diag_operator(n, inv_lam) + np.diag(alpha.reshape(-1))
    U = subspace_basis(n ** 3)
    A = U.T @ Q @ U
    Ainv = np.linalg.inv(A)
    mu = U @ (Ainv @ (U.T @ beta.reshape(-1)))
    cov = U @ Ainv @ U.T
    return mu, cov, Q, U
