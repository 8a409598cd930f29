"""Oracle: grid, DFT and k-shell bookkeeping (test infrastructure only).

Real fields live on the N^3 multi-index grid of Sec. "Notation", stored
row-major as [x][y][z].  Fourier modes use the Appendix "Discrete Fourier
transformation" convention with the symmetric (unitary) reading of the free
normalisation constants, C = C_hat = N_vox^(-1/2): the transform pair is then
an orthogonal map, so sum_i delta_i^2 = sum_k |delta_hat_k|^2.  Because the
field is real only kz in [0, N/2] is stored: shape [N][N][N/2+1].

Signed frequencies run over -(N/2-1) .. N/2, as in the inverse-transform sum
of that appendix.

k-shells (the bins m of eq. INVERSE_GAMMA and of sigma_m).  The paper fixes no
bin edges.  Reading: n_b linear shells over (0, k_corner], k_corner = sqrt(3)
(N/2) 2 pi / L, i.e. in integer form, with q = i^2 + j^2 + l^2 and
q_max = 3 (N/2)^2, mode q >= 1 belongs to the unique m in [0, n_b) with
m^2 q_max < n_b^2 q <= (m+1)^2 q_max.  q = 0 (the mean) belongs to no shell.
n_m counts modes over the full grid (k and -k both counted), which on the
stored half grid is a weight w = 1 for kz in {0, N/2} and w = 2 otherwise.
"""
import numpy as np
import scipy.fft


def signed_freq(n):
    """Signed integer frequency of stored index 0..n-1: -(n/2-1) .. n/2."""
    k = np.arange(n, dtype=np.int64)
    return np.where(k <= n // 2, k, k - n)


def half_q(n):
    """Integer |k|^2 (in units of (2 pi / L)^2) on the stored half grid."""
    fx = signed_freq(n)[:, None, None]
    fy = signed_freq(n)[None, :, None]
    fz = np.arange(n // 2 + 1, dtype=np.int64)[None, None, :]
    return fx * fx + fy * fy + fz * fz


def half_weights(n):
    """w_k = number of full-grid modes a stored half-grid entry stands for."""
    w = np.full((n, n, n // 2 + 1), 2.0)
    w[:, :, 0] = 1.0
    w[:, :, n // 2] = 1.0
    return w


def shell_of_q(q, n, nb):
    """Shell index for integer q (array); -1 for q == 0.

    m = #{m' in 1..nb-1 : m'^2 q_max < nb^2 q}, which is the m of the
    defining inequality m^2 q_max < nb^2 q <= (m+1)^2 q_max.
    """
    q = np.asarray(q, dtype=np.int64)
    qmax = 3 * (n // 2) ** 2
    m = np.zeros(q.shape, dtype=np.int64)
    for mp in range(1, nb):
        m += (mp * mp * qmax < nb * nb * q)
    return np.where(q == 0, -1, m)


def half_shells(n, nb):
    """Shell index of every stored half-grid mode ([N][N][N/2+1], int64)."""
    return shell_of_q(half_q(n), n, nb)


def mode_counts(n, nb):
    """n_m: full-grid number of modes in each shell (int64, length nb)."""
    m = half_shells(n, nb)
    w = half_weights(n).astype(np.int64)
    sel = m >= 0
    return np.bincount(m[sel], weights=w[sel], minlength=nb).astype(np.int64)


def shell_sums(dk, nb):
    """sigma_m = sum over shell m of |delta_hat_k|^2, full-grid counting."""
    n = dk.shape[0]
    m = half_shells(n, nb)
    w = half_weights(n)
    sel = m >= 0
    return np.bincount(m[sel], weights=(w * np.abs(dk) ** 2)[sel], minlength=nb)


def k_corner(n, box):
    return np.sqrt(3.0) * (n // 2) * 2.0 * np.pi / box


def fwd(x, workers=1):
    """Unitary forward real DFT, N^3 -> [N][N][N/2+1] (float64 / complex128)."""
    return scipy.fft.rfftn(np.asarray(x, dtype=np.float64), norm="ortho", workers=workers)


def inv(xk, n, workers=1):
    """Unitary inverse real DFT, [N][N][N/2+1] -> N^3."""
    return scipy.fft.irfftn(np.asarray(xk, dtype=np.complex128), s=(n, n, n), norm="ortho",
                            workers=workers)
