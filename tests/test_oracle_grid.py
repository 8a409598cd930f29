"""Pins for oracle.grid: DFT convention and k-shells, against brute force."""
import math

import numpy as np
import pytest

from oracle import grid


def naive_rdft3(x):
    """O(N^6) unitary DFT straight from the Appendix's sum, kz restricted to [0, N/2]."""
    n = x.shape[0]
    j = np.arange(n)
    E = np.exp(-2j * np.pi * np.outer(j, j) / n)          # E[k, j]
    out = np.einsum("aj,bk,cl,jkl->abc", E, E, E[: n // 2 + 1], x)
    return out / n ** 1.5


@pytest.mark.parametrize("n", [4, 8])
def test_fwd_matches_naive_dft(n):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n, n, n))
    assert np.max(np.abs(grid.fwd(x) - naive_rdft3(x))) < 1e-12


def test_parseval_and_roundtrip():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((16, 16, 16))
    xk = grid.fwd(x)
    w = grid.half_weights(16)
    assert abs(np.sum(x * x) - np.sum(w * np.abs(xk) ** 2)) < 1e-10 * np.sum(x * x)
    assert np.max(np.abs(grid.inv(xk, 16) - x)) < 1e-12


def test_hermitian_planes():
    """kz = 0 and kz = N/2 planes of a real field's transform are Hermitian in (kx, ky)."""
    rng = np.random.default_rng(3)
    n = 8
    xk = grid.fwd(rng.standard_normal((n, n, n)))
    for kz in (0, n // 2):
        p = xk[:, :, kz]
        flip = np.conj(p[(-np.arange(n)) % n][:, (-np.arange(n)) % n])
        assert np.max(np.abs(p - flip)) < 1e-12


def brute_shell(i, j, l, n, nb):
    """Smallest t >= 1 with t^2 q_max >= nb^2 q, minus one (pure integer loop)."""
    q = i * i + j * j + l * l
    if q == 0:
        return -1
    qmax = 3 * (n // 2) ** 2
    t = 1
    while t * t * qmax < nb * nb * q:
        t += 1
    return t - 1


@pytest.mark.parametrize("n,nb", [(8, 4), (8, 16), (16, 8), (12, 5)])
def test_shells_vs_full_grid_enumeration(n, nb):
    f = [k if k <= n // 2 else k - n for k in range(n)]
    counts = np.zeros(nb, dtype=np.int64)
    for a in f:
        for b in f:
            for c in f:
                m = brute_shell(a, b, c, n, nb)
                if m >= 0:
                    counts[m] += 1
    assert np.array_equal(counts, grid.mode_counts(n, nb))
    assert counts.sum() == n ** 3 - 1
    # the half-grid index agrees with the brute rule entry by entry
    sh = grid.half_shells(n, nb)
    for a in range(n):
        for b in range(n):
            for c in range(n // 2 + 1):
                assert sh[a, b, c] == brute_shell(f[a], f[b], c, n, nb)


def test_shell_edges_float_reading():
    """Bin m holds k in (m/nb, (m+1)/nb] k_corner (checked away from exact edges)."""
    n, nb = 32, 16
    q = grid.half_q(n)
    sh = grid.half_shells(n, nb)
    frac = np.sqrt(q / (3.0 * (n // 2) ** 2)) * nb
    sel = (q > 0) & (np.abs(frac - np.round(frac)) > 1e-9)
    assert np.array_equal(sh[sel], np.ceil(frac[sel]).astype(np.int64) - 1)


def test_shell_sums_full_grid():
    """sigma_m from the half grid equals the sum over the full complex grid."""
    n, nb = 8, 4
    rng = np.random.default_rng(4)
    x = rng.standard_normal((n, n, n))
    full = np.fft.fftn(x, norm="ortho")
    f = [k if k <= n // 2 else k - n for k in range(n)]
    ref = np.zeros(nb)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                m = brute_shell(f[a], f[b], f[c], n, nb)
                if m >= 0:
                    ref[m] += abs(full[a, b, c]) ** 2
    assert np.allclose(grid.shell_sums(grid.fwd(x), nb), ref, rtol=1e-12, atol=0)


def test_config_shells_nonempty():
    for n, nb in [(32, 16), (64, 20), (128, 40), (192, 60), (256, 60), (8, 4), (16, 8)]:
        assert (grid.mode_counts(n, nb) > 0).all(), (n, nb)
    assert math.isclose(grid.k_corner(32, 500.0), math.sqrt(3) * 16 * 2 * math.pi / 500.0)
