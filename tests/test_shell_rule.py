"""The k-shell rule as the k-space passes evaluate it (32-bit integers and one
float32 square root, then one integer correction upwards and one downwards) equals the
integer rule of the oracle for every q at every supported grid size, also when
the square root is off by up to two units in the last place."""
import numpy as np
import pytest

from oracle import grid


def fast_rule(q, n, nb, ulps):
    qmax = np.uint64(3 * (n // 2) ** 2)
    q = q.astype(np.uint64)
    lhs = np.uint64(nb * nb) * q
    x = lhs.astype(np.float32) * (np.float32(1.0) / np.float32(qmax))
    s = np.sqrt(x).astype(np.float32)
    for _ in range(abs(ulps)):
        s = np.nextafter(s, np.float32(np.inf) if ulps > 0 else np.float32(-np.inf))
    t = np.maximum(np.ceil(s).astype(np.int64), 1).astype(np.uint64)
    t = np.where(t * t * qmax < lhs, t + 1, t)
    t = np.where((t > 1) & ((t - 1) * (t - 1) * qmax >= lhs), t - 1, t)
    out = t.astype(np.int64) - 1
    return np.where(q == 0, -1, out)


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 192, 256])
def test_fast_shell_rule_is_exact(n):
    qmax = 3 * (n // 2) ** 2
    q = np.arange(qmax + 1)
    assert (128 * 128 * qmax) < 2 ** 31 and (129 * 129 * qmax) < 2 ** 31   # 32-bit headroom
    for nb in (4, 16, 40, 60, 97, 128):
        ref = grid.shell_of_q(q, n, nb)
        for ulps in (-2, -1, 0, 1, 2):
            assert np.array_equal(fast_rule(q, n, nb, ulps), ref), (n, nb, ulps)
