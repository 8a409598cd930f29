"""Pins for oracle.philox: published known answers and distribution checks."""
import os

import numpy as np
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def load_kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_known_answers():
    rows = load_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = philox.philox4x32_10(*[np.array([c], dtype=np.uint64) for c in ctr], *key)
        assert [int(g[0]) for g in got] == want


def test_counter_layout():
    """words() places (block, draw, chain<<8|stream, sub) in the counter, seed in the key."""
    seed = 0x0123456789ABCDEF
    w = philox.words(seed, 5, 3, 77, 9, [11])[0]
    ref = philox.philox4x32_10(np.array([11]), np.array([77]), np.array([(5 << 8) | 3]),
                               np.array([9]), seed & 0xFFFFFFFF, seed >> 32)
    assert [int(r[0]) for r in ref] == [int(x) for x in w]


def test_uniform_open_interval():
    assert philox.to_uniform(0) > 0.0
    assert philox.to_uniform(0xFFFFFFFF) < 1.0


def test_normals_distribution():
    z = philox.normals(42, 0, philox.STREAM_MOMENTA, 0, 200000)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # neighbouring lanes are uncorrelated
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / np.sqrt(z.size)


def test_streams_differ():
    a = philox.normals(1, 0, 3, 0, 64)
    b = philox.normals(1, 0, 4, 0, 64)
    c = philox.normals(1, 1, 3, 0, 64)
    d = philox.normals(1, 0, 3, 1, 64)
    for o in (b, c, d):
        assert not np.allclose(a, o)
