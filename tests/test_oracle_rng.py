"""Pins of the oracle's counter-based noise (Philox4x32-10 + Box-Muller)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    for ctr, key, out in _kat():
        got = oracle_lib.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == out


def test_pair_normals_symmetric_and_distinct(oracle_lib):
    z1 = oracle_lib.pair_normals(0, 17, 4242, 9)
    z2 = oracle_lib.pair_normals(0, 4242, 17, 9)
    assert np.array_equal(z1, z2)
    assert not np.array_equal(z1, oracle_lib.pair_normals(0, 17, 4242, 10))
    assert not np.array_equal(z1, oracle_lib.pair_normals(0, 17, 4243, 9))
    assert not np.array_equal(z1, oracle_lib.pair_normals(1, 17, 4242, 9))


def test_normals_moments(oracle_lib):
    rng = np.random.default_rng(0)
    zs = []
    for k in range(6000):
        a, b = rng.integers(0, 1 << 20, size=2)
        zs.append(oracle_lib.pair_normals(7, int(a), int(b), int(k)))
    z = np.asarray(zs)  # 6000 x 4 = 24000 samples
    n = z.shape[0]
    # each of the four components is standard normal and they are uncorrelated
    assert np.all(np.abs(z.mean(axis=0)) < 5.0 / np.sqrt(n))
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 6.0 * np.sqrt(2.0 / n))
    c = np.corrcoef(z.T)
    off = c[~np.eye(4, dtype=bool)]
    assert np.all(np.abs(off) < 5.0 / np.sqrt(n))
    flat = z.ravel()
    # fourth moment of a standard normal is 3
    assert abs(np.mean(flat ** 4) - 3.0) < 0.1
    # tails exist but stay within the Box-Muller bound sqrt(-2 ln 2^-24)
    assert np.abs(flat).max() <= np.sqrt(-2.0 * np.log(2.0 ** -24)) + 1e-12
