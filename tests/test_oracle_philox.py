"""Pins of the oracle's counter-based RNG (Philox4x64-10) and its normals.

The generator is checked bit for bit against numpy's independent
implementation of the same published algorithm; numpy increments its counter
before producing a block, so block c is numpy's output at counter c - 1.
"""
import numpy as np
import pytest
from scipy import stats


def _numpy_block(ctr, key):
    c = [int(v) for v in ctr]
    # subtract one from the 256-bit counter (little-endian words)
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = (1 << 64) - 1
    bg = np.random.Philox()
    st = bg.state
    st["state"]["counter"] = np.array(c, dtype=np.uint64)
    st["state"]["key"] = np.array([int(key[0]), int(key[1])], dtype=np.uint64)
    st["buffer_pos"] = 4
    bg.state = st
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [0, 0]),
    ([0, 0, 0, 1], [1, 2]),
    ([5, 7, 3, 2], [12345, 0]),
    ([2**64 - 1, 2**63, 17, 99], [2**64 - 1, 2**64 - 1]),
    ([200, 131071, 4, 3], [0, 0]),
])
def test_philox_matches_numpy(oracle, ctr, key):
    got = oracle.philox(ctr, key)
    want = _numpy_block(ctr, key)
    assert np.array_equal(got, want)


def test_philox_many_counters(oracle):
    rng = np.random.default_rng(3)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(1, 2**63, 4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, 2, dtype=np.int64)]
        assert np.array_equal(oracle.philox(ctr, key), _numpy_block(ctr, key))


def test_u01_open_interval(oracle):
    assert oracle.u01(0) == 0.5 * 2.0**-53
    assert oracle.u01(2**64 - 1) == 1.0 - 0.5 * 2.0**-53
    assert 0.0 < oracle.u01(2**63) < 1.0


def test_normals_use_box_muller_of_the_block(oracle):
    # first pair of block 0 from the raw words, via the polar form of the pair
    w = oracle.philox([3, 11, 4, 0], [9, 0])
    u = [oracle.u01(int(v)) for v in w]
    z = oracle.normals(9, 3, 11, 4, 4)
    r = np.hypot(z[0], z[1])
    assert r == pytest.approx(np.sqrt(-2 * np.log(u[0])), rel=1e-14)
    ang = np.arctan2(z[1], z[0]) % (2 * np.pi)
    assert ang == pytest.approx(2 * np.pi * u[1], rel=1e-12, abs=1e-12)
    # the count only truncates: a longer request starts with the same values
    z7 = oracle.normals(9, 3, 11, 4, 7)
    assert np.array_equal(z7[:4], z)


def test_normals_distribution(oracle):
    z = np.concatenate([oracle.normals(1, 0, n, 1, 12) for n in range(4000)])
    assert abs(z.mean()) < 4 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / len(z))
    assert stats.kstest(z, "norm").pvalue > 1e-3
