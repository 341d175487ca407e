"""Pins of the oracle's Omega stream (Philox4x64-10 + Box-Muller).

The integer words are pinned bit for bit to numpy.random.Philox, an
independent implementation of the same SC'11 generator (numpy increments its
counter before each block, so our block c is numpy's output for counter c-1).
The Gaussian map is pinned by its distribution, not by retyping it.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

MASK = (1 << 64) - 1


def _numpy_block(seed, ctr):
    c = list(ctr)
    # subtract one from the 256-bit counter (little-endian words)
    for w in range(4):
        if c[w] > 0:
            c[w] -= 1
            break
        c[w] = MASK
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                           counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("seed", [0, 1, 12345, (1 << 63) + 7])
def test_philox_words_match_numpy(seed):
    rng = np.random.default_rng(seed % 1000)
    ctrs = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 5, 0, 0), (MASK, 3, 0, 0)]
    ctrs += [(int(rng.integers(0, 1 << 40)), int(rng.integers(0, 1 << 20)), 0, 0) for _ in range(20)]
    # the probe streams of the SRQR test: stream q >= 1 in the third word
    ctrs += [(int(rng.integers(0, 1 << 12)), int(rng.integers(0, 64)), int(rng.integers(1, 1 << 16)), 0)
             for _ in range(10)]
    for c in ctrs:
        mine = oracle.philox4x64_10(*[np.array([v], dtype=np.uint64) for v in c],
                                    np.uint64(seed), np.uint64(0))
        assert [int(x[0]) for x in mine] == _numpy_block(seed, c), c


def test_philox_vectorised_equals_scalar():
    t = np.arange(50, dtype=np.uint64)
    i = np.full(50, 7, dtype=np.uint64)
    z = np.zeros(50, dtype=np.uint64)
    x0, x1, x2, x3 = oracle.philox4x64_10(t, i, z, z, np.uint64(3), np.uint64(0))
    for j in (0, 17, 49):
        s = oracle.philox4x64_10(np.array([j], np.uint64), np.array([7], np.uint64),
                                 np.array([0], np.uint64), np.array([0], np.uint64),
                                 np.uint64(3), np.uint64(0))
        assert (int(s[0][0]), int(s[1][0])) == (int(x0[j]), int(x1[j]))


def test_uniform_open_interval():
    words = np.array([0, 1, 4095, 4096, MASK], dtype=np.uint64)
    u = oracle.uniform_open(words)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    # the extreme words map to the half-ulp points next to 0 and 1
    assert u[0] == u[2] == 0.5 * 2.0 ** -52
    assert u[3] == 1.5 * 2.0 ** -52
    assert u[-1] == 1.0 - 0.5 * 2.0 ** -52


def test_omega_is_standard_normal():
    om = oracle.omega(0, 64, 4000)
    x = om.ravel()
    n = x.size
    assert abs(x.mean()) < 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # rows are uncorrelated
    c = np.corrcoef(om[:8])
    assert np.max(np.abs(c - np.eye(8))) < 6.0 / np.sqrt(om.shape[1])


def test_omega_counter_addressed():
    big = oracle.omega(9, 12, 300)
    small = oracle.omega(9, 5, 120)
    assert np.array_equal(big[:5, :120], small)
    assert not np.array_equal(oracle.omega(10, 5, 120), small)
