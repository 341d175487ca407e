"""Oracle side of the Gaussian test matrix Omega (Algorithm 2, first step).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this file.

The paper only asks for i.i.d. N(0,1) entries.  Both the oracle and the GPU
path regenerate the same Omega from a seed, each with its own implementation
of one published counter-based generator:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 4 x 64-bit counter, 2 x 64-bit key, ten rounds of the
  multiply/xor S-box with the two published multipliers and the two Weyl key
  increments.
* Box-Muller (1958): z = sqrt(-2 ln u1) * cos(2 pi u2).

Omega stream definition (shared by both sides, written independently):
  key      = (seed, 0)
  entry    Omega[i, t], 0 <= i < l (row), 0 <= t < m (column)
  counter  = (t, i, s, 0)  ->  output words x0..x3 = Philox4x64-10(counter, key)
           s = 0 for the sketch's Omega; s = q >= 1 for the q-th random probe
           of the SRQR test (a d x (l+1) matrix, Algorithm 4's g2 estimate)
  u1 = ((x0 >> 12) + 0.5) * 2^-52,  u2 = ((x1 >> 12) + 0.5) * 2^-52
           (exact in FP64, both in [2^-53, 1 - 2^-53], so inside (0, 1))
  Omega[i, t] = sqrt(-2 ln u1) * cos((2 pi) * u2)   in FP64; x2, x3 unused.

Pins (tests): the integer words equal numpy.random.Philox (an independent
library implementation; it pre-increments its counter, so block c is its
output for counter c-1); the normals pass moment and Kolmogorov-Smirnov
checks against N(0,1).
"""
from __future__ import annotations

import numpy as np

# Philox4x64 round multipliers and Weyl key increments (SC'11, Table/Section 2).
_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """Full 64x64 -> 128-bit product, returned as (hi, lo) uint64 arrays."""
    a_lo = a & _LO32
    a_hi = a >> _S32
    b_lo = b & _LO32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (hl & _LO32) + (lh & _LO32)
    lo = (ll & _LO32) | (cross << _S32)
    hi = hh + (hl >> _S32) + (lh >> _S32) + (cross >> _S32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x64 rounds on arrays of counters; returns four uint64 arrays."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64).copy()
        x1 = np.asarray(c1, dtype=np.uint64).copy()
        x2 = np.asarray(c2, dtype=np.uint64).copy()
        x3 = np.asarray(c3, dtype=np.uint64).copy()
        key0 = np.uint64(k0)
        key1 = np.uint64(k1)
        for rnd in range(10):
            if rnd:
                key0 = key0 + _W0
                key1 = key1 + _W1
            hi0, lo0 = _mulhilo(x0, _M0)
            hi1, lo1 = _mulhilo(x2, _M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ key0, lo1, hi0 ^ x3 ^ key1, lo0
    return x0, x1, x2, x3


def uniform_open(x: np.ndarray) -> np.ndarray:
    """Top 52 bits of a 64-bit word mapped exactly into the open interval (0, 1)."""
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def omega(seed: int, l: int, m: int, stream: int = 0) -> np.ndarray:
    """Omega (l x m), FP64, entry (i, t) from counter (t, i, stream, 0), key
    (seed, 0).  Stream 0 is the sketch's Omega; stream q >= 1 is the q-th
    random probe of the SRQR test's g2 estimate (d x (l+1))."""
    t = np.arange(m, dtype=np.uint64)[None, :].repeat(l, axis=0)
    i = np.arange(l, dtype=np.uint64)[:, None].repeat(m, axis=1)
    z = np.zeros_like(t)
    c2 = np.full_like(t, np.uint64(stream))
    x0, x1, _, _ = philox4x64_10(t, i, c2, z, np.uint64(seed), np.uint64(0))
    u1 = uniform_open(x0)
    u2 = uniform_open(x1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos((2.0 * np.pi) * u2)
