"""Pins of the oracle's bfloat16 sketch mode (the mixed-precision form's
definition of B = Omega A): the rounding function against an exhaustive
nearest-value search over every bfloat16 bit pattern and against torch's
float32 -> bfloat16 conversion, and the bf16-mode sketch against exactly
rounded sums of exact products."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _all_bf16_values() -> np.ndarray:
    """Every finite bfloat16 value as FP64 (the top 16 bits of a float32)."""
    bits = np.arange(1 << 16, dtype=np.uint32) << np.uint32(16)
    with np.errstate(invalid="ignore"):
        v = bits.view(np.float32).astype(np.float64)
    pattern = np.arange(1 << 16, dtype=np.int64)
    keep = np.isfinite(v)
    return v[keep], pattern[keep]


_VALS, _PAT = _all_bf16_values()
_ORDER = np.argsort(_VALS, kind="stable")
_SORTED = _VALS[_ORDER]
_SORTED_PAT = _PAT[_ORDER]


def _nearest_bf16_brute(x: float) -> float:
    """Nearest bfloat16 value to x by search over all values; a tie goes to
    the neighbour whose bit pattern is even (ties to even)."""
    i = int(np.searchsorted(_SORTED, x))
    cands = []
    for j in (i - 1, i, i + 1):
        if 0 <= j < _SORTED.shape[0]:
            cands.append((abs(Fraction(_SORTED[j]) - Fraction(x)), _SORTED_PAT[j] & 1, _SORTED[j]))
    cands.sort(key=lambda t: (t[0], t[1]))
    return float(cands[0][2])


def test_round_bf16_matches_exhaustive_search_on_doubles():
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.standard_normal(400) * 10.0 ** rng.uniform(-30, 30, 400),
        rng.uniform(-1, 1, 200),
    ])
    got = oracle.round_bf16(xs)
    for x, g in zip(xs, got):
        assert g == _nearest_bf16_brute(float(x)), x


def test_round_bf16_ties_and_double_rounding():
    one = 1.0
    cases = {
        one + 2.0 ** -8: one,                         # tie, 1.0 has the even pattern
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,         # tie between 1+2^-7 (odd) and 1+2^-6 (even)
        one + 2.0 ** -8 + 2.0 ** -40: one + 2.0 ** -7,  # above the tie: FP32 first would give 1.0
        2.0 - 2.0 ** -8: 2.0,                         # tie at a binade edge rounds up to 2
        -(one + 2.0 ** -8 + 2.0 ** -40): -(one + 2.0 ** -7),
        0.0: 0.0,
        10 * 2.0 ** -133 + 2.0 ** -134: 10 * 2.0 ** -133,  # subnormal tie (spacing 2^-133), even 10
        11 * 2.0 ** -133 + 2.0 ** -134: 12 * 2.0 ** -133,  # subnormal tie, odd 11 -> 12
    }
    for x, want in cases.items():
        assert oracle.round_bf16(np.array([x]))[0] == want, x
        assert _nearest_bf16_brute(x) == want, x


def test_round_bf16_matches_torch_on_float32_inputs():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-20, 20, 20000)).astype(np.float32)
    # add exact ties: bfloat16 values plus half a spacing (exactly representable in FP32)
    b = oracle.round_bf16(x32.astype(np.float64)[:1000])
    _, e = np.frexp(b)
    ties = (b + np.ldexp(1.0, np.maximum(e, -125) - 9)).astype(np.float32)
    x32 = np.concatenate([x32, ties])
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.round_bf16(x32.astype(np.float64))
    assert np.array_equal(got, ref)


def test_bf16_sketch_is_the_exactly_rounded_sum_of_exact_products():
    rng = np.random.default_rng(2)
    Om = rng.standard_normal((5, 40))
    A = (rng.standard_normal((40, 7)) * 3).astype(np.float32).astype(np.float64)
    B = oracle.sketch(Om, A, mode="bf16")
    Ob = oracle.round_bf16(Om)
    Ab = oracle.round_bf16(A)
    for i in range(5):
        for j in range(7):
            prods = [Ob[i, t] * Ab[t, j] for t in range(40)]
            for t in range(40):   # every product is exact in FP64
                assert Fraction(prods[t]) == Fraction(Ob[i, t]) * Fraction(Ab[t, j])
            exact = math.fsum(prods)
            bound = 40 * 2.0 ** -53 * sum(abs(p) for p in prods)
            assert abs(B[i, j] - exact) <= bound


def test_bf16_sketch_within_rounding_of_fp64_sketch():
    rng = np.random.default_rng(3)
    Om = rng.standard_normal((6, 300))
    A = rng.standard_normal((300, 20))
    d = np.abs(oracle.sketch(Om, A, "bf16") - oracle.sketch(Om, A, "fp64"))
    # |bf16(a) bf16(b) - a b| <= (2 u + u^2) |a b| with u = 2^-9
    u = 2.0 ** -9
    assert np.all(d <= (2 * u + u * u) * (np.abs(Om) @ np.abs(A)) * (1 + 1e-12))
    assert d.max() > 0
    with pytest.raises(ValueError):
        oracle.sketch(Om, A, "fp8")
