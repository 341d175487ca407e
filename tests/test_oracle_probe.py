"""Pins of the oracle's randomized g2 estimate (Algorithm 4, the g2 step;
Section 2.2, definition of g2) and of the swap loop that uses it.

* With a probe whose rows are sqrt(d) times an orthonormal basis (d = l+1)
  the estimate equals the exact g2 quantities rho_i of srqr_rho (which the
  path tests pin by a closed form and brute force): Om^T Om = d I makes
  ||Om x||^2 / d = ||x||^2 exactly.
* With the Philox probes, est_i^2 / rho_i^2 is chi-squared with d degrees
  of freedom over d: mean 1, variance 2/d.  The average over many probe
  streams lands within a few standard errors of 1 for every position; a
  missing 1/sqrt(d), a dropped alpha column or a transposed inverse (column
  norms instead of row norms of R-tilde^{-1}) does not.
* In the loop, every swap multiplies |det R11| by the exact rho of the
  position it removes (the block-determinant identity of a round-robin
  rotation), whatever the estimate that triggered it.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth


def kahan(n, c=0.285, pert=1e-10):
    s = np.sqrt(1 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.triu(-c * np.ones((n, n)), 1) + np.eye(n))
    return K @ np.diag(1 - pert * np.arange(n))


def _test_state(A, S):
    """R11, a = R(:, j*), alpha and j* of the SRQR test on leading set S."""
    perm, Q1, R11, R, W = oracle.factor_leading_set(A, S)
    l = len(S)
    trailing = perm[l:]
    gam = oracle.residual_norms(A, Q1, W, trailing)
    j = int(trailing[int(np.argmax(gam))])
    return R11, W[:, j], float(gam.max()), j


@pytest.fixture(scope="module")
def kahan_state():
    A = np.vstack([kahan(48), np.zeros((6, 48))])
    r = oracle.ffsrqr(A, 20, 0, seed=0, max_swaps=0)
    S = list(r.perm[:20])
    return A, S, _test_state(A, S)


def test_probe_stream_is_standard_normal_and_apart_from_the_sketch():
    P = np.concatenate([oracle.probe_omega(3, q, 8, 40).ravel() for q in range(1, 60)])
    assert abs(P.mean()) < 0.05 and abs(P.std() - 1.0) < 0.05
    assert stats.kstest(P, "norm").pvalue > 1e-3
    # stream q differs from the sketch's stream 0 and from stream q + 1
    S0 = oracle.omega(3, 8, 41)
    P1, P2 = oracle.probe_omega(3, 1, 8, 40), oracle.probe_omega(3, 2, 8, 40)
    assert abs(np.corrcoef(S0.ravel(), P1.ravel())[0, 1]) < 0.2
    assert abs(np.corrcoef(P1.ravel(), P2.ravel())[0, 1]) < 0.2
    with pytest.raises(ValueError):
        oracle.probe_omega(3, 0, 8, 40)


def test_probe_words_are_philox_with_the_stream_in_the_third_counter_word():
    # the probe's uniforms come from words 0 and 1 of Philox(counter (i, t, q, 0))
    seed, q, d, l = 11, 5, 3, 9
    i = np.arange(l + 1, dtype=np.uint64)[None, :].repeat(d, 0)
    t = np.arange(d, dtype=np.uint64)[:, None].repeat(l + 1, 1)
    x0, x1, _, _ = oracle.philox4x64_10(i, t, np.full_like(i, q), np.zeros_like(i), np.uint64(seed), np.uint64(0))
    u1, u2 = oracle.uniform_open(x0), oracle.uniform_open(x1)
    P = oracle.probe_omega(seed, q, d, l)
    # Box-Muller: the radius depends on u1 only and the angle on u2 only
    r = np.sqrt(-2.0 * np.log(u1))
    assert np.all(np.abs(P) <= r * (1 + 1e-15))
    assert np.array_equal(np.sign(P), np.sign(np.cos(2 * np.pi * u2)))


@pytest.mark.parametrize("l", [1, 7, 20])
def test_orthogonal_probe_gives_the_exact_rho(l):
    rng = np.random.default_rng(l)
    R11 = np.triu(rng.standard_normal((l, l))) + 4 * np.eye(l)
    a = rng.standard_normal(l)
    alpha = 0.3
    d = l + 1
    H, _ = np.linalg.qr(rng.standard_normal((d, d)))
    est = oracle.g2_probe_estimate(R11, a, alpha, np.sqrt(d) * H)
    rho = oracle.srqr_rho(R11, a, alpha)
    assert np.max(np.abs(est - rho) / rho) < 1e-12
    # the last position: |alpha| ||row l+1 of R-tilde^{-1}|| = 1
    assert abs(est[-1] - 1.0) < 1e-12


def test_probe_estimate_is_unbiased_over_the_probe_streams(kahan_state):
    A, S, (R11, a, alpha, _) = kahan_state
    l, d, nq = len(S), 4, 3000
    rho = oracle.srqr_rho(R11, a, alpha)
    acc = np.zeros(l + 1)
    for q in range(1, nq + 1):
        est = oracle.g2_probe_estimate(R11, a, alpha, oracle.probe_omega(7, q, d, l))
        acc += est * est
    ratio = acc / nq / (rho * rho)
    se = np.sqrt(2.0 / (d * nq))
    assert np.max(np.abs(ratio - 1.0)) < 5 * se, np.max(np.abs(ratio - 1.0))
    # the test has power against a transposed inverse: column norms differ
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l], Rt[:l, l], Rt[l, l] = R11, a, alpha
    X = oracle.upper_inverse(Rt)
    col = alpha * np.sqrt(np.sum(X * X, axis=0))
    assert np.max(np.abs(col * col / (rho * rho) - 1.0)) > 20 * se


def test_probe_loop_swaps_follow_the_determinant_identity():
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    r = oracle.ffsrqr(A, 40, 0, seed=0, g2_probe=8)
    assert r.swaps >= 1 and not r.flags & oracle.FLAG_SWAPCAP
    assert r.probes == len(r.history) and r.g2 == r.history[-1][1] <= 2.0
    assert r.history[0][1] > 2.0
    for i in range(1, len(r.history)):
        S0, S1 = r.history[i - 1][0], r.history[i][0]
        if S0 == S1:
            continue  # an identity rotation: a fresh probe on the same set
        # S1 = S0 without S0[istar], followed by j* of the previous test
        assert S1[-1] == r.history[i - 1][2]
        istar = next(t for t in range(len(S0)) if S0[:t] + S0[t + 1:] == S1[:-1])
        R11, a, alpha, _ = _test_state(A, S0)
        rho = oracle.srqr_rho(R11, a, alpha)
        _, Ra = oracle.householder_qr(A[:, S0])
        _, Rb = oracle.householder_qr(A[:, S1])
        growth = np.sum(np.log(np.abs(np.diag(Rb)))) - np.sum(np.log(np.abs(np.diag(Ra))))
        assert abs(growth - np.log(rho[istar])) < 1e-8
    # the probe stops where the exact g2 is moderate: the estimate's error is
    # a chi-squared factor, not a blow-up
    R11, a, alpha, _ = _test_state(A, list(r.perm[:40]))
    assert oracle.srqr_rho(R11, a, alpha).max() < 4.0


def test_identity_rotation_draws_a_fresh_probe_and_counts_toward_the_cap():
    # d = 1 and g close to 1: |omega| of the last position often exceeds g,
    # so the argmax is sometimes position l+1, whose rotation is the identity
    A = synth.spectrum_matrix(60, 40, 0.9 ** np.arange(40), seed=3, noise=1e-10)
    found = False
    for seed in range(40):
        r = oracle.ffsrqr(A, 6, 2, seed=seed, g=1.05, g2_probe=1, max_swaps=30)
        same = [i for i in range(1, len(r.history)) if r.history[i][0] == r.history[i - 1][0]]
        if same:
            found = True
            i = same[0]
            assert r.history[i][2] == r.history[i - 1][2]      # same j*
            assert r.history[i][3] == r.history[i - 1][3]      # same alpha
            assert r.history[i][1] != r.history[i - 1][1]      # a fresh estimate
            break
    assert found
    # the cap counts identity rotations: with max_swaps rotations at most
    # max_swaps + 1 tests run
    r = oracle.ffsrqr(A, 6, 2, seed=0, g=1.001, g2_probe=1, max_swaps=3)
    assert len(r.history) <= 4 and r.swaps <= 3


def test_exact_default_is_unchanged():
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    r = oracle.ffsrqr(A, 40, 0, seed=0)
    assert r.probes == 0
    for S, g2, j, alpha in r.history:
        R11, a, al, jj = _test_state(A, S)
        assert jj == j and abs(oracle.srqr_rho(R11, a, al).max() - g2) <= 1e-12 * g2
