"""Pins of the oracle's sample-estimated residual norms (Algorithm 4, the
norm estimate and its downdates and updates; Algorithm 2, the sample update).

* After the blocked selection the updated sample is exactly Omega times the
  residual of the remaining columns, B(:, i) = Omega (I - P_S) a_i (each
  block's update B(:, rest) -= B(:, piv) R11^{-1} R12 is that identity for
  one block), checked against a brute-force projection with Omega regenerated
  from its pinned stream.
* Every downdate and update is an exact change of a squared residual norm,
  so the estimate's initial error is carried unchanged: at exit
  r_i - ||(I - P_S) a_i||^2 equals r_i(initial) - ||(I - P_S0) a_i||^2 for a
  column never in the leading set, and is zero for a column that left it
  (its estimate is reset to an exact R entry).
* The same holds for the one-block selection, whose sample update takes
  all l pivots as one block.
* With enough sample rows the estimates pick the same j* as exact norms on
  a matrix with well separated residual norms.
"""
import numpy as np
import pytest

import oracle
import synth


def _resid2(A, S, cols):
    Q, _ = np.linalg.qr(A[:, list(S)])
    X = A[:, cols]
    X = X - Q @ (Q.T @ X)
    X = X - Q @ (Q.T @ X)
    return np.sum(X * X, axis=0)


@pytest.mark.parametrize("b,p", [(4, 2), (8, 6), (30, 5)])
def test_final_sample_is_omega_times_the_residual(b, p):
    A = synth.spectrum_matrix(200, 150, 0.95 ** np.arange(150), seed=4, noise=1e-9)
    l = 30
    trace = []
    S, _ = oracle.trqrcp_pivots(A, l, b, p, seed=9, trace=trace)
    B = trace[-1][1]
    rows = min(b + p, A.shape[0])
    Om = oracle.omega(9, rows, A.shape[0])
    rest = [c for c in range(A.shape[1]) if c not in set(S)]
    Q, _ = np.linalg.qr(A[:, list(S)])
    Rz = A[:, rest] - Q @ (Q.T @ A[:, rest])
    ref = Om @ Rz
    assert np.max(np.abs(B[:, rest] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_estimate_errors_are_carried_exactly_through_the_swaps():
    A = synth.spectrum_matrix(300, 200, 0.97 ** np.arange(200), seed=5, noise=1e-8)
    k, p, b, seed = 20, 6, 8, 1
    res = oracle.ffsrqr(A, k, p, seed, g=1.05, block=b, est_norms=True, max_swaps=12)
    assert res.swaps >= 1
    l = res.l
    S0 = res.history[0][0]
    trace = []
    S_init, _ = oracle.trqrcp_pivots(A, l, b, p, seed, trace=trace)
    assert list(S_init) == list(S0)
    Bs = trace[-1][1]
    r0 = np.sum(Bs * Bs, axis=0) / Bs.shape[0]
    S = list(res.perm[:l])
    ever = set()
    for h in res.history:
        ever |= set(h[0])
    trailing = [c for c in range(A.shape[1]) if c not in set(S)]
    g_fin = _resid2(A, S, trailing)
    never = [c for c in trailing if c not in ever]
    left = [c for c in trailing if c in ever]
    assert left, "some column must have left the leading set"
    g_ini = _resid2(A, S0, never)
    scale = float(np.max(np.sum(A * A, axis=0)))
    est = res.norm_estimates
    e_fin = est[never] - g_fin[[trailing.index(c) for c in never]]
    e_ini = r0[never] - g_ini
    assert np.max(np.abs(e_fin - e_ini)) <= 1e-12 * scale
    assert np.max(np.abs(est[left] - g_fin[[trailing.index(c) for c in left]])) <= 1e-12 * scale


def test_identity_rotation_resets_the_estimate_of_jstar():
    A = synth.spectrum_matrix(60, 40, 0.9 ** np.arange(40), seed=3, noise=1e-10)
    r = oracle.ffsrqr(A, 6, 2, 1, g=1.05, g2_probe=1, max_swaps=30, block=4, est_norms=True)
    same = [i for i in range(1, len(r.history)) if r.history[i][0] == r.history[i - 1][0]]
    assert same
    i = same[0]
    S, jstar, alpha = r.history[i][0], r.history[i][2], r.history[i][3]
    # alpha is exact: the residual norm of column j* against the leading set
    assert abs(alpha ** 2 - _resid2(A, S, [jstar])[0]) <= 1e-12 * float(np.sum(A[:, jstar] ** 2))


def test_estimates_agree_with_exact_norms_on_separated_columns():
    # orthogonal columns with norms spaced by 1.3: residual norms are the
    # column norms themselves, far apart relative to a 64-row sample's error
    A = synth.separated_columns_matrix(400, 120, ratio=1.3, seed=2)
    ex = oracle.ffsrqr(A, 10, 54, 3, block=10)
    es = oracle.ffsrqr(A, 10, 54, 3, block=10, est_norms=True)
    assert list(ex.perm) == list(es.perm) and ex.jstar == es.jstar
    assert abs(ex.alpha - es.alpha) <= 1e-12 * ex.alpha


def test_one_block_sample_update_is_omega_times_the_residual():
    # the one-block selection: an l-row sample, all l pivots as the block
    A = synth.spectrum_matrix(200, 150, 0.95 ** np.arange(150), seed=4, noise=1e-9)
    l, seed = 30, 9
    Om = oracle.omega(seed, l, A.shape[0])
    B = Om @ A
    piv, _, _ = oracle.qrcp_sketch(B, l)
    S = [int(s) for s in piv[:l]]
    from oracle.ffsrqr import sample_update
    Bu = sample_update(A, B, S)
    rest = [c for c in range(A.shape[1]) if c not in set(S)]
    Q, _ = np.linalg.qr(A[:, S])
    ref = Om @ (A[:, rest] - Q @ (Q.T @ A[:, rest]))
    assert np.max(np.abs(Bu[:, rest] - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert np.all(Bu[:, S] == 0.0)


def test_one_block_estimates_carry_their_errors_through_the_swaps():
    A = synth.spectrum_matrix(300, 200, 0.97 ** np.arange(200), seed=5, noise=1e-8)
    k, p, seed = 20, 6, 1
    res = oracle.ffsrqr(A, k, p, seed, g=1.05, est_norms=True, max_swaps=12)
    l = res.l
    S0 = res.history[0][0]
    B = oracle.sketch(oracle.omega(seed, l, A.shape[0]), A)
    from oracle.ffsrqr import sample_update
    Bu = sample_update(A, B, S0)
    r0 = np.sum(Bu * Bu, axis=0) / l
    S = list(res.perm[:l])
    ever = set()
    for h in res.history:
        ever |= set(h[0])
    trailing = [c for c in range(A.shape[1]) if c not in set(S)]
    never = [c for c in trailing if c not in ever]
    scale = float(np.max(np.sum(A * A, axis=0)))
    e_fin = res.norm_estimates[never] - _resid2(A, S, never)
    e_ini = r0[never] - _resid2(A, S0, never)
    assert res.swaps >= 1
    assert np.max(np.abs(e_fin - e_ini)) <= 1e-12 * scale
