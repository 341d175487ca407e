"""Pins of the oracle's Algorithm 9 completion (tmp = A Pi Qhat1, its SVD,
U_k, Sigma_k, V_k) and of the margin of the residual-norm argmax j*."""
import numpy as np

import oracle
import synth
from oracle import diagnostics as dg


def _solve(A, k, p, seed=0):
    r = oracle.ffsrqr(A, k, p, seed)
    return r, oracle.alg9(A, r, k)


def test_alg9_sigma_matches_lapack_and_factors_are_consistent():
    A = synth.spectrum_matrix(300, 200, np.exp(-np.arange(200) / 12.0), seed=51, noise=1e-9)
    k = 15
    r, a9 = _solve(A, k, 8)
    ref = dg.alg9_sigma(A, r, k)            # LAPACK SVD of A V
    assert np.max(np.abs(a9.sigma - ref) / ref) < 1e-12
    assert np.linalg.norm(a9.U.T @ a9.U - np.eye(k)) < 1e-13
    assert np.linalg.norm(a9.V.T @ a9.V - np.eye(k)) < 1e-13
    # A V_k = U_k Sigma_k (tmp V_t = U_tmp Sigma and V_k = V V_t(:, 1:k))
    assert np.linalg.norm(A @ a9.V - a9.U * a9.sigma) < 1e-13 * np.linalg.norm(A)
    # column sign convention: the largest-magnitude entry of each U column is positive
    idx = np.argmax(np.abs(a9.U), axis=0)
    assert np.all(a9.U[idx, np.arange(k)] > 0)


def test_alg9_at_full_rank_is_the_svd_of_A():
    s = np.logspace(0, -5, 40)
    A = synth.spectrum_matrix(90, 40, s, seed=52)
    r, a9 = _solve(A, 40, 0)
    assert r.l == 40
    assert np.max(np.abs(a9.sigma - s) / s) < 1e-10
    U, sv, Vt = np.linalg.svd(A, full_matrices=False)
    # singular vectors agree up to sign where the singular values are separated
    d = np.abs(np.sum(U * a9.U, axis=0))
    assert np.all(np.abs(d - 1.0) < 1e-8)
    dv = np.abs(np.sum(Vt.T * a9.V, axis=0))
    assert np.all(np.abs(dv - 1.0) < 1e-8)


def test_alg9_error_floor_theorem_1_1():
    # ||A - U_k Sigma_k V_k^T||_2 >= sigma_{k+1}(A) (Eckart-Young-Mirsky), and the
    # Alg-9 values interlace the true ones
    A = synth.spectrum_matrix(200, 150, 0.85 ** np.arange(150), seed=53, noise=1e-10)
    k = 12
    r, a9 = _solve(A, k, 6)
    s = np.linalg.svd(A, compute_uv=False)
    E = A - (a9.U * a9.sigma) @ a9.V.T
    assert np.linalg.svd(E, compute_uv=False)[0] >= s[k] * (1 - 1e-12)
    assert np.all(a9.sigma <= s[:k] * (1 + 1e-12))


def test_jstar_margin_on_orthogonal_columns():
    # orthogonal columns: the trailing residual norms are the trailing column
    # norms themselves, so the margin is a closed form of the two largest
    A = synth.separated_columns_matrix(120, 60, seed=54, ratio=1.3)
    k, p = 10, 0
    r = oracle.ffsrqr(A, k, p, seed=0)
    norms = np.linalg.norm(A, axis=0)
    trailing = np.sort(norms[r.perm[r.l:]] ** 2)
    want = (trailing[-1] - trailing[-2]) / trailing[-1]
    assert abs(r.jstar_margin - want) < 1e-12
    assert r.jstar == int(r.perm[r.l:][np.argmax(norms[r.perm[r.l:]])])
