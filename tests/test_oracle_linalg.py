"""Pins of the oracle's building blocks against LAPACK (numpy/scipy used as
black boxes), closed forms and brute force on tiny inputs."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


def _rng(s):
    return np.random.default_rng(s)


# ----------------------------------------------------------------- reflector
@pytest.mark.parametrize("x", [[3.0, 4.0], [-3.0, 4.0, 12.0], [0.0, 1.0, 1.0], [2.0, 0.0, 0.0], [-1e-300, 1e-300]])
def test_householder_maps_to_beta_e1(x):
    x = np.array(x)
    scale = np.abs(x).max()
    nx = scale * np.linalg.norm(x / scale)
    v, tau, beta = oracle.householder(x)
    H = np.eye(len(x)) - tau * np.outer(v, v)
    y = (H @ (x / scale)) * scale
    assert abs(y[0] - beta) <= 1e-15 * abs(beta)
    assert np.all(np.abs(y[1:]) <= 1e-15 * nx)
    assert np.allclose(H @ H.T, np.eye(len(x)), atol=1e-15)
    assert abs(abs(beta) - nx) <= 1e-15 * nx
    if np.any(x[1:] != 0):
        # LAPACK convention: beta has the opposite sign of x[0] (sign(0) = +)
        assert beta == -math.copysign(abs(beta), x[0])


# ---------------------------------------------------------- Householder QR
@pytest.mark.parametrize("shape", [(7, 7), (50, 13), (300, 40), (33, 1)])
def test_householder_qr_matches_lapack(shape):
    P = _rng(1).standard_normal(shape)
    Q, R = oracle.householder_qr(P)
    Ql, Rl = np.linalg.qr(P)
    d = np.sign(np.diag(Rl))
    Ql, Rl = Ql * d, Rl * d[:, None]
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.max(np.abs(Q - Ql)) < 1e-12
    assert np.max(np.abs(R - Rl)) < 1e-12 * np.abs(Rl).max()
    assert np.linalg.norm(Q.T @ Q - np.eye(shape[1])) < 1e-13
    assert np.linalg.norm(P - Q @ R) < 1e-14 * np.linalg.norm(P)


def test_householder_qr_rank_deficient_panel():
    # a zero column and a repeated column: Householder still returns an
    # orthonormal Q and an exact factorization
    P = _rng(2).standard_normal((40, 6))
    P[:, 2] = 0.0
    P[:, 4] = P[:, 1]
    Q, R = oracle.householder_qr(P)
    assert np.linalg.norm(Q.T @ Q - np.eye(6)) < 1e-13
    assert np.linalg.norm(P - Q @ R) < 1e-14 * np.linalg.norm(P)


# --------------------------------------------------------------- QRCP on B
@pytest.mark.parametrize("seed,shape,l", [(3, (20, 300), 20), (4, (40, 90), 40), (5, (30, 30), 30), (6, (12, 500), 8)])
def test_qrcp_pivots_match_dgeqp3(seed, shape, l):
    B = _rng(seed).standard_normal(shape)
    perm, margins, Bout = oracle.qrcp_sketch(B, l)
    _, Rl, Pl = sla.qr(B, pivoting=True, mode="economic")
    assert margins.min() > 1e-10           # well separated: the pivot order is unique
    assert list(perm[:l]) == list(Pl[:l])
    # the transformed leading block is R of the pivoted QR (up to row signs)
    assert np.allclose(np.abs(np.diag(Bout[:l, :l])), np.abs(np.diag(Rl)[:l]), rtol=1e-12)
    assert np.allclose(np.tril(Bout[:, :l], -1), 0.0)
    # B Pi = Qb Bout holds: the column norms are preserved by the orthogonal updates
    assert np.allclose(np.linalg.norm(Bout, axis=0), np.linalg.norm(B[:, perm], axis=0), rtol=1e-12)


def test_qrcp_orthogonal_columns_pick_descending_norms():
    # orthogonal columns: every step just removes the chosen column, so the
    # greedy order is the descending column-norm order
    A = synth.separated_columns_matrix(60, 25, seed=7, ratio=1.3)
    norms = np.linalg.norm(A, axis=0)
    perm, _, _ = oracle.qrcp_sketch(A, 25)
    assert list(perm) == list(np.argsort(-norms, kind="stable"))


def test_qrcp_ties_go_to_smallest_index():
    B = np.zeros((3, 6))
    B[0, 4] = 1.0
    B[1, 1] = 1.0      # columns 1 and 4 tie, then 5 and 2 tie (all zero after)
    perm, _, _ = oracle.qrcp_sketch(B, 3)
    assert list(perm[:3]) == [1, 4, 0]


# ------------------------------------------------------------------ SRQR g2
def test_srqr_rho_matches_block_inverse_closed_form():
    # R-tilde^{-1} = [[R11^{-1}, -R11^{-1} a / alpha], [0, 1/alpha]], so
    # rho_i^2 = (R11^{-1} a)_i^2 + alpha^2 ||row_i(R11^{-1})||^2 and rho_{l+1} = 1
    rng = _rng(8)
    l = 12
    R11 = np.triu(rng.standard_normal((l, l))) + 4 * np.eye(l)
    a = rng.standard_normal(l)
    alpha = 0.37
    rho = oracle.srqr_rho(R11, a, alpha)
    X = sla.solve_triangular(R11, np.eye(l))
    z = sla.solve_triangular(R11, a)
    closed = np.sqrt(z * z + alpha * alpha * np.sum(X * X, axis=1))
    assert np.allclose(rho[:l], closed, rtol=1e-13)
    assert abs(rho[l] - 1.0) < 1e-15
    # and the definition through LAPACK's inverse of R-tilde^T
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l], Rt[:l, l], Rt[l, l] = R11, a, alpha
    Xt = np.linalg.inv(Rt.T)
    assert abs(rho.max() - alpha * np.sqrt(np.sum(Xt * Xt, axis=0)).max()) < 1e-13 * rho.max()


def test_upper_inverse_and_back_substitution():
    rng = _rng(9)
    U = np.triu(rng.standard_normal((15, 15))) + 3 * np.eye(15)
    b = rng.standard_normal(15)
    assert np.allclose(oracle.back_substitute(U, b), np.linalg.solve(U, b), rtol=1e-12)
    assert np.allclose(oracle.upper_inverse(U) @ U, np.eye(15), atol=1e-13)


# ------------------------------------------------------------------- Jacobi
def test_jacobi_2x2_closed_form():
    # sigma_{1,2}^2 = (S +- sqrt(S^2 - 4 det^2)) / 2 with S the squared Frobenius norm
    for a, b, c, d in [(1.0, 2.0, 3.0, 4.0), (2.0, 0.0, 0.0, 1e-8), (1.0, 1.0, 1.0, 1.0)]:
        M = np.array([[a, b], [c, d]])
        S = a * a + b * b + c * c + d * d
        det = a * d - b * c
        disc = math.sqrt(S * S - 4 * det * det)
        s1 = math.sqrt((S + disc) / 2)
        s2 = abs(det) / s1
        sig, _ = oracle.jacobi_svd(M)
        assert abs(sig[0] - s1) < 1e-15 * s1 and abs(sig[1] - s2) <= 1e-14 * s1


@pytest.mark.parametrize("shape,kind", [((30, 30), "gauss"), ((25, 25), "graded"), ((40, 12), "gauss"),
                                        ((20, 20), "lower"), ((16, 16), "rankdef")])
def test_jacobi_matches_lapack_svd(shape, kind):
    rng = _rng(10)
    M = rng.standard_normal(shape)
    if kind == "graded":
        M = M * (10.0 ** -np.arange(shape[1]) * 0.5)
    if kind == "lower":
        M = np.tril(M) * np.exp(-np.arange(shape[1]) / 4.0)
    if kind == "rankdef":
        M[:, 5:] = M[:, :5] @ rng.standard_normal((5, shape[1] - 5))
    sig, U, V, sweeps = oracle.jacobi_svd(M, want_vectors=True)
    ref = np.linalg.svd(M, compute_uv=False)
    assert sweeps < 30
    assert np.max(np.abs(sig - ref)) < 1e-13 * ref[0]
    keep = ref > 1e-12 * ref[0]
    if kind in ("graded", "lower", "gauss"):
        # one-sided Jacobi is accurate relative to each singular value here
        assert np.max(np.abs(sig[keep] - ref[keep]) / ref[keep]) < 1e-12
    r = int(keep.sum())
    assert np.linalg.norm(M @ V[:, :r] - U[:, :r] * sig[:r]) < 1e-13 * ref[0]
    assert np.linalg.norm(V.T @ V - np.eye(shape[1])) < 1e-13


@pytest.mark.parametrize("rows,n,l,seed", [(40, 300, 40, 1), (25, 120, 20, 2), (60, 61, 60, 3)])
def test_qrcp_margins_match_projection_residuals(rows, n, l, seed):
    """Independent pin of the QRCP margins: at step j the trailing column
    norms of partial QRCP are the squared residuals of the unchosen columns of
    B against the span of the j chosen ones, computed here by LAPACK QR of
    B(:, chosen) and a projection; the step's pivot is their argmax and its
    margin (r_max - r_2nd) / r_max."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((rows, n)) * rng.uniform(0.5, 2.0, size=n)
    perm, margins, _ = oracle.qrcp_sketch(B, l)
    for j in range(l):
        chosen = list(perm[:j])
        rest = [c for c in range(n) if c not in set(chosen)]
        X = B[:, rest]
        if chosen:
            Q, _ = np.linalg.qr(B[:, chosen])
            X = X - Q @ (Q.T @ X)
            X = X - Q @ (Q.T @ X)
        r = np.sum(X * X, axis=0)
        order = np.argsort(-r, kind="stable")
        assert rest[order[0]] == perm[j]
        if len(rest) > 1:
            ref = (r[order[0]] - r[order[1]]) / r[order[0]]
            assert abs(margins[j] - ref) <= 1e-9 * max(ref, 1e-3), (j, margins[j], ref)
