"""Pins of the whole oracle path: closed forms, the paper's bounds (Lemma 3.1,
Theorem 3.1, Theorem 1.1), SRQR post-conditions and metamorphic relations."""
import numpy as np
import pytest

import oracle
import synth
from oracle import diagnostics as dg


def kahan(n, c=0.285, pert=1e-10):
    s = np.sqrt(1 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.triu(-c * np.ones((n, n)), 1) + np.eye(n))
    return K @ np.diag(1 - pert * np.arange(n))


@pytest.fixture(scope="module")
def small():
    w = synth.WORKLOADS["small_fp64"]
    A = synth.make_workload("small_fp64")
    res = oracle.ffsrqr(A, w.k, w.p, w.seed)
    return w, A, res


def test_generator_spectrum_is_prescribed(small):
    w, A, _ = small
    s = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - w.sigma()) / w.sigma()) < 1e-9


def test_small_outputs_structure(small):
    w, A, r = small
    l = w.l
    assert r.l == 30 and r.flags == 0
    assert sorted(r.perm) == list(range(w.n))
    assert list(r.perm[l:]) == sorted(r.perm[l:])
    assert np.linalg.norm(r.Q.T @ r.Q - np.eye(l)) < 1e-13
    assert np.all(np.diag(r.R[:, :l]) > 0)
    assert np.allclose(np.tril(r.R[:, :l], -1), 0.0)
    assert np.allclose(np.triu(r.L, 1), 0.0) and np.all(np.diag(r.L) >= 0)
    assert np.linalg.norm(r.V.T @ r.V - np.eye(l)) < 1e-13
    # Q1 R11 reproduces the pivoted columns
    P = A[:, r.perm[:l]]
    assert np.linalg.norm(P - r.Q @ r.R[:, :l]) < 1e-14 * np.linalg.norm(A)
    # R = Q1^T A Pi and A ~ Q L V^T: L V^T = R Pi^T
    assert np.allclose(r.L @ r.V.T, r.R[:, np.argsort(r.perm)], atol=1e-14 * np.abs(r.R).max())
    # sigma(L) = sigma(R) (R^T = Qhat1 Rhat11), through LAPACK's SVD
    sR = np.linalg.svd(r.R, compute_uv=False)
    assert np.max(np.abs(r.sigma - sR) / sR) < 1e-12
    assert r.g2 <= 2.0


def test_full_rank_reconstruction():
    # l = min(m, n): A Pi = Q R exactly and sigma(L) = sigma(A)
    A = synth.spectrum_matrix(80, 50, np.logspace(0, -6, 50), seed=11)
    r = oracle.ffsrqr(A, 40, 10, seed=3)
    assert r.l == 50
    assert np.linalg.norm(A[:, r.perm] - r.Q @ r.R) < 1e-13 * np.linalg.norm(A)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(r.sigma - s) / s) < 1e-9
    assert np.max(np.abs(r.sigma - s)) < 1e-13 * s[0]
    assert dg.residual_fro(A, r.Q, r.L, r.V) < 1e-13 * np.linalg.norm(A)


def test_exact_low_rank_is_recovered():
    sig = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    A = synth.spectrum_matrix(120, 90, sig, seed=12)
    r = oracle.ffsrqr(A, 6, 0, seed=1)
    assert np.max(np.abs(r.sigma[:6] - sig) / sig) < 1e-11
    assert dg.residual_fro(A, r.Q, r.L, r.V) < 1e-12 * np.linalg.norm(A)


def test_rank_deficient_flag():
    sig = np.array([5.0, 3.0, 2.0])
    A = synth.spectrum_matrix(60, 40, sig, seed=13)
    r = oracle.ffsrqr(A, 5, 2, seed=0)
    assert r.flags & oracle.FLAG_RANK_DEFICIENT
    assert r.numerical_rank == 3
    assert np.max(np.abs(r.sigma[:3] - sig) / sig) < 1e-11


def test_clamped_l_flag():
    A = synth.random_matrix(30, 20, seed=14)
    r = oracle.ffsrqr(A, 18, 10, seed=0)
    assert r.l == 20 and r.flags & oracle.FLAG_L_CLAMPED


def test_nonfinite_flag():
    A = synth.random_matrix(30, 20, seed=15)
    A[3, 4] = np.nan
    with np.errstate(invalid="ignore"):
        r = oracle.ffsrqr(A, 5, 2, seed=0)
    assert r.flags & oracle.FLAG_NONFINITE


@pytest.mark.parametrize("name_or_seed", ["small", 21, 22, 23])
def test_singular_value_bounds(small, name_or_seed):
    """Interlacing sigma_j(L) <= sigma_j(A); Lemma 3.1 applied to R^T split into
    ((R11 R12)^T, (0 R22)^T): sigma_j(A)^2 <= sigma_j(L)^2 + ||R22||_2^2;
    Pythagoras for the residual; Theorem 1.1 floors for rank l and rank k."""
    if name_or_seed == "small":
        w, A, r = small
        k = w.k
    else:
        rng = np.random.default_rng(name_or_seed)
        m, n = int(rng.integers(60, 200)), int(rng.integers(40, 150))
        sig = np.exp(-np.arange(min(m, n)) / rng.uniform(3, 30))
        A = synth.spectrum_matrix(m, n, sig, seed=name_or_seed, noise=1e-9)
        k = int(rng.integers(3, 15))
        r = oracle.ffsrqr(A, k, int(rng.integers(0, 8)), seed=name_or_seed)
    s = np.linalg.svd(A, compute_uv=False)
    l = r.l
    r22_2, r22_12 = dg.r22_norms(A, r)
    assert np.all(r.sigma <= s[:l] * (1 + 1e-12))
    assert np.all(s[:l] ** 2 <= r.sigma ** 2 + r22_2 ** 2 + 1e-12 * s[0] ** 2)
    res_l = dg.residual_fro(A, r.Q, r.L, r.V)
    assert abs(res_l ** 2 - (np.sum(s ** 2) - np.sum(r.sigma ** 2))) < 1e-12 * np.sum(s ** 2)
    assert res_l >= np.sqrt(np.sum(s[l:] ** 2)) * (1 - 1e-12)
    # g1 = 1 in the exact reading: alpha is the largest trailing residual norm
    assert abs(r.alpha - r22_12) <= 1e-12 * r22_12


@pytest.mark.parametrize("case", ["small", "decay", "kahan"])
def test_theorem_3_1(small, case):
    if case == "small":
        w, A, r = small
        k = w.k
    elif case == "decay":
        A = synth.spectrum_matrix(150, 110, 0.8 ** np.arange(110), seed=31, noise=1e-8)
        k = 10
        r = oracle.ffsrqr(A, k, 5, seed=2)
    else:
        A = np.vstack([kahan(80), np.zeros((10, 80))])
        k = 40
        r = oracle.ffsrqr(A, k, 0, seed=0)
    s = np.linalg.svd(A, compute_uv=False)
    checks = dg.theorem31(A, r, k, s)
    assert any(name.startswith("lower_") for name in checks)
    for name, (lhs, rhs) in checks.items():
        assert lhs <= rhs * (1 + 1e-10) + 1e-14 * s[0], name


def test_srqr_swaps_kahan():
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    r = oracle.ffsrqr(A, 40, 0, seed=0)
    assert r.swaps >= 1 and r.g2 <= 2.0 and not r.flags & oracle.FLAG_SWAPCAP
    assert r.history[0][1] > 2.0
    # each swap multiplies |det R11| by the g2 of the test that triggered it
    logdet = []
    for S, g2, _, _ in r.history:
        _, R11 = oracle.householder_qr(A[:, S])
        logdet.append(np.sum(np.log(np.abs(np.diag(R11)))))
    for i in range(1, len(logdet)):
        growth = logdet[i] - logdet[i - 1]
        assert growth > np.log(2.0)
        assert abs(growth - np.log(r.history[i - 1][1])) < 1e-8
    # the swapped-in column is the argmax residual column of the previous test
    for i in range(1, len(r.history)):
        assert r.history[i][0][-1] == r.history[i - 1][2]


def test_swap_cap():
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    r = oracle.ffsrqr(A, 40, 0, seed=0, max_swaps=0)
    assert r.swaps == 0 and r.flags & oracle.FLAG_SWAPCAP and r.g2 > 2.0


def test_tighter_g_swaps_until_satisfied():
    A = synth.spectrum_matrix(120, 90, 0.9 ** np.arange(90), seed=41, noise=1e-10)
    r = oracle.ffsrqr(A, 10, 2, seed=0, g=1.1)
    assert r.swaps >= 1 and r.g2 <= 1.1


def test_permuting_columns_permutes_pivots(small):
    w, A, r = small
    rng = np.random.default_rng(5)
    P = rng.permutation(w.n)
    r2 = oracle.ffsrqr(A[:, P], w.k, w.p, w.seed)
    assert list(P[r2.perm[: w.l]]) == list(r.perm[: w.l])
    assert np.max(np.abs(r2.sigma - r.sigma) / r.sigma) < 1e-12


def test_scaling_by_power_of_two(small):
    w, A, r = small
    r2 = oracle.ffsrqr(A * 2.0 ** 7, w.k, w.p, w.seed)
    assert list(r2.perm) == list(r.perm)
    assert np.array_equal(r2.sigma, r.sigma * 2.0 ** 7)


def test_result_depends_only_on_leading_set(small):
    # sigma(L) and the residual are functions of set(S) and A only
    w, A, r = small
    S = list(r.perm[: w.l])
    perm2, Q2, R11, R2, W2 = oracle.factor_leading_set(A, S[::-1])
    L2, _, V2 = oracle.flip_flop_lq(R2, perm2)
    s2, _ = oracle.jacobi_svd(L2)
    assert np.max(np.abs(s2 - r.sigma) / r.sigma) < 1e-12
    assert abs(dg.residual_fro(A, Q2, L2, V2) - dg.residual_fro(A, r.Q, r.L, r.V)) < 1e-12


def _integer_low_rank(m, n, r, seed):
    """A = X Y^T with small integer factors: every entry is an integer below
    2^24, so the matrix is exactly the same in FP32 and FP64 storage and has
    exact rank r."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-2, 3, size=(m, r)).astype(np.float64)
    Y = rng.integers(-2, 3, size=(n, r)).astype(np.float64)
    return np.asfortranarray(X @ Y.T)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_rank_tolerance_finds_exact_integer_rank(storage):
    """Exactly dependent columns held in either precision: the rule of the
    storage flags RANK_DEFICIENT and counts the exact rank (r = 20 < l = 30,
    past the first 16-column block)."""
    A = _integer_low_rank(200, 150, 20, seed=5)
    assert np.linalg.matrix_rank(A) == 20
    r = oracle.ffsrqr(A, 25, 5, seed=0, storage=storage)
    assert r.flags & oracle.FLAG_RANK_DEFICIENT
    assert r.numerical_rank == 20


def test_rank_tolerance_fp32_keeps_a_conditioned_full_rank_matrix():
    """sigma_min / sigma_1 = 1e-3 is far above FP32 rounding: not flagged."""
    A = synth.spectrum_matrix(300, 200, np.logspace(0, -3, 200), seed=6).astype(np.float32)
    r = oracle.ffsrqr(A.astype(np.float64), 30, 5, seed=0, storage="fp32")
    assert not r.flags & oracle.FLAG_RANK_DEFICIENT
    assert r.numerical_rank == r.l


def test_rank_tolerance_values():
    """The two thresholds written out: max(m, n) 2^-52 a_max for FP64 storage and
    8 sqrt(max(m, n)) 2^-24 a_max for FP32 storage."""
    assert oracle.rank_tolerance(100, 400, 2.0, "fp64") == 400 * 2.0 ** -52 * 2.0
    assert oracle.rank_tolerance(400, 100, 2.0, "fp32") == 8 * 20 * 2.0 ** -24 * 2.0
    with pytest.raises(ValueError):
        oracle.rank_tolerance(1, 1, 1.0, "bf16")
