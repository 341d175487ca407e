"""Pins of the robust PCA (IALM) oracle, oracle/ialm.py: the shrinkage
operator against its closed form, and recovery of the planted low-rank and
sparse parts of the paper's test matrices (rank 0.1 m, 5% of the entries
corrupted by values uniform on [-500, 500]) with Flip-Flop SRQR as the SVD
and, as a cross-check, with LAPACK's SVD in the same loop."""
import numpy as np
import pytest

import synth
from oracle import ialm


def test_shrink_closed_form():
    x = np.array([-3.0, -1.0, -0.5, 0.0, 0.25, 1.0, 2.5])
    assert np.array_equal(ialm.shrink(x, 1.0), np.array([-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.5]))
    assert np.array_equal(ialm.shrink(x, 0.0), x)


@pytest.fixture(scope="module")
def problem():
    return synth.rpca_problem(200, 200, 20, 0.05, seed=3)


def test_recovers_planted_parts(problem):
    M, X0, E0 = problem
    r = ialm.rpca_ialm(M, p=10, seed=0)
    err = np.linalg.norm(r.X - X0) / np.linalg.norm(X0)
    assert err < 1e-5, err
    assert r.sv == 20
    assert r.residual < 1e-7
    # the corrupted entries, and only they, are carried by E
    assert np.count_nonzero(np.abs(r.E - E0) > 1e-3) == 0
    assert 10 <= r.iterations <= 60


def test_lapack_svd_in_the_same_loop(problem):
    M, X0, _ = problem

    def exact(D, k):
        U, s, Vt = np.linalg.svd(D, full_matrices=False)
        return U[:, :k], s[:k], Vt[:k].T

    a = ialm.rpca_ialm(M, p=10, seed=0)
    b = ialm.rpca_ialm(M, p=10, seed=0, svd=exact)
    eb = np.linalg.norm(b.X - X0) / np.linalg.norm(X0)
    assert eb < 1e-5
    assert abs(a.iterations - b.iterations) <= 3
    assert np.linalg.norm(a.X - b.X) / np.linalg.norm(X0) < 1e-5


def test_spectral_estimate_bounds():
    # sigma_1(L) = sigma_1(Q1^T A Pi) lies between the norm of the first
    # pivot column (the first column of R) and ||M||_2 (interlacing)
    import oracle
    M, _, _ = synth.rpca_problem(150, 120, 12, 0.05, seed=4)
    est = ialm.spectral_estimate(M, 10, 0)
    first = oracle.ffsrqr(M, 1, 10, 0).perm[0]
    assert np.linalg.norm(M[:, first]) * (1 - 1e-12) <= est <= np.linalg.norm(M, 2) * (1 + 1e-12)
