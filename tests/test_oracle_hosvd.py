"""Pins of the ST-HOSVD oracle (oracle/hosvd.py) against definitions and
closed forms: the unfolding against index arithmetic written out entry by
entry, the mode product against its defining sum, exact recovery of a
Tucker tensor of the requested multilinear rank, and the subspaces and
error of ST-HOSVD with exact truncated SVDs on a tensor with a gap."""
import itertools

import numpy as np
import pytest

import synth
from oracle import hosvd


def _unfold_by_index(X, n):
    # column index c = sum over k != n of i_k * prod_{m < k, m != n} I_m
    dims = X.shape
    rest = [k for k in range(len(dims)) if k != n]
    M = np.zeros((dims[n], int(np.prod([dims[k] for k in rest]))))
    for idx in itertools.product(*[range(s) for s in dims]):
        c, stride = 0, 1
        for k in rest:
            c += idx[k] * stride
            stride *= dims[k]
        M[idx[n], c] = X[idx]
    return M


@pytest.mark.parametrize("n", [0, 1, 2])
def test_unfold_matches_index_formula(n):
    X = np.random.default_rng(1).standard_normal((3, 4, 5))
    assert np.array_equal(hosvd.unfold(X, n), _unfold_by_index(X, n))
    assert np.array_equal(hosvd.fold(hosvd.unfold(X, n), n, X.shape), X)


def test_unfold_four_way():
    X = np.random.default_rng(2).standard_normal((2, 3, 2, 3))
    for n in range(4):
        assert np.array_equal(hosvd.unfold(X, n), _unfold_by_index(X, n))


@pytest.mark.parametrize("n", [0, 1, 2])
def test_mode_product_matches_its_sum(n):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 4, 5))
    U = rng.standard_normal((2, X.shape[n]))
    Y = hosvd.mode_product(X, U, n)
    shape = list(X.shape)
    shape[n] = 2
    Z = np.zeros(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        acc = 0.0
        for jn in range(X.shape[n]):
            src = list(idx)
            src[n] = jn
            acc += X[tuple(src)] * U[idx[n], jn]
        Z[idx] = acc
    assert np.allclose(Y, Z, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("order", [None, [2, 0, 1]])
def test_exact_tucker_is_recovered(order):
    # multilinear rank (5, 4, 3) exactly: every unfolding has rank <= l, so
    # the rank-k SVDs span the unfoldings' column spaces and the Tucker form
    # reproduces X to rounding
    X = synth.tucker_tensor((30, 25, 20), (5, 4, 3), seed=4)
    res = hosvd.st_hosvd(X, (5, 4, 3), p=3, seed=0, order=order)
    Xr = hosvd.tucker_full(res.core, res.U)
    assert np.linalg.norm(Xr - X) <= 1e-12 * np.linalg.norm(X)
    for U in res.U:
        assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) < 1e-13
    assert abs(np.linalg.norm(res.core) - np.linalg.norm(X)) <= 1e-12 * np.linalg.norm(X)


def test_close_to_exact_st_hosvd_with_a_gap():
    # noise 1e-6 below a rank-(6, 6, 6) Tucker signal: the FFSRQR subspaces
    # agree with the exact truncated SVDs' to about the noise over the gap
    X = synth.tucker_tensor((40, 35, 30), (6, 6, 6), seed=5, noise=1e-6)

    def exact(M, k):
        return np.linalg.svd(M, full_matrices=False)[0][:, :k]

    a = hosvd.st_hosvd(X, (6, 6, 6), p=4, seed=1)
    b = hosvd.st_hosvd(X, (6, 6, 6), p=4, seed=1, svd=exact)
    for Ua, Ub in zip(a.U, b.U):
        assert np.linalg.norm(Ua @ Ua.T - Ub @ Ub.T, 2) < 1e-4
    ea = np.linalg.norm(hosvd.tucker_full(a.core, a.U) - X)
    eb = np.linalg.norm(hosvd.tucker_full(b.core, b.U) - X)
    assert ea <= 1.01 * eb


def test_core_norm_is_projected_norm():
    # G = X x_1 U_1^T x_2 U_2^T x_3 U_3^T, so ||G|| = ||X (projected)|| <= ||X||
    X = synth.tucker_tensor((20, 18, 16), (4, 4, 4), seed=6, noise=1e-2)
    res = hosvd.st_hosvd(X, (4, 4, 4), p=2, seed=2)
    P = X
    for n, U in enumerate(res.U):
        P = hosvd.mode_product(P, U.T, n)
    assert np.allclose(P, res.core, rtol=1e-12, atol=1e-12)
    assert np.linalg.norm(res.core) <= np.linalg.norm(X)
