"""CPU FP64 oracle of ST-HOSVD driven by Flip-Flop SRQR (Section 2,
tensor notation and the ST-HOSVD algorithm; Section 4, the tensor
experiment, which runs ST-HOSVD with FFSRQR as the rank-k SVD).

TEST INFRASTRUCTURE ONLY: imported by tests/ alone, never by the product.

Conventions (the paper's definitions, written out):
  * Tensors are stored in Fortran order: the first index runs fastest.
  * The mode-n unfolding X_(n) is I_n x prod_{j != n} I_j; entry
    (i_n, c) holds x_{i_1..i_d}, where c is the Fortran-order linear index of
    the remaining indices (i_1, .., i_{n-1}, i_{n+1}, .., i_d) in their
    original order.
  * The mode-n product Y = X x_n U (U k x I_n) sums x over i_n against
    u_{j, i_n}; equivalently Y_(n) = U X_(n) (the identity the paper states).
  * ST-HOSVD: G <- X; for each mode r in the processing order, a rank-k_r
    approximate SVD of G_(r) ~ U Sigma V^T, U_r <- U, and G_(r) <- U_r^T G_(r),
    the mode-r product with U_r^T (the paper equates this with
    Sigma V^T, which holds for an exact SVD only).  The rank-k_r SVD is
    Flip-Flop SRQR with oversampling p followed by Algorithm 9's completion
    (ffsrqr, alg9).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .ffsrqr import alg9, ffsrqr


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding (I_n x prod of the other dimensions)."""
    X = np.asarray(X)
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def fold(M: np.ndarray, n: int, shape) -> np.ndarray:
    """Inverse of unfold for a tensor of the given shape."""
    rest = tuple(s for j, s in enumerate(shape) if j != n)
    return np.moveaxis(np.reshape(M, (shape[n],) + rest, order="F"), 0, n)


def mode_product(X: np.ndarray, U: np.ndarray, n: int) -> np.ndarray:
    """X x_n U through Y_(n) = U X_(n)."""
    shape = list(X.shape)
    shape[n] = U.shape[0]
    return fold(U @ unfold(X, n), n, shape)


def tucker_full(G: np.ndarray, Us) -> np.ndarray:
    """G x_1 U_1 x_2 U_2 ... x_d U_d."""
    X = G
    for n, U in enumerate(Us):
        X = mode_product(X, U, n)
    return X


@dataclasses.dataclass
class TuckerResult:
    core: np.ndarray     # k_1 x .. x k_d, Fortran order
    U: list              # U_n, I_n x k_n, orthonormal columns
    sigma: list          # Sigma_k of each mode's rank-k SVD, in processing order
    order: list          # the processing order used


def st_hosvd(X: np.ndarray, ranks, p: int, seed: int, order=None, storage: str = "fp64",
             sketch_mode: str = "fp64", svd=None) -> TuckerResult:
    """ST-HOSVD with the rank-k_r SVD of each unfolding from Flip-Flop SRQR
    (ffsrqr with target rank k_r, oversampling p and the given sketch seed,
    then alg9).  `svd`, if given, replaces that step: svd(M, k) -> U (a
    hook for comparing against exact truncated SVDs)."""
    X = np.asarray(X, dtype=np.float64)
    d = X.ndim
    order = list(range(d)) if order is None else list(order)
    G = X
    Us = [None] * d
    sig = []
    for r in order:
        Gr = unfold(G, r)
        k = int(ranks[r])
        if svd is None:
            res = ffsrqr(Gr, k, p, seed, storage=storage, sketch_mode=sketch_mode)
            a9 = alg9(Gr, res, k)
            U, s = a9.U, a9.sigma
        else:
            U = svd(Gr, k)
            s = np.linalg.svd(U.T @ Gr, compute_uv=False)
        Us[r] = U
        sig.append(s)
        shape = list(G.shape)
        shape[r] = k
        G = fold(U.T @ Gr, r, shape)
    return TuckerResult(core=np.asfortranarray(G), U=Us, sigma=sig, order=order)
