"""CPU FP64 oracle of robust PCA by the inexact augmented Lagrange multiplier
method with Flip-Flop SRQR as its SVD (Section 2, nuclear norm minimization
and the robust PCA algorithm; Section 4, the robust PCA experiment).

TEST INFRASTRUCTURE ONLY: imported by tests/ alone, never by the product.

The problem: min ||X||_* + lambda ||E||_1 subject to M = X + E.  Iteration
k (the robust PCA algorithm of Section 2):
  D = M - E_k + Y_k / mu_k;  (U, Sigma, V) = the SVD of D (here: rank-sv
      Flip-Flop SRQR with oversampling p, completed by Algorithm 9);
  X_{k+1} = U S_{1/mu_k}(Sigma) V^T;
  E_{k+1} = S_{lambda/mu_k}(M - X_{k+1} + Y_k / mu_k);
  Y_{k+1} = Y_k + mu_k (M - X_{k+1} - E_{k+1});  mu_{k+1} = min(rho mu_k, mu_bar);
  stop when ||M - X_{k+1} - E_{k+1}||_F / ||M||_F < tol,
with S_w(x) = sgn(x) max(|x| - w, 0) and, initially, E_0 = 0,
Y_0 = M / J(M), J(M) = max(||M||_2, max_ij |M_ij|).

Settings the paper leaves to the IALM code it uses (the readings of the
design notes): mu_0 = 1.25 / ||M||_2, mu_bar = 1e7 mu_0, rho = 1.5,
tol = 1e-7, lambda = 1 / sqrt(max(m, n)); the partial SVD's rank starts at
sv = 10 and is predicted from the previous iteration: with svp the number of
singular values above 1 / mu_k, sv <- svp + 1 if svp < sv, else
svp + round(0.05 n), capped at min(m, n); ||M||_2 is taken as sigma_1 of the
flip-flop factor L of M (ffsrqr with k = 1 and the same p and seed), the
method's own estimate of the largest singular value.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .ffsrqr import alg9, ffsrqr


def shrink(x, w: float):
    """Soft shrinkage S_w(x) = sgn(x) max(|x| - w, 0), elementwise."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.maximum(np.abs(x) - w, 0.0)


def spectral_estimate(M: np.ndarray, p: int, seed: int) -> float:
    """sigma_1 of the flip-flop factor L of M (k = 1, oversampling p)."""
    return float(ffsrqr(M, 1, p, seed).sigma[0])


@dataclasses.dataclass
class RpcaResult:
    X: np.ndarray
    E: np.ndarray
    iterations: int
    sv: int               # rank of the final X (singular values kept)
    residual: float       # ||M - X - E||_F / ||M||_F at exit
    history: list         # (sv requested, svp kept, residual) per iteration


def rpca_ialm(M: np.ndarray, p: int = 10, seed: int = 0, lam: float | None = None, tol: float = 1e-7,
              max_iter: int = 500, rho: float = 1.5, svd=None) -> RpcaResult:
    """Robust PCA by IALM with Flip-Flop SRQR (plus Algorithm 9) as the
    rank-sv SVD.  `svd`, if given, replaces that step: svd(D, sv) -> (U,
    sigma, V) with sigma descending (for comparing with exact SVDs)."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    r = min(m, n)
    if lam is None:
        lam = 1.0 / math.sqrt(max(m, n))
    norm2 = spectral_estimate(M, p, seed)
    J = max(norm2, float(np.max(np.abs(M))))
    Y = M / J
    E = np.zeros_like(M)
    X = np.zeros_like(M)
    mu = 1.25 / norm2
    mu_bar = mu * 1e7
    nM = float(np.linalg.norm(M))
    sv = min(10, r)
    history = []
    it = 0
    svp = 0
    res = float("inf")
    while it < max_iter:
        it += 1
        D = M - E + Y / mu
        if svd is None:
            f = ffsrqr(D, sv, p, seed)
            a9 = alg9(D, f, sv)
            U, s, V = a9.U, a9.sigma, a9.V
        else:
            U, s, V = svd(D, sv)
        svp = int(np.sum(s[:sv] > 1.0 / mu))
        X = (U[:, :svp] * (s[:svp] - 1.0 / mu)) @ V[:, :svp].T
        E = shrink(M - X + Y / mu, lam / mu)
        Z = M - X - E
        Y = Y + mu * Z
        res = float(np.linalg.norm(Z)) / nM
        history.append((sv, svp, res))
        sv = min(svp + 1, r) if svp < sv else min(svp + int(round(0.05 * n)), r)
        mu = min(mu * rho, mu_bar)
        if res < tol:
            break
    return RpcaResult(X=X, E=E, iterations=it, sv=svp, residual=res, history=history)
