"""Untimed diagnostics of a Flip-Flop SRQR result (test infrastructure only).

Quantities from the paper's quality analysis (Section 3.3): the trailing block
R22 (never formed by the method; here it is the residual E = A Pi - Q1 R
restricted to the trailing columns, whose spectral norm equals ||R22||_2),
tau and tau-hat (their definition in the proof of Theorem 3.1), the Algorithm 9
singular values Sigma_k = sigma(A Pi Qhat1), and the residuals used by
Theorem 1.1 (Eckart-Young-Mirsky).
"""
from __future__ import annotations

import numpy as np


def residual_matrix(A, res):
    """E = A Pi - Q1 R (m x n, in Pi order)."""
    A = np.asarray(A, dtype=np.float64)
    return A[:, res.perm] - res.Q @ res.R


def residual_fro(A, Q, L, V):
    """||A - Q L V^T||_F in FP64 from the returned factors."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - Q @ (L @ V.T)))


def r22_norms(A, res):
    """(||R22||_2, ||R22||_{1,2}) from the residual of the trailing columns."""
    E = residual_matrix(A, res)[:, res.l:]
    if E.shape[1] == 0:
        return 0.0, 0.0
    two = float(np.linalg.svd(E, compute_uv=False)[0])
    one_two = float(np.sqrt(np.sum(E * E, axis=0)).max())
    return two, one_two


def alg9_sigma(A, res, k):
    """Sigma_k: leading k singular values of A Pi Qhat1 = A V (Algorithm 9)."""
    A = np.asarray(A, dtype=np.float64)
    T = A @ res.V
    return np.linalg.svd(T, compute_uv=False)[:k]


def rtilde_inv_row_norm_max(R11, a, alpha):
    """||R-tilde^{-T}||_{1,2} (largest row norm of R-tilde^{-1})."""
    l = R11.shape[0]
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l] = R11
    Rt[:l, l] = a
    Rt[l, l] = alpha
    X = np.linalg.inv(Rt)
    return float(np.sqrt(np.sum(X * X, axis=1)).max())


def r11_inv_row_norm_max(R11):
    X = np.linalg.inv(R11)
    return float(np.sqrt(np.sum(X * X, axis=1)).max())


def theorem31(A, res, k, sigma_A, g1=1.0):
    """Both sides of the four inequalities of Theorem 3.1 and the tau bounds.

    sigma_A: the exact singular values of A (at least l+1 of them).
    Returns a dict of (lhs, rhs) pairs, each meant to satisfy lhs <= rhs
    (up to rounding).
    """
    l = res.l
    n = res.R.shape[1]
    r22_2, r22_12 = r22_norms(A, res)
    Sk = alg9_sigma(A, res, k)
    a = res.R[:, l] if l < n else np.zeros(l)
    alpha = res.alpha
    R11 = res.R[:, :l]
    g2 = res.g2
    out = {}
    # auxiliary lower bound: sigma_j(A) / (1 + 2||R22||^4/sigma_j(S)^4)^(1/4) <= sigma_j(S)
    for j in range(k):
        rhs = Sk[j]
        lhs = sigma_A[j] / (1.0 + 2.0 * r22_2 ** 4 / Sk[j] ** 4) ** 0.25
        out[f"aux_lower_{j}"] = (lhs, rhs)
    s_kp1 = sigma_A[k]
    # residual of the rank-k approximation in the 2-norm
    Aff = np.asarray(A, dtype=np.float64)
    T = Aff @ res.V
    U, s, Wt = np.linalg.svd(T, full_matrices=False)
    Ak = (U[:, :k] * s[:k]) @ (res.V @ Wt[:k, :].T).T
    err2 = float(np.linalg.svd(Aff - Ak, compute_uv=False)[0])
    out["aux_upper"] = (err2, s_kp1 * (1.0 + 2.0 * (r22_2 / s_kp1) ** 4) ** 0.25)
    if l < n and r22_12 > 0:
        tau = g1 * g2 * (r22_2 / r22_12) / rtilde_inv_row_norm_max(R11, a, alpha) / sigma_A[l]
        tau_hat = g1 * g2 * (r22_2 / r22_12) / r11_inv_row_norm_max(R11) / Sk[k - 1]
        out["tau_dim"] = (tau, g1 * g2 * np.sqrt((l + 1) * (n - l)))
        out["tau_hat_dim"] = (tau_hat, g1 * g2 * np.sqrt(l * (n - l)))
        out["r22_tau"] = (r22_2, tau * sigma_A[l] * (1 + 1e-12))
        for j in range(k):
            denom = (1.0 + min(2.0 * tau_hat ** 4,
                               tau ** 4 * (2.0 + 4.0 * tau_hat ** 4)
                               * (sigma_A[l] / sigma_A[j]) ** 4)) ** 0.25
            out[f"lower_{j}"] = (sigma_A[j] / denom, Sk[j])
        out["upper"] = (err2, s_kp1 * (1.0 + 2.0 * tau ** 4 * (sigma_A[l] / s_kp1) ** 4) ** 0.25)
    return out
