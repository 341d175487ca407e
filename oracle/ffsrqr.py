"""Plain FP64 CPU oracle of the Flip-Flop SRQR hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything under ``oracle/``.
It shares no code with the GPU library and never imports it.

Every step follows the paper's text in the paper's order, written for a reader
to check by eye; numpy matmul is used as a library primitive and nothing is
blocked, fused or reordered.  All arithmetic is FP64.

Steps (Feng, Xiao & Gu, "Low-Rank Matrix Approximations with Flip-Flop
Spectrum-Revealing QR Factorization"):

  sketch       Algorithm 2 (TRQRCP), first two steps: B = Omega A; in the
               "bf16" mode both factors are first rounded to bfloat16 and the
               exact products are summed in FP64 (the mixed-precision form's
               definition of the sample matrix).
  qrcp_sketch  Algorithm 1 (Partial QRCP) run for l steps on B; pivots only.
  qr_panel     Householder QR without pivoting of A(:, S) (Algorithm 2, the
               "QR on the pivoted block" step; compact-WY form in Section 2.1),
               returned as explicit Q1 and R11.
  project      R = Q1^T A Pi: the (R11 R12) block of the partial QR
               factorization (Section 2.1, block form; Section 3.1, partial
               QRCP on A to l steps).
  srqr_rho     g2 of Section 2.2 (definitions of R-tilde, g1, g2), computed
               exactly.
  g2_probe_estimate
               Algorithm 4's randomized estimate of the same quantity: the
               column norms of Omega_q R-tilde^{-T} scaled by |alpha| / sqrt(d),
               Omega_q a fresh d x (l+1) Gaussian probe per test (an option of
               ffsrqr; the exact g2 is the default).
  ffsrqr       Algorithm 4 (SRQR) swap loop around the above, then Section
               3.1: QR without pivoting of (R11 R12)^T, L = Rhat11^T,
               V = Pi Qhat1, and sigma(L) by one-sided Jacobi.
  alg9         Algorithm 9, last three steps: tmp = A Pi Qhat1 = A V, its thin
               SVD (Householder QR of tmp, then one-sided Jacobi with vectors
               on the triangular factor), U = U_tmp(:, 1:k), Sigma_k and
               V_k = Pi Qhat1 V_tmp(:, 1:k).

Readings of the paper taken here (each is listed with its reason in the
design notes):
  * Omega has l = min(k+p, m, n) rows and QRCP on B runs all l steps (one
    block: the block size b only tiles work, it does not change results).
  * Column norms on B are recomputed from scratch at every step (no
    downdating), ties go to the smallest original column index.
  * Residual norms gamma_j of the trailing columns are exact,
    ||(I - Q1 Q1^T) a_j||, by default.  With est_norms they are Algorithm
    4's estimates instead: r_i = ||B(:, i)||^2 / (sample rows) from the
    sample after the last block's update (for the one-block selection, the
    update of Algorithm 2 with all l pivots as the block, B(:, rest) -=
    B(:, S) R11^{-1} R12), j* = argmax r_i, alpha the exact residual
    norm of column j*; before each test r_i -= (row l+1 of R of [S, j*])_i^2;
    after a swap r_i += (row l+1 of R of [S', i*])_i^2 for the trailing
    columns and r_{i*} = R_{l+1,l+1}^2 (the squared rows of the retriangularised
    R, taken here from a fresh QR of the same ordered columns: the thin QR is
    unique up to row signs); after an identity rotation r_{j*} = alpha^2 and
    the other estimates return to their values before the downdate.
  * g2 is exact by default: |alpha| * max row norm of R-tilde^{-1}.  With
    g2_probe = d > 0 it is Algorithm 4's estimate instead: the q-th test of a
    solve (q = 1, 2, ...) draws Omega_q (d x (l+1)) from the Philox stream q,
    g2 is the largest estimated column norm over all l+1 positions and i* its
    argmax; when i* is position l+1 the round-robin rotation is the identity
    and the next test only draws a fresh probe.  The swap cap counts these
    identity rotations too.
  * A swap (Algorithm 4's round-robin rotation) replaces S[i*] by j*: the new
    ordered leading set is S without S[i*], followed by j*.  The factorization
    of the new set is recomputed from scratch instead of Givens updates; thin
    QR is unique up to row signs, and signs are normalised.
  * The swap loop is capped at max_swaps (default 4 l); the flag SWAPCAP
    records when the cap stops it.
  * Outputs are normalised to diag(R11) > 0 and diag(L) >= 0.
  * sigma_j := sigma_j(L), L the whole l x l factor.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .philox import omega as _omega

FLAG_RANK_DEFICIENT = 1
FLAG_SWAPCAP = 2
FLAG_NONFINITE = 4
FLAG_L_CLAMPED = 8


# ---------------------------------------------------------------------------
# Householder reflector (LAPACK xLARFG convention)
# ---------------------------------------------------------------------------
def _norm2(x: np.ndarray) -> float:
    """Euclidean norm, scaled by max |x_i| so that tiny entries do not underflow."""
    s = float(np.max(np.abs(x))) if x.size else 0.0
    if s == 0.0 or not math.isfinite(s):
        return s
    y = x / s
    return s * math.sqrt(float(y @ y))


def householder(x: np.ndarray):
    """Reflector H = I - tau v v^T with v[0] = 1 and H x = beta e_1.

    beta = -sign(x[0]) ||x|| (sign(0) = +), tau = (beta - x[0]) / beta.
    When x[1:] is zero, H = I (tau = 0, beta = x[0]).
    """
    alpha = float(x[0])
    xnorm = _norm2(x[1:]) if x.shape[0] > 1 else 0.0
    v = np.zeros_like(x, dtype=np.float64)
    v[0] = 1.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    beta = -math.copysign(math.hypot(alpha, xnorm), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


# ---------------------------------------------------------------------------
# a1: sketch
# ---------------------------------------------------------------------------
def omega(seed: int, l: int, m: int) -> np.ndarray:
    return _omega(seed, l, m)


def round_bf16(x) -> np.ndarray:
    """Each FP64 value rounded to the nearest bfloat16 value, ties to even.

    bfloat16 keeps 8 significant bits and the FP32 exponent range, so near
    x = f 2^e (1/2 <= |f| < 1) its values are spaced 2^(e-8) apart, and
    2^-133 apart below 2^-126 (subnormals).  The rounding is taken from the
    FP64 value directly (not through FP32, which could round twice).
    Finite inputs below the bfloat16 overflow threshold only.
    """
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)
    return np.rint(x / q) * q


def sketch(Omega: np.ndarray, A: np.ndarray, mode: str = "fp64") -> np.ndarray:
    """B = Omega A (Algorithm 2: form the initial sample matrix).

    mode "fp64": FP64 product.  mode "bf16": B = bf16(Omega) bf16(A), i.e.
    B_ij = sum_t bf16(Omega_it) bf16(A_tj) with every product exact in FP64
    (8 x 8 significant bits) and the sum taken in FP64.
    """
    A = np.asarray(A, dtype=np.float64)
    if mode == "fp64":
        return Omega @ A
    if mode == "bf16":
        return round_bf16(Omega) @ round_bf16(A)
    raise ValueError(f"unknown sketch mode {mode!r}")


# ---------------------------------------------------------------------------
# a2: partial QRCP on the sketch
# ---------------------------------------------------------------------------
def qrcp_sketch(B: np.ndarray, l: int):
    """Algorithm 1 (Partial QRCP) on B for l steps.

    Returns (perm, margins, Bout): perm is the full column order (the first l
    entries are the pivots in the order chosen, the rest is where the swaps
    left them), margins[j] = (r_max - r_second) / r_max at step j, and Bout
    the transformed B (upper trapezoidal in its leading l columns).
    """
    B = np.array(B, dtype=np.float64, copy=True)
    rows, n = B.shape
    perm = np.arange(n)
    margins = np.zeros(l)
    for j in range(l):
        # residual column norms of the trailing matrix, recomputed from scratch
        r = np.sum(B[j:, j:] ** 2, axis=0)
        rmax = r.max()
        cands = np.flatnonzero(r == rmax)
        s = int(cands[np.argmin(perm[j + cands])])       # tie -> smallest original index
        if r.shape[0] > 1:
            rest = np.delete(r, s)
            margins[j] = (rmax - rest.max()) / rmax if rmax > 0 else 0.0
        else:
            margins[j] = 1.0
        # exchange columns j and j+s in B and Pi
        if s:
            B[:, [j, j + s]] = B[:, [j + s, j]]
            perm[[j, j + s]] = perm[[j + s, j]]
        if j < rows:
            v, tau, beta = householder(B[j:, j])
            if j + 1 < n and tau != 0.0:
                w = v @ B[j:, j + 1:]
                B[j:, j + 1:] -= tau * np.outer(v, w)
            B[j, j] = beta
            B[j + 1:, j] = 0.0
    return perm, margins, B


# ---------------------------------------------------------------------------
# a2 (blocked): Algorithm 2, truncated randomized QRCP with the sample update
# ---------------------------------------------------------------------------
def trqrcp_pivots(A: np.ndarray, l: int, b: int, p: int, seed: int, sketch_mode: str = "fp64",
                  trace: list | None = None):
    """Algorithm 2's pivot selection, l pivots in blocks of b.

    The sample B = Omega A has rows = min(b + p, m) rows (Omega from the same
    Philox stream: the first rows of the l-row Omega).  For each block of
    bj = min(b, l - j) pivots: partial QRCP (Algorithm 1) on the sample's
    columns not yet chosen gives the block's pivots; the chosen columns'
    residual after the previous blocks, A(:, piv) - Q Q^T A(:, piv), is
    factored (Householder QR, Q_b R11); R12 = Q_b^T A(:, rest); and the sample
    is updated, B(:, rest) <- B(:, rest) - B(:, piv) R11^{-1} R12, which is
    Omega times the new residual of the remaining columns.  Returns (S, margins)
    with S the l pivots in order and margins the QRCP margins of the steps
    that chose them.  With trace a list, (Q, B, rest) after each block is
    appended to it.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows = min(b + p, m)
    B = sketch(omega(seed, rows, m), A, sketch_mode)
    active = list(range(n))
    S: list = []
    margins: list = []
    Q = np.zeros((m, 0))
    while len(S) < l:
        bj = min(b, l - len(S))
        perm, mg, _ = qrcp_sketch(B[:, active], bj)
        piv = [active[int(i)] for i in perm[:bj]]
        margins.extend(float(x) for x in mg[:bj])
        P = A[:, piv]
        for _ in range(2):  # the residual after the previous blocks (two projections)
            P = P - Q @ (Q.T @ P)
        Qb, R11 = householder_qr(P)
        chosen = set(piv)
        rest = [c for c in active if c not in chosen]
        if rest:
            R12 = Qb.T @ A[:, rest]
            X = np.column_stack([back_substitute(R11, R12[:, t]) for t in range(len(rest))])
            B[:, rest] = B[:, rest] - B[:, piv] @ X
        Q = np.hstack([Q, Qb])
        S.extend(piv)
        active = rest
        if trace is not None:
            trace.append((Q.copy(), B.copy(), list(rest)))
    return S, np.asarray(margins)


# ---------------------------------------------------------------------------
# a3: Householder QR (no pivoting) of a tall panel, explicit Q1
# ---------------------------------------------------------------------------
def householder_qr(P: np.ndarray):
    """Householder QR of P (m x c), m >= c: P = Q1 R, Q1 explicit (m x c).

    Reflectors are applied one column at a time (Algorithm 1 without the
    pivot search); Q1 = H_1 ... H_c [I; 0] is accumulated backwards.
    Signs are normalised so that diag(R) >= 0.
    """
    W = np.array(P, dtype=np.float64, copy=True)
    m, c = W.shape
    if m < c:
        raise ValueError("householder_qr needs a tall panel")
    vs, taus = [], []
    for j in range(c):
        v, tau, beta = householder(W[j:, j])
        if j + 1 < c and tau != 0.0:
            W[j:, j + 1:] -= tau * np.outer(v, v @ W[j:, j + 1:])
        W[j, j] = beta
        W[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    R = np.triu(W[:c, :])
    Q = np.zeros((m, c))
    Q[:c, :c] = np.eye(c)
    for j in range(c - 1, -1, -1):
        # H_j only touches rows j:, and columns < j of the partial product are
        # still e_i there (zero in rows j:), so only Q[j:, j:] changes.
        v, tau = vs[j], taus[j]
        if tau != 0.0:
            Q[j:, j:] -= tau * np.outer(v, v @ Q[j:, j:])
    d = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * d, R * d[:, None]


# ---------------------------------------------------------------------------
# a4: projection and residual norms
# ---------------------------------------------------------------------------
def project(Q1: np.ndarray, A: np.ndarray) -> np.ndarray:
    """W = Q1^T A for every column of A, in the original column order."""
    return Q1.T @ np.asarray(A, dtype=np.float64)


def residual_norms(A: np.ndarray, Q1: np.ndarray, W: np.ndarray, cols) -> np.ndarray:
    """gamma_j = ||a_j - Q1 W(:, j)|| for j in cols (exact, column by column)."""
    A = np.asarray(A)
    cols = np.asarray(cols)
    out = np.empty(cols.shape[0])
    step = 256
    for s in range(0, cols.shape[0], step):
        c = cols[s:s + step]
        E = np.asarray(A[:, c], dtype=np.float64) - Q1 @ W[:, c]
        out[s:s + step] = np.sqrt(np.sum(E * E, axis=0))
    return out


# ---------------------------------------------------------------------------
# a5: SRQR quantities
# ---------------------------------------------------------------------------
def back_substitute(U: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve U x = b for upper-triangular U, one row at a time."""
    n = U.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (b[i] - U[i, i + 1:] @ x[i + 1:]) / U[i, i]
    return x


def upper_inverse(U: np.ndarray) -> np.ndarray:
    """Inverse of an upper-triangular matrix, column by column."""
    n = U.shape[0]
    X = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        X[: j + 1, j] = back_substitute(U[: j + 1, : j + 1], e[: j + 1])
    return X


def srqr_rho(R11: np.ndarray, a: np.ndarray, alpha: float) -> np.ndarray:
    """rho_i = |alpha| * ||row i of R-tilde^{-1}||, i = 1..l+1 (Section 2.2).

    R-tilde = [[R11, a], [0, alpha]] is the leading (l+1) x (l+1) block of R;
    g2 = |alpha| ||R-tilde^{-T}||_{1,2} is the largest rho_i (the largest
    column norm of R-tilde^{-T} is the largest row norm of R-tilde^{-1}).
    """
    l = R11.shape[0]
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l] = R11
    Rt[:l, l] = a
    Rt[l, l] = alpha
    X = upper_inverse(Rt)
    return abs(alpha) * np.sqrt(np.sum(X * X, axis=1))


def sample_update(A: np.ndarray, B: np.ndarray, S) -> np.ndarray:
    """Algorithm 2's sample update with the pivots S as one block: B(:, c) -
    B(:, S) R11^{-1} R12(:, c) for the columns c outside S (zero columns at
    S), R11 and R12 from the QR of A(:, S); equal to Omega times the residual
    of column c when B = Omega A."""
    S = list(S)
    perm, Q1, R11, R, W = factor_leading_set(A, S)
    out = np.zeros_like(B, dtype=np.float64)
    chosen = set(S)
    for c in range(A.shape[1]):
        if c not in chosen:
            out[:, c] = B[:, c] - B[:, S] @ back_substitute(R11, W[:, c])
    return out


def row_l1(A: np.ndarray, S, j: int) -> np.ndarray:
    """Row l+1 of R in the QR of A(:, S + [j]) over all columns of A:
    q^T A with q the last column of the Householder Q of those l+1 columns
    (the part of a_j outside span(A(:, S)), normalised; its squares are the
    norm downdates of Algorithm 4)."""
    Qx, _ = householder_qr(np.asarray(A[:, list(S) + [j]], dtype=np.float64))
    return Qx[:, -1] @ A


def probe_omega(seed: int, q: int, d: int, l: int) -> np.ndarray:
    """The q-th probe (q >= 1) of a solve: d x (l+1) N(0,1), Philox stream q."""
    if q < 1:
        raise ValueError("probe streams start at 1 (stream 0 is the sketch)")
    return _omega(seed, d, l + 1, stream=q)


def g2_probe_estimate(R11: np.ndarray, a: np.ndarray, alpha: float, Om: np.ndarray) -> np.ndarray:
    """Algorithm 4's estimate of g2 (Section 2.2; Algorithm 4, the g2 step):
    est_i = |alpha| / sqrt(d) * (i-th column 2-norm of Om R-tilde^{-T}),
    i = 1..l+1, for a d x (l+1) probe Om with N(0,1) entries.  Since
    E ||Om x||^2 = d ||x||^2, est_i^2 is an unbiased estimate of rho_i^2
    (srqr_rho); g2 ~ max_i est_i."""
    l = R11.shape[0]
    d = Om.shape[0]
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l] = R11
    Rt[:l, l] = a
    Rt[l, l] = alpha
    Y = Om @ upper_inverse(Rt).T
    return abs(alpha) / math.sqrt(d) * np.sqrt(np.sum(Y * Y, axis=0))


# ---------------------------------------------------------------------------
# a6: flip-flop LQ and right factor
# ---------------------------------------------------------------------------
def flip_flop_lq(R: np.ndarray, perm: np.ndarray):
    """QR without pivoting of R^T = (R11 R12)^T (Section 3.1).

    Returns (L, Qhat1, V): L = Rhat11^T (lower triangular, diag >= 0),
    Qhat1 (n x l) explicit, V = Pi Qhat1, i.e. V[perm[i], :] = Qhat1[i, :].
    """
    Qh, Rh = householder_qr(R.T)
    L = Rh.T
    V = np.empty_like(Qh)
    V[np.asarray(perm), :] = Qh
    return L, Qh, V


# ---------------------------------------------------------------------------
# a7: one-sided Jacobi singular values
# ---------------------------------------------------------------------------
def jacobi_svd(M: np.ndarray, tol: float = 1e-14, max_sweeps: int = 60,
               want_vectors: bool = False):
    """One-sided (Hestenes) Jacobi on the columns of M, cyclic by rows.

    Each pair (p, q) with |c_p . c_q| > tol ||c_p|| ||c_q|| is rotated so that
    the two columns become orthogonal (Rutishauser's formulas).  Stops after a
    sweep with no rotation.  Returns sigma descending (and U, V if asked;
    M V = U diag(sigma)).
    """
    G = np.array(M, dtype=np.float64, copy=True)
    n = G.shape[1]
    V = np.eye(n) if want_vectors else None
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                cp = G[:, p]
                cq = G[:, q]
                a = float(cp @ cp)
                b = float(cq @ cq)
                g = float(cp @ cq)
                if a == 0.0 or b == 0.0 or abs(g) <= tol * math.sqrt(a * b):
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * g)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = c * t
                new_p = c * cp - s * cq
                new_q = s * cp + c * cq
                G[:, p] = new_p
                G[:, q] = new_q
                if V is not None:
                    vp = V[:, p].copy()
                    vq = V[:, q].copy()
                    V[:, p] = c * vp - s * vq
                    V[:, q] = s * vp + c * vq
        if not rotated:
            break
    norms = np.sqrt(np.sum(G * G, axis=0))
    order = np.argsort(-norms, kind="stable")
    sigma = norms[order]
    if not want_vectors:
        return sigma, sweeps
    U = np.zeros_like(G)
    nz = sigma > 0
    U[:, nz] = G[:, order[nz]] / sigma[nz]
    return sigma, U, V[:, order], sweeps


# ---------------------------------------------------------------------------
# The whole path
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Result:
    perm: np.ndarray        # [n] pivots first (in order), the rest ascending
    Q: np.ndarray           # m x l, orthonormal columns, diag(R11) > 0
    R: np.ndarray           # l x n = [R11 R12] in perm order
    L: np.ndarray           # l x l lower triangular, diag >= 0
    V: np.ndarray           # n x l, Pi Qhat1
    sigma: np.ndarray       # [l] singular values of L, descending
    l: int
    swaps: int
    g2: float               # g2 of the final leading set
    alpha: float            # residual norm of the (l+1)-st column
    jstar: int              # original index of that column
    margins: np.ndarray     # QRCP-on-B margins per step
    jstar_margin: float     # (gamma_max^2 - gamma_2nd^2) / gamma_max^2 at the final test
    flags: int
    numerical_rank: int
    B: np.ndarray           # sketch (l x n)
    history: list           # [(S, g2, jstar, alpha)] per SRQR test
    sketch_mode: str = "fp64"
    probes: int = 0         # random probes drawn (0: exact g2)
    norm_estimates: np.ndarray | None = None  # est_norms: r_i w.r.t. the final leading set
    test_margins: list = dataclasses.field(default_factory=list)
    # per SRQR test: (relative gap of the two largest squared residual norms
    # or estimates that pick j*, relative gap of the two largest values that
    # pick i*)


def _full_perm(S, n):
    S = list(int(s) for s in S)
    chosen = np.zeros(n, dtype=bool)
    chosen[S] = True
    rest = np.flatnonzero(~chosen)
    return np.concatenate([np.asarray(S, dtype=np.int64), rest.astype(np.int64)])


def factor_leading_set(A: np.ndarray, S):
    """QR of A(:, S) and the projection for a given ordered leading set S."""
    A = np.asarray(A)
    n = A.shape[1]
    perm = _full_perm(S, n)
    P = np.asarray(A[:, perm[: len(S)]], dtype=np.float64)
    Q1, R11 = householder_qr(P)
    W = project(Q1, A)
    R = W[:, perm]
    R[:, : len(S)] = R11
    return perm, Q1, R11, R, W


def residual_margin(gam: np.ndarray) -> float:
    """(gamma_max^2 - gamma_2nd^2) / gamma_max^2 over the trailing columns
    (1 when there is one column, 0 when the largest is zero)."""
    if gam.shape[0] < 2:
        return 1.0
    g2 = np.sort(gam * gam)
    return float((g2[-1] - g2[-2]) / g2[-1]) if g2[-1] > 0 else 0.0


def rank_tolerance(m: int, n: int, max_col_norm: float, storage: str = "fp64") -> float:
    """tau_r: alpha or |R11_ii| at or below it counts as zero (numerical rank).

    For FP64 data, max(m, n) 2^-52 max_j ||a_j|| (the usual rank-revealing
    threshold).  When A and the factors are held in FP32, rounding to 2^-24
    leaves exactly dependent columns with residuals of order
    sqrt(l) 2^-24 ||a_j||, so the threshold is 8 sqrt(max(m, n)) 2^-24
    max_j ||a_j||: zero at the storage precision.
    """
    mn = float(max(m, n))
    if storage == "fp64":
        return mn * 2.0 ** -52 * max_col_norm
    if storage == "fp32":
        return 8.0 * math.sqrt(mn) * 2.0 ** -24 * max_col_norm
    raise ValueError(f"unknown storage {storage!r}")


def ffsrqr(A: np.ndarray, k: int, p: int, seed: int, g: float = 2.0,
           max_swaps: int | None = None, Omega: np.ndarray | None = None,
           sketch_mode: str = "fp64", storage: str = "fp64", block: int = 0,
           g2_probe: int = 0, est_norms: bool = False) -> Result:
    """Flip-Flop SRQR hot path, FP64 (Algorithm 9 up to the LQ, Algorithm 4 inside).

    sketch_mode selects the arithmetic of B = Omega A ("fp64" or "bf16", see
    sketch()); every later step is FP64 on the same A.  storage names the
    precision the data is held in ("fp64" or "fp32"); it only sets the rank
    tolerance (rank_tolerance()).  g2_probe = d > 0 replaces the exact g2 by
    Algorithm 4's d-row random estimate (g2_probe_estimate, probe_omega).
    est_norms replaces the exact residual norms that pick j* by Algorithm
    4's sample estimates (sample_update, row_l1, and the module notes).
    """
    A = np.asarray(A)
    m, n = A.shape
    if not (1 <= k <= min(m, n)) or p < 0 or not g > 1.0 or g2_probe < 0:
        raise ValueError("bad arguments")
    flags = 0
    l = min(k + p, m, n)
    if l < k + p:
        flags |= FLAG_L_CLAMPED
    if max_swaps is None:
        max_swaps = 4 * l
    Af = np.asarray(A, dtype=np.float64)
    if not np.all(np.isfinite(Af)):
        # a non-finite entry poisons every step: report it, factor nothing
        flags |= FLAG_NONFINITE
        nan = np.nan
        return Result(perm=np.arange(n, dtype=np.int64), Q=np.full((m, l), nan),
                      R=np.full((l, n), nan), L=np.full((l, l), nan), V=np.full((n, l), nan),
                      sigma=np.full(l, nan), l=l, swaps=0, g2=nan, alpha=nan, jstar=-1,
                      margins=np.zeros(l), jstar_margin=0.0, flags=flags, numerical_rank=0,
                      B=np.full((l, n), nan), history=[], sketch_mode=sketch_mode)
    colnorm = np.sqrt(np.sum(Af * Af, axis=0))
    tau_r = rank_tolerance(m, n, float(colnorm.max()), storage)

    if block > 0:
        # a1 + a2 blocked: Algorithm 2 with a (b + p)-row sample, b = min(block, k)
        trace = [] if est_norms else None
        S, margins = trqrcp_pivots(Af, l, min(block, k), p, seed, sketch_mode, trace=trace)
        S = [int(s) for s in S]
        B = None
        if est_norms:
            # Algorithm 4: squared column norms of the updated sample over its
            # row count estimate the squared residual norms of A's columns
            Bs = trace[-1][1]
            r = np.sum(Bs * Bs, axis=0) / Bs.shape[0]
    else:
        # a1
        Om = omega(seed, l, m) if Omega is None else Omega
        B = sketch(Om, Af, sketch_mode)
        # a2
        pivots, margins, _ = qrcp_sketch(B, l)
        S = [int(s) for s in pivots[:l]]
        if est_norms:
            Bu = sample_update(Af, B, S)
            r = np.sum(Bu * Bu, axis=0) / B.shape[0]

    swaps = 0
    est_out = None
    rotations = 0   # loop iterations: the swaps plus identity rotations of the probe
    q = 0           # SRQR tests so far (the probe stream of the next one is q + 1)
    test_margins = []
    history = []
    numerical_rank = l
    jmargin = 1.0
    while True:
        # a3 + a4
        perm, Q1, R11, R, W = factor_leading_set(Af, S)
        # a5
        if l < n:
            trailing = perm[l:]
            if est_norms:
                rt = r[trailing]
                cands = np.flatnonzero(rt == rt.max())
                jstar = int(trailing[int(cands[np.argmin(trailing[cands])])])
                alpha = float(residual_norms(Af, Q1, W, [jstar])[0])
                jmargin = residual_margin(np.sqrt(np.maximum(rt, 0.0)))
                # the one-step QR of column j* and the downdate of the estimates
                r_before = r.copy()
                est_out = r_before
                r = r - row_l1(Af, S, jstar) ** 2
            else:
                gam = residual_norms(Af, Q1, W, trailing)
                gmax = gam.max()
                cands = np.flatnonzero(gam == gmax)
                jpos = int(cands[np.argmin(trailing[cands])])
                jstar = int(trailing[jpos])
                alpha = float(gmax)
                jmargin = residual_margin(gam)
            dR = np.abs(np.diag(R11))
            if alpha <= tau_r or dR.min() <= tau_r:
                flags |= FLAG_RANK_DEFICIENT
                numerical_rank = int(np.sum(dR > tau_r))
                g2 = 1.0
                history.append((list(S), g2, jstar, alpha))
                break
            q += 1
            if g2_probe > 0:
                est = g2_probe_estimate(R11, W[:, jstar], alpha, probe_omega(seed, q, g2_probe, l))
                g2 = float(est.max())
                istar = int(np.argmax(est))       # 0..l; l is the (l+1)-st position
            else:
                rho = srqr_rho(R11, W[:, jstar], alpha)
                g2 = float(rho.max())
                istar = int(np.argmax(rho[:l]))
            history.append((list(S), g2, jstar, alpha))
            cand_i = np.sort(est if g2_probe > 0 else rho[:l])
            imargin = float((cand_i[-1] - cand_i[-2]) / cand_i[-1]) if cand_i.size > 1 and cand_i[-1] > 0 else 1.0
            test_margins.append((jmargin, imargin))
            if g2 <= g:
                break
            if rotations >= max_swaps:
                flags |= FLAG_SWAPCAP
                break
            rotations += 1
            if istar < l:
                removed = S[istar]
                S = S[:istar] + S[istar + 1:] + [jstar]
                swaps += 1
                if est_norms:
                    # the removed column at position l+1 of the new order: its
                    # row of R restores the estimates; r of it is exact
                    row = row_l1(Af, S, removed)
                    r = r + row ** 2
                    r[removed] = row[removed] ** 2
            elif est_norms:
                # the identity rotation: j* back at position l+1, r_{j*} exact
                r = r_before
                r[jstar] = alpha * alpha
        else:
            jstar, alpha, g2 = -1, 0.0, 1.0
            history.append((list(S), g2, jstar, alpha))
            break

    # a6
    L, Qhat1, V = flip_flop_lq(R, perm)
    # a7
    sigma, _ = jacobi_svd(L)
    return Result(perm=perm, Q=Q1, R=R, L=L, V=V, sigma=sigma, l=l, swaps=swaps,
                  g2=g2, alpha=alpha, jstar=jstar, margins=margins, jstar_margin=jmargin,
                  flags=flags, numerical_rank=numerical_rank, B=B, history=history,
                  sketch_mode=sketch_mode, probes=q if g2_probe > 0 else 0,
                  norm_estimates=est_out, test_margins=test_margins)


# ---------------------------------------------------------------------------
# Algorithm 9 completion: rank-k approximate SVD from the flip-flop factors
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Alg9:
    U: np.ndarray           # m x k, orthonormal columns
    sigma: np.ndarray       # [k] leading singular values of A Pi Qhat1, descending
    V: np.ndarray           # n x k, Pi Qhat1 V_tmp(:, 1:k)
    sigma_all: np.ndarray   # [l] all singular values of tmp


def alg9(A: np.ndarray, res: Result, k: int) -> Alg9:
    """Last three steps of Algorithm 9 on the result of ffsrqr().

    tmp = A Pi Qhat1; since V = Pi Qhat1 this is A V (m x l).  Its thin SVD
    is taken as tmp = Q_t R_t (Householder QR), R_t V_t = U_R diag(s) (one-
    sided Jacobi with accumulated rotations), U_tmp = Q_t U_R.  Returns
    U = U_tmp(:, 1:k), sigma = s(1:k), V_k = V V_t(:, 1:k).  Column signs are
    normalised so that the largest-magnitude entry of each column of U_k is
    positive (the SVD fixes the pairs (u_j, v_j) only up to a common sign).
    """
    A = np.asarray(A, dtype=np.float64)
    tmp = A @ res.V
    Qt, Rt = householder_qr(tmp)
    s, UR, VR, _ = jacobi_svd(Rt, want_vectors=True)
    U = Qt @ UR[:, :k]
    Vk = res.V @ VR[:, :k]
    idx = np.argmax(np.abs(U), axis=0)
    sg = np.where(U[idx, np.arange(k)] < 0, -1.0, 1.0)
    return Alg9(U=U * sg, sigma=s[:k].copy(), V=Vk * sg, sigma_all=s)
