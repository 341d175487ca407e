"""Per-step GPU parity: each stage entry point of the C ABI against the
oracle's step on the same seeded inputs (element by element), at sizes that
span several tiles and a ragged tail."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev_f, host, rel

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_1803_01982_amd as ff
    ff.load()
    return ff


# ------------------------------------------------------------------ Omega
@pytest.mark.parametrize("seed,l,m", [(0, 30, 1000), (7, 17, 333), ((1 << 63) + 5, 5, 4099)])
def test_omega_fp64(ff, seed, l, m):
    import torch
    announce(f"omega fp64 seed={seed} l={l} m={m}")
    Ot = host(ff.omega(seed, l, m, torch.float64))
    ref = oracle.omega(seed, l, m).T
    # different libm: a few ulp
    assert np.max(np.abs(Ot - ref) / np.maximum(np.abs(ref), 1e-3)) < 64 * EPS


def test_omega_fp32_is_rounded_fp64(ff):
    import torch
    announce("omega fp32 seed=3 l=9 m=700")
    Ot = host(ff.omega(3, 9, 700, torch.float32)).astype(np.float64)
    ref = oracle.omega(3, 9, 700).T
    assert np.max(np.abs(Ot - ref) / np.abs(ref)) <= 2.0 ** -24 * (1 + 1e-9)


# ----------------------------------------------------------------- sketch
# l <= 288 takes the tall-tile kernel (one row block, K split), larger l the
# 64 x 64 tiled kernel
# (eight waves from l > 112 on: odd tile counts leave a zero tile, ragged
# column blocks and K chunks)
@pytest.mark.parametrize("m,n,l", [(1000, 800, 30), (1000, 333, 30), (8192, 200, 20), (130, 70, 65),
                                   (3000, 130, 129), (5000, 517, 150), (2000, 300, 288),
                                   (16384, 2048, 272), (4096, 700, 300), (6000, 700, 544), (5000, 700, 600),
                                   (3000, 1100, 1000)])
def test_sketch_fp64(ff, m, n, l):
    announce(f"sketch fp64 m={m} n={n} l={l}")
    A = synth.random_matrix(m, n, seed=m + n)
    B, an = ff.sketch(dev_f(A), 11, l)
    Om = oracle.omega(11, l, m)
    Bref = oracle.sketch(Om, A)
    bound = 4 * m * EPS * (np.abs(Om) @ np.abs(A))
    assert np.all(np.abs(host(B) - Bref) <= bound)
    assert np.max(np.abs(host(an) - np.sum(A * A, axis=0)) / np.sum(A * A, axis=0)) < 4 * m * EPS


@pytest.mark.parametrize("l", [40, 136, 544])
def test_sketch_fp32(ff, l):
    import torch
    n = max(300, l + 100)
    announce(f"sketch fp32 m=2000 n={n} l={l}")
    A = synth.random_matrix(2000, n, seed=5).astype(np.float32)
    B, an = ff.sketch(dev_f(A, torch.float32), 4, l)
    Om32 = oracle.omega(4, l, 2000).astype(np.float32).astype(np.float64)
    A64 = A.astype(np.float64)
    Bref = Om32 @ A64
    bound = 4 * 2000 * 2.0 ** -24 * (np.abs(Om32) @ np.abs(A64))
    assert np.all(np.abs(host(B) - Bref) <= bound)
    assert np.max(np.abs(host(an) - np.sum(A64 * A64, axis=0)) / np.sum(A64 * A64, axis=0)) < 1e-12


# Mixed form: B = bf16(Omega) bf16(A) with FP32 sums.  The oracle's bf16
# sketch is the FP64 sum of the same exact products, so the difference is the
# FP32 summation error, at most m 2^-24 sum_t |bf16(Omega_it)| |bf16(A_tj)|.
# m a multiple of 64 takes the wide-column kernel (row groups of up to 17
# tiles: l = 544 two, l = 700 three, l = 300 two with a partial last tile;
# l <= 128 one group of up to eight), other m the narrow kernel (l = 544 one
# row group, l = 700 two); ragged n.
@pytest.mark.parametrize("m,n,l", [(1000, 800, 30), (3001, 517, 136), (8192, 1100, 544), (2000, 900, 700),
                                   (40000, 64, 16), (4096, 1000, 300), (2048, 700, 700), (16384, 300, 64)])
def test_sketch_mixed(ff, m, n, l):
    import torch
    announce(f"sketch mixed m={m} n={n} l={l}")
    A = synth.random_matrix(m, n, seed=m + 3 * n).astype(np.float32)
    B, an = ff.sketch(dev_f(A, torch.float32), 6, l, mixed=True)
    A64 = A.astype(np.float64)
    Om = oracle.omega(6, l, m)
    Bref = oracle.sketch(Om, A64, "bf16")
    bound = m * 2.0 ** -24 * (np.abs(oracle.round_bf16(Om)) @ np.abs(oracle.round_bf16(A64)))
    err = np.abs(host(B).astype(np.float64) - Bref)
    print(f"[gpu-case] max err / bound {np.max(err / bound):.3e}", flush=True)
    assert np.all(err <= bound)
    an_ref = np.sum(A64 * A64, axis=0)
    assert np.max(np.abs(host(an) - an_ref) / an_ref) < 1e-12


# Split-BF16 projection: each product q a is replaced by
# qhi ahi + qhi alo + qlo ahi, whose error is at most about 3 2^-18 |q a|
# (the dropped qlo alo and the two representation remainders), plus the FP32
# summation error m 2^-24 of the sum of |q a|.
@pytest.mark.parametrize("m,n,c", [(1000, 800, 30), (4100, 1100, 200), (8192, 700, 544), (2049, 300, 17),
                                   (6400, 1500, 300), (8192, 300, 100), (16384, 2000, 1000)])
def test_project_mixed(ff, m, n, c):
    import torch
    announce(f"project mixed m={m} n={n} c={c}")
    A = synth.random_matrix(m, n, seed=c + 1000).astype(np.float32)
    Qr, _ = oracle.householder_qr(synth.random_matrix(m, c, seed=c + 1001))
    Q32 = Qr.astype(np.float32)
    A64, Q64 = A.astype(np.float64), Q32.astype(np.float64)
    an = np.sum(A64 * A64, axis=0)
    W, g2 = ff.project(dev_f(Q32, torch.float32), dev_f(A, torch.float32), torch.from_numpy(an).cuda(), mixed=True)
    Wr = oracle.project(Q64, A64)
    bound = (3.0 * 2.0 ** -18 * 1.01 + m * 2.0 ** -24) * (np.abs(Q64.T) @ np.abs(A64))
    err = np.abs(host(W).astype(np.float64) - Wr)
    print(f"[gpu-case] max err / bound {np.max(err / bound):.3e}", flush=True)
    assert np.all(err <= bound)


# ------------------------------------------------------------------- QRCP
# register-resident kernel (l <= 288 and few enough columns) and the LDS /
# global-memory kernel (larger l or n) are both covered
@pytest.mark.parametrize("l,n,seed", [(30, 800, 1), (30, 1001, 2), (64, 5000, 3), (100, 60000, 4), (8, 8, 5),
                                      (1, 50, 6), (200, 4000, 7), (272, 8192, 8), (300, 2000, 9),
                                      (544, 16384, 10), (400, 3000, 11), (544, 20000, 12)])
def test_qrcp_pivots_fp64(ff, l, n, seed):
    announce(f"qrcp fp64 l={l} n={n} seed={seed}")
    B = synth.random_matrix(l, n, seed=seed)
    piv_ref, marg_ref, _ = oracle.qrcp_sketch(B, l)
    piv, marg = ff.qrcp(dev_f(B))
    piv = host(piv)
    marg = host(marg)
    # exact up to the first step whose margin is below the FP64 threshold
    bad = np.flatnonzero(marg_ref < 1e-12)
    upto = bad[0] if bad.size else l
    assert list(piv[:upto]) == list(piv_ref[:upto])
    assert np.max(np.abs(marg[:upto] - marg_ref[:upto])) < 1e-9


def test_qrcp_pivots_fp32(ff):
    import torch
    announce("qrcp fp32 l=40 n=3000")
    B = synth.random_matrix(40, 3000, seed=9).astype(np.float32)
    piv_ref, marg_ref, _ = oracle.qrcp_sketch(B.astype(np.float64), 40)
    piv, _ = ff.qrcp(dev_f(B, torch.float32))
    piv = host(piv)
    bad = np.flatnonzero(marg_ref < 1e-4)
    upto = bad[0] if bad.size else 40
    assert upto >= 10
    assert list(piv[:upto]) == list(piv_ref[:upto])


def test_qrcp_orthogonal_columns(ff):
    announce("qrcp orthogonal columns 40x40")
    A = synth.separated_columns_matrix(40, 40, seed=3, ratio=1.3)
    piv, _ = ff.qrcp(dev_f(A), 40)
    ref, _, _ = oracle.qrcp_sketch(A, 40)
    assert list(host(piv)) == list(ref)
    assert list(ref) == list(np.argsort(-np.linalg.norm(A, axis=0), kind="stable"))


# --------------------------------------------------------- Householder QR
# M goes through the blocked back substitution with two 256-row slots per
# column up to c = 512, three up to c = 592 (c = 520, 544), and through the
# column-per-wave kernel beyond (c = 600); from 32768 rows on the row blocks
# are 128 rows (256 workgroups), 40000 rows gives blocks of 157 rows with a
# short last one
@pytest.mark.parametrize("m,n,c,seed", [(1000, 800, 30, 1), (1000, 800, 37, 2), (300, 50, 5, 3),
                                        (5000, 400, 100, 4), (64, 64, 64, 5), (16384, 300, 17, 6),
                                        (1100, 600, 512, 8), (1300, 600, 520, 9), (20000, 600, 544, 10),
                                        (32768, 600, 544, 11), (40000, 300, 100, 12), (2000, 700, 600, 13)])
def test_panel_qr_fp64(ff, m, n, c, seed):
    import torch
    announce(f"panel_qr fp64 m={m} n={n} c={c}")
    A = synth.random_matrix(m, n, seed=seed)
    cols = np.random.default_rng(seed).permutation(n)[:c]
    Q, R = ff.panel_qr(dev_f(A), torch.from_numpy(cols).cuda())
    Qr, Rr = oracle.householder_qr(A[:, cols])
    Q, R = host(Q), host(R)
    assert np.max(np.abs(Q - Qr)) < 1e-11
    assert np.max(np.abs(R - Rr)) < 1e-12 * np.abs(Rr).max()
    assert np.linalg.norm(Q.T @ Q - np.eye(c)) < 1e-13
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) >= 0)


# Columns that are (nearly) dependent on earlier ones of their panel: the
# panel reflectors recovered from the panel's Gram matrix would lose most of
# such a column's remaining norm to cancellation, so the kernel takes those
# columns through the exact per-column reductions.  The leading columns are
# well conditioned and must match the oracle; the whole factorization must
# be orthogonal and reproduce A(:, cols) to rounding.
@pytest.mark.parametrize("m,c,bad", [(3000, 40, ((5, 4, 1e-9), (20, 19, 0.0), (33, None, 0.0))),
                                     (16384, 48, ((1, 0, 1e-7), (17, 3, 1e-12), (40, 39, 1e-5))),
                                     (32768, 40, ((3, 2, 1e-8), (18, None, 0.0), (35, 34, 1e-11)))])
def test_panel_qr_dependent_columns_fp64(ff, m, c, bad):
    import torch
    announce(f"panel_qr dependent columns fp64 m={m} c={c}")
    A = synth.random_matrix(m, c, seed=c)
    noise = synth.random_matrix(m, c, seed=c + 1)
    for j, k, eps in bad:
        A[:, j] = 0.0 if k is None else A[:, k] + eps * noise[:, j]
    cols = np.arange(c)
    Q, R = ff.panel_qr(dev_f(A), torch.from_numpy(cols).cuda())
    Q, R = host(Q), host(R)
    first = min(j for j, _, _ in bad)
    Qr, Rr = oracle.householder_qr(A)
    assert np.max(np.abs(Q[:, :first] - Qr[:, :first])) < 1e-11
    assert np.max(np.abs(R[:first, :] - Rr[:first, :])) < 1e-12 * np.abs(Rr).max()
    assert np.linalg.norm(Q.T @ Q - np.eye(c)) < 1e-13
    assert np.linalg.norm(A - Q @ R) < 1e-14 * np.linalg.norm(A)
    assert np.allclose(np.tril(R, -1), 0.0) and np.all(np.diag(R) >= 0)
    for j, k, eps in bad:
        if k is None:
            assert R[j, j] == 0.0
        else:
            assert R[j, j] <= 4 * eps * np.linalg.norm(noise[:, j]) + 1e-12 * np.abs(Rr).max()


def test_panel_qr_fp32(ff):
    import torch
    announce("panel_qr fp32 m=3000 c=50")
    A = synth.random_matrix(3000, 200, seed=7).astype(np.float32)
    cols = np.arange(0, 200, 4)[:50]
    Q, R = ff.panel_qr(dev_f(A, torch.float32), torch.from_numpy(cols).cuda())
    Qr, Rr = oracle.householder_qr(A[:, cols].astype(np.float64))
    Q = host(Q).astype(np.float64)
    assert np.max(np.abs(Q - Qr)) < 1e-5
    assert np.linalg.norm(Q.T @ Q - np.eye(50)) < 1e-5 * np.sqrt(50)


# -------------------------------------------------------------- projection
@pytest.mark.parametrize("m,n,c", [(1000, 800, 30), (2049, 513, 45), (4100, 1100, 200), (3000, 1000, 290)])
def test_project_fp64(ff, m, n, c):
    announce(f"project fp64 m={m} n={n} c={c}")
    A = synth.random_matrix(m, n, seed=c)
    Qr, _ = oracle.householder_qr(synth.random_matrix(m, c, seed=c + 1))
    an = np.sum(A * A, axis=0)
    import torch
    W, g2 = ff.project(dev_f(Qr), dev_f(A), torch.from_numpy(an).cuda())
    Wr = oracle.project(Qr, A)
    bound = 4 * m * EPS * (np.abs(Qr.T) @ np.abs(A))
    assert np.all(np.abs(host(W) - Wr) <= bound)
    gr = an - np.sum(Wr * Wr, axis=0)
    assert np.max(np.abs(host(g2) - gr) / an) < 1e-13


# ------------------------------------------------------------------- SRQR
@pytest.mark.parametrize("l,seed", [(12, 1), (30, 2), (100, 3), (272, 4)])
def test_srqr_rho_fp64(ff, l, seed):
    announce(f"srqr_rho fp64 l={l}")
    rng = np.random.default_rng(seed)
    R11 = np.triu(rng.standard_normal((l, l))) * 0.3 + np.diag(np.exp(-np.arange(l) / 40.0) + 0.5)
    a = rng.standard_normal(l) * 0.1
    alpha = 0.05
    import torch
    rho = host(ff.srqr_rho(dev_f(R11), torch.from_numpy(a).cuda(), alpha))
    ref = oracle.srqr_rho(R11, a, alpha)[:l]
    assert np.max(np.abs(rho - ref) / ref) < 1e-11


# --------------------------------------------------------------- flip-flop
@pytest.mark.parametrize("l,n,seed", [(30, 800, 1), (37, 500, 2), (5, 5, 3), (64, 3000, 4), (544, 4000, 5)])
def test_lq_fp64(ff, l, n, seed):
    import torch
    announce(f"lq fp64 l={l} n={n}")
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((l, n))
    R[:, :l] = np.triu(R[:, :l])
    perm = rng.permutation(n)
    Lg, Vg = ff.lq(dev_f(R), torch.from_numpy(perm).cuda())
    Lr, _, Vr = oracle.flip_flop_lq(R, perm)
    assert np.max(np.abs(host(Lg) - Lr)) < 1e-12 * np.abs(Lr).max()
    assert np.max(np.abs(host(Vg) - Vr)) < 1e-11


# --------------------------------------------------------------- small SVD
# l = 700 and 1000: the block pairs' rows are split over two and three
# workgroups (their partial Gram matrices exchanged every round); the
# reference is LAPACK's SVD on a well-conditioned factor (kappa ~ 1e2, where
# its singular values are accurate to a few u relative as well)
@pytest.mark.parametrize("l", [700, 1000])
def test_svd_small_row_split_fp64(ff, l):
    announce(f"svd_small fp64 l={l} (row-split block pairs)")
    rng = np.random.default_rng(l)
    M = np.tril(rng.standard_normal((l, l))) * 0.02 + np.diag(np.linspace(1.0, 0.01, l))
    sig = host(ff.svd_small(dev_f(M)))
    ref = np.linalg.svd(M, compute_uv=False)
    nrm = np.linalg.norm(M, axis=0)
    kappa_s = np.linalg.cond(M / nrm)
    rel_tol = 8.0 * l * EPS * kappa_s
    print(f"[gpu-case] kappa_s {kappa_s:.3e}, bound {rel_tol:.2e}, worst {np.max(np.abs(sig - ref) / ref):.2e}",
          flush=True)
    assert np.all(np.abs(sig - ref) <= rel_tol * ref)

# FP32 data: the iteration stops after a sweep whose rotations all had
# cosines <= 1e-4; the singular values then differ from the oracle's (Jacobi
# run until nothing rotates, on the same FP32 values, in FP64) by second-order
# terms.  Well-conditioned factors (kappa_s small), where relative
# differences are meaningful: "diag", a dominant decaying diagonal under a
# small random lower triangle, and "cluster", eight equal singular values
# then a decay, through the LQ of U diag(s) V^T (the shape of the flip-flop
# factor).  The FP32 forms' tolerance is 1e-4; the bound here is 1e-6.
@pytest.mark.parametrize("l,kind", [(272, "diag"), (544, "diag"), (544, "cluster"), (64, "cluster")])
def test_svd_small_fp32_stop(ff, l, kind):
    import torch
    announce(f"svd_small fp32 l={l} kind={kind}")
    rng = np.random.default_rng(l + 7)
    if kind == "diag":
        M = np.tril(rng.standard_normal((l, l))) * 0.02 + np.diag(np.linspace(1.0, 0.01, l))
    else:
        j = np.arange(1, l + 1)
        s = np.where(j <= 8, 1.0, 10.0 ** (-3.0 * (j - 8) / 1000.0))
        U, _ = np.linalg.qr(rng.standard_normal((l, l)))
        V, _ = np.linalg.qr(rng.standard_normal((2 * l, l)))
        X = (U * s) @ V.T
        M = np.linalg.qr(X.T, mode="r").T
    M32 = M.astype(np.float32)
    sig = host(ff.svd_small(dev_f(M32, torch.float32)))
    ref, _ = oracle.jacobi_svd(M32.astype(np.float64))
    nrm = np.linalg.norm(M32.astype(np.float64), axis=0)
    kappa_s = np.linalg.cond(M32 / nrm)
    worst = np.max(np.abs(sig - ref) / ref)
    print(f"[gpu-case] kappa_s {kappa_s:.2e}, worst relative difference {worst:.2e}", flush=True)
    assert worst < 1e-6


@pytest.mark.parametrize("l,kind", [(30, "qlp"), (2, "gauss"), (31, "gauss"), (100, "graded"), (272, "qlp"),
                                    (16, "rankdef"), (544, "qlp")])
def test_svd_small_fp64(ff, l, kind):
    announce(f"svd_small fp64 l={l} kind={kind}")
    rng = np.random.default_rng(l)
    if kind == "qlp":
        M = np.tril(rng.standard_normal((l, l))) * 0.05 + np.diag(np.exp(-np.arange(l) / 20.0))
    elif kind == "graded":
        M = np.tril(rng.standard_normal((l, l))) * (0.9 ** np.arange(l))
    elif kind == "rankdef":
        M = rng.standard_normal((l, 4)) @ rng.standard_normal((4, l))
    else:
        M = rng.standard_normal((l, l))
    sig = host(ff.svd_small(dev_f(M)))
    ref, _ = oracle.jacobi_svd(M)
    # Both sides are one-sided Jacobi, whose computed singular values carry a
    # relative error of at most about l u kappa_s, kappa_s the condition
    # number of M with its columns scaled to unit norm (Demmel and Veselic):
    # each sigma_j is compared to that bound, and in absolute terms to
    # 8 l u sigma_1, the order of the backward error of l sweeps' worth of
    # plane rotations on each side (u = 2^-53).
    nrm = np.linalg.norm(M, axis=0)
    cols = nrm > 0
    kappa_s = np.linalg.cond(M[:, cols] / nrm[cols]) if np.all(cols) else np.inf
    assert np.max(np.abs(sig - ref)) < 4.0 * l * EPS * ref[0]
    if np.isfinite(kappa_s):
        rel_tol = 8.0 * l * EPS * kappa_s
        print(f"[gpu-case] kappa_s {kappa_s:.3e}, relative bound {rel_tol:.2e}, worst "
              f"{np.max(np.abs(sig - ref) / ref):.2e}", flush=True)
        assert np.all(np.abs(sig - ref) <= rel_tol * ref)
