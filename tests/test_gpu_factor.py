"""End-to-end GPU parity of ffsrqr_factor against the oracle: pivots exact
(where the QRCP margins separate them), sigma_j, the residual
||A - Q L V^T||_F, the factors and the SRQR outcome within the FP64 bound
(1e-10 relative), or 1e-4 for the FP32 form; plus the edge cases."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev_f, host
from oracle import diagnostics as dg

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_1803_01982_amd as ff
    ff.load()
    return ff


def kahan(n, c=0.285, pert=1e-10):
    s = np.sqrt(1 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.triu(-c * np.ones((n, n)), 1) + np.eye(n))
    return K @ np.diag(1 - pert * np.arange(n))


def rtilde_cond(ref):
    """Condition number of R-tilde = [[R11, R(:, j*)], [0, alpha]] (the
    oracle's): the relative error of g2 grows with it."""
    l = ref.l
    jpos = int(np.flatnonzero(ref.perm == ref.jstar)[0])
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l] = ref.R[:, :l]
    Rt[:l, l] = ref.R[:, jpos]
    Rt[l, l] = ref.alpha
    return float(np.linalg.cond(Rt))


def compare(ff, A, k, p, seed, g=2.0, max_swaps=None, dtype=None, tol=FP64_TOL, margin_floor=1e-12,
            mixed=False):
    """GPU vs oracle on the same bytes.  FP64: pivots, swaps and j* exact where
    the oracle's QRCP and j* margins separate them, g2 within 1e-8.  FP32:
    the same comparisons under FP32 error bounds derived from the condition
    of the quantity compared (stated inline); the rank rule is the FP32
    storage one on both sides."""
    import torch
    fp32 = tol != FP64_TOL
    Ad = dev_f(A, dtype)
    Ahost = host(Ad).astype(np.float64)  # the exact bytes the GPU reads
    ms = -1 if max_swaps is None else max_swaps
    out = ff.factor(Ad, k, p, seed, g=g, max_swaps=ms, mixed=mixed)
    ref = oracle.ffsrqr(Ahost, k, p, seed, g=g, max_swaps=max_swaps, storage="fp32" if fp32 else "fp64",
                        sketch_mode="bf16" if mixed else "fp64")
    l = ref.l
    info = out.info
    u = 2.0 ** -24 if fp32 else 2.0 ** -53
    assert info["l"] == l
    assert info["flags"] == ref.flags, (info["flags"], ref.flags)
    perm = host(out.perm)
    deficient = bool(ref.flags & oracle.FLAG_RANK_DEFICIENT)
    # g2 error bound: a relative perturbation e of R-tilde moves g2 by about
    # cond(R-tilde) e relatively; e ~ sqrt(l) u for FP32-rounded factors
    g2_tol = 1e-8 if not fp32 else 10.0 * np.sqrt(l) * u * (rtilde_cond(ref) if 0 <= ref.jstar else 1.0)
    # the swap decisions are robust when every SRQR test of the oracle's
    # trajectory had g2 clearly away from g
    decided = all(abs(h[1] - g) > 2.0 * g2_tol * g for h in ref.history)
    jm_floor = 1e-3 if fp32 else 1e-10
    if deficient:
        # pivots past the numerical rank pick among noise-level columns
        r = ref.numerical_rank
        assert info["numerical_rank"] == r
        assert list(perm[:r]) == list(ref.perm[:r])
    elif ref.margins.min() >= margin_floor and decided:
        assert list(perm) == list(ref.perm)
        assert info["swaps"] == ref.swaps
        if ref.jstar_margin >= jm_floor:
            assert info["jstar"] == ref.jstar
            assert info["jstar_margin"] > 0.0
        assert abs(info["alpha"] - ref.alpha) <= (1e-8 if not fp32 else 1e-3) * ref.alpha
    # else: near-tie in QRCP or a g2 at the threshold; only set-level
    # results are compared
    Q, L, V = host(out.Q).astype(np.float64), host(out.L).astype(np.float64), host(out.V).astype(np.float64)
    sig = host(out.sigma)
    # backward-stable arithmetic: relative tol plus a floor at the rounding
    # level of sigma_1 (1e-14 for FP64, 1e-5 for FP32 storage)
    floor = (1e-14 if not fp32 else 1e-5) * ref.sigma[0]
    err = np.abs(sig - ref.sigma)
    print(f"[gpu-case] sigma: max rel err {np.max(err / ref.sigma):.3e}, "
          f"max abs err / sigma_1 {np.max(err) / ref.sigma[0]:.3e}", flush=True)
    assert np.all(err <= tol * ref.sigma + floor)
    orth = 1e-13 if not fp32 else 1e-5 * np.sqrt(l)
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < orth
    assert np.linalg.norm(V.T @ V - np.eye(l)) < orth
    assert np.allclose(np.triu(L, 1), 0.0) and np.all(np.diag(L) >= 0)
    res = dg.residual_fro(Ahost, Q, L, V)
    res_ref = dg.residual_fro(Ahost, ref.Q, ref.L, ref.V)
    nA = np.linalg.norm(Ahost)
    # absolute floor: the rounding of the returned factors themselves, about
    # u ||A||_F per factor (FP32 factors: 4 sqrt(l) 2^-24 ||A||_F)
    res_floor = (1e-13 if not fp32 else 4.0 * np.sqrt(l) * 2.0 ** -24) * nA
    assert abs(res - res_ref) <= tol * max(res_ref, 1e-3 * nA) + res_floor
    if ref.margins.min() >= margin_floor and not deficient and decided and ref.jstar >= 0:
        assert abs(info["g2"] - ref.g2) <= g2_tol * ref.g2, (info["g2"], ref.g2, g2_tol)
    if ref.margins.min() >= margin_floor and not deficient and decided:
        # L entries: the unpivoted QR of R^T moves them by about
        # cond(L) sqrt(l) u max|L| (FP32), far less for FP64
        lt = 1e-7 if not fp32 else 20.0 * np.linalg.cond(ref.L) * np.sqrt(l) * u
        assert np.max(np.abs(L - ref.L)) < lt * np.abs(ref.L).max()
    return out, ref


def test_small_fp64_workload(ff):
    announce("factor small_fp64 1000x800 k=20 p=10")
    w = synth.WORKLOADS["small_fp64"]
    A = synth.make_workload("small_fp64")
    out, ref = compare(ff, A, w.k, w.p, w.seed)
    assert ref.margins.min() > 1e-12
    assert out.info["min_margin"] > 1e-12


def test_small_fp32(ff):
    import torch
    announce("factor small fp32 1000x800 k=20 p=10")
    A = synth.make_workload("small_fp64").astype(np.float32)
    compare(ff, A, 20, 10, 0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)


def test_kahan_swaps(ff):
    announce("factor kahan 90x80 k=40 p=0 (swaps)")
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    out, ref = compare(ff, A, 40, 0, 0)
    assert ref.swaps >= 1 and out.info["swaps"] == ref.swaps


def test_tight_g_swaps(ff):
    announce("factor decay 120x90 g=1.1 (swaps)")
    A = synth.spectrum_matrix(120, 90, 0.9 ** np.arange(90), seed=41, noise=1e-10)
    out, ref = compare(ff, A, 10, 2, 0, g=1.1)
    assert ref.swaps >= 1


def test_swap_cap(ff):
    announce("factor kahan max_swaps=0 (SWAPCAP)")
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    out, ref = compare(ff, A, 40, 0, 0, max_swaps=0)
    assert out.info["flags"] & 2


def test_kahan_swaps_fp32(ff):
    import torch
    announce("factor kahan fp32 90x80 k=40 p=0 (swaps)")
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    out, ref = compare(ff, A, 40, 0, 0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)
    assert ref.swaps >= 1 and out.info["swaps"] == ref.swaps


def test_tight_g_swaps_fp32(ff):
    import torch
    announce("factor decay fp32 120x90 g=1.1 (swaps)")
    A = synth.spectrum_matrix(120, 90, 0.9 ** np.arange(90), seed=41, noise=1e-10)
    out, ref = compare(ff, A, 10, 2, 0, g=1.1, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)
    assert ref.swaps >= 1 and out.info["swaps"] == ref.swaps


def test_swap_cap_fp32(ff):
    import torch
    announce("factor kahan fp32 max_swaps=0 (SWAPCAP)")
    A = np.vstack([kahan(80), np.zeros((10, 80))])
    out, ref = compare(ff, A, 40, 0, 0, max_swaps=0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)
    assert out.info["flags"] & 2


def slow_decay(m, n, seed, decay):
    """U diag(decay^j) V^T with U, V from the QR of seeded Gaussians: a
    spectrum flat enough that with g just above 1 nearly every SRQR test
    asks for a swap."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * decay ** np.arange(n)) @ V.T


@pytest.mark.parametrize("form", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("case", [(600, 300, 30, 6, 0.97, 6), (400, 200, 40, 0, 0.99, 6), (500, 260, 20, 4, 0.9, 6)])
def test_forced_swaps(ff, form, case):
    """Several swaps in a row, each an in-place update of Q, R11 and W
    (rotations, a new column, a pass over A), against the oracle, which
    factors every new leading set from scratch: the same swaps and
    pivots, and the final factors within the form's bound."""
    import torch
    m, n, k, p, decay, cap = case
    announce(f"factor forced swaps {form} {m}x{n} k={k} p={p} decay={decay} max_swaps={cap}")
    A = slow_decay(m, n, 11, decay)
    if form == "fp64":
        out, ref = compare(ff, A, k, p, 0, g=1.0 + 1e-6, max_swaps=cap)
    else:
        out, ref = compare(ff, A, k, p, 0, g=1.0 + 1e-6, max_swaps=cap, dtype=torch.float32, tol=FP32_TOL,
                           margin_floor=1e-5, mixed=form == "mixed")
    print(f"[gpu-case] swaps oracle {ref.swaps} gpu {out.info['swaps']}", flush=True)
    assert ref.swaps >= 2
    assert out.info["swaps"] == ref.swaps


def test_swap_update_matches_fresh_qr_mid(ff):
    """At the mid workload's size (16384 x 8192, l = 272): two forced swaps;
    the updated Q must equal the Householder QR of the final leading set
    A(:, perm[:l]) computed from scratch (the thin QR with a positive
    diagonal is unique; the difference is bounded by the conditioning of
    A(:, S) times the rounding of either side), and the per-swap device time
    is reported."""
    import torch
    w = synth.WORKLOADS["mid"]
    announce("factor mid fp64 with two forced swaps vs a fresh QR of the final set")
    A = dev_f(synth.make_workload("mid"))
    ff.profile_enable(True)
    try:
        out = ff.factor(A, w.k, w.p, w.seed, g=1.0 + 1e-9, max_swaps=2)
        torch.cuda.synchronize()
        prof = ff.profile_read()
    finally:
        ff.profile_enable(False)
    info = out.info
    assert info["swaps"] == 2 and info["flags"] & 2
    ms, cnt = prof["swap"]
    assert cnt == 2
    print(f"[gpu-case] swap update: {1000.0 * ms / cnt:.1f} us per swap "
          f"(panel {prof['panel'][0]:.3f} ms, projection {prof['project'][0]:.3f} ms once)", flush=True)
    l = info["l"]
    cols = out.perm[:l].clone()
    Qf, Rf = ff.panel_qr(A, cols)
    Qu = host(out.Q)
    Qfh = host(Qf)
    S = host(A)[:, host(cols)]
    kappa = np.linalg.cond(S)
    d = np.abs(Qu - Qfh).max()
    print(f"[gpu-case] cond(A(:, S)) {kappa:.3e}, max |Q_update - Q_fresh| {d:.3e}", flush=True)
    assert d <= 1e-13 * kappa * np.sqrt(l)
    assert np.linalg.norm(Qu.T @ Qu - np.eye(l)) < 1e-12


# Mixed form against the oracle in its bf16 sketch mode on the same FP32
# bytes: the sample matrices differ only by the FP32 summation of the GPU
# (relative about sqrt(m) 2^-24), so pivots are compared where the QRCP
# margins exceed 1e-4; the projection's split-BF16 error (about 2^-16 per
# product) stays inside the FP32 forms' 1e-4 tolerance for sigma.
def test_small_mixed(ff):
    import torch
    announce("factor small mixed 1000x800 k=20 p=10")
    A = synth.make_workload("small_fp64").astype(np.float32)
    compare(ff, A, 20, 10, 0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-4, mixed=True)


@pytest.mark.parametrize("m,n,k,p", [(3000, 2000, 100, 10), (2050, 4100, 250, 22), (600, 500, 40, 0)])
def test_shapes_mixed(ff, m, n, k, p):
    import torch
    announce(f"factor mixed m={m} n={n} k={k} p={p}")
    r = min(m, n)
    A = synth.spectrum_matrix(m, n, np.exp(-np.arange(r) / 30.0), seed=m + n, noise=1e-6).astype(np.float32)
    compare(ff, A, k, p, 1, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-4, mixed=True)


def _integer_low_rank(m, n, r, seed):
    rng = np.random.default_rng(seed)
    X = rng.integers(-2, 3, size=(m, r)).astype(np.float64)
    Y = rng.integers(-2, 3, size=(n, r)).astype(np.float64)
    return np.asfortranarray(X @ Y.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rank_deficient_integer_columns(ff, prec):
    """Exactly dependent columns (integer X Y^T of rank 20, identical in both
    storages), l = 30 > 16: RANK_DEFICIENT, the exact rank and no swaps."""
    import torch
    announce(f"factor integer rank 20 of 400x300 l=30 {prec}")
    A = _integer_low_rank(400, 300, 20, seed=5)
    if prec == "fp64":
        out, ref = compare(ff, A, 25, 5, 0)
    else:
        out, ref = compare(ff, A, 25, 5, 0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)
    assert out.info["flags"] & 1 and out.info["numerical_rank"] == 20
    assert out.info["swaps"] == 0


# (1500, 1200, 290, 10): l = 300 > 288 takes the general kernels (LDS QRCP,
# 64 x 64 GEMM tiles); (20000, 3000, 100, 8): row blocks of 256 rows in the
# panel QR and the register QRCP at l = 108
@pytest.mark.parametrize("m,n,k,p", [(300, 200, 150, 50), (200, 300, 10, 5), (50, 400, 7, 3), (400, 33, 5, 2),
                                     (70, 70, 1, 0), (64, 1, 1, 0), (1, 64, 1, 0), (257, 129, 16, 16),
                                     (1500, 1200, 290, 10), (20000, 3000, 100, 8)])
def test_shapes(ff, m, n, k, p):
    announce(f"factor shape m={m} n={n} k={k} p={p}")
    r = min(m, n)
    A = synth.spectrum_matrix(m, n, np.exp(-np.arange(r) / 7.0), seed=m * 7 + n, noise=1e-9)
    compare(ff, A, k, p, 3)


def test_full_rank(ff):
    announce("factor full rank 80x50 l=50")
    A = synth.spectrum_matrix(80, 50, np.logspace(0, -6, 50), seed=11)
    out, ref = compare(ff, A, 40, 10, 3)
    Q, L, V = host(out.Q), host(out.L), host(out.V)
    assert np.linalg.norm(A - Q @ L @ V.T) < 1e-13 * np.linalg.norm(A)


def test_clamped(ff):
    announce("factor clamped 30x20 k=18 p=10")
    A = synth.random_matrix(30, 20, seed=14)
    out, ref = compare(ff, A, 18, 10, 0)
    assert out.info["flags"] & 8


def test_rank_deficient(ff):
    announce("factor rank deficient 60x40 rank 3")
    A = synth.spectrum_matrix(60, 40, np.array([5.0, 3.0, 2.0]), seed=13)
    out, ref = compare(ff, A, 5, 2, 0)
    assert out.info["flags"] & 1 and out.info["numerical_rank"] == 3


def test_nonfinite(ff):
    announce("factor non-finite 30x20")
    A = synth.random_matrix(30, 20, seed=15)
    A[3, 4] = np.nan
    out = ff.factor(dev_f(A), 5, 2, 0)
    assert out.info["flags"] & 4
    assert np.all(np.isnan(host(out.sigma)))


def test_repeat_is_deterministic(ff):
    announce("factor determinism small_fp64 x2")
    A = dev_f(synth.make_workload("small_fp64"))
    a = ff.factor(A, 20, 10, 0)
    b = ff.factor(A, 20, 10, 0)
    assert np.array_equal(host(a.perm), host(b.perm))
    assert np.array_equal(host(a.sigma), host(b.sigma))
    assert np.array_equal(host(a.Q), host(b.Q))


def test_profiled_solve_matches_unprofiled(ff):
    """Per-step timing (events on the solve's stream and on the side stream
    that runs the Jacobi step concurrently with the forming of V) leaves the
    results unchanged and accounts for every step once per solve."""
    import torch
    announce("factor small_fp64 with step profiling")
    A = dev_f(synth.make_workload("small_fp64"))
    ref = ff.factor(A, 20, 10, 0)
    ff.profile_enable(True)
    try:
        out = ff.factor(A, 20, 10, 0)
        torch.cuda.synchronize()
        prof = ff.profile_read()
    finally:
        ff.profile_enable(False)
    assert np.array_equal(host(out.sigma), host(ref.sigma))
    assert np.array_equal(host(out.V), host(ref.V))
    for step in ("sketch", "qrcp", "panel", "project", "lq", "svd"):
        ms, launches = prof[step]
        assert launches == 1 + out.info["swaps"] and ms > 0.0, (step, prof[step])
    # a later unprofiled call still works (no stale error left behind)
    again = ff.factor(A, 20, 10, 0)
    assert np.array_equal(host(again.sigma), host(ref.sigma))
