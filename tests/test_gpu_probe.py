"""GPU parity of Algorithm 4's randomized g2 estimate against the oracle on
the same inputs and the same Philox probe streams:

* ffsrqr_srqr_probe: est[0:l+1] within the FP64 bound of the two sides'
  triangular solves (both compute in FP64 from the same, possibly
  FP32-rounded, R11 and a), across l = 1 .. 545 and d = 1 .. 64;
* ffsrqr_factor with opts.g2_probe: the same probe count, swaps, identity
  rotations, pivots and final estimate as the oracle where every decision
  of the oracle's trajectory is clear of its threshold (g2 against g, the
  argmax against the runner-up), the final factors within the form's bound;
* the 8192 x 4096, l = 544 workload in the mixed form (the headline
  workload's l and spectrum at a quarter of its rows and columns): with the
  probe the solve runs through the same kernels, and when neither run swaps
  the results are bit-identical to the exact test's.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, dev_f, host

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


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


def slow_decay(m, n, seed, decay):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * decay ** np.arange(n)) @ V.T


def rtilde(R11, a, alpha):
    l = R11.shape[0]
    Rt = np.zeros((l + 1, l + 1))
    Rt[:l, :l], Rt[:l, l], Rt[l, l] = R11, a, alpha
    return Rt


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("l,d", [(1, 1), (37, 8), (100, 64), (545, 10)])
def test_probe_step_matches_oracle(ff, prec, l, d):
    import torch
    announce(f"srqr_probe l={l} d={d} {prec}")
    rng = np.random.default_rng(l * 100 + d)
    _, R11 = np.linalg.qr(rng.standard_normal((2 * l + 2, l)))
    a = 0.5 * rng.standard_normal(l)
    alpha = 0.7
    dt = torch.float64 if prec == "fp64" else torch.float32
    Rd, ad = dev_f(R11, dt), dev_f(a[:, None], dt)
    # the oracle reads the exact values the GPU reads
    R11h, ah = host(Rd).astype(np.float64), host(ad).astype(np.float64)[:, 0]
    seed, q = 77, 3
    est = host(ff.srqr_probe(Rd, ad, alpha, d, seed, q))
    ref = oracle.g2_probe_estimate(R11h, ah, alpha, oracle.probe_omega(seed, q, d, l))
    # both sides solve in FP64: the error is about cond(R-tilde) l u of the
    # largest estimate (the probe's Box-Muller differs by a few ulps at most)
    tol = 10.0 * np.linalg.cond(rtilde(R11h, ah, alpha)) * l * U64 + 1e-14
    err = np.max(np.abs(est - ref)) / np.max(ref)
    print(f"[gpu-case] probe est: max err / max est {err:.3e} (tol {tol:.3e})", flush=True)
    assert est.shape == (l + 1,) and err <= tol
    # and the exact rho is what the estimate's square averages to: a fresh
    # stream gives a different estimate of the same quantity
    est2 = host(ff.srqr_probe(Rd, ad, alpha, d, seed, q + 1))
    assert not np.array_equal(est, est2)


def trajectory_is_clear(A, ref, d, seed, g, rel):
    """Every SRQR test of the oracle's trajectory decided clearly: g2 away
    from g and the argmax ahead of the runner-up by more than rel."""
    l = ref.l
    for q, (S, g2, j, alpha) in enumerate(ref.history, start=1):
        if abs(g2 - g) <= rel * g:
            return False
        perm, Q1, R11, R, W = oracle.factor_leading_set(A, S)
        est = oracle.g2_probe_estimate(R11, W[:, j], alpha, oracle.probe_omega(seed, q, d, l))
        top = np.sort(est)[-2:]
        if top[1] - top[0] <= rel * top[1]:
            return False
    return True


def run_pair(ff, A, k, p, seed, g, d, max_swaps, dtype=None, mixed=False):
    import torch
    fp32 = dtype is not None
    Ad = dev_f(A, dtype)
    Ah = host(Ad).astype(np.float64)
    out = ff.factor(Ad, k, p, seed, g=g, max_swaps=max_swaps, mixed=mixed, g2_probe=d)
    torch.cuda.synchronize()
    ref = oracle.ffsrqr(Ah, k, p, seed, g=g, max_swaps=max_swaps, g2_probe=d,
                        storage="fp32" if fp32 else "fp64", sketch_mode="bf16" if mixed else "fp64")
    return Ah, out, ref


@pytest.mark.parametrize("case", ["kahan", "identity_rotations"])
def test_probe_factor_matches_oracle_fp64(ff, case):
    if case == "kahan":
        announce("factor kahan 90x80 k=40 p=0 g2_probe=8 fp64")
        A = np.vstack([kahan(80), np.zeros((10, 80))])
        k, p, seed, g, d, cap = 40, 0, 0, 2.0, 8, 320
    else:
        announce("factor 60x40 k=6 p=2 g=1.05 g2_probe=1 fp64 (identity rotations)")
        A = synth.spectrum_matrix(60, 40, 0.9 ** np.arange(40), seed=3, noise=1e-10)
        k, p, seed, g, d, cap = 6, 2, 2, 1.05, 1, 30
    Ah, out, ref = run_pair(ff, A, k, p, seed, g, d, cap)
    info = out.info
    clear = trajectory_is_clear(Ah, ref, d, seed, g, 1e-8) and ref.margins.min() > 1e-10
    idle = sum(1 for i in range(1, len(ref.history)) if ref.history[i][0] == ref.history[i - 1][0])
    print(f"[gpu-case] oracle: tests {ref.probes}, swaps {ref.swaps}, identity rotations {idle}, "
          f"g2 {ref.g2:.6f}; gpu: tests {info['probes']}, swaps {info['swaps']}, g2 {info['g2']:.6f}; "
          f"clear {clear}", flush=True)
    assert clear, "the chosen case must decide clearly"
    if case == "identity_rotations":
        assert idle >= 1
    assert info["probes"] == ref.probes and info["swaps"] == ref.swaps and info["flags"] == ref.flags
    assert list(host(out.perm)) == list(ref.perm)
    assert abs(info["g2"] - ref.g2) <= 1e-8 * ref.g2
    sig = host(out.sigma)
    assert np.all(np.abs(sig - ref.sigma) <= 1e-10 * ref.sigma + 1e-14 * ref.sigma[0])


@pytest.mark.parametrize("form", ["fp64", "fp32", "mixed"])
def test_probe_forced_swaps(ff, form):
    """g just above 1: the estimate exceeds it at every test, so the loop
    runs to its cap (6 rotations, 7 probes) on both sides; where each
    decision is clear the same swaps and pivots follow."""
    import torch
    announce(f"factor forced swaps with g2_probe=8 {form} 600x300 k=30 p=6")
    A = slow_decay(600, 300, 11, 0.97)
    dt = None if form == "fp64" else torch.float32
    Ah, out, ref = run_pair(ff, A, 30, 6, 0, 1.0 + 1e-6, 8, 6, dtype=dt, mixed=form == "mixed")
    info = out.info
    assert ref.probes == 7 and ref.flags & oracle.FLAG_SWAPCAP
    assert info["probes"] == 7 and info["flags"] & oracle.FLAG_SWAPCAP
    rel = 1e-8 if form == "fp64" else 1e-3
    clear = trajectory_is_clear(Ah, ref, 8, 0, 1.0 + 1e-6, rel) and ref.margins.min() > rel
    print(f"[gpu-case] swaps oracle {ref.swaps} gpu {info['swaps']}; clear {clear}", flush=True)
    if clear:
        assert info["swaps"] == ref.swaps
        assert list(host(out.perm)) == list(ref.perm)
        tol = 1e-10 if form == "fp64" else 1e-4
        sig = host(out.sigma)
        floor = (1e-14 if form == "fp64" else 1e-5) * ref.sigma[0]
        assert np.all(np.abs(sig - ref.sigma) <= tol * ref.sigma + floor)


def test_probe_l544_mixed(ff):
    """The 8192 x 4096, l = 544 workload in the mixed form with a 10-row
    probe: every solve runs the same kernels; when neither the exact nor the
    probed test swaps, the two results are bit-identical (only the SRQR test
    differs); the SRQR step's device time is reported for both."""
    import torch
    w = synth.WORKLOADS["large_q"]
    announce(f"generate large_q {w.m}x{w.n}")
    A = dev_f(synth.make_workload("large_q"), torch.float32)
    res = {}
    for d in (0, 10):
        announce(f"factor large mixed g2_probe={d}")
        ff.profile_enable(True)
        try:
            out = ff.factor(A, w.k, w.p, w.seed, mixed=True, g2_probe=d)
            torch.cuda.synchronize()
            prof = ff.profile_read()
        finally:
            ff.profile_enable(False)
        res[d] = out
        ms, cnt = prof["srqr"]
        print(f"[gpu-case] g2_probe={d}: swaps {out.info['swaps']}, probes {out.info['probes']}, "
              f"g2 {out.info['g2']:.4f}, SRQR step {ms:.3f} ms over {cnt} launches", flush=True)
    ex, pr = res[0].info, res[10].info
    assert ex["probes"] == 0 and pr["probes"] >= 1
    assert pr["g2"] <= 2.0 or pr["flags"] & oracle.FLAG_SWAPCAP
    if ex["swaps"] == 0 and pr["swaps"] == 0:
        assert torch.equal(res[0].perm, res[10].perm)
        assert torch.equal(res[0].sigma, res[10].sigma)
        assert torch.equal(res[0].L, res[10].L)
    del A
