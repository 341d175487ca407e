"""Parity at l = 544: the 32768 x 16384 workload (sigma_j = 1 for j <= 8,
then 10^(-3 (j - 8) / 1000) up to r = 1024, plus 1e-5 noise; k = 512,
p = 32) and its quarter-size twin (8192 x 4096, same spectrum and k, p).

The twin is compared with the whole oracle output (pivots, swaps, j*, g2,
sigma, residual, orthogonality).  At full size the oracle's whole solve
takes too long for a test, so the full-size GPU solve (the benchmark's
launch configuration) is checked on what the oracle computes there in
seconds, the sketch and its QRCP pivots (rows a1 and a2), and on properties
that hold at any size: orthonormal Q and V, Pythagoras for the residual
(||A - Q L V^T||_F^2 = ||A||_F^2 - ||L||_F^2) and interlacing of sigma(L)
with the prescribed spectrum."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, host
from oracle import diagnostics as dg

pytestmark = pytest.mark.gpu


def _dev(A, dtype):
    import torch
    import paper_1803_01982_amd as ff
    return ff.fortran(torch.from_numpy(A).to(dtype).cuda())


@pytest.fixture(scope="module")
def large_q():
    return synth.WORKLOADS["large_q"], synth.make_workload("large_q")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_large_q(large_q, prec):
    import torch
    import paper_1803_01982_amd as ff
    w, A = large_q
    dtype = torch.float64 if prec == "fp64" else torch.float32
    Ad = _dev(A, dtype)
    Ah = Ad.cpu().numpy().astype(np.float64)
    announce(f"factor large_q {w.m}x{w.n} l={w.l} {prec}")
    out = ff.factor(Ad, w.k, w.p, w.seed, mixed=prec == "mixed")
    torch.cuda.synchronize()
    announce("oracle large_q")
    ref = oracle.ffsrqr(Ah, w.k, w.p, w.seed, storage="fp64" if prec == "fp64" else "fp32",
                        sketch_mode="bf16" if prec == "mixed" else "fp64")
    fp32 = prec != "fp64"
    tol, floor, mfloor = (1e-10, 1e-14, 1e-12) if not fp32 else (1e-4, 1e-5, 1e-5 if prec == "fp32" else 1e-4)
    perm, sig = host(out.perm), host(out.sigma)
    assert out.info["l"] == ref.l == 544
    assert out.info["flags"] == ref.flags
    Q, L, V = (host(t).astype(np.float64) for t in (out.Q, out.L, out.V))
    l = ref.l
    orth = 1e-13 if not fp32 else 1e-5 * np.sqrt(l)
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < orth
    assert np.linalg.norm(V.T @ V - np.eye(l)) < orth
    res = dg.residual_fro(Ah, Q, L, V)
    res_ref = dg.residual_fro(Ah, ref.Q, ref.L, ref.V)
    err = np.abs(sig - ref.sigma)
    print(f"[gpu-case] sigma vs oracle: max rel err {np.max(err / ref.sigma):.3e}, j <= k "
          f"{np.max(err[:w.k] / ref.sigma[:w.k]):.3e}, max abs / sigma_1 {np.max(err) / ref.sigma[0]:.3e}; "
          f"residual {res:.6e} vs {res_ref:.6e}", flush=True)
    if ref.margins.min() >= mfloor:
        assert np.array_equal(perm, ref.perm)
        assert out.info["swaps"] == ref.swaps
        if ref.jstar_margin >= (1e-3 if fp32 else 1e-10):
            assert out.info["jstar"] == ref.jstar
        if not fp32:
            assert abs(out.info["g2"] - ref.g2) < 1e-8 * ref.g2
        assert np.all(err <= tol * ref.sigma + floor * ref.sigma[0])
        assert abs(res - res_ref) <= tol * res_ref
    else:
        # A QRCP step of the oracle whose margin is below what this form's
        # rounding resolves: the pivots are exact up to it, and after it the
        # two leading sets may differ, so sigma(L) and the residual (functions
        # of the set) are only held to what every SRQR-certified set meets:
        # g2 <= g, interlacing with sigma(A), the residual within 1% of the
        # oracle's, and sigma_j(L)^2 >= sigma_j(A)^2 - res^2.
        bad = int(np.flatnonzero(ref.margins < mfloor)[0])
        print(f"[gpu-case] QRCP near-tie at step {bad} (margin {ref.margins[bad]:.2e}): "
              f"pivots compared up to it, set-level bounds after it", flush=True)
        assert np.array_equal(perm[:bad], ref.perm[:bad])
        assert out.info["g2"] <= 2.0
        s_true = w.sigma()[:l]
        nn = w.noise * (np.sqrt(w.m) + np.sqrt(w.n)) * 1.01
        assert np.all(sig <= s_true + nn)
        assert res <= 1.01 * res_ref
        assert np.all(sig ** 2 >= np.maximum(s_true - nn, 0.0) ** 2 - res ** 2)


def test_large_fp64_full_size():
    import torch
    import paper_1803_01982_amd as ff
    w = synth.WORKLOADS["large"]
    announce(f"generate large {w.m}x{w.n}")
    A = synth.make_workload("large")
    Ad = _dev(A, torch.float64)
    announce(f"factor large {w.m}x{w.n} l={w.l} fp64")
    out = ff.factor(Ad, w.k, w.p, w.seed)
    torch.cuda.synchronize()
    l = w.l
    assert out.info["l"] == l and out.info["flags"] == 0
    # rows a1 + a2 against the oracle at full size: B = Omega A, QRCP pivots
    announce("oracle sketch + QRCP on B at full size")
    B = oracle.sketch(oracle.omega(w.seed, l, w.m), A)
    piv, margins, _ = oracle.qrcp_sketch(B, l)
    del B
    perm = host(out.perm)
    mfloor = 1e-12
    if margins.min() >= mfloor and out.info["swaps"] == 0:
        assert np.array_equal(perm[:l], piv[:l])
    else:
        bad = int(np.flatnonzero(margins < mfloor)[0]) if margins.min() < mfloor else l
        assert np.array_equal(perm[:bad], piv[:bad]) or out.info["swaps"] > 0
    # properties at any size
    Q, L, V = (host(t) for t in (out.Q, out.L, out.V))
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < 1e-12
    assert np.linalg.norm(V.T @ V - np.eye(l)) < 1e-12
    assert np.allclose(np.triu(L, 1), 0.0) and np.all(np.diag(L) >= 0)
    announce("residual at full size")
    res = dg.residual_fro(A, Q, L, V)
    nA2 = float(np.sum(A * A))
    pyth = np.sqrt(max(nA2 - float(np.sum(L * L)), 0.0))
    assert abs(res - pyth) <= 1e-6 * res
    # interlacing with the prescribed spectrum: sigma_j(L) <= sigma_j(A) and,
    # A = U S V^T + N with ||N||_2 <= 1e-5 (sqrt(m) + sqrt(n)) (1 + 1e-2),
    # so sigma_j(L) <= sigma_j(U S V^T) + ||N||_2
    s_true = w.sigma()[:l]
    nn = 1e-5 * (np.sqrt(w.m) + np.sqrt(w.n)) * 1.01
    sig = host(out.sigma)
    assert np.all(sig <= s_true + nn)
    # the leading k values: sigma_j(L)^2 >= sigma_j(A)^2 - ||R22||_2^2 with
    # ||R22||_2 <= ||A - Q Q^T A||_F = res
    assert np.all(sig[: w.k] ** 2 >= (np.maximum(s_true[: w.k] - nn, 0.0)) ** 2 - res ** 2)
