"""The path with Algorithm 2's blocked pivot selection (opts.block > 0:
TRQRCP with a (block + p)-row sample and the sample update) on the GPU
against the oracle's blocked selection on the same bytes: the pivots where
the QRCP margins of the oracle's blocks separate them, sigma, the residual
and the factors' orthogonality within each form's bound; at the mid size
the time per solve is reported beside the one-block path's."""
import time

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


def _compare(ff, A, k, p, seed, block, form="fp64"):
    import torch
    fp32 = form != "fp64"
    Ad = dev_f(A, torch.float32 if fp32 else torch.float64)
    Ah = host(Ad).astype(np.float64)
    out = ff.factor(Ad, k, p, seed, block=block, mixed=form == "mixed")
    ref = oracle.ffsrqr(Ah, k, p, seed, block=block, storage="fp32" if fp32 else "fp64",
                        sketch_mode="bf16" if form == "mixed" else "fp64")
    tol = FP32_TOL if fp32 else FP64_TOL
    floor_m = 1e-4 if form == "mixed" else (1e-5 if fp32 else 1e-12)
    perm = host(out.perm)
    l = ref.l
    assert out.info["l"] == l and out.info["flags"] == ref.flags
    mg = ref.margins
    if mg.min() >= floor_m:
        assert list(perm[:l]) == list(ref.perm[:l])
        assert out.info["swaps"] == ref.swaps
        first_tie = l
    else:
        first_tie = int(np.flatnonzero(mg < floor_m)[0])
        assert list(perm[:first_tie]) == list(ref.perm[:first_tie])
    sig = host(out.sigma)
    err = np.abs(sig - ref.sigma)
    floor = (1e-14 if not fp32 else 1e-5) * ref.sigma[0]
    print(f"[gpu-case] pivots equal up to {first_tie} of {l}; sigma max rel err {np.max(err / ref.sigma):.3e}",
          flush=True)
    if first_tie == l:
        assert np.all(err <= tol * ref.sigma + floor)
    Q, L, V = (host(t).astype(np.float64) for t in (out.Q, out.L, out.V))
    orth = 1e-13 if not fp32 else 1e-5 * np.sqrt(l)
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < orth
    assert np.linalg.norm(V.T @ V - np.eye(l)) < orth
    res = dg.residual_fro(Ah, Q, L, V)
    res_ref = dg.residual_fro(Ah, ref.Q, ref.L, ref.V)
    nA = np.linalg.norm(Ah)
    res_floor = (1e-13 if not fp32 else 4.0 * np.sqrt(l) * 2.0 ** -24) * nA
    if first_tie == l:
        assert abs(res - res_ref) <= tol * max(res_ref, 1e-3 * nA) + res_floor
    return out, ref


@pytest.mark.parametrize("block", [4, 8, 30])
def test_blocked_small_fp64(ff, block):
    announce(f"factor blocked b={block} small_fp64 1000x800 k=20 p=10")
    w = synth.WORKLOADS["small_fp64"]
    _compare(ff, synth.make_workload("small_fp64"), w.k, w.p, w.seed, block)


def test_blocked_decay_fp64(ff):
    announce("factor blocked b=16 600x500 decay 0.97 k=40 p=8")
    sig = 0.97 ** np.arange(500)
    A = synth.spectrum_matrix(600, 500, sig, seed=31, noise=1e-6)
    _compare(ff, A, 40, 8, 2, 16)


@pytest.mark.parametrize("form", ["fp32", "mixed"])
def test_blocked_fp32_forms(ff, form):
    announce(f"factor blocked b=8 small 1000x800 k=20 p=10 {form}")
    A = synth.make_workload("small_fp64").astype(np.float32)
    _compare(ff, A, 20, 10, 0, 8, form)


def test_blocked_mid_fp64(ff):
    """The mid workload (16384 x 8192, k = 256, p = 16) with blocks of 32:
    parity with the oracle's blocked selection, and the time per solve
    beside the one-block path's."""
    import torch
    w = synth.WORKLOADS["mid"]
    announce("factor blocked b=32 mid 16384x8192 k=256 p=16 fp64")
    A = synth.make_workload("mid")
    _compare(ff, A, w.k, w.p, w.seed, 32)
    Ad = dev_f(A)
    for block in (0, 32):
        ff.factor(Ad, w.k, w.p, w.seed, block=block)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            ff.factor(Ad, w.k, w.p, w.seed, block=block)
        torch.cuda.synchronize()
        print(f"[gpu-case] mid fp64 block={block}: {(time.perf_counter() - t) / 3 * 1e3:.2f} ms per solve",
              flush=True)
