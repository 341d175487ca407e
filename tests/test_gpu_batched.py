"""ffsrqr_factor_batched over 64 problems of mixed shapes (m, n uniform on
[500, 4000], sigma_j = j^-1.5, k uniform on [10, 100], p = 10, FP32): every
problem's outputs equal those of its own ffsrqr_factor call bit for bit (the
batch runs the same kernels one problem after another), a sample is
compared with the oracle, and the batch's time is reported."""
import time

import numpy as np
import pytest

import synth
from gpu_util import announce, dev_f, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_1803_01982_amd as ff
    ff.load()
    return ff


@pytest.fixture(scope="module")
def batch():
    return synth.batch_problems(64, seed=6)


def test_batched_equals_single_calls(ff, batch):
    import torch
    announce("factor_batched 64 problems, fp32, p=10")
    As = [dev_f(A, torch.float32) for A, _ in batch]
    ks = [k for _, k in batch]
    ps = [10] * len(As)
    ff.factor_batched(As, ks, ps)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = ff.factor_batched(As, ks, ps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    t = time.perf_counter()
    singles = [ff.factor(A, k, 10) for A, k in zip(As, ks)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    print(f"[gpu-case] batch of {len(As)}: {tb * 1e3:.1f} ms ({len(As) / tb:.1f} solves/s); one call each: "
          f"{ts * 1e3:.1f} ms", flush=True)
    for i, (b, s) in enumerate(zip(outs, singles)):
        assert np.array_equal(host(b.perm), host(s.perm)), i
        assert np.array_equal(host(b.sigma), host(s.sigma)), i
        assert np.array_equal(host(b.Q), host(s.Q)), i
        assert np.array_equal(host(b.V), host(s.V)), i
        assert b.info["swaps"] == s.info["swaps"] and b.info["flags"] == s.info["flags"]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_batched_sample_against_oracle(ff, batch, idx):
    # the three smallest problems of the batch, through the factor parity
    # helper (FP32 storage bounds)
    import torch
    from test_gpu_factor import FP32_TOL, compare
    order = sorted(range(len(batch)), key=lambda i: batch[i][0].size)
    A, k = batch[order[idx]]
    announce(f"batch problem {order[idx]}: {A.shape[0]}x{A.shape[1]} k={k} fp32 vs oracle")
    compare(ff, A, k, 10, 0, dtype=torch.float32, tol=FP32_TOL, margin_floor=1e-5)


def test_batched_with_probe_equals_single_calls(ff, batch):
    """The options reach every problem of a batch: with the random g2 probe
    (d = 8) the first 16 problems give the same results as single calls with
    the same option (the probe streams restart with each problem)."""
    import torch
    announce("factor_batched 16 problems, fp32, p=10, g2_probe=8")
    sub = batch[:16]
    As = [dev_f(A, torch.float32) for A, _ in sub]
    ks = [k for _, k in sub]
    outs = ff.factor_batched(As, ks, [10] * len(As), g2_probe=8)
    singles = [ff.factor(A, k, 10, g2_probe=8) for A, k in zip(As, ks)]
    torch.cuda.synchronize()
    for i, (b, s) in enumerate(zip(outs, singles)):
        assert b.info["probes"] >= 1 and b.info["probes"] == s.info["probes"], i
        assert np.array_equal(host(b.perm), host(s.perm)), i
        assert np.array_equal(host(b.sigma), host(s.sigma)), i
        assert b.info["swaps"] == s.info["swaps"] and b.info["g2"] == s.info["g2"], i
