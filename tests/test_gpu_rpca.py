"""Robust PCA by IALM with Flip-Flop SRQR as the partial SVD, on the GPU
through the C ABI (ffsrqr_rpca_ialm), against the oracle (oracle/ialm.py)
on the same bytes: iterations, the rank kept, the low-rank and sparse parts
and the recovery of the planted parts (the paper's test matrices: rank
0.1 m, 5% of the entries corrupted by values uniform on [-500, 500]); at
1000 x 1000 and 2000 x 2000 the device time per solve is reported."""
import time

import numpy as np
import pytest

import synth
from gpu_util import announce, dev_f, host
from oracle import ialm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_1803_01982_amd as ff
    ff.load()
    return ff


def _check(ff, m, n, rank, seed, oracle_too=True, tol=1e-7, dtype=None, mixed=False, x_tol=1e-6):
    import torch
    M, X0, E0 = synth.rpca_problem(m, n, rank, 0.05, seed=seed)
    Md = dev_f(M, dtype)
    Mh = host(Md).astype(np.float64)
    ff.rpca_ialm(Md, tol=tol, mixed=mixed)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = ff.rpca_ialm(Md, tol=tol, mixed=mixed)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    X, E = host(out.X).astype(np.float64), host(out.E).astype(np.float64)
    err = np.linalg.norm(X - X0) / np.linalg.norm(X0)
    info = out.info
    print(f"[gpu-case] rpca {m}x{n} rank {rank}: {ms:.1f} ms, {info['iterations']} iterations, rank "
          f"{info['rank']}, residual {info['residual']:.2e}, ||X - X*|| / ||X*|| {err:.2e}, "
          f"nnz(E) {np.count_nonzero(E)}", flush=True)
    assert info["converged"] == 1 and info["rank"] == rank
    assert err < (1e-5 if tol <= 1e-7 else 1e-3)
    if oracle_too:
        ref = ialm.rpca_ialm(Mh, tol=tol)
        dx = np.linalg.norm(X - ref.X) / np.linalg.norm(ref.X)
        de = np.linalg.norm(E - ref.E) / np.linalg.norm(ref.E)
        print(f"[gpu-case] vs oracle: iterations {ref.iterations}, rank {ref.sv}, X {dx:.2e}, E {de:.2e}", flush=True)
        assert abs(info["iterations"] - ref.iterations) <= (1 if x_tol <= 1e-6 else 3)
        assert info["rank"] == ref.sv
        assert dx < x_tol and de < x_tol
    return out, ms


@pytest.mark.parametrize("m,n,rank,seed", [(200, 200, 20, 3), (300, 250, 25, 5)])
def test_rpca_fp64(ff, m, n, rank, seed):
    announce(f"rpca fp64 {m}x{n} rank {rank}")
    _check(ff, m, n, rank, seed)


def test_rpca_fp32(ff):
    import torch
    announce("rpca fp32 200x200 rank 20 tol 1e-5")
    _check(ff, 200, 200, 20, 3, tol=1e-5, dtype=torch.float32, x_tol=1e-4)


def test_rpca_1000(ff):
    """The paper's first robust PCA size (1000 x 1000, rank 100)."""
    announce("rpca fp64 1000x1000 rank 100")
    _check(ff, 1000, 1000, 100, 1)


@pytest.mark.parametrize("m", [2000, 4000, 6000])
def test_rpca_large_gpu_only(ff, m):
    """The paper's larger robust PCA sizes (rank 0.1 m): the oracle's run
    would take many minutes, so the result is checked against the planted
    parts only."""
    announce(f"rpca fp64 {m}x{m} rank {m // 10}")
    _check(ff, m, m, m // 10, 2, oracle_too=False)
