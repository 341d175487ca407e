"""ffsrqr_svd_small_noalloc (the entry point that allocates nothing; its
scratch is a static device array of the library) called through the C ABI
and compared with ffsrqr_svd_small, which runs the same kernels on a caller
workspace: the singular values must be identical bit for bit, on two calls in
a row (the second smaller, so it runs on what the first left in the static
array), in FP64 and FP32 storage; sizes above the maximum are rejected."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def _factor(l, seed):
    rng = np.random.default_rng(seed)
    return np.tril(rng.standard_normal((l, l))) * 0.05 + np.diag(np.exp(-np.arange(l) / 20.0))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_entry_point(prec):
    import torch
    import paper_1803_01982_amd as ff
    from paper_1803_01982_amd import _lib
    lib = _lib.load()
    dtype = torch.float64 if prec == "fp64" else torch.float32
    code = _lib.FP64 if prec == "fp64" else _lib.FP32
    stream = torch.cuda.current_stream().cuda_stream
    for l, seed in ((300, 1), (97, 2)):
        announce(f"svd_small_noalloc {prec} l={l}")
        Ld = ff.fortran(torch.from_numpy(_factor(l, seed)).to(dtype).cuda())
        ref = ff.svd_small(Ld)
        sig = torch.full((l,), float("nan"), dtype=torch.float64, device="cuda")
        st = lib.ffsrqr_svd_small_noalloc(Ld.data_ptr(), l, l, sig.data_ptr(), code, stream)
        assert st == _lib.FFSRQR_OK, lib.ffsrqr_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(sig.cpu().numpy(), ref.cpu().numpy())
    # above the static array's maximum: a clear error, nothing enqueued
    big = torch.zeros((1025, 1025), dtype=dtype, device="cuda")
    out = torch.zeros(1025, dtype=torch.float64, device="cuda")
    st = lib.ffsrqr_svd_small_noalloc(big.data_ptr(), 1025, 1025, out.data_ptr(), code, stream)
    assert st == _lib.FFSRQR_EINVAL
    assert b"1024" in lib.ffsrqr_last_error()
