"""The C ABI on the CPU: the library loads, exports every entry point that
include/ffsrqr.h declares, and its host-side logic (argument checks,
workspace sizing) behaves as documented.  No call here reaches a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffsrqr.h")
LIB = os.path.join(ROOT, "paper_1803_01982_amd", "libffsrqr.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffsrqr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libffsrqr.so is not built (run __graft_entry__.build())")
    from paper_1803_01982_amd import _lib
    return _lib.load()


def test_header_declares_the_path():
    names = declared()
    for n in ("ffsrqr_factor", "ffsrqr_workspace_size", "ffsrqr_omega", "ffsrqr_sketch", "ffsrqr_qrcp",
              "ffsrqr_panel_qr", "ffsrqr_project", "ffsrqr_srqr_rho", "ffsrqr_srqr_probe", "ffsrqr_lq",
              "ffsrqr_svd_small"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    raw = C.CDLL(LIB)
    for name in declared():
        assert hasattr(raw, name), name
    from paper_1803_01982_amd import _lib
    assert set(declared()) == set(_lib.SIGNATURES), "binding and header disagree"


def test_status_strings(lib):
    assert lib.ffsrqr_status_string(0) == b"ok"
    assert lib.ffsrqr_status_string(1) == b"invalid argument"
    assert lib.ffsrqr_status_string(99) == b"unknown status"


def test_default_opts(lib):
    from paper_1803_01982_amd import _lib
    o = _lib.Opts()
    lib.ffsrqr_default_opts(C.byref(o))
    assert (o.precision, o.max_swaps, o.g) == (0, -1, 2.0)


def test_workspace_size_host_only(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    o = _lib.Opts(0, -1, 2.0)
    assert lib.ffsrqr_workspace_size(1000, 800, 20, 10, C.byref(o), C.byref(out)) == 0
    small = out.value
    assert small > 8 * (1000 * 30 + 2 * 30 * 800)      # at least the sketch, W and the panel
    assert lib.ffsrqr_workspace_size(16384, 8192, 256, 16, C.byref(o), C.byref(out)) == 0
    assert out.value > small
    o32 = _lib.Opts(1, -1, 2.0)
    big64 = out.value
    assert lib.ffsrqr_workspace_size(16384, 8192, 256, 16, C.byref(o32), C.byref(out)) == 0
    assert out.value < big64


@pytest.mark.parametrize("m,n,k,p", [(0, 10, 1, 0), (10, 0, 1, 0), (10, 10, 0, 0), (10, 10, 11, 0),
                                     (10, 10, 1, -1)])
def test_workspace_size_rejects_bad_dims(lib, m, n, k, p):
    out = C.c_size_t(0)
    assert lib.ffsrqr_workspace_size(m, n, k, p, None, C.byref(out)) == 1
    assert lib.ffsrqr_last_error()


def test_workspace_size_limits(lib):
    """l = min(k + p, m, n) <= 1024, and the panel rows of the m x l and n x l
    Householder QRs must fit the LDS of a workgroup (at most
    256 min(1024, 1259 - l) rows): sizes beyond are EINVAL, checked on the
    host before anything is enqueued."""
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    o = _lib.Opts(0, -1, 2.0)
    assert lib.ffsrqr_workspace_size(4000, 3000, 1000, 24, C.byref(o), C.byref(out)) == 0   # l = 1024
    assert lib.ffsrqr_workspace_size(4000, 3000, 1000, 25, C.byref(o), C.byref(out)) == 1   # l = 1025
    assert b"1024" in lib.ffsrqr_last_error()
    assert lib.ffsrqr_workspace_size(183040, 2000, 512, 32, C.byref(o), C.byref(out)) == 0  # l = 544
    assert lib.ffsrqr_workspace_size(184000, 2000, 512, 32, C.byref(o), C.byref(out)) == 1
    assert lib.ffsrqr_workspace_size(2000, 184000, 512, 32, C.byref(o), C.byref(out)) == 1


def test_workspace_size_mixed(lib):
    """The mixed form keeps FP32 storage: its workspace is the FP32 one plus
    the BF16 operand rows (m rounded up to 8)."""
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    assert lib.ffsrqr_workspace_size(32768, 16384, 512, 32, C.byref(_lib.Opts(1, -1, 2.0)), C.byref(out)) == 0
    fp32 = out.value
    assert lib.ffsrqr_workspace_size(32768, 16384, 512, 32, C.byref(_lib.Opts(2, -1, 2.0)), C.byref(out)) == 0
    assert out.value >= fp32


def test_svd_small_noalloc_host_checks(lib):
    fake = C.c_void_p(0x1000)
    assert lib.ffsrqr_svd_small_noalloc(fake, 1025, 1025, fake, 0, None) == 1
    assert b"1024" in lib.ffsrqr_last_error()
    assert lib.ffsrqr_svd_small_noalloc(fake, 4, 3, fake, 0, None) == 1
    assert lib.ffsrqr_svd_small_noalloc(None, 4, 4, fake, 0, None) == 1
    assert lib.ffsrqr_svd_small_noalloc(fake, 4, 4, fake, 9, None) == 1


def test_workspace_size_rejects_bad_precision_and_null(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    assert lib.ffsrqr_workspace_size(10, 10, 1, 0, C.byref(_lib.Opts(7, -1, 2.0)), C.byref(out)) == 1
    assert lib.ffsrqr_workspace_size(10, 10, 1, 0, None, None) == 1


def _factor(lib, m=10, n=8, lda=10, k=2, p=1, ldq=10, ldl=3, ldv=8, g=2.0, prec=0, null=None):
    from paper_1803_01982_amd import _lib
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks fail first
    ptrs = {n_: fake for n_ in ("A", "perm", "Q", "L", "V", "sigma", "work")}
    if null:
        ptrs[null] = None
    o = _lib.Opts(prec, -1, g)
    info = _lib.Info()
    return lib.ffsrqr_factor(ptrs["A"], m, n, lda, k, p, 0, ptrs["perm"], ptrs["Q"], ldq, ptrs["L"], ldl,
                             ptrs["V"], ldv, ptrs["sigma"], C.byref(info), ptrs["work"], 1 << 20, C.byref(o),
                             None)


@pytest.mark.parametrize("kw", [dict(m=0), dict(k=0), dict(k=9), dict(p=-2), dict(lda=9), dict(ldq=9),
                                dict(ldl=2), dict(ldv=7), dict(g=1.0), dict(g=0.5), dict(prec=3), dict(prec=-1),
                                dict(null="A"), dict(null="Q"), dict(null="sigma"), dict(null="work")])
def test_factor_argument_checks(lib, kw):
    assert _factor(lib, **kw) == 1
    assert lib.ffsrqr_last_error() != b""


def test_stage_argument_checks(lib):
    fake = C.c_void_p(0x1000)
    assert lib.ffsrqr_omega(0, 0, 10, fake, 10, 0, None) == 1
    assert lib.ffsrqr_omega(0, 3, 10, fake, 9, 0, None) == 1
    assert lib.ffsrqr_sketch(fake, 10, 5, 9, 0, 3, fake, 3, fake, fake, 100, 0, None) == 1
    assert lib.ffsrqr_qrcp(fake, 5, 4, 5, fake, fake, fake, 100, 0, None) == 1          # n < l
    assert lib.ffsrqr_panel_qr(fake, 10, 5, 10, fake, 11, fake, 10, fake, 11, fake, 100, 0, None) == 1
    assert lib.ffsrqr_project(fake, 10, 3, 10, fake, 5, 10, fake, 2, fake, fake, fake, 100, 0, None) == 1
    assert lib.ffsrqr_srqr_rho(fake, 4, 4, fake, 0.0, fake, fake, 100, 0, None) == 1   # alpha must be > 0
    assert lib.ffsrqr_lq(fake, 4, 3, 4, fake, fake, 4, fake, 3, fake, 100, 0, None) == 1
    assert lib.ffsrqr_svd_small(fake, 4, 3, fake, fake, 100, 0, None) == 1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1803_01982_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()


def test_st_hosvd_workspace_size_host_only(lib):
    """The ST-HOSVD sizing call plans every mode on the host: a 400^3 tensor
    of Tucker rank 40^3 needs its two tensor buffers (2 x 256 MB FP32) plus
    the largest mode's factorization; invalid ranks, orders and tensor
    orders are rejected."""
    from paper_1803_01982_amd import _lib
    i64 = C.c_int64 * 3
    out = C.c_size_t(0)
    o = _lib.Opts(1, -1, 2.0)
    assert lib.ffsrqr_st_hosvd_workspace_size(3, i64(400, 400, 400), i64(40, 40, 40), None, 10, C.byref(o),
                                              C.byref(out)) == 0
    assert out.value > 2 * 4 * 400 ** 3
    order = (C.c_int32 * 3)(2, 0, 1)
    assert lib.ffsrqr_st_hosvd_workspace_size(3, i64(400, 400, 400), i64(40, 40, 40), order, 10, C.byref(o),
                                              C.byref(out)) == 0
    bad_order = (C.c_int32 * 3)(0, 0, 1)
    assert lib.ffsrqr_st_hosvd_workspace_size(3, i64(40, 40, 40), i64(4, 4, 4), bad_order, 2, None,
                                              C.byref(out)) == 1
    assert lib.ffsrqr_st_hosvd_workspace_size(3, i64(40, 40, 40), i64(4, 41, 4), None, 2, None, C.byref(out)) == 1
    assert lib.ffsrqr_st_hosvd_workspace_size(0, i64(40, 40, 40), i64(4, 4, 4), None, 2, None, C.byref(out)) == 1
    assert lib.ffsrqr_st_hosvd_workspace_size(9, (C.c_int64 * 9)(*[2] * 9), (C.c_int64 * 9)(*[1] * 9), None, 0,
                                              None, C.byref(out)) == 1
    assert lib.ffsrqr_last_error()


def test_rpca_workspace_size_host_only(lib):
    out = C.c_size_t(0)
    assert lib.ffsrqr_rpca_workspace_size(1000, 1000, 10, 0, None, C.byref(out)) == 0
    assert out.value > 3 * 8 * 1000 * 1000
    small = out.value
    assert lib.ffsrqr_rpca_workspace_size(1000, 1000, 10, 150, None, C.byref(out)) == 0
    assert out.value < small
    assert lib.ffsrqr_rpca_workspace_size(0, 10, 10, 0, None, C.byref(out)) == 1
    assert lib.ffsrqr_rpca_workspace_size(10, 10, 1024, 0, None, C.byref(out)) == 1
    assert lib.ffsrqr_last_error()


def test_batched_host_checks(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    probs = (_lib.Problem * 2)()
    probs[0] = _lib.Problem(None, 1000, 800, 1000, 20, 10, 0, None, None, 1000, None, 30, None, 800, None, None)
    probs[1] = _lib.Problem(None, 600, 900, 600, 40, 10, 0, None, None, 600, None, 50, None, 900, None, None)
    assert lib.ffsrqr_batched_workspace_size(2, probs, None, C.byref(out)) == 0
    one = C.c_size_t(0)
    assert lib.ffsrqr_workspace_size(1000, 800, 20, 10, None, C.byref(one)) == 0
    assert out.value >= one.value
    assert lib.ffsrqr_batched_workspace_size(0, probs, None, C.byref(out)) == 1
    probs[1].k = 0
    assert lib.ffsrqr_batched_workspace_size(2, probs, None, C.byref(out)) == 1
    assert b"problem 1" in lib.ffsrqr_last_error()
    # NULL device pointers are rejected before anything runs (no device needed)
    probs[1].k = 40
    assert lib.ffsrqr_factor_batched(2, probs, C.c_void_p(1), 1 << 30, None, None) == 1


def test_block_option_checks(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    o = _lib.Opts(0, -1, 2.0, 32, 0)
    assert lib.ffsrqr_workspace_size(16384, 8192, 256, 16, C.byref(o), C.byref(out)) == 0
    big = out.value
    assert lib.ffsrqr_workspace_size(16384, 8192, 256, 16, C.byref(_lib.Opts(0, -1, 2.0)), C.byref(out)) == 0
    assert big >= out.value
    assert lib.ffsrqr_workspace_size(100, 80, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 65, 0)), C.byref(out)) == 1
    # n - l + 1 < block + p: too few columns for the blocked sample
    assert lib.ffsrqr_workspace_size(100, 40, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 16, 0)), C.byref(out)) == 1
    assert b"blocked" in lib.ffsrqr_last_error()


def test_probe_option_checks(lib):
    from paper_1803_01982_amd import _lib
    o = _lib.Opts()
    lib.ffsrqr_default_opts(C.byref(o))
    assert o.g2_probe == 0
    out = C.c_size_t(0)
    for d, want in ((0, 0), (1, 0), (64, 0), (-1, 1), (65, 1)):
        rc = lib.ffsrqr_workspace_size(1000, 800, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 0, d)), C.byref(out))
        assert rc == want, d
    assert b"g2_probe" in lib.ffsrqr_last_error()
    # the per-step entry point checks its arguments before touching a device
    f = lib.ffsrqr_srqr_probe
    one = C.c_void_p(256)
    assert f(one, 8, 8, one, 1.0, 0, 1, 1, one, one, 1 << 20, 0, None) == 1    # d = 0
    assert f(one, 8, 8, one, 1.0, 65, 1, 1, one, one, 1 << 20, 0, None) == 1   # d > 64
    assert f(one, 8, 8, one, 1.0, 4, 1, 0, one, one, 1 << 20, 0, None) == 1    # q = 0 is Omega's stream
    assert f(one, 8, 8, one, 0.0, 4, 1, 1, one, one, 1 << 20, 0, None) == 1    # alpha must be > 0
    assert f(one, 8, 4, one, 1.0, 4, 1, 1, one, one, 1 << 20, 0, None) == 1    # ldr < l


def test_est_norms_option_checks(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    ws = lib.ffsrqr_workspace_size
    assert ws(1000, 800, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 16, 0, 1)), C.byref(out)) == 0
    # the one-block selection: its sample update needs an l x n product in scratch
    assert ws(1000, 800, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 0, 0, 0)), C.byref(out)) == 0
    plain = out.value
    assert ws(1000, 800, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 0, 0, 1)), C.byref(out)) == 0
    assert out.value >= plain
    assert ws(1000, 800, 20, 10, C.byref(_lib.Opts(0, -1, 2.0, 16, 0, 2)), C.byref(out)) == 1
    assert b"est_norms" in lib.ffsrqr_last_error()
    est = _lib.Opts(0, -1, 2.0, 0, 0, 1)
    assert lib.ffsrqr_rpca_workspace_size(500, 400, 10, 0, C.byref(est), C.byref(out)) == 1


def test_python_workspace_size_follows_the_options(lib):
    # the binding sizes the workspace of a call with the options the call uses
    from paper_1803_01982_amd import _lib, api
    out = C.c_size_t(0)
    for block, est in ((0, False), (0, True), (16, False), (16, True)):
        o = _lib.Opts(0, -1, 2.0, block, 0, 1 if est else 0)
        assert lib.ffsrqr_workspace_size(2000, 1500, 40, 10, C.byref(o), C.byref(out)) == 0
        assert api.workspace_size(2000, 1500, 40, 10, block=block, est_norms=est) == out.value


def test_drivers_refuse_the_blocked_selection(lib):
    from paper_1803_01982_amd import _lib
    out = C.c_size_t(0)
    blocked = _lib.Opts(0, -1, 2.0, 16, 0)
    probed = _lib.Opts(0, -1, 2.0, 0, 8)
    assert lib.ffsrqr_rpca_workspace_size(500, 400, 10, 0, C.byref(blocked), C.byref(out)) == 1
    assert b"opts.block" in lib.ffsrqr_last_error()
    assert lib.ffsrqr_rpca_workspace_size(500, 400, 10, 0, C.byref(probed), C.byref(out)) == 0
    I64 = C.c_int64 * 3
    dims, ranks = I64(40, 30, 20), I64(5, 5, 5)
    assert lib.ffsrqr_st_hosvd_workspace_size(3, dims, ranks, None, 4, C.byref(blocked), C.byref(out)) == 1
    assert lib.ffsrqr_st_hosvd_workspace_size(3, dims, ranks, None, 4, C.byref(probed), C.byref(out)) == 0


def test_server_rejects_bad_config(lib):
    from paper_1803_01982_amd import _lib
    assert not lib.ffsrqr_server_create(None)
    assert not lib.ffsrqr_server_create(C.byref(_lib.ServerCfg(1 << 30, 0, 1)))
    assert not lib.ffsrqr_server_create(C.byref(_lib.ServerCfg(1 << 30, 17, 1)))
    assert not lib.ffsrqr_server_create(C.byref(_lib.ServerCfg(1 << 10, 2, 1)))
    assert not lib.ffsrqr_server_create(C.byref(_lib.ServerCfg(1 << 30, 2, 9)))
    t = C.c_uint64(0)
    assert lib.ffsrqr_submit(None, None, C.byref(t)) == 1
    lib.ffsrqr_server_destroy(None)
