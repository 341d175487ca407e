"""Python binding of the C ABI: the same names, argument marshalling only.

Matrices are column-major torch tensors on the current HIP device: a (rows x
cols) tensor with strides (1, ld).  ``fortran(t)`` makes one.  Every step of
the method runs in libffsrqr.so; torch only allocates device memory and
provides the current stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import threading

import torch

from . import _lib as L

_WORK: dict = {}


def fortran(t: torch.Tensor) -> torch.Tensor:
    """Column-major copy (strides (1, rows)) of a 2-D tensor."""
    return t.t().contiguous().t()


def empty_fortran(rows: int, cols: int, dtype, device) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    rows, cols = t.shape
    if t.stride(0) != 1 and rows > 1:
        raise ValueError("expected a column-major tensor (stride(0) == 1); use fortran()")
    return max(t.stride(1), rows, 1)


def _prec(dtype, mixed: bool = False) -> int:
    if dtype == torch.float64:
        if mixed:
            raise TypeError("the mixed form takes float32 data")
        return L.FP64
    if dtype == torch.float32:
        return L.MIXED if mixed else L.FP32
    raise TypeError(f"unsupported dtype {dtype}; use float64 or float32")


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def opts(precision=L.FP64, g: float = 2.0, max_swaps: int = -1, block: int = 0, g2_probe: int = 0,
         est_norms: bool = False) -> L.Opts:
    return L.Opts(precision=precision, max_swaps=max_swaps, g=g, block=block, g2_probe=g2_probe,
                  est_norms=1 if est_norms else 0, reserved=0)


def workspace_size(m: int, n: int, k: int, p: int, precision=L.FP64, block: int = 0,
                   est_norms: bool = False) -> int:
    lib = L.load()
    out = C.c_size_t(0)
    o = opts(precision, block=block, est_norms=est_norms)
    L.check(lib.ffsrqr_workspace_size(m, n, k, p, C.byref(o), C.byref(out)), "ffsrqr_workspace_size")
    return out.value


def workspace(nbytes: int, device, stream=None) -> torch.Tensor:
    """A cached device workspace of at least nbytes (grown on demand), one per
    (device, stream, host thread): calls on one workspace must not overlap, so
    work on different streams or from different threads never shares one.
    A buffer that is replaced is first recorded on its stream, so the caching
    allocator does not hand its memory out while work queued there may still
    use it."""
    dev = torch.device(device)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    key = (dev.type, dev.index, s.cuda_stream, threading.get_ident())
    w = _WORK.get(key)
    if w is None or w.numel() < nbytes:
        if w is not None:
            w.record_stream(s)
        w = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _WORK[key] = w
    return w


def release() -> None:
    """Drop the cached workspaces and the library's per-thread streams and
    events (registered to run at exit, while the HIP runtime is alive)."""
    _WORK.clear()
    if L._lib is not None:
        L._lib.ffsrqr_release()


atexit.register(release)


@dataclasses.dataclass
class Factorization:
    perm: torch.Tensor
    Q: torch.Tensor
    L: torch.Tensor
    V: torch.Tensor
    sigma: torch.Tensor
    info: dict


def factor(A: torch.Tensor, k: int, p: int, seed: int = 0, g: float = 2.0, max_swaps: int = -1,
           work: torch.Tensor | None = None, stream=None, mixed: bool = False, block: int = 0,
           g2_probe: int = 0, est_norms: bool = False) -> Factorization:
    """ffsrqr_factor: A (m x n, column-major, float64 or float32) -> perm, Q, L, V, sigma, info.
    mixed=True (float32 A) selects FFSRQR_MIXED (BF16 sketch, split-BF16 projection);
    block > 0 Algorithm 2's blocked selection; g2_probe = d > 0 the d-row random g2 estimate;
    est_norms (with block > 0) Algorithm 4's sample-estimated residual norms."""
    lib = L.load()
    m, n = A.shape
    lda = _ld(A)
    prec = _prec(A.dtype, mixed)
    l = min(k + p, m, n)
    dev = A.device
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    Q = empty_fortran(m, l, A.dtype, dev)
    Lf = empty_fortran(l, l, A.dtype, dev)
    V = empty_fortran(n, l, A.dtype, dev)
    sigma = torch.empty(l, dtype=torch.float64, device=dev)
    if work is None:
        work = workspace(workspace_size(m, n, k, p, prec, block, est_norms), dev, stream)
    info = L.Info()
    o = opts(prec, g, max_swaps, block, g2_probe, est_norms)
    L.check(lib.ffsrqr_factor(_ptr(A), m, n, lda, k, p, seed, _ptr(perm), _ptr(Q), m, _ptr(Lf), l,
                              _ptr(V), n, _ptr(sigma), C.byref(info), _ptr(work), work.numel(),
                              C.byref(o), _stream(stream)), "ffsrqr_factor")
    return Factorization(perm, Q, Lf, V, sigma, info.as_dict())


def omega(seed: int, l: int, m: int, dtype=torch.float64, device="cuda", stream=None) -> torch.Tensor:
    """ffsrqr_omega: Omega^T as an m x l column-major tensor."""
    lib = L.load()
    Ot = empty_fortran(m, l, dtype, device)
    L.check(lib.ffsrqr_omega(seed, l, m, _ptr(Ot), m, _prec(dtype), _stream(stream)), "ffsrqr_omega")
    return Ot


def sketch(A: torch.Tensor, seed: int, l: int, work=None, stream=None, mixed: bool = False):
    """ffsrqr_sketch: (B = Omega A, anorm2); mixed=True: BF16 operands, FP32 sums."""
    lib = L.load()
    m, n = A.shape
    prec = _prec(A.dtype, mixed)
    B = empty_fortran(l, n, A.dtype, A.device)
    an = torch.empty(n, dtype=torch.float64, device=A.device)
    if work is None:
        work = workspace(workspace_size(m, n, l, 0, prec), A.device, stream)
    L.check(lib.ffsrqr_sketch(_ptr(A), m, n, _ld(A), seed, l, _ptr(B), l, _ptr(an), _ptr(work), work.numel(),
                              prec, _stream(stream)), "ffsrqr_sketch")
    return B, an


def qrcp(B: torch.Tensor, l: int | None = None, work=None, stream=None):
    """ffsrqr_qrcp: (piv[l], margins[l]) of partial QRCP on B (l x n)."""
    lib = L.load()
    rows, n = B.shape
    l = rows if l is None else l
    piv = torch.empty(l, dtype=torch.int64, device=B.device)
    mg = torch.empty(l, dtype=torch.float64, device=B.device)
    if work is None:
        work = workspace(workspace_size(max(rows, l), n, l, 0, _prec(B.dtype)), B.device, stream)
    L.check(lib.ffsrqr_qrcp(_ptr(B), l, n, _ld(B), _ptr(piv), _ptr(mg), _ptr(work), work.numel(),
                            _prec(B.dtype), _stream(stream)), "ffsrqr_qrcp")
    return piv, mg


def panel_qr(A: torch.Tensor, cols: torch.Tensor, work=None, stream=None):
    """ffsrqr_panel_qr: explicit (Q, R) of A(:, cols)."""
    lib = L.load()
    m, n = A.shape
    c = cols.numel()
    Q = empty_fortran(m, c, A.dtype, A.device)
    R = empty_fortran(c, c, A.dtype, A.device)
    if work is None:
        work = workspace(workspace_size(m, n, min(c, m, n), 0, _prec(A.dtype)) + m * c * 8, A.device, stream)
    L.check(lib.ffsrqr_panel_qr(_ptr(A), m, n, _ld(A), _ptr(cols), c, _ptr(Q), m, _ptr(R), c, _ptr(work),
                                work.numel(), _prec(A.dtype), _stream(stream)), "ffsrqr_panel_qr")
    return Q, R


def project(Q: torch.Tensor, A: torch.Tensor, anorm2: torch.Tensor, work=None, stream=None, mixed: bool = False):
    """ffsrqr_project: (W = Q^T A, gamma2); mixed=True: the split-BF16 product."""
    lib = L.load()
    m, c = Q.shape
    n = A.shape[1]
    prec = _prec(A.dtype, mixed)
    W = empty_fortran(c, n, A.dtype, A.device)
    g2 = torch.empty(n, dtype=torch.float64, device=A.device)
    if work is None:
        work = workspace(workspace_size(m, n, min(c, m, n), 0, prec), A.device, stream)
    L.check(lib.ffsrqr_project(_ptr(Q), m, c, _ld(Q), _ptr(A), n, _ld(A), _ptr(W), c, _ptr(anorm2), _ptr(g2),
                               _ptr(work), work.numel(), prec, _stream(stream)), "ffsrqr_project")
    return W, g2


def srqr_rho(R11: torch.Tensor, a: torch.Tensor, alpha: float, work=None, stream=None) -> torch.Tensor:
    """ffsrqr_srqr_rho: rho[l] of R-tilde = [[R11, a], [0, alpha]]."""
    lib = L.load()
    l = R11.shape[0]
    rho = torch.empty(l, dtype=torch.float64, device=R11.device)
    if work is None:
        work = workspace(8 * (l + 1) * l + (1 << 16), R11.device, stream)
    L.check(lib.ffsrqr_srqr_rho(_ptr(R11), l, _ld(R11), _ptr(a), float(alpha), _ptr(rho), _ptr(work),
                                work.numel(), _prec(R11.dtype), _stream(stream)), "ffsrqr_srqr_rho")
    return rho


def srqr_probe(R11: torch.Tensor, a: torch.Tensor, alpha: float, d: int, seed: int, q: int, work=None,
               stream=None) -> torch.Tensor:
    """ffsrqr_srqr_probe: est[l+1], the randomized g2 estimate with the q-th d-row probe."""
    lib = L.load()
    l = R11.shape[0]
    est = torch.empty(l + 1, dtype=torch.float64, device=R11.device)
    if work is None:
        work = workspace(8 * ((d + 1) * l + d * (l + 1)) + (1 << 16), R11.device, stream)
    L.check(lib.ffsrqr_srqr_probe(_ptr(R11), l, _ld(R11), _ptr(a), float(alpha), int(d), int(seed), int(q),
                                  _ptr(est), _ptr(work), work.numel(), _prec(R11.dtype), _stream(stream)),
            "ffsrqr_srqr_probe")
    return est


def lq(R: torch.Tensor, perm: torch.Tensor, work=None, stream=None):
    """ffsrqr_lq: (L, V) with R^T = Qhat1 Rhat11, L = Rhat11^T, V = Pi Qhat1."""
    lib = L.load()
    l, n = R.shape
    Lf = empty_fortran(l, l, R.dtype, R.device)
    V = empty_fortran(n, l, R.dtype, R.device)
    if work is None:
        work = workspace(workspace_size(n, n, l, 0, _prec(R.dtype)) + n * l * 8, R.device, stream)
    L.check(lib.ffsrqr_lq(_ptr(R), l, n, _ld(R), _ptr(perm), _ptr(Lf), l, _ptr(V), n, _ptr(work), work.numel(),
                          _prec(R.dtype), _stream(stream)), "ffsrqr_lq")
    return Lf, V


def svd_small(Lm: torch.Tensor, work=None, stream=None) -> torch.Tensor:
    """ffsrqr_svd_small: singular values of L (descending, float64)."""
    lib = L.load()
    l = Lm.shape[0]
    sig = torch.empty(l, dtype=torch.float64, device=Lm.device)
    if work is None:
        work = workspace(workspace_size(l, l, l, 0, _prec(Lm.dtype)), Lm.device, stream)
    L.check(lib.ffsrqr_svd_small(_ptr(Lm), l, _ld(Lm), _ptr(sig), _ptr(work), work.numel(), _prec(Lm.dtype),
                                 _stream(stream)), "ffsrqr_svd_small")
    return sig


@dataclasses.dataclass
class Alg9Result:
    U: torch.Tensor       # m x k
    sigma: torch.Tensor   # [l] descending (the first k are Sigma_k)
    Vk: torch.Tensor      # n x k


def alg9_svd(A: torch.Tensor, V: torch.Tensor, k: int, work=None, stream=None, mixed: bool = False) -> Alg9Result:
    """ffsrqr_alg9_svd: rank-k SVD A ~ U diag(sigma[:k]) Vk^T from V = Pi Qhat1."""
    lib = L.load()
    m, n = A.shape
    l = V.shape[1]
    prec = _prec(A.dtype, mixed)
    U = empty_fortran(m, k, A.dtype, A.device)
    Vk = empty_fortran(n, k, A.dtype, A.device)
    sigma = torch.empty(l, dtype=torch.float64, device=A.device)
    if work is None:
        out = C.c_size_t(0)
        L.check(lib.ffsrqr_alg9_workspace_size(m, n, l, k, prec, C.byref(out)), "ffsrqr_alg9_workspace_size")
        work = workspace(out.value, A.device, stream)
    L.check(lib.ffsrqr_alg9_svd(_ptr(A), m, n, _ld(A), _ptr(V), _ld(V), l, k, _ptr(U), m, _ptr(sigma), _ptr(Vk), n,
                                _ptr(work), work.numel(), prec, _stream(stream)), "ffsrqr_alg9_svd")
    return Alg9Result(U, sigma, Vk)


def fortran_nd(t: torch.Tensor) -> torch.Tensor:
    """Fortran-order copy (the first index runs fastest) of a tensor."""
    rev = tuple(range(t.dim() - 1, -1, -1))
    return t.permute(rev).contiguous().permute(rev)


def empty_fortran_nd(shape, dtype, device) -> torch.Tensor:
    rev = tuple(range(len(shape) - 1, -1, -1))
    return torch.empty(tuple(shape[::-1]), dtype=dtype, device=device).permute(rev)


@dataclasses.dataclass
class TuckerResult:
    core: torch.Tensor    # ranks[0] x .. x ranks[d-1], Fortran order
    U: list               # U[n]: dims[n] x ranks[n], column-major


def st_hosvd(X: torch.Tensor, ranks, p: int, seed: int = 0, order=None, mixed: bool = False, work=None,
             stream=None) -> TuckerResult:
    """ffsrqr_st_hosvd: Tucker decomposition X ~ core x_1 U[0] .. x_d U[d-1]
    by ST-HOSVD with Flip-Flop SRQR (plus Algorithm 9) as each mode's rank-k
    SVD.  X must be in Fortran order (fortran_nd)."""
    lib = L.load()
    d = X.dim()
    dims = [int(x) for x in X.shape]
    step = 1
    for j in range(d):
        if X.stride(j) != step and dims[j] > 1:
            raise ValueError("expected a Fortran-order tensor; use fortran_nd()")
        step *= dims[j]
    ranks = [int(r) for r in ranks]
    if len(ranks) != d:
        raise ValueError("one rank per mode")
    prec = _prec(X.dtype, mixed)
    i64 = C.c_int64 * d
    dims_c, ranks_c = i64(*dims), i64(*ranks)
    order_c = (C.c_int32 * d)(*[int(o) for o in order]) if order is not None else None
    o = opts(prec)
    if work is None:
        out = C.c_size_t(0)
        L.check(lib.ffsrqr_st_hosvd_workspace_size(d, dims_c, ranks_c, order_c, p, C.byref(o), C.byref(out)),
                "ffsrqr_st_hosvd_workspace_size")
        work = workspace(out.value, X.device, stream)
    core = empty_fortran_nd(ranks, X.dtype, X.device)
    Us = [empty_fortran(dims[j], ranks[j], X.dtype, X.device) for j in range(d)]
    u_c = (C.c_void_p * d)(*[u.data_ptr() for u in Us])
    L.check(lib.ffsrqr_st_hosvd(_ptr(X), d, dims_c, ranks_c, order_c, p, seed, _ptr(core), u_c, i64(*dims),
                                _ptr(work), work.numel(), C.byref(o), _stream(stream)), "ffsrqr_st_hosvd")
    return TuckerResult(core, Us)


def factor_batched(As, ks, ps, seeds=None, g: float = 2.0, max_swaps: int = -1, mixed: bool = False, work=None,
                   stream=None, g2_probe: int = 0) -> list:
    """ffsrqr_factor_batched: one call over many problems (column-major A's
    of one dtype); returns one Factorization per problem."""
    lib = L.load()
    cnt = len(As)
    seeds = [0] * cnt if seeds is None else list(seeds)
    prec = _prec(As[0].dtype, mixed)
    o = opts(prec, g, max_swaps, g2_probe=g2_probe)
    probs = (L.Problem * cnt)()
    outs, infos = [], []
    for i, A in enumerate(As):
        if A.dtype != As[0].dtype:
            raise TypeError("one dtype for the whole batch")
        m, n = A.shape
        k, p = int(ks[i]), int(ps[i])
        l = min(k + p, m, n)
        dev = A.device
        f = Factorization(torch.empty(n, dtype=torch.int64, device=dev), empty_fortran(m, l, A.dtype, dev),
                          empty_fortran(l, l, A.dtype, dev), empty_fortran(n, l, A.dtype, dev),
                          torch.empty(l, dtype=torch.float64, device=dev), {})
        info = L.Info()
        infos.append(info)
        outs.append(f)
        probs[i] = L.Problem(_ptr(A), m, n, _ld(A), k, p, int(seeds[i]), _ptr(f.perm), _ptr(f.Q), m, _ptr(f.L), l,
                             _ptr(f.V), n, _ptr(f.sigma), C.pointer(info))
    if work is None:
        out = C.c_size_t(0)
        L.check(lib.ffsrqr_batched_workspace_size(cnt, probs, C.byref(o), C.byref(out)),
                "ffsrqr_batched_workspace_size")
        work = workspace(out.value, As[0].device, stream)
    L.check(lib.ffsrqr_factor_batched(cnt, probs, _ptr(work), work.numel(), C.byref(o), _stream(stream)),
            "ffsrqr_factor_batched")
    for f, info in zip(outs, infos):
        f.info.update(info.as_dict())
    return outs


class Server:
    """ffsrqr_server_*: a serving loop (continuous batching) over the path.
    submit() allocates the request's outputs on A's device and keeps them
    (and A) alive until poll() reports the request done; A must be ready on
    the device (its producing stream synchronised) when it is submitted."""

    def __init__(self, budget_bytes: int, slots: int = 4, precision=L.FP32):
        self._lib = L.load()
        cfg = L.ServerCfg(int(budget_bytes), int(slots), int(precision))
        self._h = self._lib.ffsrqr_server_create(C.byref(cfg))
        if not self._h:
            raise L.FfsrqrError(1, "ffsrqr_server_create (configuration or device allocation)")
        self._live = {}

    def submit(self, A: torch.Tensor, k: int, p: int, seed: int = 0) -> int:
        m, n = A.shape
        l = min(k + p, m, n)
        dev = A.device
        f = Factorization(torch.empty(n, dtype=torch.int64, device=dev), empty_fortran(m, l, A.dtype, dev),
                          empty_fortran(l, l, A.dtype, dev), empty_fortran(n, l, A.dtype, dev),
                          torch.empty(l, dtype=torch.float64, device=dev), {})
        torch.cuda.current_stream(dev).synchronize()  # outputs allocated, A ready
        prob = L.Problem(_ptr(A), m, n, _ld(A), k, p, seed, _ptr(f.perm), _ptr(f.Q), m, _ptr(f.L), l, _ptr(f.V), n,
                         _ptr(f.sigma), None)
        t = C.c_uint64(0)
        L.check(self._lib.ffsrqr_submit(self._h, C.byref(prob), C.byref(t)), "ffsrqr_submit")
        self._live[t.value] = (A, f)
        return t.value

    def poll(self, ticket: int):
        """(done, Factorization or None); a done ticket is forgotten."""
        info = L.Info()
        done = C.c_int32(0)
        st = self._lib.ffsrqr_poll(self._h, ticket, C.byref(info), C.byref(done))
        if not done.value:
            L.check(st, "ffsrqr_poll")
            return False, None
        A, f = self._live.pop(ticket)
        L.check(st, "ffsrqr_poll")
        f.info.update(info.as_dict())
        return True, f

    def close(self) -> None:
        if self._h:
            self._lib.ffsrqr_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class RpcaResult:
    X: torch.Tensor       # low-rank part, m x n column-major
    E: torch.Tensor       # sparse part, m x n column-major
    info: dict


def rpca_ialm(M: torch.Tensor, p: int = 10, seed: int = 0, lam: float = 0.0, tol: float = 1e-7,
              max_iter: int = 500, max_rank: int = 0, mixed: bool = False, work=None, stream=None) -> RpcaResult:
    """ffsrqr_rpca_ialm: robust PCA M ~ X + E by IALM with Flip-Flop SRQR
    (plus Algorithm 9) as the partial SVD; lam <= 0 selects
    1 / sqrt(max(m, n))."""
    lib = L.load()
    m, n = M.shape
    prec = _prec(M.dtype, mixed)
    o = opts(prec)
    if work is None:
        out = C.c_size_t(0)
        L.check(lib.ffsrqr_rpca_workspace_size(m, n, p, max_rank, C.byref(o), C.byref(out)),
                "ffsrqr_rpca_workspace_size")
        work = workspace(out.value, M.device, stream)
    X = empty_fortran(m, n, M.dtype, M.device)
    E = empty_fortran(m, n, M.dtype, M.device)
    info = L.RpcaInfo()
    L.check(lib.ffsrqr_rpca_ialm(_ptr(M), m, n, _ld(M), lam, tol, max_iter, p, seed, max_rank, _ptr(X), m, _ptr(E),
                                 m, C.byref(info), _ptr(work), work.numel(), C.byref(o), _stream(stream)),
            "ffsrqr_rpca_ialm")
    return RpcaResult(X, E, info.as_dict())


def profile_enable(on: bool = True) -> None:
    """Enable (and reset) the per-step device-time accounting of factor()."""
    L.load().ffsrqr_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{step: (milliseconds, launches)} accumulated since profile_enable()."""
    lib = L.load()
    n = len(L.STEPS)
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    lib.ffsrqr_profile_read(ms, cnt, n)
    return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STEPS)}
