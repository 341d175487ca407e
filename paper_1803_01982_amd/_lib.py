"""ctypes declarations of libffsrqr.so (the C ABI in include/ffsrqr.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffsrqr.so")

FFSRQR_OK, FFSRQR_EINVAL, FFSRQR_EWORKSPACE, FFSRQR_EHIP, FFSRQR_ENODEV = range(5)
FP64, FP32, MIXED = 0, 1, 2
FLAG_RANK_DEFICIENT, FLAG_SWAPCAP, FLAG_NONFINITE, FLAG_L_CLAMPED, FLAG_TIMEOUT = 1, 2, 4, 8, 16


class LibraryMissing(RuntimeError):
    pass


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_swaps", C.c_int32), ("g", C.c_double), ("block", C.c_int32),
                ("g2_probe", C.c_int32), ("est_norms", C.c_int32), ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("l", C.c_int64), ("swaps", C.c_int32), ("flags", C.c_uint32), ("g2", C.c_double),
                ("alpha", C.c_double), ("jstar", C.c_int64), ("numerical_rank", C.c_int64),
                ("min_margin", C.c_double), ("jacobi_sweeps", C.c_int32), ("probes", C.c_int32),
                ("jstar_margin", C.c_double), ("jstar_candidates", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [("A", C.c_void_p), ("m", C.c_int64), ("n", C.c_int64), ("lda", C.c_int64), ("k", C.c_int64),
                ("p", C.c_int64), ("seed", C.c_uint64), ("perm", C.c_void_p), ("Q", C.c_void_p),
                ("ldq", C.c_int64), ("L", C.c_void_p), ("ldl", C.c_int64), ("V", C.c_void_p),
                ("ldv", C.c_int64), ("sigma", C.c_void_p), ("info", C.POINTER(Info))]


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("slots", C.c_int32), ("precision", C.c_int32)]


class RpcaInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rank", C.c_int32), ("residual", C.c_double), ("mu", C.c_double),
                ("norm2", C.c_double), ("converged", C.c_int32), ("rank_capped", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_SZ = C.c_size_t
_U64 = C.c_uint64
_D = C.c_double

SIGNATURES = {
    "ffsrqr_default_opts": (None, [C.POINTER(Opts)]),
    "ffsrqr_release": (None, []),
    "ffsrqr_status_string": (C.c_char_p, [C.c_int]),
    "ffsrqr_last_error": (C.c_char_p, []),
    "ffsrqr_workspace_size": (C.c_int, [_I64, _I64, _I64, _I64, C.POINTER(Opts), C.POINTER(_SZ)]),
    "ffsrqr_factor": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I64, _U64, _P, _P, _I64, _P, _I64, _P, _I64, _P,
                                C.POINTER(Info), _P, _SZ, C.POINTER(Opts), _P]),
    "ffsrqr_omega": (C.c_int, [_U64, _I64, _I64, _P, _I64, _I32, _P]),
    "ffsrqr_sketch": (C.c_int, [_P, _I64, _I64, _I64, _U64, _I64, _P, _I64, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_qrcp": (C.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_panel_qr": (C.c_int, [_P, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _SZ, _I32, _P]),
    "ffsrqr_project": (C.c_int, [_P, _I64, _I64, _I64, _P, _I64, _I64, _P, _I64, _P, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_srqr_rho": (C.c_int, [_P, _I64, _I64, _P, _D, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_srqr_probe": (C.c_int, [_P, _I64, _I64, _P, _D, _I32, _U64, _U64, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_lq": (C.c_int, [_P, _I64, _I64, _I64, _P, _P, _I64, _P, _I64, _P, _SZ, _I32, _P]),
    "ffsrqr_svd_small": (C.c_int, [_P, _I64, _I64, _P, _P, _SZ, _I32, _P]),
    "ffsrqr_svd_small_noalloc": (C.c_int, [_P, _I64, _I64, _P, _I32, _P]),
    "ffsrqr_alg9_workspace_size": (C.c_int, [_I64, _I64, _I64, _I64, _I32, C.POINTER(_SZ)]),
    "ffsrqr_alg9_svd": (C.c_int, [_P, _I64, _I64, _I64, _P, _I64, _I64, _I64, _P, _I64, _P, _P, _I64, _P, _SZ,
                                  _I32, _P]),
    "ffsrqr_st_hosvd_workspace_size": (C.c_int, [_I32, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32), _I64,
                                                 C.POINTER(Opts), C.POINTER(_SZ)]),
    "ffsrqr_st_hosvd": (C.c_int, [_P, _I32, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32), _I64, _U64, _P,
                                  C.POINTER(_P), C.POINTER(_I64), _P, _SZ, C.POINTER(Opts), _P]),
    "ffsrqr_batched_workspace_size": (C.c_int, [_I32, C.POINTER(Problem), C.POINTER(Opts), C.POINTER(_SZ)]),
    "ffsrqr_factor_batched": (C.c_int, [_I32, C.POINTER(Problem), _P, _SZ, C.POINTER(Opts), _P]),
    "ffsrqr_server_create": (C.c_void_p, [C.POINTER(ServerCfg)]),
    "ffsrqr_submit": (C.c_int, [_P, C.POINTER(Problem), C.POINTER(_U64)]),
    "ffsrqr_poll": (C.c_int, [_P, _U64, C.POINTER(Info), C.POINTER(_I32)]),
    "ffsrqr_server_destroy": (None, [_P]),
    "ffsrqr_rpca_workspace_size": (C.c_int, [_I64, _I64, _I64, _I64, C.POINTER(Opts), C.POINTER(_SZ)]),
    "ffsrqr_rpca_ialm": (C.c_int, [_P, _I64, _I64, _I64, _D, _D, _I32, _I64, _U64, _I64, _P, _I64, _P, _I64,
                                   C.POINTER(RpcaInfo), _P, _SZ, C.POINTER(Opts), _P]),
    "ffsrqr_profile_enable": (None, [C.c_int]),
    "ffsrqr_profile_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
}

STEPS = ["omega", "sketch", "check", "qrcp", "panel", "project", "resid", "srqr", "lq", "svd", "swap"]

_lib = None


def load() -> C.CDLL:
    """Load libffsrqr.so (once) and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -m paper_1803_01982_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FfsrqrError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.ffsrqr_last_error().decode()
        text = lib.ffsrqr_status_string(status).decode()
        super().__init__(f"{where}: {text} ({status}): {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != FFSRQR_OK:
        raise FfsrqrError(status, where)
