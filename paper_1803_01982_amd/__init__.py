"""MI355X (gfx950) Flip-Flop SRQR hot path.

Python binding over libffsrqr.so (C ABI: include/ffsrqr.h).  Build the
library with ``python -m paper_1803_01982_amd.build``; importing works without
it, and the first call raises ``LibraryMissing`` if it is absent.
"""
from ._lib import (FLAG_L_CLAMPED, FLAG_NONFINITE, FLAG_RANK_DEFICIENT, FLAG_SWAPCAP, FLAG_TIMEOUT, FP32, FP64,
                   MIXED, FfsrqrError, LibraryMissing, load)
from .api import (Alg9Result, Factorization, TuckerResult, alg9_svd, empty_fortran, empty_fortran_nd, factor,
                  fortran, fortran_nd, lq, omega, panel_qr, profile_enable, profile_read, project, qrcp, sketch,
                  rpca_ialm, RpcaResult, factor_batched, Server, srqr_probe, srqr_rho, st_hosvd, svd_small, workspace,
                  workspace_size)

__all__ = [
    "FLAG_L_CLAMPED", "FLAG_NONFINITE", "FLAG_RANK_DEFICIENT", "FLAG_SWAPCAP", "FLAG_TIMEOUT", "FP32", "FP64",
    "MIXED", "FfsrqrError", "LibraryMissing", "load", "Alg9Result", "alg9_svd", "Factorization", "empty_fortran", "factor", "fortran", "lq", "omega",
    "panel_qr", "profile_enable", "profile_read", "project", "qrcp", "sketch", "srqr_probe", "srqr_rho", "svd_small", "workspace", "workspace_size",
    "TuckerResult", "st_hosvd", "fortran_nd", "empty_fortran_nd", "RpcaResult", "rpca_ialm", "factor_batched", "Server",
]
