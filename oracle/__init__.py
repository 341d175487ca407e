"""CPU FP64 oracle of the Flip-Flop SRQR hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import, call or run anything under
``oracle/``.  The product library never does, and the oracle never imports
the product; the two share no code.  Inputs come from the separate ``synth``
module, which holds none of the method's arithmetic.

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: numpy's Philox, LAPACK (numpy/scipy) QR, pivoted QR and SVD used as
black boxes, closed forms, brute force on tiny inputs, Lemma 3.1, Theorem 3.1
and Theorem 1.1 of the paper, and metamorphic relations.

Parity unpinned (no printed example exists in the paper to fix them):
  * the exact pivot trajectory of QRCP on generic inputs beyond what LAPACK's
    dgeqp3 reproduces on well-separated inputs;
  * the exact swap-loop trajectory of Algorithm 4 (only its post-condition
    g2 <= g and its monotone determinant growth are pinned);
  * the choice of Box-Muller for the Gaussian map (its output distribution is
    pinned, the choice itself is a documented convention).
"""
from .philox import omega, philox4x64_10, uniform_open
from .ffsrqr import (
    FLAG_L_CLAMPED,
    FLAG_NONFINITE,
    FLAG_RANK_DEFICIENT,
    FLAG_SWAPCAP,
    Alg9,
    Result,
    alg9,
    back_substitute,
    factor_leading_set,
    ffsrqr,
    flip_flop_lq,
    g2_probe_estimate,
    householder,
    householder_qr,
    jacobi_svd,
    probe_omega,
    project,
    qrcp_sketch,
    rank_tolerance,
    residual_margin,
    residual_norms,
    round_bf16,
    sketch,
    srqr_rho,
    trqrcp_pivots,
    upper_inverse,
)
from . import diagnostics
from . import hosvd
from . import ialm

__all__ = [
    "omega", "philox4x64_10", "uniform_open", "FLAG_L_CLAMPED", "FLAG_NONFINITE",
    "FLAG_RANK_DEFICIENT", "FLAG_SWAPCAP", "Alg9", "Result", "alg9", "back_substitute",
    "factor_leading_set", "ffsrqr", "flip_flop_lq", "g2_probe_estimate", "householder",
    "householder_qr", "jacobi_svd", "probe_omega", "project", "qrcp_sketch", "rank_tolerance", "residual_margin", "residual_norms", "round_bf16",
    "sketch", "srqr_rho", "trqrcp_pivots",
    "upper_inverse", "diagnostics", "hosvd", "ialm",
]
