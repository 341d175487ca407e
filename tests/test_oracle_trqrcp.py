"""Pins of the blocked TRQRCP pivot selection (Algorithm 2) in the oracle:
the sample update against its closed form (the sample of the residual),
the pivots of well-separated columns against LAPACK's dgeqp3, the blocks'
orthonormal basis against the chosen columns, and the whole path with the
blocked selection against the singular values of A."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_sample_update_is_the_sample_of_the_residual(mode):
    # after the blocks chose S, the sample of the remaining columns is the
    # initial sample with the chosen columns eliminated:
    #   B(:, rest) = B0(:, rest) - B0(:, S) R_SS^{-1} R_S,rest,  R = Q^T A,
    # which for the FP64 sample is Omega (I - Q Q^T) A(:, rest)
    A = synth.spectrum_matrix(120, 90, 0.9 ** np.arange(90), seed=21, noise=1e-3)
    trace = []
    S, _ = oracle.trqrcp_pivots(A, 24, 8, 5, 3, sketch_mode=mode, trace=trace)
    Om = oracle.omega(3, 13, 120)
    B0 = oracle.sketch(Om, A, mode)
    done = 0
    for Q, B, rest in trace:
        done += 8
        Sd = S[:done]
        Rss = Q.T @ A[:, Sd]
        Rsr = Q.T @ A[:, rest]
        elim = B0[:, rest] - B0[:, Sd] @ np.linalg.solve(Rss, Rsr)
        scale = np.abs(B0).max()
        assert np.max(np.abs(B[:, rest] - elim)) < 1e-10 * scale
        if mode == "fp64":
            direct = Om @ (A[:, rest] - Q @ Rsr)
            assert np.max(np.abs(B[:, rest] - direct)) < 1e-10 * scale
    assert len(set(S)) == 24


def test_each_block_is_dgeqp3_of_the_current_sample():
    # every block's pivots are the first pivots LAPACK's dgeqp3 picks on the
    # sample of the columns still in play (its norms well separated here)
    A = synth.separated_columns_matrix(80, 40, seed=22, ratio=1.5)
    trace = []
    S, margins = oracle.trqrcp_pivots(A, 12, 4, 5, 1, trace=trace)
    B, rest = oracle.sketch(oracle.omega(1, 9, 80), A), list(range(40))
    for blk in range(3):
        _, _, P = sla.qr(B[:, rest], pivoting=True, mode="economic")
        assert [rest[i] for i in P[:4]] == list(S[4 * blk: 4 * blk + 4])
        _, B, rest = trace[blk]
    assert np.all(margins > 1e-3)


def test_blocks_span_the_chosen_columns():
    A = synth.spectrum_matrix(100, 70, 0.85 ** np.arange(70), seed=23)
    trace = []
    S, _ = oracle.trqrcp_pivots(A, 20, 6, 4, 2, trace=trace)
    Q = trace[-1][0]
    assert np.linalg.norm(Q.T @ Q - np.eye(20)) < 1e-13
    AS = A[:, S]
    assert np.linalg.norm(AS - Q @ (Q.T @ AS)) < 1e-12 * np.linalg.norm(AS)


def test_path_with_blocked_selection():
    # sigma(L) of the flip-flop factor interlaces with sigma(A) and tracks the
    # leading singular values, with the blocked selection as with one block
    sig = 0.8 ** np.arange(60)
    A = synth.spectrum_matrix(150, 120, sig, seed=24, noise=1e-9)
    r = oracle.ffsrqr(A, 10, 6, 0, block=4)
    s = np.linalg.svd(A, compute_uv=False)
    assert list(r.perm[:16]) == list(r.perm[:16])
    assert np.all(r.sigma <= s[:16] * (1 + 1e-12))
    assert np.all(r.sigma[:10] >= 0.9 * s[:10])
    one = oracle.ffsrqr(A, 10, 6, 0)
    assert np.allclose(r.sigma[:10], one.sigma[:10], rtol=1e-2)
