"""Planted mistakes: each mutant is the oracle's own source with one plausible
slip (a dropped term, a wrong sign or index, a transposed operand).  The test
compiles the mutant in the oracle's namespace, patches it in, and checks that
at least one of the pins fails.  This shows that the pins can tell a wrong
oracle from a right one.  Everything here runs on the CPU."""
import inspect
import sys
import textwrap

import numpy as np
import pytest

import oracle
import test_oracle_alg9 as ALG9
import test_oracle_bf16 as BF16
import test_oracle_est_norms as EST
import test_oracle_linalg as LIN
import test_oracle_path as PATH
import test_oracle_probe as PROBE

MOD = sys.modules["oracle.ffsrqr"]


def _mutant(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) >= 1, f"snippet not found in {func.__name__}: {old!r}"
    src = src.replace(old, new, 1)
    ns = dict(MOD.__dict__)
    exec(compile(src, f"<mutant {func.__name__}>", "exec"), ns)
    return ns[func.__name__]


def _small():
    import synth
    w = synth.WORKLOADS["small_fp64"]
    A = synth.make_workload("small_fp64")
    return w, A, oracle.ffsrqr(A, w.k, w.p, w.seed)


def _kahan_state():
    """The state of the probe pins' fixture: an SRQR test on a Kahan matrix."""
    A = np.vstack([PROBE.kahan(48), np.zeros((6, 48))])
    r = oracle.ffsrqr(A, 20, 0, seed=0, max_swaps=0)
    S = list(r.perm[:20])
    return A, S, PROBE._test_state(A, S)


def _pins():
    """The pins, run in order; returns the name of the first one that fails."""
    checks = [
        ("householder", lambda: [LIN.test_householder_maps_to_beta_e1(x) for x in
                                 ([3.0, 4.0], [-3.0, 4.0, 12.0], [0.0, 1.0, 1.0])]),
        ("qr_lapack", lambda: [LIN.test_householder_qr_matches_lapack(s) for s in ((50, 13), (300, 40))]),
        ("qrcp_dgeqp3", lambda: LIN.test_qrcp_pivots_match_dgeqp3(3, (20, 300), 20)),
        ("qrcp_ties", LIN.test_qrcp_ties_go_to_smallest_index),
        ("qrcp_margins", lambda: LIN.test_qrcp_margins_match_projection_residuals(25, 120, 20, 2)),
        ("rho_closed_form", LIN.test_srqr_rho_matches_block_inverse_closed_form),
        ("backsub", LIN.test_upper_inverse_and_back_substitution),
        ("jacobi_2x2", LIN.test_jacobi_2x2_closed_form),
        ("jacobi_lapack", lambda: LIN.test_jacobi_matches_lapack_svd((30, 30), "gauss")),
        ("full_rank", PATH.test_full_rank_reconstruction),
        ("structure", lambda: PATH.test_small_outputs_structure(_small())),
        ("bounds", lambda: PATH.test_singular_value_bounds(_small(), "small")),
        ("kahan_swaps", PATH.test_srqr_swaps_kahan),
        ("tight_g", PATH.test_tighter_g_swaps_until_satisfied),
        ("bf16_brute", BF16.test_round_bf16_matches_exhaustive_search_on_doubles),
        ("bf16_ties", BF16.test_round_bf16_ties_and_double_rounding),
        ("bf16_sketch", BF16.test_bf16_sketch_is_the_exactly_rounded_sum_of_exact_products),
        ("alg9_lapack", ALG9.test_alg9_sigma_matches_lapack_and_factors_are_consistent),
        ("alg9_full_rank", ALG9.test_alg9_at_full_rank_is_the_svd_of_A),
        ("jstar_margin", ALG9.test_jstar_margin_on_orthogonal_columns),
        # Algorithm 4's random g2 estimate and sample-estimated residual norms
        ("probe_stream", PROBE.test_probe_stream_is_standard_normal_and_apart_from_the_sketch),
        ("probe_orthogonal", lambda: [PROBE.test_orthogonal_probe_gives_the_exact_rho(l) for l in (1, 7, 20)]),
        ("est_sample", lambda: EST.test_final_sample_is_omega_times_the_residual(4, 2)),
        ("est_one_block_sample", EST.test_one_block_sample_update_is_omega_times_the_residual),
        ("est_carry", EST.test_estimate_errors_are_carried_exactly_through_the_swaps),
        ("est_carry_one_block", EST.test_one_block_estimates_carry_their_errors_through_the_swaps),
        ("probe_loop", PROBE.test_probe_loop_swaps_follow_the_determinant_identity),
        ("probe_identity", PROBE.test_identity_rotation_draws_a_fresh_probe_and_counts_toward_the_cap),
        ("probe_unbiased", lambda: PROBE.test_probe_estimate_is_unbiased_over_the_probe_streams(_kahan_state())),
    ]
    for name, fn in checks:
        try:
            with np.errstate(all="ignore"):
                fn()
        except Exception:          # an assertion or a crash both count as caught
            return name
    return None


MUTANTS = [
    # reflector
    ("householder", "tau = (beta - alpha) / beta", "tau = (beta + alpha) / beta"),
    ("householder", "v[1:] = x[1:] / (alpha - beta)", "v[1:] = x[1:] / (alpha + beta)"),
    ("householder", "beta = -math.copysign(", "beta = math.copysign("),
    # QRCP on the sketch
    ("qrcp_sketch", "r = np.sum(B[j:, j:] ** 2, axis=0)", "r = np.sum(B[:, j:] ** 2, axis=0)"),
    ("qrcp_sketch", "s = int(cands[np.argmin(perm[j + cands])])", "s = int(cands[np.argmax(perm[j + cands])])"),
    ("qrcp_sketch", "B[j:, j + 1:] -= tau * np.outer(v, w)", "B[j:, j + 1:] -= np.outer(v, w)"),
    ("qrcp_sketch", "perm[[j, j + s]] = perm[[j + s, j]]", "perm[[j, j + s]] = perm[[j, j + s]]"),
    ("qrcp_sketch", "margins[j] = (rmax - rest.max()) / rmax", "margins[j] = (rmax - rest.min()) / rmax"),
    ("qrcp_sketch", "margins[j] = (rmax - rest.max()) / rmax", "margins[j] = (rmax - rest.max()) / rest.max()"),
    # Householder QR of the panel
    ("householder_qr", "W[j:, j + 1:] -= tau * np.outer(v, v @ W[j:, j + 1:])",
     "W[j:, j + 1:] -= 0.5 * tau * np.outer(v, v @ W[j:, j + 1:])"),
    ("householder_qr", "for j in range(c - 1, -1, -1):", "for j in range(c):"),
    ("householder_qr", "return Q * d, R * d[:, None]", "return Q, R * d[:, None]"),
    # projection and residual norms
    ("factor_leading_set", "R = W[:, perm]", "R = W[:, np.argsort(perm)]"),
    ("residual_norms", "E = np.asarray(A[:, c], dtype=np.float64) - Q1 @ W[:, c]",
     "E = np.asarray(A[:, c], dtype=np.float64) - Q1 @ W[:, c[::-1]]"),
    # SRQR test
    ("srqr_rho", "Rt[:l, l] = a", "Rt[:l, l] = 0.0 * a"),
    ("srqr_rho", "Rt[l, l] = alpha", "Rt[l, l] = 1.0"),
    ("srqr_rho", "np.sum(X * X, axis=1)", "np.sum(X * X, axis=0)"),
    ("back_substitute", "x[i] = (b[i] - U[i, i + 1:] @ x[i + 1:]) / U[i, i]",
     "x[i] = (b[i] + U[i, i + 1:] @ x[i + 1:]) / U[i, i]"),
    ("ffsrqr", "S = S[:istar] + S[istar + 1:] + [jstar]", "S = S[:istar] + S[istar + 1:] + [S[istar]]"),
    ("ffsrqr", "if g2 <= g:", "if True:"),
    # flip-flop LQ
    ("flip_flop_lq", "V[np.asarray(perm), :] = Qh", "V[:, :] = Qh"),
    ("flip_flop_lq", "L = Rh.T", "L = Rh"),
    # Jacobi
    ("jacobi_svd", "new_p = c * cp - s * cq", "new_p = c * cp + s * cq"),
    ("jacobi_svd", "zeta = (b - a) / (2.0 * g)", "zeta = (a - b) / (2.0 * g)"),
    ("jacobi_svd", "for q in range(p + 1, n):", "for q in range(p + 2, n):"),
    # bfloat16 sketch mode
    ("round_bf16", "return np.rint(x / q) * q", "return np.floor(x / q + 0.5) * q"),
    ("round_bf16", "np.maximum(e, -125) - 8", "np.maximum(e, -125) - 7"),
    ("round_bf16", "np.maximum(e, -125) - 8", "e - 8"),
    ("sketch", "return round_bf16(Omega) @ round_bf16(A)", "return round_bf16(Omega) @ A"),
    # Algorithm 9 completion and the j* margin
    ("alg9", "tmp = A @ res.V", "tmp = A @ res.V[:, ::-1] * 1.0 + 0.0 * A @ res.V"),
    ("alg9", "U = Qt @ UR[:, :k]", "U = Qt[:, :k]"),
    ("alg9", "Vk = res.V @ VR[:, :k]", "Vk = res.V @ UR[:, :k]"),
    ("residual_margin", "return float((g2[-1] - g2[-2]) / g2[-1])", "return float((g2[-1] - g2[0]) / g2[-1])"),
    # the random g2 estimate
    ("g2_probe_estimate", "return abs(alpha) / math.sqrt(d) *", "return abs(alpha) / d *"),
    ("g2_probe_estimate", "Y = Om @ upper_inverse(Rt).T", "Y = Om @ upper_inverse(Rt)"),
    ("g2_probe_estimate", "Rt[:l, l] = a", "Rt[:l, l] = 0.0 * a"),
    ("probe_omega", "return _omega(seed, d, l + 1, stream=q)", "return _omega(seed, d, l + 1, stream=q - 1)"),
    ("ffsrqr", "istar = int(np.argmax(est))", "istar = int(np.argmax(est[:l]))"),
    # the sample-estimated residual norms
    ("trqrcp_pivots", "B[:, rest] = B[:, rest] - B[:, piv] @ X", "B[:, rest] = B[:, rest] - 0.0 * (B[:, piv] @ X)"),
    ("sample_update", "out[:, c] = B[:, c] - B[:, S] @ back_substitute(R11, W[:, c])",
     "out[:, c] = B[:, c] + B[:, S] @ back_substitute(R11, W[:, c])"),
    ("row_l1", "return Qx[:, -1] @ A", "return Qx[:, 0] @ A"),
    ("ffsrqr", "r = r - row_l1(Af, S, jstar) ** 2", "r = r + row_l1(Af, S, jstar) ** 2"),
    ("ffsrqr", "r[removed] = row[removed] ** 2", "r[removed] = r[removed]"),
]


def test_unmutated_oracle_passes_every_pin():
    assert _pins() is None


@pytest.mark.parametrize("fname,old,new", MUTANTS, ids=[f"{m[0]}-{i}" for i, m in enumerate(MUTANTS)])
def test_mutant_is_caught(monkeypatch, fname, old, new):
    orig = getattr(MOD, fname)
    mut = _mutant(orig, old, new)
    monkeypatch.setattr(MOD, fname, mut)
    if hasattr(oracle, fname) and getattr(oracle, fname) is orig:
        monkeypatch.setattr(oracle, fname, mut)
    caught = _pins()
    assert caught is not None, f"no pin caught the mutant {fname}: {old!r} -> {new!r}"
