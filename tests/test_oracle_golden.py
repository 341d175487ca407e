"""The oracle reproduces the values stored under tests/golden/ (written by
tests/golden/make_golden.py, which calls only the oracle).  Guards against
silent drift of the oracle's arithmetic."""
import json
import os

import numpy as np

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


def test_small_fp64_golden():
    g = GOLD["small_fp64"]
    w = synth.WORKLOADS["small_fp64"]
    r = oracle.ffsrqr(synth.make_workload("small_fp64"), w.k, w.p, w.seed)
    assert list(r.perm[: r.l]) == g["pivots"]
    assert np.max(np.abs(r.sigma - g["sigma"]) / np.asarray(g["sigma"])) < 1e-12
    assert abs(r.g2 - g["g2"]) < 1e-10 * g["g2"] and r.swaps == g["swaps"]


def test_kahan_golden():
    from test_oracle_path import kahan
    g = GOLD["kahan80_k40_p0_seed0"]
    r = oracle.ffsrqr(np.vstack([kahan(80), np.zeros((10, 80))]), 40, 0, 0)
    assert list(r.perm[: r.l]) == g["pivots"] and r.swaps == g["swaps"]
    assert np.max(np.abs(r.sigma - g["sigma"]) / np.asarray(g["sigma"])) < 1e-10


def test_omega_golden():
    assert np.array_equal(oracle.omega(0, 4, 6), np.asarray(GOLD["omega_seed0_4x6"]))
