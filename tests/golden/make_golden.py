"""Writes the stored expected values under tests/golden/ by calling only the
oracle (and the seeded input generators).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402


def kahan(n, c=0.285, pert=1e-10):
    s = np.sqrt(1 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.triu(-c * np.ones((n, n)), 1) + np.eye(n))
    return K @ np.diag(1 - pert * np.arange(n))


def record(res, k):
    return {
        "l": int(res.l),
        "pivots": [int(x) for x in res.perm[: res.l]],
        "sigma": [float(x) for x in res.sigma],
        "g2": float(res.g2),
        "alpha": float(res.alpha),
        "jstar": int(res.jstar),
        "swaps": int(res.swaps),
        "flags": int(res.flags),
        "min_margin": float(res.margins.min()),
        "k": int(k),
    }


def main():
    out = {}
    w = synth.WORKLOADS["small_fp64"]
    A = synth.make_workload("small_fp64")
    out["small_fp64"] = record(oracle.ffsrqr(A, w.k, w.p, w.seed), w.k)
    K = np.vstack([kahan(80), np.zeros((10, 80))])
    out["kahan80_k40_p0_seed0"] = record(oracle.ffsrqr(K, 40, 0, 0), 40)
    om = oracle.omega(0, 4, 6)
    out["omega_seed0_4x6"] = [[float(x) for x in row] for row in om]
    with open(os.path.join(HERE, "oracle_values.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
