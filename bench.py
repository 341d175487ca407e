#!/usr/bin/env python3
"""Throughput of the Flip-Flop SRQR hot path on one MI355X.

One step = one whole ffsrqr_factor solve (sketch, QRCP on the sketch,
Householder QR of the pivoted columns, projection, SRQR test, flip-flop LQ,
singular values of L) on the "mid" workload:
  A = U_r diag(exp(-j/50)) V_r^T + 1e-6 G,  16384 x 8192, r = 1024,
  k = 256, p = 16 (l = 272), sketch seed 0, FP64 (default) or FP32.
A is synthetic (seeded), generated on the host and resident in HBM before the
timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision fp64|fp32]
                  [--no-cpu-baseline] [--no-second-form]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK = {"fp64": 78.6, "fp32": 157.3}  # MI355X dense MFMA, TFLOP/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_solves(ff, torch, A, w, steps, warmup, mixed=False):
    for _ in range(warmup):
        ff.factor(A, w.k, w.p, w.seed, mixed=mixed)
    ff.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = ff.factor(A, w.k, w.p, w.seed, mixed=mixed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ff.profile_read()
    ff.profile_enable(False)
    return out, (t1 - t0), prof


def gemm_traffic(w, prec):
    """HBM bytes per GEMM launch from the committed rocprofv3 counter summary
    (profiles/gemm_tall_mid_fp64_pmc.json), or None when the summary is for
    another kernel or workload, or the kernel source has changed since."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "gemm_tall_mid_fp64_pmc.json")
    try:
        with open(path) as f:
            d = json.load(f)
        with open(os.path.join(here, d["source_file"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if sha != d.get("source_sha256") or prec != "fp64" or w.name != "mid":
        return None
    return int(d["bytes_per_launch"])


def mixed_roofline(prof, w):
    # mixed form: the sketch is bound by HBM (A read once in FP32, Omega^T in
    # BF16, B written in FP32), the split-BF16 projection by BF16 MFMA (three
    # products of 2 l m n flops each)
    sk_ms, sk_n = prof["sketch"]
    pj_ms, pj_n = prof["project"]
    if sk_n == 0 or pj_n == 0:
        return None
    sk_s = sk_ms / sk_n / 1e3
    pj_s = pj_ms / pj_n / 1e3
    sk_bytes = 4.0 * w.m * w.n + 2.0 * w.m * w.l + 4.0 * w.l * w.n
    pj_flop = 3 * 2.0 * w.l * w.m * w.n
    pj = pj_flop / pj_s / 1e12
    sk = sk_bytes / sk_s / 1e9
    return {"bound": "mfma", "achieved": round(pj, 3), "peak": 2500.0, "unit": "TFLOP/s",
            "frac": round(pj / 2500.0, 4), "traffic": None, "kernel": "gemm_bf16_kernel<3, *> (split-BF16 projection)",
            "flop_per_launch": pj_flop, "avg_launch_ms": round(pj_s * 1e3, 4), "launches": pj_n,
            "sketch": {"bound": "hbm", "achieved": round(sk, 1), "peak": 8000.0, "unit": "GB/s",
                       "frac": round(sk / 8000.0, 4), "bytes_per_launch": sk_bytes,
                       "avg_launch_ms": round(sk_s * 1e3, 4), "kernel": "gemm_bf16_kernel<1, *> (BF16 sketch)"}}


def gemm_roofline(prof, w, prec):
    if prec == "mixed":
        return mixed_roofline(prof, w)
    # the sketch (B = Omega A) and the projection (W = Q1^T A) are launches of
    # the same MFMA GEMM (for l <= 288 the tall-tile kernel, K split over two
    # halves plus the fixed-order sum of the halves, both inside the timed
    # interval); each performs 2 l m n flops
    ms = prof["sketch"][0] + prof["project"][0]
    n_launch = prof["sketch"][1] + prof["project"][1]
    if n_launch == 0:
        return None
    avg_s = ms / n_launch / 1e3
    flop = 2.0 * w.l * w.m * w.n
    achieved = flop / avg_s / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[prec], 4), "traffic": gemm_traffic(w, prec),
            "kernel": (f"{'gemm_tall8_kernel' if w.l > 112 else 'gemm_tall_kernel'}"
                       f"<{'double' if prec == 'fp64' else 'float'}, {(w.l + 15) // 16}> + splitk_reduce"
                       if w.l <= 288 else f"gemm_tn_kernel<{'double' if prec == 'fp64' else 'float'}>"),
            "flop_per_launch": flop, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": n_launch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32", "mixed"], default="fp64")
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-second-form", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1803_01982_amd as ff

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ff.load()
    w = synth.WORKLOADS[args.workload]
    log(f"generating {args.workload}: {w.m}x{w.n} k={w.k} p={w.p}")
    t = time.perf_counter()
    A = synth.make_workload(args.workload)
    log(f"generated in {time.perf_counter() - t:.1f} s")
    dt = torch.float64 if args.precision == "fp64" else torch.float32
    Ad = ff.fortran(torch.from_numpy(A).to(dt).cuda())
    torch.cuda.synchronize()

    log(f"{args.precision}: warmup {args.warmup}, timing {args.steps} solves")
    out, secs, prof = timed_solves(ff, torch, Ad, w, args.steps, args.warmup, mixed=args.precision == "mixed")
    value = args.steps / secs
    log(f"{args.precision}: {secs / args.steps * 1e3:.3f} ms per solve")
    stages = {k: {"ms_per_solve": round(v[0] / args.steps, 4), "launches_per_solve": v[1] / args.steps}
              for k, v in prof.items()}

    result = {
        "metric": "FF-SRQR solves/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic (seeded prescribed-spectrum matrix, generated on the host, resident in HBM)",
        "config": {"workload": f"{args.workload}: A = U_r diag(exp(-j/50)) V_r^T + 1e-6 G, r = 1024",
                   "m": w.m, "n": w.n, "k": w.k, "p": w.p, "l": w.l, "seed": w.seed,
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": gemm_roofline(prof, w, args.precision),
        "stages": stages,
        "info": out.info,
    }

    sig_gpu = out.sigma.cpu().numpy()
    perm_gpu = out.perm.cpu().numpy()

    if not args.no_second_form:
        other = "fp32" if args.precision == "fp64" else "fp64"
        dt2 = torch.float32 if other == "fp32" else torch.float64
        A2 = ff.fortran(torch.from_numpy(A).to(dt2).cuda())
        log(f"{other}: timing {args.steps} solves")
        out2, secs2, prof2 = timed_solves(ff, torch, A2, w, args.steps, args.warmup)
        del A2
        result["second_form"] = {
            "precision": other, "value": round(args.steps / secs2, 4), "unit": "solves/s",
            "ms_per_step": round(secs2 / args.steps * 1e3, 4),
            "roofline": gemm_roofline(prof2, w, other),
            "sigma_rel_err_vs_first_form": float(np.max(np.abs(out2.sigma.cpu().numpy() - sig_gpu) / sig_gpu)),
            "pivots_match_first_form": bool(np.array_equal(out2.perm.cpu().numpy()[: w.l], perm_gpu[: w.l])),
            "stages": {k: {"ms_per_solve": round(v[0] / args.steps, 4)} for k, v in prof2.items()},
        }

    if not args.no_cpu_baseline:
        import oracle
        from oracle import diagnostics as dg
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:  # pragma: no cover - threadpoolctl missing
            cores = int(os.environ.get("OMP_NUM_THREADS", "1"))
        A64 = A if args.precision == "fp64" else A.astype(np.float32).astype(np.float64)
        log("oracle: one full solve on the host")
        t = time.perf_counter()
        ref = oracle.ffsrqr(A64, w.k, w.p, w.seed)
        osecs = time.perf_counter() - t
        log(f"oracle: {osecs:.1f} s")
        result["cpu_baseline"] = {"value": round(1.0 / osecs, 6), "unit": "solves/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"one full FP64 oracle solve of the {args.workload} workload "
                                            f"({w.m}x{w.n}, l={w.l}); {osecs:.1f} s"}
        Q, L, V = (out.Q.cpu().numpy().astype(np.float64), out.L.cpu().numpy().astype(np.float64),
                   out.V.cpu().numpy().astype(np.float64))
        res = dg.residual_fro(A64, Q, L, V)
        res_ref = dg.residual_fro(A64, ref.Q, ref.L, ref.V)
        result["parity_vs_oracle"] = {
            "pivots_match": bool(np.array_equal(perm_gpu, ref.perm)),
            "sigma_max_rel_err": float(np.max(np.abs(sig_gpu - ref.sigma) / ref.sigma)),
            "residual_rel_diff": float(abs(res - res_ref) / res_ref),
            "residual_fro": res, "oracle_min_margin": float(ref.margins.min()),
            "swaps": [int(out.info["swaps"]), int(ref.swaps)],
        }

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
