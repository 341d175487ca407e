#!/usr/bin/env python3
"""Throughput of the Flip-Flop SRQR hot path on one MI355X.

One step = one whole ffsrqr_factor solve (sketch, QRCP on the sketch,
Householder QR of the pivoted columns, projection, SRQR test, flip-flop LQ,
singular values of L).  Default workload, the mixed-precision configuration:
  A = U_r diag(sigma) V_r^T + 1e-5 G, 32768 x 16384, r = 1024,
  sigma_j = 1 (j <= 8), 10^(-3 (j - 8) / 1000) (8 < j <= 1024),
  FP32 storage, k = 512, p = 32 (l = 544), sketch seed 0,
  BF16 sketch, split-BF16 projection, FP64 l x l steps (FFSRQR_MIXED).
The same matrix is also solved with the plain FP64 form (second_form), and
the FP64 "mid" workload (16384 x 8192, l = 272) is reported beside it.  A is
synthetic (seeded), generated on the host and resident in HBM before the
timed region.  Every solve is timed on its own (ffsrqr_factor returns after
its stream has finished): value = solves / total time of the timed solves,
p50 / p99 from the per-solve times.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload large|mid|...]
                  [--precision mixed|fp64|fp32] [--no-cpu-baseline]
                  [--no-second-form] [--cpu-baseline-full]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # MI355X dense MFMA, TFLOP/s
HBM_PEAK = 8000.0  # GB/s
DTYPE = {"fp64": "f64", "fp32": "f32", "mixed": "bf16"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_solves(ff, torch, A, w, steps, warmup, mixed=False, **opts):
    """Warm up, then time `steps` solves one by one (each call returns after
    the stream is done).  Returns (last output, per-solve seconds, step
    accounting accumulated over the timed solves).  opts: options of the
    SRQR test and the pivot selection (block, g2_probe, est_norms)."""
    for _ in range(warmup):
        ff.factor(A, w.k, w.p, w.seed, mixed=mixed, **opts)
    torch.cuda.synchronize()
    ff.profile_enable(True)
    times = []
    out = None
    for _ in range(steps):
        t0 = time.perf_counter()
        out = ff.factor(A, w.k, w.p, w.seed, mixed=mixed, **opts)
        times.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    prof = ff.profile_read()
    ff.profile_enable(False)
    return out, np.array(times), prof


def latency(times):
    return {"p50_ms": round(float(np.percentile(times, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(times, 99)) * 1e3, 4),
            "mean_ms": round(float(np.mean(times)) * 1e3, 4),
            "min_ms": round(float(np.min(times)) * 1e3, 4), "solves": int(times.size)}


def traffic_from_profile(name, source_rel):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (profiles/<name>.json), or None when it is missing or the kernel
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", name + ".json")
    try:
        with open(path) as f:
            d = json.load(f)
        with open(os.path.join(HERE, d["source_file"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if d.get("source_file") != source_rel or sha != d.get("source_sha256"):
        return None
    return int(d["bytes_per_launch"])


def roofline(prof, w, prec):
    """Roofline of the dominant kernel, measured live: the step accounting
    records HIP events on the solve's stream around each GEMM step."""
    sk_ms, sk_n = prof["sketch"]
    pj_ms, pj_n = prof["project"]
    if sk_n == 0 or pj_n == 0:
        return None
    sk_s, pj_s = sk_ms / sk_n / 1e3, pj_ms / pj_n / 1e3
    flop = 2.0 * w.l * w.m * w.n
    if prec == "mixed":
        # the split-BF16 projection (three BF16 products) is MFMA-bound; the
        # BF16 sketch reads A once (FP32) and is HBM-bound
        pj_flop = 3 * flop
        pj = pj_flop / pj_s / 1e12
        sk_bytes = 4.0 * w.m * w.n + 2.0 * w.m * w.l + 4.0 * w.l * w.n
        sk = sk_bytes / sk_s / 1e9
        return {"bound": "mfma", "achieved": round(pj, 2), "peak": PEAK["bf16"], "unit": "TFLOP/s",
                "frac": round(pj / PEAK["bf16"], 4),
                "traffic": traffic_from_profile("gemm_bf16_split_large_pmc", "paper_1803_01982_amd/csrc/gemm_bf16.hip"),
                "kernel": ("gemm_bf16_xl_kernel<3, 17, 2> (split-BF16 projection; the timed interval also holds "
                           "split_bf16_kernel and splitk_reduce_f32)"),
                "flop_per_launch": pj_flop, "avg_launch_ms": round(pj_s * 1e3, 4), "launches": int(pj_n),
                "sketch": {"bound": "hbm", "achieved": round(sk, 1), "peak": HBM_PEAK, "unit": "GB/s",
                           "frac": round(sk / HBM_PEAK, 4), "bytes_per_launch": sk_bytes,
                           "avg_launch_ms": round(sk_s * 1e3, 4), "kernel": ("gemm_bf16_xl_kernel<1, 17, 2> (BF16 sketch; the timed interval also "
                                      "holds splitk_reduce_f32)")}}
    avg_s = (sk_ms + pj_ms) / (sk_n + pj_n) / 1e3
    achieved = flop / avg_s / 1e12
    kern = "gemm_tall8_kernel" if w.l > 112 else "gemm_tall_kernel"
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[prec], 4),
            "traffic": (traffic_from_profile(f"gemm_tall_{w.name}_{prec}_pmc", "paper_1803_01982_amd/csrc/gemm.hip")),
            "kernel": f"{kern}<{'double' if prec == 'fp64' else 'float'}, *> (sketch and projection)",
            "flop_per_launch": flop, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": int(sk_n + pj_n)}


def stages(prof, steps):
    return {k: round(v[0] / steps, 4) for k, v in prof.items()}


def host_cpu():
    model, cores = platform.processor() or "unknown", os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return model, cores


def oracle_flops(w):
    # algorithmic work of one solve (leading terms): the two GEMM passes
    # 4 l m n, the panel QR 2 m l^2, the flip-flop QR 2 n l^2 and the
    # QRCP on the l x n sketch 2 l^2 n
    return 4.0 * w.l * w.m * w.n + 2.0 * w.m * w.l ** 2 + 4.0 * w.n * w.l ** 2


def cpu_baseline(w, full):
    """The oracle (numpy FP64, as it stands) on the host's cores, on a bounded
    sample of the workload: the same spectrum, k and p at an eighth of m and
    n (4096 x 2048 for the default workload, so the same l).  The sample's
    time splits into the SVD of the l x l factor L, whose cost depends on l
    alone and carries over unscaled (timed on its own on the sample's L), and
    the rest, scaled to the workload by the ratio of algorithmic work."""
    import synth
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    name = {"large": "large_s"}.get(w.name, w.name)
    ws = synth.WORKLOADS[name]
    A = synth.make_workload(name)
    if w.name == "large":
        A = A.astype(np.float32).astype(np.float64)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    runs = 3 if full else 1
    secs = []
    ref = None
    for _ in range(runs):
        t = time.perf_counter()
        ref = oracle.ffsrqr(A, ws.k, ws.p, ws.seed, storage="fp64")
        secs.append(time.perf_counter() - t)
        log(f"oracle {name}: {secs[-1]:.1f} s ({threads} threads)")
    t = time.perf_counter()
    oracle.jacobi_svd(ref.L)
    tj = time.perf_counter() - t
    log(f"oracle {name}: SVD of L alone {tj:.1f} s")
    scale = oracle_flops(w) / oracle_flops(ws)
    med = float(np.median(secs))
    est = tj + max(med - tj, 0.0) * scale
    one = None
    if full:
        with threadpool_limits(limits=1):
            t = time.perf_counter()
            oracle.ffsrqr(A, ws.k, ws.p, ws.seed, storage="fp64")
            one = time.perf_counter() - t
        log(f"oracle {name}: {one:.1f} s (1 thread)")
    model, ncpu = host_cpu()
    res = {"value": round(1.0 / est, 6), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": (f"oracle (numpy FP64) solve of {name} ({ws.m}x{ws.n}, k={ws.k}, p={ws.p}, the same l), "
                      f"median of {runs} run(s) {med:.1f} s with {threads} BLAS threads, of which the SVD of L "
                      f"(timed alone) {tj:.1f} s carries over unscaled and the rest is scaled by the "
                      f"algorithmic-work ratio {scale:.2f}: {est:.1f} s per {w.name} solve"),
           "host_cpu": model, "host_cpus_visible": ncpu, "sample_seconds": [round(x, 2) for x in secs],
           "svd_of_L_seconds": round(tj, 2), "estimated_seconds_per_solve": round(est, 2)}
    if one is not None:
        est1 = tj + max(one - tj, 0.0) * scale
        res["one_thread_value"] = round(1.0 / est1, 6)
        res["one_thread_sample_seconds"] = round(one, 2)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64", "fp32"], default="mixed")
    ap.add_argument("--workload", default="large")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="median of 3 oracle runs plus a 1-thread run (several minutes)")
    ap.add_argument("--no-second-form", action="store_true")
    ap.add_argument("--no-mid", action="store_true")
    # options of the first form (the defaults are the headline configuration)
    ap.add_argument("--block", type=int, default=0, help="Algorithm 2's blocked selection, block size")
    ap.add_argument("--g2-probe", type=int, default=0, help="Algorithm 4's random g2 estimate, probe rows")
    ap.add_argument("--est-norms", action="store_true", help="Algorithm 4's sample-estimated residual norms")
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
    prec = args.precision
    log(f"generating {args.workload}: {w.m}x{w.n} k={w.k} p={w.p}")
    t = time.perf_counter()
    A = synth.make_workload(args.workload)
    log(f"generated in {time.perf_counter() - t:.1f} s")
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = ff.fortran(torch.from_numpy(A).to(dt).cuda())
    torch.cuda.synchronize()

    log(f"{prec}: warmup {args.warmup}, timing {args.steps} solves")
    sopts = {"block": args.block, "g2_probe": args.g2_probe, "est_norms": args.est_norms}
    out, times, prof = timed_solves(ff, torch, Ad, w, args.steps, args.warmup, mixed=prec == "mixed", **sopts)
    secs = float(np.sum(times))
    log(f"{prec}: {secs / args.steps * 1e3:.3f} ms per solve")
    del Ad

    desc = {"large": "A = U_r diag(sigma) V_r^T + 1e-5 G, sigma_j = 1 (j <= 8), 10^(-3 (j - 8) / 1000) "
                     "(j <= r = 1024), FP32 storage",
            "mid": "A = U_r diag(exp(-j/50)) V_r^T + 1e-6 G, r = 1024"}.get(w.name, w.spectrum)
    result = {
        "metric": "FF-SRQR solves/s",
        "value": round(args.steps / secs, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic (seeded prescribed-spectrum matrix, generated on the host, resident in HBM)",
        "config": {"workload": f"{w.name} {w.m}x{w.n}: {desc}", "m": w.m, "n": w.n, "k": w.k, "p": w.p,
                   "l": w.l, "seed": w.seed,
                   "form": {"mixed": "BF16 sketch, split-BF16 projection (FP32 accumulation), FP32 storage, "
                                     "FP64 l x l steps",
                            "fp64": "plain FP64", "fp32": "FP32 storage and GEMMs, FP64 l x l steps"}[prec],
                   "parallelism": "single GPU"},
        "latency": latency(times),
        "roofline": roofline(prof, w, prec),
        "stages_ms": stages(prof, args.steps),
        "info": {k: out.info[k] for k in ("l", "swaps", "flags", "g2", "jstar", "jstar_margin", "min_margin",
                                          "jacobi_sweeps")},
    }
    if args.block or args.g2_probe or args.est_norms:
        result["config"]["srqr_options"] = sopts
        result["info"]["probes"] = out.info["probes"]
    sig_gpu = out.sigma.cpu().numpy()
    perm_gpu = out.perm.cpu().numpy()
    result["accuracy"] = {"sigma_rel_err_vs_prescribed_spectrum_j<=k":
                          float(np.max(np.abs(sig_gpu[: w.k] - w.sigma()[: w.k]) / w.sigma()[: w.k]))}

    if not args.no_second_form and prec != "fp64":
        # the same FP32 bytes, held in FP64
        A2 = ff.fortran(torch.from_numpy(A).to(torch.float32).to(torch.float64).cuda())
        log(f"fp64: timing {args.steps} solves")
        out2, times2, prof2 = timed_solves(ff, torch, A2, w, args.steps, args.warmup)
        del A2
        secs2 = float(np.sum(times2))
        sig2 = out2.sigma.cpu().numpy()
        result["second_form"] = {
            "form": "plain FP64 on the same matrix", "value": round(args.steps / secs2, 4), "unit": "solves/s",
            "ms_per_step": round(secs2 / args.steps * 1e3, 4), "latency": latency(times2),
            "roofline": roofline(prof2, w, "fp64"), "stages_ms": stages(prof2, args.steps),
            "speedup_of_first_form": round(secs2 / secs, 3),
            "first_form_sigma_rel_err_vs_fp64_j<=k": float(np.max(np.abs(sig_gpu[: w.k] - sig2[: w.k]) / sig2[: w.k])),
            "pivots_match_first_form": bool(np.array_equal(out2.perm.cpu().numpy()[: w.l], perm_gpu[: w.l])),
            "swaps": int(out2.info["swaps"]),
        }

    if not args.no_mid and w.name != "mid":
        wm = synth.WORKLOADS["mid"]
        Am = ff.fortran(torch.from_numpy(synth.make_workload("mid")).cuda())
        log("mid fp64: timing")
        outm, tm, profm = timed_solves(ff, torch, Am, wm, args.steps, args.warmup)
        del Am
        result["mid_fp64"] = {"workload": "mid 16384x8192, l = 272, FP64", "value": round(tm.size / float(np.sum(tm)), 4),
                              "unit": "solves/s", "latency": latency(tm), "roofline": roofline(profm, wm, "fp64"),
                              "stages_ms": stages(profm, tm.size)}

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_baseline_full)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
