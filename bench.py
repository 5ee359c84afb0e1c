"""Throughput of the AVU-GSR LSQR hot path on one MI355X.

A step is one LSQR iteration (aprod 1, aprod 2 with its tail pass, the
x / w / variance update and the scalar recurrences) on the one-GPU share:
1,000,000 stars with U[50,90] observations each (m ~ 7.0e7 rows,
~1.7e9 nonzeros), 3 x 40,000 attitude, 200 instrumental and 1 global
unknown, FP64 coefficients N(0,1), plain (unscaled) FP64 LSQR with damp 0.

Prints one JSON line: iterations/s, the roofline of the dominant product
kernel (HIP-event timing inside the timed region), and the CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per row / per star (FP64 values, int32 indices)
APROD1_B_ROW = 192 + 4 + 24 + 16  # coefficients, attitude start, 6 instr columns, y read+write
APROD2_B_ROW = 192 + 4 + 24 + 8  # coefficients, attitude start, 6 instr columns, u read
APROD2_B_STAR = 80  # astrometric x read+write


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("aprod.hip", "device_common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2503_22863_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(f"{kernel}:{workload}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(full_m: int, budget_s: float = 15.0):
    """The oracle, as it stands, on a bounded sample: a 20,000-star system of the same
    construction (same attitude / instrumental sizes, same distributions)."""
    import numpy as np

    import gsr_synth
    import oracle

    g = gsr_synth.share_1m(seed=2505, n_stars=20_000)
    o = oracle.OSystem(g)
    b = oracle.known_terms(o, g.x_true, g.noise)
    t = time.perf_counter()
    oracle.lsqr(o, b, atol=0, btol=0, itmax=1, precond=False)
    t1 = time.perf_counter() - t
    k = max(2, min(50, int(budget_s / max(t1, 1e-3))))
    t = time.perf_counter()
    r = oracle.lsqr(o, b, atol=0, btol=0, itmax=k, precond=False)
    tk = time.perf_counter() - t
    per_it = (tk - t1) / max(1, k - 1)  # remove the one-time setup
    per_it_full = per_it * full_m / g.dims.m
    del np
    return {"value": 1.0 / per_it_full, "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{g.dims.n_stars} stars ({g.dims.m} rows) of the same construction, "
                      f"{r['itn']} unscaled LSQR iterations in {tk:.1f} s, scaled by rows to m={full_m}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--stars", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU row split is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import gsr_synth
    import paper_2503_22863_amd as gsr

    torch.cuda.set_device(0)
    t = time.time()
    g = gsr_synth.share_1m(n_stars=args.stars)
    m, n, ns = g.dims.m, g.dims.n, g.dims.n_stars
    print(f"# generated m={m} n={n} in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    S = gsr.System.from_generated(g)
    xt = torch.from_numpy(g.x_true).cuda()
    b = torch.from_numpy(g.noise).cuda()
    del g
    S.aprod1(xt, b, scale=1.0)  # b = A x_true + noise
    torch.cuda.synchronize()

    K, W = args.steps, args.warmup
    S.lsqr_begin(b, atol=0.0, btol=0.0, itmax=W + K + 1, precond=False)
    S.lsqr_iterate(W)
    st = S.lsqr_status()
    assert st["itn"] == W, st
    S.timing_enable(True)
    S.timing_get()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.lsqr_iterate(K)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    tm = S.timing_get()
    S.timing_enable(False)
    st = S.lsqr_status()
    if st["itn"] != W + K:
        raise RuntimeError(f"solve stopped early (itn={st['itn']}, istop={st['istop']}): timed steps not all real")
    S.lsqr_end(want_var=False)

    a1 = tm["aprod1_ms"] / max(1, tm["aprod1_n"])
    a2 = tm["aprod2_ms"] / max(1, tm["aprod2_n"])
    bytes1 = APROD1_B_ROW * m
    bytes2 = APROD2_B_ROW * m + APROD2_B_STAR * ns
    if a2 >= a1:
        kname, ms, by = "k_aprod2", a2, bytes2
    else:
        kname, ms, by = "k_aprod1", a1, bytes1
    achieved = by / (ms * 1e-3) / 1e9
    workload = "share_1m"
    traffic = load_traffic(kname, workload)
    out = {
        "metric": "LSQR iterations/s (FP64, one-GPU share)",
        "value": K / T,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * T / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{workload}: {ns} stars x U[50,90] obs (m={m}), 3x40000 attitude, 200 instr, "
                               f"1 global (n={n}); unscaled FP64 LSQR, damp 0, variances on",
                   "global_batch": m, "seq_len": None, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": by, "avg_ms": ms},
        "aprod": {"aprod1_ms": a1, "aprod1_gbs": bytes1 / (a1 * 1e-3) / 1e9,
                  "aprod2_ms": a2, "aprod2_gbs": bytes2 / (a2 * 1e-3) / 1e9,
                  "tail_ms": tm["tail_ms"] / max(1, tm["tail_n"]),
                  "update_ms": tm["update_ms"] / max(1, tm["update_n"]),
                  "aprod_pair_frac": (bytes1 + bytes2) / ((a1 + a2) * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    S.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
