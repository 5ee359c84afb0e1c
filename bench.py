"""Throughput of the AVU-GSR LSQR hot path on one MI355X.

A step is one LSQR iteration (both products A v and A^T u in one pass over
the rows regrouped by attitude window, the star-segment reduction, the tail
pass with the scalar recurrences, the x / w / variance update) on the one-GPU
share: 1,000,000 stars with U[50,90] observations each (m ~ 7.0e7 rows,
~1.7e9 nonzeros), 3 x 40,000 attitude, 200 instrumental and 1 global
unknown, FP64 coefficients N(0,1), plain (unscaled) FP64 LSQR with damp 0.
The caller places its rows in the regrouped order at load time, so the
library holds no copy of A.

Prints one JSON line: iterations/s (graph replay on, as shipped), the
roofline of the dominant kernel (HIP events around every kernel over a
separate run of iterations right after the timed region; besides the HBM
peak, its rate against the memory probe's stream of the same reads with the
pass's two write streams, measured first in a child process), the same for
the 3e6-star share with the covariances of 4,000 unknowns, the time to 1e-10
of the FP32 forms and of the warm start, and the CPU oracle timed on a
bounded sample of the same workload.
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
# Algorithmic bytes of the fused row pass (one per LSQR iteration), FP64 values and
# int32 indices: per row the 24 coefficients, the attitude start, the 6 instrumental
# columns, u read and u written; per star the 5 astrometric v read and the 5 raw
# column sums written.
FUSED_B_ROW = 192 + 4 + 24 + 8 + 8
FUSED_B_STAR = 40 + 40
# the same with FP32 values (the FP32 forms)
FUSED_B_ROW_F32 = 96 + 4 + 24 + 8 + 8
# The pass over the copy regrouped by attitude window: per row the 24 coefficients,
# the 12-byte row record, u read and u written; per 64-row tile the star of its
# first row; per star segment the star's 5 v read and the 5 partial sums written;
# per workgroup its attitude window of sums written.
FBLK_B_ROW = 192 + 12 + 8 + 8
FBLK_B_ROW_F32 = 96 + 12 + 8 + 8
FBLK_B_TILE = 4
FBLK_B_SEG = 40 + 40
# The standalone products on the caller's rows: aprod 1 reads the coefficients, the
# attitude start and the 6 instrumental columns and reads and writes y; aprod 2
# reads the same and y, and per star reads and writes the 5 astrometric x.
APROD1_B_ROW = 192 + 4 + 24 + 8 + 8
APROD2_B_ROW = 192 + 4 + 24 + 8
APROD2_B_STAR = 40 + 40


def pass_bytes(info, m, ns, f32=False):
    """(kernel, algorithmic bytes per launch) of the iteration's row pass."""
    if info and info.get("active"):
        by = (FBLK_B_ROW_F32 if f32 else FBLK_B_ROW) * m + FBLK_B_TILE * (info["padded_rows"] // 64) + \
            FBLK_B_SEG * info["segments"] + 24 * (info["window"] + 3) * info["workgroups"]
        return "k_fblk", by
    return "k_fused", (FUSED_B_ROW_F32 if f32 else FUSED_B_ROW) * m + FUSED_B_STAR * ns


# the sources each row-pass kernel is compiled from
KERNEL_SOURCES = {
    "k_fblk": ("blocked.hip", "row_tiles.h", "device_common.h", "internal.h"),
    "k_fused": ("fused.hip", "row_tiles.h", "device_common.h", "internal.h"),
}


def kernel_source_hash(kernel: str = "k_fblk") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
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
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def stream_copy_gbps(nbytes: int = 1 << 31, reps: int = 5) -> float:
    """Device-to-device copy of nbytes (read + written), HIP events: the measured
    stream-copy rate that a read-and-write pass can be held against."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    c = torch.empty_like(a)
    for _ in range(2):
        c.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        c.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, c
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _usable_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))  # at most 16 threads: the host cores that go with one GPU


def cpu_baseline(full_m: int, budget_s: float = 12.0):
    """The oracle, as it stands, on a bounded sample: a 20,000-star system of the same
    construction (same attitude / instrumental sizes, same distributions), timed on
    one thread and on every usable core (its products are threaded by stars and by
    fixed chunks of stars), the per-iteration time scaled by rows to the full share."""
    import gsr_synth
    import oracle

    g = gsr_synth.share_1m(seed=2505, n_stars=20_000)
    o = oracle.OSystem(g)
    b = oracle.known_terms(o, g.x_true, g.noise)

    def per_iteration(threads, budget):
        oracle.set_threads(threads)
        t = time.perf_counter()
        oracle.lsqr(o, b, atol=0, btol=0, itmax=1, precond=False)
        t1 = time.perf_counter() - t
        k = max(2, min(200, int(budget / max(t1, 1e-3))))
        t = time.perf_counter()
        r = oracle.lsqr(o, b, atol=0, btol=0, itmax=k, precond=False)
        tk = time.perf_counter() - t
        return (tk - t1) / max(1, k - 1), r["itn"], tk  # the one-time setup removed

    try:
        per1, it1, t1 = per_iteration(1, budget_s)
        P = _usable_cores()
        perP, itP, tP = per_iteration(P, budget_s / 2)
    finally:
        oracle.set_threads(0)
    scale = full_m / g.dims.m
    return {"value": 1.0 / (per1 * scale), "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{g.dims.n_stars} stars ({g.dims.m} rows) of the same construction, {it1} unscaled LSQR "
                      f"iterations in {t1:.1f} s on one thread, scaled by rows to m={full_m}",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "all_cores": {"value": 1.0 / (perP * scale), "unit": "iterations/s", "cores": P, "kind": "oracle",
                          "sample": f"the same sample, {itP} iterations in {tP:.1f} s on {P} threads, scaled "
                                    f"by rows to m={full_m}"}}


def _rel(a, b):
    import torch

    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def _median_time(fn, reps=5):
    import torch

    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    ts.sort()
    return ts[len(ts) // 2]


def _iters_to(S, b, x_ref, tol, cap, x0=None, **opts):
    """Trace run: iterations of a warm- or cold-start solve until ||x - x_ref|| <= tol ||x_ref||."""
    S.lsqr_begin(b, x0=x0, atol=0.0, btol=0.0, itmax=cap, **opts)
    x = None
    for it in range(1, cap + 1):
        S.lsqr_iterate(1)
        x = S.lsqr_peek(x)
        if _rel(x, x_ref) <= tol:
            S.lsqr_end(want_var=False)
            return it
    S.lsqr_end(want_var=False)
    return None


def _pass_rates(S, b, product, m, ns, f32, iters=10):
    """Average row pass and second pass (bucketed attitude sums, or the segment
    reduction of the regrouped pass) times (HIP events) over `iters` iterations of a
    column-scaled solve with the given product mode, and the row pass's algorithmic
    GB/s."""
    import torch

    S.lsqr_begin(b, atol=0.0, btol=0.0, itmax=iters + 3, precond=True, product=product)
    S.lsqr_iterate(2)
    S.timing_enable(True)
    S.timing_get()
    S.lsqr_iterate(iters)
    torch.cuda.synchronize()
    tm = S.timing_get()
    S.timing_enable(False)
    S.lsqr_end(want_var=False)
    f_ms = tm["aprod1_ms"] / max(1, tm["aprod1_n"])
    kname, by = pass_bytes(S.blocked_info(), m, ns, f32)
    return {"row_pass": kname, "row_pass_ms": f_ms, "second_pass_ms": tm["aprod2_ms"] / max(1, tm["aprod2_n"]),
            "row_pass_bytes": by, "row_pass_GBps": by / (f_ms * 1e-3) / 1e9}


def time_to_tolerance_fp32(gsr, g, tol=1e-10, label="", inner_tol=1e-5, packed=False):
    """FP64 LSQR vs the FP32 forms on the same FP32-representable matrix: FP32 products
    with FP64 iterative refinement (inner atol = btol = inner_tol, outer_tol 1e-11), and
    FP32 storage with FP64 products.  Reference: the FP64 solve converged to
    atol = btol = 1e-14; the FP64 and storage-only counts are the fewest iterations
    that reach `tol` of it."""
    import numpy as np
    import torch

    import copy

    g32 = g.as_f32()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if packed:
        # rows placed by the caller in the regrouped order, as the headline runs them
        g64 = copy.copy(g32)
        g64.vals = g32.vals.astype(np.float64)
        S64 = gsr.System.packed_from_generated(g64)
        del g64
        S32 = gsr.System.packed_from_generated(g32)
    else:
        rp, at, ic = t(g.star_row_ptr), t(g.att_start), t(g.instr_col)
        v32 = t(g32.vals)
        S64 = gsr.System(v32.double(), rp, at, ic, g.dims.n_att, g.dims.n_instr, g.dims.n_glob)
        S32 = gsr.System(v32, rp, at, ic, g.dims.n_att, g.dims.n_instr, g.dims.n_glob)
    b = t(g.noise)
    S64.aprod1(t(g.x_true), b, scale=1.0)
    x_ref, _, rref = S64.lsqr_solve(b, atol=1e-14, btol=1e-14, itmax=5000, precond=True, want_var=False)
    n64 = _iters_to(S64, b, x_ref, tol, 2000, precond=True)
    t64 = _median_time(lambda: S64.lsqr_solve(b, atol=0, btol=0, itmax=n64, precond=True, want_var=False))
    ropts = dict(atol=inner_tol, btol=inner_tol, itmax=2000, precond=True, outer_max=10, outer_tol=1e-11)
    xr, rr = S32.lsqr_refine(b, **ropts)
    err32 = _rel(xr, x_ref)
    t32 = _median_time(lambda: S32.lsqr_refine(b, **ropts))
    # bytes-only form: FP32 storage, FP64 products (no refinement needed)
    nb = _iters_to(S32, b, x_ref, tol, 2000, precond=True, product="f64")
    tb = _median_time(lambda: S32.lsqr_solve(b, atol=0, btol=0, itmax=nb, precond=True, want_var=False,
                                             product="f64"))
    m, ns = g.dims.m, g.dims.n_stars
    rates = {"fp64": _pass_rates(S64, b, "f64", m, ns, False),
             "fp32_products": _pass_rates(S32, b, "f32", m, ns, True),
             "fp32_storage_fp64_products": _pass_rates(S32, b, "f64", m, ns, True)}
    S64.close()
    S32.close()
    return {"workload": label, "tol": tol, "fp64": {"iterations": n64, "seconds": t64},
            "fp32_refine": {"inner_tol": inner_tol, "outer": rr["outer_steps"], "inner_total": rr["inner_total"],
                            "seconds": t32, "rel_err_vs_fp64": err32},
            "speedup": t64 / t32,
            "fp32_storage_fp64_products": {"iterations": nb, "seconds": tb, "speedup": t64 / tb},
            "per_iteration": rates}


def time_to_tolerance_warm(gsr, tol=1e-10, train_steps=1500):
    """Family of 16 related systems on the 1,000-star matrix; train on 0-7, warm-start 8-15."""
    import numpy as np
    import torch

    import gsr_synth

    base = gsr_synth.tiny()
    S = gsr.System.from_generated(base)
    ns = base.dims.n_stars
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    opts = dict(atol=1e-12, btol=1e-12, itmax=500, precond=True)
    bs = []
    for s in range(16):
        fm = gsr_synth.family_member(base, s)
        b = t(fm.noise)
        S.aprod1(t(fm.x_true), b, scale=1.0)
        bs.append(b)
    sols = [S.lsqr_solve(bs[s], want_var=False, **opts)[0] for s in range(8)]
    x_mean = gsr.mean_rows(torch.stack(sols))
    xo = x_mean[5 * ns:].contiguous()
    F = torch.cat([S.features(bs[s], xo) for s in range(8)])
    T = torch.cat([sols[s][: 5 * ns].reshape(ns, 5) for s in range(8)])
    net = gsr.MLP(gsr_synth.mlp_init(28, 128, 5, seed=11))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.fit_norm(F, T)
    loss = net.train(F, T, steps=train_steps, lr=1e-3)
    train_s = time.perf_counter() - t0

    def mlp_x0(b):
        x0 = torch.empty(base.dims.n, dtype=torch.float64, device="cuda")
        x0[: 5 * ns] = net.forward(S.features(b, xo)).reshape(-1)
        x0[5 * ns:] = xo
        return x0

    rows = []
    for s in range(8, 16):
        b = bs[s]
        x_ref, _, _ = S.lsqr_solve(b, atol=1e-14, btol=1e-14, itmax=5000, precond=True, want_var=False)
        k0 = _iters_to(S, b, x_ref, tol, 500, precond=True)
        km = _iters_to(S, b, x_ref, tol, 500, x0=x_mean, precond=True)
        kn = _iters_to(S, b, x_ref, tol, 500, x0=mlp_x0(b), precond=True)
        t0_ = _median_time(lambda: S.lsqr_solve(b, atol=0, btol=0, itmax=k0, precond=True, want_var=False))
        tm_ = _median_time(lambda: S.lsqr_solve(b, x0=x_mean, atol=0, btol=0, itmax=km, precond=True,
                                                want_var=False))
        tn_ = _median_time(lambda: S.lsqr_solve(b, x0=mlp_x0(b), atol=0, btol=0, itmax=kn, precond=True,
                                                want_var=False))
        rows.append((k0, km, kn, t0_, tm_, tn_))
    net.close()
    S.close()
    a = np.array(rows, dtype=float)
    return {"workload": "family of 16 systems on the 1,000-star matrix (train 0-7, test 8-15)", "tol": tol,
            "train_loss": loss, "train_seconds": train_s,
            "iterations": {"zero": a[:, 0].mean(), "mean_x0": a[:, 1].mean(), "mlp_x0": a[:, 2].mean()},
            "seconds": {"zero": a[:, 3].mean(), "mean_x0": a[:, 4].mean(), "mlp_x0_incl_inference": a[:, 5].mean()},
            "speedup_mlp_vs_zero": a[:, 3].mean() / a[:, 5].mean()}


def aprods_bench(S, m, n, ns, workload, reps=10):
    """The standalone products y = 0.5 y + A x and x = 0.5 x + A^T y on the caller's
    rows (HIP events on the stream they run on), against their algorithmic bytes."""
    import torch

    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.randn(m, dtype=torch.float64, device="cuda")
    out = {"metric": "standalone aprod HBM rate", "workload": workload, "unit": "GB/s", "peak": HBM_PEAK_GBS}
    for name, f, by in (("aprod1", lambda: S.aprod1(x, y, scale=0.5), APROD1_B_ROW * m),
                        ("aprod2", lambda: S.aprod2(y, x, scale=0.5), APROD2_B_ROW * m + APROD2_B_STAR * ns)):
        f()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        gbs = by / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "bytes": by, "GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    return out


def syrk_bench(gsr, k=4000, reps=20):
    """The covariance update C += D D^T alone (upper 32x32 tiles, FP64 MFMA) for
    k selected unknowns and blocks of 64, 256 and 512 buffered iterations."""
    import torch

    rows = []
    T = (k + 31) // 32
    for cols in (64, 256, 512):
        D = torch.randn(k, cols, dtype=torch.float64, device="cuda")
        Cm = torch.zeros(k, k, dtype=torch.float64, device="cuda")
        gsr.syrk(D, k, cols, cols, Cm)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            gsr.syrk(D, k, cols, cols, Cm)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        flops = 2.0 * cols * 32 * 32 * (T * (T + 1) // 2)  # the upper tiles computed
        rows.append({"k": k, "cols": cols, "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                     "frac_of_fp64_mfma_peak": flops / (ms * 1e-3) / 78.6e12})
    return {"metric": "covariance SYRK FP64 MFMA rate", "unit": "TFLOP/s", "peak": 78.6, "results": rows}


def stream_probe_rows():
    """Rows of the memory-system probe (csrc/stream_probe.hip), run as a child process
    of its own; None if it is not built."""
    import subprocess

    probe = os.path.join(ROOT, "paper_2503_22863_amd", "stream_probe")
    if not os.path.exists(probe):
        return None
    r = subprocess.run([probe], capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise SystemExit(f"stream_probe failed ({r.returncode}): {r.stderr.strip()}")
    return [json.loads(line) for line in r.stdout.splitlines() if line.startswith("{")]


def _attach_floor(roof, floor):
    """The row pass's rate against the probe's two-stream floor (FP64 rows only)."""
    if floor and roof.get("kernel") == "k_fblk" and roof.get("bytes_per_launch"):
        roof["probe_floor"] = floor
        roof["frac_of_probe_floor"] = roof["achieved"] / floor["GBps"]


def two_stream_floor(rows):
    """The probe's FP64 form with both of the row pass's write streams (u, and 35
    values per 64-row tile: a tile's segment sums), as bytes read + written per
    second."""
    if not rows:
        return None
    r = next((x for x in rows if x["chunks"] == 12 and x["store"].endswith("two streams")), None)
    if r is None:
        return None
    n, tiles = r["rows"], (r["rows"] + 63) // 64
    by = n * (12 * 16 + 16 + 8) + n * 8 + tiles * 35 * 8
    return {"form": r["store"], "rows": n, "ms": r["ms"], "GBps": by / (r["ms"] * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--stars", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1e-10 comparisons")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 2 GiB device copy (known bytes, for scaling HBM counters)")
    ap.add_argument("--workload", choices=("share_1m", "share_3m"), default="share_1m",
                    help="share_3m: 3e6 stars, 3x120,000 attitude, 500 instrumental unknowns")
    ap.add_argument("--cov", type=int, default=0,
                    help="covariances of this many selected unknowns (blocks of 64 iterations) during the run")
    ap.add_argument("--export", type=int, default=0,
                    help="export the whole d_i every this many iterations to pinned host memory during the run, "
                         "then form covariances of --cov unknowns from the export")
    ap.add_argument("--pairs", type=int, default=0,
                    help="covariances of this many random index pairs (blocks of 64 iterations) during the run")
    ap.add_argument("--constraints", action="store_true",
                    help="add 6 constraint equations: the sums over all stars of astrometric unknowns 0-2 and "
                         "the sums over each attitude axis")
    ap.add_argument("--library-copy", action="store_true",
                    help="hand the rows over in star order and let the library make its regrouped copy (instead of "
                         "placing them in the regrouped order first)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 3e6-star leg with the covariances of 4,000 unknowns")
    ap.add_argument("--star-order", action="store_true",
                    help="iterate on the rows in star order (bucketed attitude pass) instead of the copy "
                         "regrouped by attitude window")
    ap.add_argument("--stream-probe", action="store_true",
                    help="run the memory-system calibration (the row pass's byte stream with its u store in "
                         "several forms) and print its results")
    ap.add_argument("--syrk-bench", action="store_true",
                    help="time the covariance SYRK alone (k = 4000) and print its MFMA rate instead")
    ap.add_argument("--aprods", action="store_true",
                    help="time the standalone aprod 1 and aprod 2 on the workload's rows and print their "
                         "HBM rates instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU row split is not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.stream_probe:
        rows = stream_probe_rows()
        if rows is None:
            raise SystemExit("stream_probe is not built (run the package build first)")
        print(json.dumps({"stream_probe": rows}), flush=True)
        return
    # the row pass's own memory floor on this chip, measured before this process
    # touches the GPU: the probe's stream of the same reads with u and a
    # segment-sized second store stream
    probe_floor = None if args.aprods or args.syrk_bench else two_stream_floor(stream_probe_rows())

    import numpy as np
    import torch

    import gsr_synth
    import paper_2503_22863_amd as gsr

    torch.cuda.set_device(0)
    if args.syrk_bench:
        print(json.dumps(syrk_bench(gsr)), flush=True)
        return
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        c.copy_(a)  # reads and writes 2 GiB
        torch.cuda.synchronize()
        del a, c
    workload = args.workload
    if args.aprods:
        g = _generate(gsr_synth, workload, args.stars)
        S = gsr.System.from_generated(g)  # the standalone products on the caller's rows in star order
        print(json.dumps(aprods_bench(S, g.dims.m, g.dims.n, g.dims.n_stars, workload)), flush=True)
        S.close()
        return
    layout = "star_order" if args.star_order else ("library_copy" if args.library_copy else "packed")
    g = _generate(gsr_synth, workload, args.stars)
    g_share = None if args.no_ttt else g  # the FP32 forms are timed on the same system
    out, extra = share_leg(gsr, g, args.steps, args.warmup, layout=layout, cov=args.cov, export=args.export,
                           pairs=args.pairs, constraints=args.constraints,
                           # with covariances, 64 kernel-timed iterations hold one covariance flush
                           timed_kernels=64 if (args.cov or args.pairs) else min(args.steps, 20))
    del g
    m, n, ns = out["_m"], out["_n"], out["_ns"]
    res = {
        "metric": "LSQR iterations/s (FP64, one-GPU share)",
        "value": out["value"],
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": out["workload"], "global_batch": m, "seq_len": None, "parallelism": "single-gpu"},
        "roofline": out["roofline"],
        "iteration_ms": out["iteration_ms"],
        "row_layout": out["row_layout"],
    }
    res.update(extra)
    _attach_floor(res["roofline"], probe_floor)
    if "covariances" in out:
        res["covariances"] = out["covariances"]
    if not args.no_large and workload == "share_1m" and args.stars == 1_000_000 and layout == "packed":
        # the largest single-GPU configuration: 3e6 stars with the covariances of 4,000
        # unknowns in blocks of 64 iterations (one graph block warm-up, one timed block,
        # one block with per-kernel events)
        g3 = _generate(gsr_synth, "share_3m", 3_000_000)
        o3, _ = share_leg(gsr, g3, 64, 64, layout="packed", cov=4000, timed_kernels=64)
        del g3
        res["share_3m_cov4000"] = {k: v for k, v in o3.items() if not k.startswith("_")}
        _attach_floor(res["share_3m_cov4000"]["roofline"], probe_floor)
    if not args.no_ttt:
        import gsr_synth as _gs

        res["time_to_1e-10"] = {
            "fp32_forms_tiny": time_to_tolerance_fp32(gsr, _gs.tiny(), label="tiny: 1,000 stars x 20 rows"),
            "fp32_forms_share": time_to_tolerance_fp32(gsr, g_share, label=f"{workload}: {ns} stars x U[50,90] rows",
                                                       packed=True),
            "warm_start": time_to_tolerance_warm(gsr),
        }
    del g_share
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(m)
    print(json.dumps(res), flush=True)


def _generate(gsr_synth, workload, stars):
    t = time.time()
    if workload == "share_3m":
        g = gsr_synth.share_3m() if stars in (1_000_000, 3_000_000) else gsr_synth.share_3m(n_stars=stars)
    else:
        g = gsr_synth.share_1m(n_stars=stars)
    print(f"# generated {workload}: m={g.dims.m} n={g.dims.n} in {time.time() - t:.1f}s", file=sys.stderr,
          flush=True)
    return g


def share_leg(gsr, g, K, W, layout="packed", cov=0, export=0, pairs=0, constraints=False, timed_kernels=20):
    """One timed LSQR run on a share.  The handle is made over rows the caller placed
    in the regrouped order (layout "packed": the library holds no copy of A), over the
    rows in star order with the library's regrouped copy ("library_copy"), or in star
    order with the bucketed attitude pass ("star_order").  A throwaway solve first
    captures the iteration graph; then W untimed warm-up iterations and exactly K timed
    ones with graph replay on (the shipped configuration) give the iteration rate;
    then `timed_kernels` more iterations with HIP events around every kernel (graph
    replay off) give the per-kernel times the roofline uses."""
    import numpy as np
    import torch

    import gsr_synth

    m, n, ns = g.dims.m, g.dims.n, g.dims.n_stars
    t = time.time()
    if layout == "packed":
        S = gsr.System.packed_from_generated(g)
    else:
        S = gsr.System.from_generated(g)
        S.set_blocked(layout == "library_copy")
    print(f"# handle ({layout}) in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    sel = None
    if cov > 0:
        nst = (cov * 3 // 5) // 5
        sel = gsr_synth.covariance_selection(g.dims, nst, cov * 3 // 10 // 3, cov - 5 * nst - 3 * (cov * 3 // 10 // 3),
                                             seed=19)
        S.cov_request(sel, block=64)
    if pairs > 0:
        rngp = np.random.default_rng(29)
        S.cov_request_pairs(rngp.integers(0, n, size=(pairs, 2)), block=64)
    if constraints:
        d = g.dims
        rows = [np.arange(k, d.n_astro, 5) for k in range(3)]
        rows += [d.n_astro + a * d.n_att + np.arange(d.n_att) for a in range(3)]
        ptr = np.cumsum([0] + [r.size for r in rows]).astype(np.int64)
        col = np.concatenate(rows).astype(np.int64)
        val = np.concatenate([np.full(r.size, np.sqrt(24.0 / r.size)) for r in rows])
        rhs = np.array([val[ptr[i]:ptr[i + 1]] @ g.x_true[col[ptr[i]:ptr[i + 1]]] for i in range(6)])
        S.set_constraints(ptr, col, val, rhs)
    ehost = None
    if export > 0:
        nblk = (W + K + timed_kernels + export - 1) // export + 1
        ehost = torch.empty((nblk, export, n), dtype=torch.float64).pin_memory()
        S.cov_export(ehost, export)
    xt = torch.from_numpy(g.x_true).cuda()
    b = torch.from_numpy(g.noise).cuda()
    S.aprod1(xt, b, scale=1.0)  # b = A x_true + noise
    del xt
    torch.cuda.synchronize()
    G = 64 if (cov > 0 or pairs > 0) else 16
    if export == 0:
        # capture the iteration graph once (it is replayed by later solves of the same configuration)
        S.lsqr_begin(b, atol=0.0, btol=0.0, itmax=G + 1, precond=False)
        S.lsqr_iterate(G)
        S.lsqr_end(want_var=False)
    S.lsqr_begin(b, atol=0.0, btol=0.0, itmax=W + K + timed_kernels + 1, precond=False)
    S.lsqr_iterate(W)
    st = S.lsqr_status()
    assert st["itn"] == W, st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.lsqr_iterate(K)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    st = S.lsqr_status()
    if st["itn"] != W + K:
        raise RuntimeError(f"solve stopped early (itn={st['itn']}, istop={st['istop']}): timed steps not all real")
    # per-kernel HIP events on the solve's stream, over a separate run of iterations
    S.timing_enable(True)
    S.timing_get()  # reset
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.lsqr_iterate(timed_kernels)
    torch.cuda.synchronize()
    Tk = time.perf_counter() - t1
    tm = S.timing_get()
    S.timing_enable(False)
    if S.lsqr_status()["itn"] != W + K + timed_kernels:
        raise RuntimeError("solve stopped early in the per-kernel timing run")
    cov_ms = None
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    S.lsqr_end(want_var=False)  # flushes the last partial covariance block
    if cov > 0:
        C = S.cov_get()
        torch.cuda.synchronize()
        cov_ms = 1e3 * (time.perf_counter() - t2)
        del C
    f_ms = tm["aprod1_ms"] / max(1, tm["aprod1_n"])
    info = S.blocked_info()
    kname, by = pass_bytes(info, m, ns)
    achieved = by / (f_ms * 1e-3) / 1e9
    copy_gbps = stream_copy_gbps()
    wl = "share_3m" if g.dims.n_att == 120_000 else "share_1m"
    d = g.dims
    out = {
        "_m": m, "_n": n, "_ns": ns,
        "workload": f"{wl}: {ns} stars x U[50,90] obs (m={m}), 3x{d.n_att} attitude, {d.n_instr} instr, "
                    f"{d.n_glob} global (n={n}); unscaled FP64 LSQR, damp 0, variances on"
                    + (f", covariances of {cov} unknowns in blocks of 64 iterations" if cov else "")
                    + (", 6 constraint equations" if constraints else "")
                    + {"packed": "; rows placed by the caller in the regrouped order (no library copy of A)",
                       "library_copy": "; rows in star order, library's regrouped copy",
                       "star_order": "; rows in star order, bucketed attitude pass"}[layout],
        "value": K / T, "ms_per_step": 1e3 * T / K, "steps": K, "warmup": W,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(kname, wl),
                     "bytes_per_launch": by, "avg_ms": f_ms,
                     "timed_over": f"{timed_kernels} iterations with HIP events around every kernel on the solve's "
                                   f"stream, right after the timed region ({1e3 * Tk / timed_kernels:.3f} ms per "
                                   f"iteration there, graph replay off)",
                     "stream_copy_GBps": copy_gbps, "frac_of_stream_copy": achieved / copy_gbps},
        "iteration_ms": {"row_pass": f_ms, "second_pass": tm["aprod2_ms"] / max(1, tm["aprod2_n"]),
                         "tail": tm["tail_ms"] / max(1, tm["tail_n"]),
                         "update": tm["update_ms"] / max(1, tm["update_n"])},
        "row_layout": info if kname == "k_fblk" else "star order",
    }
    extra = {}
    if export > 0:
        nb, lc = S.cov_export_status()
        extra["export"] = {"block": export, "blocks": nb, "last_cols": lc, "bytes_per_block": 8 * export * n,
                           "iteration_ms_with_export": 1e3 * T / K}
        if sel is not None:
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            Cx = gsr.cov_from_export(ehost, n, export, nb, lc, sel)
            torch.cuda.synchronize()
            extra["export"]["read_cov_ms_per_block"] = 1e3 * (time.perf_counter() - t3) / max(1, nb)
            extra["export"]["k"] = int(sel.size)
            del Cx
    if pairs > 0:
        extra["pair_covariances"] = {"pairs": pairs, "block": 64,
                                     "pair_dots_ms_per_block": tm["syrk_ms"] / max(1, tm["syrk_n"]),
                                     "blocks_timed": tm["syrk_n"]}
    if cov > 0:
        out["covariances"] = {"k": cov, "block": 64, "syrk_ms_per_block": tm["syrk_ms"] / max(1, tm["syrk_n"]),
                              "syrk_blocks_timed": tm["syrk_n"], "final_flush_and_get_ms": cov_ms}
    S.close()
    del b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out, extra


if __name__ == "__main__":
    main()
