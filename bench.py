"""Benchmark: 2D low-rank Poisson solves per second on one MI355X.

Workload (the headline case): 2D 5-point Dirichlet Poisson, n = 4096 interior
points per axis, RHS = sum of r = 16 separable Gaussian bumps, eps = 1e-8
(acceptance: relative Frobenius error <= 1e-7 against the float64 full-grid
solution).  One step = one batched call that runs the whole path (forward
sine transform of the factors, cross sweeps with maxvol, rounding, inverse
transform) for a batch of B = 2048 right-hand sides already resident in
device memory (64 distinct ones, each 32 times; every problem is solved on
its own).  The call's argument array and output buffers are prepared once.
`value` is the AUTO plan (at n = 4096: both transforms by the float64
chirp-z FFT, everything else float64); the float64 GEMM plan and the int8
slice plan are timed beside it.
Every distinct RHS of the batch is checked against the CPU oracle.

Also reported: served p50/p99 latency of a Poisson-arrival request stream
(200 req/s; 2D grids 512..8192 and 3D grids 128..512, ranks 4..64, eps
1e-6/1e-8) through the library's continuous-batching loop; the transform
kernel's roofline from HIP-event timing of its dispatches during the timed
steps; the CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The served stream runs one stream per slot group (up to eight groups); give
# each its own hardware queue so that a long 3D launch never sits in front of
# another group's short ones (HIP reads this when it initialises).
if int(os.environ.get("GPU_MAX_HW_QUEUES") or 0) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15, "int8": 5.0e15}
PRECS = ("fp64", "fp32", "bf16x3", "int8", "fft64", "bf16x6")
# arithmetic of each transform plan (everything else is float64)
DTYPE = {"fp64": "f64", "fft64": "f64", "int8": "i8-slices+f64", "fp32": "f32+f64",
         "bf16x3": "bf16x3+f64", "bf16x6": "bf16x6+f64"}

# HBM bytes moved per launch of a transform kernel in this workload, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch averaged over the kernel's dispatches), each scaled by what the same
# counter reads for a plain device copy of 1 GiB (FETCH_SIZE reads half the
# copied bytes: x2; WRITE_SIZE reads them exactly: x1).  A figure holds only
# for the kernel source it was taken on (the sha1 over the listed sources must
# match) and for dispatches of the same average column count (the default
# workload and batch); otherwise the traffic is reported as null.  k_dst_i8
# averages over the dispatches of both its tile shapes (64-column tiles and
# the narrow tail launch), as the timed launch average does.
TRAFFIC = {
    "k_dst_fft4096": {"sources": ["dst_fft.hip", "lrp_internal.h"],
                      "sha1": "b7409872572ad5116ca93bc8a2598df84db30252",
                      "columns": 83968, "fetch_kib": 1351473.0, "write_kib": 2686983.9},
    "k_dst_i8": {"sources": ["dst_i8.hip", "lrp_internal.h"],
                 "sha1": "5fd4f8c754166ab32eeabd320b2ba49e58c03a73",
                 "columns": 13989.333, "fetch_kib": 229131.2, "write_kib": 448128.0},
    "k_dst_f64": {"sources": ["dst.hip", "lrp_internal.h"],
                  "sha1": "89e1060fe35e75a54761a80325908be97c1b3497",
                  "columns": 83968, "fetch_kib": 1350067.9, "write_kib": 2818574.6},
}


def traffic_bytes(kernel, columns):
    import hashlib
    t = TRAFFIC.get(kernel)
    if not t or t["sha1"] is None or abs(columns - t["columns"]) > 0.5:
        return None
    h = hashlib.sha1()
    for f in t["sources"]:
        with open(os.path.join(ROOT, "paper_1306_2150_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != t["sha1"]:
        return None
    return (2.0 * t["fetch_kib"] + 1.0 * t["write_kib"]) * 1024.0


METRIC = "2D n=4096 r=16 solves/s at rel err<=1e-7, mixed vs FP64 path; served p99 ms"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--distinct", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-expsum", action="store_true",
                    help="skip the exponential-sum comparator timing")
    ap.add_argument("--expsum-batches", type=str, default="1,256",
                    help="batch sizes of the exponential-sum comparison")
    ap.add_argument("--only-stokes", action="store_true",
                    help="run only the Stokes driver on Section 6's test problem (one JSON line)")
    ap.add_argument("--only-expsum", action="store_true",
                    help="run only the exponential-sum comparator timing (one JSON line)")
    ap.add_argument("--cpu-sample", type=int, default=5)
    ap.add_argument("--serve-check", type=int, default=1,
                    help="served requests per (dim, n) shape checked against the oracle")
    ap.add_argument("--batch-sweep", type=str, default="",
                    help="comma-separated batch sizes: also report solves/s of both "
                         "plans at each (e.g. 1,8,32,128,256,512,1024)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy this many MiB once first (HBM counter calibration)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(hostrhs, eps, runs):
    """The oracle timed on the host cores: the float64 full-grid solve
    (scipy.fft, threaded) and, beside it, the naive float64 low-rank solver
    (threaded LAPACK); each the median of ``runs`` solves after one warm-up,
    on the first ``runs`` distinct right-hand sides."""
    import numpy as np
    from oracle import lowrank, poisson
    workers = min(16, os.cpu_count() or 1)

    def median_time(fn):
        fn(*hostrhs[0])
        ts = []
        for i in range(runs):
            t0 = time.perf_counter()
            fn(*hostrhs[i % len(hostrhs)])
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_full = median_time(lambda U, V: poisson.full_solve2d_factors(U, V, workers=workers))
    t_lr = median_time(lambda U, V: lowrank.lr_solve2d(U, V, eps))
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"median of {runs} full-grid float64 DST solves at n=4096 after one "
                      f"warm-up (scipy.fft, {workers} workers)",
            "lowrank_oracle": {"value": 1.0 / t_lr, "unit": "solves/s",
                               "sample": f"median of {runs} naive float64 low-rank solves "
                                         f"(eps={eps}, numpy/LAPACK threads)"}}


def expsum_vs_cross(ctx, workers, batches=(1, 256)):
    """Section 6.1's comparison on its case: n = 1024, eps = 1e-7, a rank-30
    right-hand side; the exponential-sum route (quadrature, Hadamard product
    of rank R r, rounding) against the cross, on one problem (latency, median
    of 5) and on a batch of 256 (throughput), both checked against the
    float64 full-grid oracle."""
    import numpy as np
    import torch

    from oracle import metrics, poisson
    from paper_1306_2150_amd import binding, inputs
    n, r, eps = 1024, 30, 1e-7
    host = [inputs.rhs2d_bumps(n, r, 6001 + i) for i in range(8)]
    dev = [(binding.colmajor(U), binding.colmajor(V)) for U, V in host]
    rec = {"workload": "2D Poisson n=1024 r=30 eps=1e-7 Gaussian-bump RHS", "n": n, "r": r,
           "eps": eps}
    X = poisson.full_solve2d_factors(*host[0], workers=workers)
    for nb in batches:
        reps = 5 if nb <= 16 else 2
        probs = [(dev[i % 8][0], dev[i % 8][1], eps) for i in range(nb)]
        for method in ("cross", "expsum"):
            b = ctx.batch2d(probs, prec="fp64", method=method)
            res = b.run()
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.run(results=False)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            res = b.results()
            dt = float(np.median(times))
            info = res[0][2]
            key = f"{method}_batch{nb}"
            rec[key] = {"ms": dt * 1e3, "solves_per_s": nb / dt, "rank": info["rank"],
                        "status": info["status"]}
            if method == "expsum":
                rec[key]["terms"] = info["k"]
                rec[key]["steps"] = info["sweeps"]
            if nb == 1:
                Ux, Vx = res[0][0].cpu().numpy(), res[0][1].cpu().numpy()
                rec[key]["rel_err"] = metrics.rel_err_factored(Ux, Vx, X)
        rec[f"ratio_batch{nb}"] = rec[f"expsum_batch{nb}"]["ms"] / rec[f"cross_batch{nb}"]["ms"]
        print(f"[bench] Section 6.1 case, batch {nb}: expsum {rec[f'expsum_batch{nb}']['ms']:.2f} ms, "
              f"cross {rec[f'cross_batch{nb}']['ms']:.2f} ms", file=sys.stderr, flush=True)
    return rec


# Section 6's test problem on the grids of Table 1, with the thresholds the
# 64-column rounding panels allow (the paper: 5e-9 at every n)
STOKES_CASES = [(64, 5e-9), (128, 5e-9), (256, 1e-7), (512, 2e-7), (1024, 5e-7)]


def stokes_table(ctx, workers):
    """Table 1's columns for the low-rank Uzawa-GMRES driver on the GPU and
    the full-format Uzawa (CG) of the CPU oracle: time and relative error of
    p against the prescribed solution (eq. "ansin2d")."""
    import numpy as np
    import torch

    from oracle import stokes
    from paper_1306_2150_amd import binding
    rows = []
    for n, eps in STOKES_CASES:
        fu, fv, g = stokes.ansin2d_factors(n)
        d = lambda pr: (binding.colmajor(pr[0]), binding.colmajor(pr[1]))
        args = (d(fu), d(fv), d(g))
        ctx.stokes2d(*args, eps)          # warm-up (tables, groups)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (pU, pV), _, _, info = ctx.stokes2d(*args, eps)
        torch.cuda.synchronize()
        t_lr = time.perf_counter() - t0
        P = pU.cpu().numpy() @ pV.cpu().numpy().T
        Fu, Fv, Gd, _, _, p_ex = stokes.ansin2d(n)
        t0 = time.perf_counter()
        pf, _, _, its = stokes.uzawa_cg(Fu, Fv, Gd, tol=1e-12)
        t_full = time.perf_counter() - t0
        pe = stokes.project(p_ex)
        rec = {"n": n, "eps": eps, "lr_s": t_lr, "full_cpu_s": t_full,
               "err_p_lr": float(np.linalg.norm(P - pe) / np.linalg.norm(pe)),
               "err_p_full": float(np.linalg.norm(stokes.project(pf) - pe) / np.linalg.norm(pe)),
               "gmres_iterations": info["iterations"], "restarts": info["restarts"],
               "rank_p": info["ranks"][0], "max_krylov_rank": info["max_krylov_rank"],
               "true_residual": info["true_residual"], "full_cg_iterations": its}
        print(f"[bench] Stokes n={n} eps={eps}: LR {t_lr:.3f} s (GPU), full {t_full:.3f} s (CPU), "
              f"err p {rec['err_p_lr']:.2e}/{rec['err_p_full']:.2e}", file=sys.stderr, flush=True)
        rows.append(rec)
    return {"problem": "Section 6 eq. ansin2d on n x n pressure cells", "rows": rows}


# HBM bytes the cross phase (a3-a6: entries, TSQR, maxvol, core, factors,
# change) moves per call of the default workload (CROSS_BATCH solves),
# summed over its kernels from the FETCH_SIZE / WRITE_SIZE counters of
# profiles/kernel_traffic_n4096_b2048.md (2 x FETCH + WRITE, calibrated by a
# device copy)
CROSS_BATCH = 2048
CROSS_BYTES_PER_CALL = 235460.5 * 2 ** 20


def cross_phase(res, batch):
    """Device time of the cross sweeps of one call (HIP events around the
    phase), per sweep of its longest solve, and the bandwidth it implies."""
    sweeps = [r[2]["sweeps"] for r in res]
    us = res[0][2]["us_phase"]["cross"]
    rec = {"us_per_call": us, "sweeps_mean": sum(sweeps) / len(sweeps),
           "sweeps_max": max(sweeps), "us_per_sweep": us / max(1, max(sweeps)),
           "solves": batch}
    if batch == CROSS_BATCH and CROSS_BYTES_PER_CALL:
        rec["bytes_per_call_counters"] = CROSS_BYTES_PER_CALL
        rec["GB_per_s"] = CROSS_BYTES_PER_CALL / (us * 1e-6) / 1e9 if us > 0 else None
    return rec


def timed_steps(ctx, problems, prec, steps, warmup):
    import torch
    # the argument array and output buffers are prepared once; every step
    # solves all problems of the batch from their inputs
    batch = ctx.batch2d(problems, prec=prec)
    for _ in range(warmup):
        res = batch.run()
    torch.cuda.synchronize()
    for p in PRECS:
        ctx.kernel_stats(p, reset=True)
    ctx.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        # the call returns when every solve of the batch is done and its
        # factors, ranks and reports are in the batch's buffers; the Python
        # views of them are built once, after the timed steps
        batch.run(results=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_kernel_timing(False)
    ks = {p: ctx.kernel_stats(p, reset=True) for p in PRECS}
    return dt, batch.results(), ks


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "requests are independent, see the design notes for the multi-GPU "
              "routing design", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1306_2150_amd import binding, inputs

    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        # a plain device copy of known size, for scaling the HBM byte counters
        a = torch.ones(args.copy_probe_mb << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ctx = binding.Context(0, workspace_bytes=128 << 30)
    if args.only_stokes:
        print(json.dumps({"stokes_table1": stokes_table(ctx, min(16, os.cpu_count() or 1))}),
              flush=True)
        ctx.close()
        return
    if args.only_expsum:
        batches = [int(x) for x in args.expsum_batches.split(",") if x]
        print(json.dumps({"expsum_vs_cross": expsum_vs_cross(ctx, min(16, os.cpu_count() or 1),
                                                             batches)}), flush=True)
        ctx.close()
        return
    n, r, eps = 4096, 16, 1e-8
    B = args.batch
    # distinct RHS instances (seed 2000 + i), repeated to fill the batch
    hostrhs = [inputs.workload_rhs(2, 1 + i) for i in range(args.distinct)]
    devrhs = [(binding.colmajor(U), binding.colmajor(V)) for U, V in hostrhs]
    problems = [(devrhs[i % args.distinct][0], devrhs[i % args.distinct][1], eps)
                for i in range(B)]
    print(f"[bench] batch {B} x (n={n}, r={r}, eps={eps}), {args.steps} steps "
          f"after {args.warmup} warmup", file=sys.stderr, flush=True)

    out = {}
    for plan in ("auto", "fp64", "int8"):
        dt, res, ks = timed_steps(ctx, problems, plan, args.steps, args.warmup)
        out[plan] = dict(seconds=dt, res=res, ks=ks,
                         solves_per_s=B * args.steps / dt,
                         ms_per_step=dt / args.steps * 1e3)
        print(f"[bench] {plan}: {out[plan]['solves_per_s']:.1f} solves/s, "
              f"{out[plan]['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)

    # accuracy of every distinct RHS against the float64 full-grid oracle
    from oracle import metrics, poisson
    workers = min(16, os.cpu_count() or 1)
    errs = {"auto": [], "fp64": [], "int8": []}
    for i, (U, V) in enumerate(hostrhs):
        X = poisson.full_solve2d_factors(U, V, workers=workers)
        for plan in ("auto", "fp64", "int8"):
            Ux, Vx, info = out[plan]["res"][i]
            e = metrics.rel_err_factored(Ux.cpu().numpy(), Vx.cpu().numpy(), X)
            errs[plan].append(e)
    print(f"[bench] max rel err auto {max(errs['auto']):.3e} fp64 "
          f"{max(errs['fp64']):.3e} int8 {max(errs['int8']):.3e}", file=sys.stderr, flush=True)
    print("[bench] rel err per instance auto: " +
          " ".join(f"{e:.2e}" for e in errs["auto"]), file=sys.stderr, flush=True)

    # Roofline of the dominant kernel of the measured (AUTO) step: the int8
    # slice transform (the float64 transform of the FP64 plan beside it).
    # frac is the HBM fraction: the method's minimum bytes of one launch (each
    # column's input read once and its transform written once) over the
    # launch's average duration, against 8 TB/s.  The dense-GEMM form does far
    # more arithmetic than the FFT form (5 N log2(2N) flops per column), so it
    # runs far from this bound; its matrix-core figures are kept beside it:
    #  - folded GEMM work per column: 2 (H0^2 + H1^2) flops, H0 = ceil(n/2),
    #    H1 = floor(n/2) (the library's count);
    #  - the int8 scheme executes 8 v_mfma_i32_16x16x64 per 16 grid points
    #    and 16 x 16 output tile: 32 int8 products per multiply-add, of which
    #    21 are needed (slice levels a + b <= 5 of the six 7-bit slices of
    #    each operand; the rest multiply zero padding).
    def kstat_roof(ks, name, peak, unit, ops_per_flop, needed_per_flop, bytes_per_col):
        launches = max(1, ks["launches"])
        avg_ms = ks["ms"] / launches
        flops = ks["flops"] / launches
        cols = ks["columns"] / launches
        sec = avg_ms * 1e-3
        alg = cols * bytes_per_col
        gbs = alg / sec / 1e9 if sec > 0 else 0.0
        ach = flops * ops_per_flop / sec if sec > 0 else 0.0
        need = flops * needed_per_flop / sec if sec > 0 else 0.0
        fft = cols * 5.0 * (n + 1) * np.log2(2.0 * (n + 1)) / sec if sec > 0 else 0.0
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": 8000.0,
                "unit": "GB/s", "frac": gbs / 8000.0, "traffic": None,
                "algorithmic_bytes": alg,
                "avg_launch_ms": avg_ms, "launches": ks["launches"],
                "columns_per_launch": cols,
                "mfma_executed": {"achieved": ach / 1e12, "peak": peak / 1e12, "unit": unit,
                                  "frac": ach / peak},
                "mfma_needed": {"achieved": need / 1e12, "frac": need / peak},
                "fft_form_tflops": fft / 1e12,
                "dense_equiv_tflops": 2.0 * n * n * cols / sec / 1e12 if sec > 0 else 0.0}
    kauto = out["auto"]["ks"]
    # minimum bytes of a column: its n float64 inputs read, n outputs written
    colbytes = 16.0 * n
    if kauto["fft64"]["launches"]:
        # the chirp-z FFT transform: float64 vector arithmetic, two forward and
        # two inverse 4096-point complex FFTs per column (the library's count)
        # It is bound by float64 vector arithmetic, not by HBM: 983040 flops
        # against 64 KiB of minimum traffic per column (15 flop/byte; the
        # chip's balance point is 78.6e12 / 8e12 = 9.8), so its roofline is
        # the float64 VALU peak and the HBM fraction is reported beside it.
        fr = kstat_roof(kauto["fft64"], "k_dst_fft4096", PEAK["fp64"], "TFLOP/s", 1.0, 1.0,
                        colbytes)
        valu = fr.pop("mfma_executed")
        fr.pop("mfma_needed")
        roofline = {"kernel": fr["kernel"], "bound": "alu", "achieved": valu["achieved"],
                    "peak": valu["peak"], "unit": "TFLOP/s", "frac": valu["frac"],
                    "traffic": traffic_bytes("k_dst_fft4096", fr["columns_per_launch"]),
                    "algorithmic_flops": fr["avg_launch_ms"] * 1e-3 * valu["achieved"] * 1e12,
                    "hbm": {"achieved": fr["achieved"], "peak": 8000.0, "unit": "GB/s",
                            "frac": fr["frac"], "algorithmic_bytes": fr["algorithmic_bytes"]},
                    "avg_launch_ms": fr["avg_launch_ms"], "launches": fr["launches"],
                    "columns_per_launch": fr["columns_per_launch"]}
    elif kauto["int8"]["launches"]:
        roofline = kstat_roof(kauto["int8"], "k_dst_i8", PEAK["int8"], "TOP/s", 32.0, 21.0,
                              colbytes)
        # the kernel itself reads each column's two parity slice records (8
        # bytes per point, each padded to 32 points) and exponents, written by
        # the slicing pass, and writes the float64 transform
        hpad = -(-((n + 1) // 2) // 32) * 32
        roofline["kernel_bytes"] = roofline["columns_per_launch"] * (2 * hpad * 8 + 8 + n * 8)
        roofline["traffic"] = traffic_bytes("k_dst_i8", roofline["columns_per_launch"])
    else:
        roofline = kstat_roof(kauto["fp64"], "k_dst_f64", PEAK["fp64"], "TFLOP/s", 1.0, 1.0,
                              colbytes)
    roofline["fp64_plan_kernel"] = kstat_roof(out["fp64"]["ks"]["fp64"], "k_dst_f64",
                                              PEAK["fp64"], "TFLOP/s", 1.0, 1.0, colbytes)
    f64 = roofline["fp64_plan_kernel"]
    f64["traffic"] = traffic_bytes("k_dst_f64", f64["columns_per_launch"])
    if out["int8"]["ks"]["int8"]["launches"]:
        i8 = kstat_roof(out["int8"]["ks"]["int8"], "k_dst_i8", PEAK["int8"], "TOP/s", 32.0, 21.0,
                        colbytes)
        i8["traffic"] = traffic_bytes("k_dst_i8", i8["columns_per_launch"])
        roofline["int8_plan_kernel"] = i8

    line = {
        "metric": METRIC,
        "value": out["auto"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out["auto"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE.get(out["auto"]["res"][0][2]["fwd_prec"], "f64"),
        "data": "synthetic",
        "config": {"workload": "2D Poisson n=4096 r=16 eps=1e-8 Gaussian-bump RHS",
                   "n": n, "r": r, "eps": eps, "batch": B,
                   "distinct_rhs": args.distinct, "plan": "auto",
                   "transform": out["auto"]["res"][0][2]["fwd_prec"]},
        "fp64_path": {"value": out["fp64"]["solves_per_s"],
                      "ms_per_step": out["fp64"]["ms_per_step"], "dtype": "f64",
                      "transform": "float64 MFMA GEMM"},
        "int8_path": {"value": out["int8"]["solves_per_s"],
                      "ms_per_step": out["int8"]["ms_per_step"], "dtype": "i8-slices+f64",
                      "transform": "int8 MFMA GEMM on exact 7-bit slices"},
        "accuracy": {"bar": 1e-7, "max_rel_err_auto": max(errs["auto"]),
                     "max_rel_err_fp64": max(errs["fp64"]),
                     "max_rel_err_int8": max(errs["int8"]),
                     "checked": len(hostrhs)},
        "roofline": roofline,
        "cross_phase": cross_phase(out["auto"]["res"], B),
    }

    if args.batch_sweep:
        sweep = []
        for b in [int(x) for x in args.batch_sweep.split(",") if x]:
            probs = [(devrhs[i % args.distinct][0], devrhs[i % args.distinct][1], eps)
                     for i in range(b)]
            rec = {"batch": b}
            for plan in ("auto", "fp64"):
                steps = max(2, min(20, 2048 // max(b, 1)))
                dt, _, _ = timed_steps(ctx, probs, plan, steps, 1)
                rec[plan] = {"solves_per_s": b * steps / dt, "ms_per_step": dt / steps * 1e3}
            print(f"[bench] batch {b}: auto {rec['auto']['solves_per_s']:.1f} solves/s "
                  f"({rec['auto']['ms_per_step']:.2f} ms), fp64 "
                  f"{rec['fp64']['solves_per_s']:.1f}", file=sys.stderr, flush=True)
            sweep.append(rec)
        line["batch_sweep"] = sweep

    if not args.no_serve:
        from paper_1306_2150_amd import serving
        reqs = serving.default_stream(args.serve_requests + args.serve_warmup)
        facs = serving.prepare(reqs)
        sv = {}
        for plan in ("auto", "fp64"):
            s = serving.run_stream(ctx, reqs, facs, prec=plan, warmup=args.serve_warmup)
            recs = s.pop("records")
            meas = recs[args.serve_warmup:]
            counts = {}
            for d in meas:
                name = binding.STATUS_NAME.get(d["status"], str(d["status"]))
                counts[name] = counts.get(name, 0) + 1
            s["status_counts"] = counts
            # accuracy of a sample: the first measured request of every shape
            s["checked"] = serving.check_sample(reqs, meas, per_shape=args.serve_check,
                                                workers=min(16, os.cpu_count() or 1))
            del recs, meas
            sv[plan] = s
            worst = max([c["rel_err"] / c["eps"] for c in s["checked"]] or [0.0])
            print(f"[bench] served {plan}: p50 {s['p50_ms']:.2f} ms p99 "
                  f"{s['p99_ms']:.2f} ms {s['solves_per_s']:.1f} solves/s, statuses {counts}, "
                  f"checked {len(s['checked'])} (worst err {worst:.2f} eps)",
                  file=sys.stderr, flush=True)
        line["serving"] = {"stream": "Poisson arrivals 200 req/s, 2D n in 512..8192 and "
                                     "3D n in 128..512, r 4..64, eps 1e-6/1e-8",
                           "p50_ms": sv["auto"]["p50_ms"], "p99_ms": sv["auto"]["p99_ms"],
                           "solves_per_s": sv["auto"]["solves_per_s"],
                           "by_dim": sv["auto"]["by_dim"],
                           "status_counts": sv["auto"]["status_counts"],
                           "checked": sv["auto"]["checked"],
                           "fp64": {k: sv["fp64"][k] for k in ("p50_ms", "p99_ms", "solves_per_s",
                                                                "by_dim", "status_counts",
                                                                "checked")},
                           "requests": args.serve_requests, "warmup": args.serve_warmup}

    if not args.no_expsum:
        batches = [int(x) for x in args.expsum_batches.split(",") if x]
        line["expsum_vs_cross"] = expsum_vs_cross(ctx, min(16, os.cpu_count() or 1), batches)

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(hostrhs, eps, args.cpu_sample)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
