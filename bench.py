#!/usr/bin/env python
"""Benchmark: Householder QR factor time of a BLR kernel matrix on one MI355X.

A step = compress the synthetic kernel matrix (untimed; the factorization is
in place, so every step starts from a freshly compressed matrix resident in
HBM) and then factor it (timed with HIP events on the stream).  Prints one
JSON line.  Workloads (synthetic points from the seeded splitmix64 generator,
Morton sorted, kernel evaluated on the device):
  c1  2048 x 1024,     2D -log(r+1e-3),  b = 128,  adjacent boxes dense, eps 1e-8, cap 16
  c2  32768 x 16384,   3D 1/(r+1e-3),    b = 256,  gap > diameter low-rank, eps 1e-8, cap 32
  c3  131072 x 65536,  3D 1/(r+1e-3),    b = 1024, gap > diameter low-rank, eps 1e-8, cap 50
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    "c1": dict(m=2048, n=1024, b=128, dim=2, kernel="log2d", rule="adjacent", tol=1e-8, cap=16),
    "c2": dict(m=32768, n=16384, b=256, dim=3, kernel="inv_r", rule="dist_gt_diam", tol=1e-8, cap=32),
    "c3": dict(m=131072, n=65536, b=1024, dim=3, kernel="inv_r", rule="dist_gt_diam", tol=1e-8, cap=50),
}
PEAK = {"fp64": 78.6e12, "mixed": 157.3e12}   # MI355X dense matrix-core peaks (FP64, FP32)


def dense_equiv_flops(m, n):
    return 2.0 * m * n * n - 2.0 / 3.0 * n ** 3


def cpu_baseline(cfg, seed):
    """The oracle (numpy FP64, untuned) timed on a bounded sample of the same
    workload: the leading (4b x 2b) block of the same kernel matrix with the
    same tile size, rule and tolerance.  Scaled to the full matrix by
    dense-equivalent flops (2mn^2 - 2n^3/3)."""
    import synth
    from oracle import blrmat, tiled
    b = cfg["b"]
    x, y = synth.kernel_points(seed, cfg["m"], cfg["n"], cfg["dim"])
    ms, ns = min(4 * b, cfg["m"]), min(2 * b, cfg["n"])
    spent = 0.0
    while True:
        xs, ys = x[:ms], y[:ns]
        A = blrmat.kernel_matrix(xs, ys, cfg["kernel"])
        mask = blrmat.lowrank_mask(xs, ys, b, cfg["rule"], ms // b, ns // b)
        blr = blrmat.compress(A, b, cfg["tol"], cfg["cap"], mask)
        t0 = time.perf_counter()
        tiled.factor(blr, cfg["tol"], cfg["cap"], copy=False)
        el = time.perf_counter() - t0
        spent += el
        # grow the sample until it holds about 8 s of work (or is the whole matrix)
        if el >= 4.0 or spent >= 15.0 or (ms == cfg["m"] and ns == cfg["n"]):
            break
        ms, ns = min(2 * ms, cfg["m"]), min(2 * ns, cfg["n"])
    rate = dense_equiv_flops(ms, ns) / el
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return {
        "value": dense_equiv_flops(cfg["m"], cfg["n"]) / rate, "unit": "s",
        "cores": cores, "kind": "oracle",
        "sample": f"oracle tiled factor of the leading {ms}x{ns} block (b={b}) of the same matrix took "
                  f"{el:.2f} s ({rate / 1e9:.2f} GFLOP/s dense-equivalent); value extrapolated to "
                  f"{cfg['m']}x{cfg['n']} by dense-equivalent flops",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default=os.environ.get("BLR_BENCH_CONFIG", "c3"), choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--variant", default="tiled", choices=["tiled", "block_column"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--stop-after-k", type=int, default=-1,
                    help="exploration only: factor the first K block columns (not a valid metric)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2208_06194_amd as P

    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    x, y = synth.kernel_points(args.seed, cfg["m"], cfg["n"], cfg["dim"])
    xd, yd = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    print(f"[bench] {args.config}: points ready in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    times, comp_times = [], []
    prof = None
    info = None
    stream = torch.cuda.current_stream()
    for step in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        tc = time.perf_counter()
        G = P.BLRMatrix.compress_kernel(xd, yd, cfg["kernel"], cfg["b"], cfg["tol"], cfg["cap"],
                                        admissibility=cfg["rule"], overflow="dense", seed=args.seed)
        torch.cuda.synchronize()
        comp_times.append(time.perf_counter() - tc)
        timed = step >= args.warmup
        if timed:
            G.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        G.factor(args.variant, args.precision, stop_after_k=args.stop_after_k)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(f"[bench] step {step} ({'timed' if timed else 'warmup'}): compress {comp_times[-1]:.2f}s "
              f"factor {ms / 1e3:.3f}s", file=sys.stderr, flush=True)
        if timed:
            times.append(ms / 1e3)
            n, tot_ms, tot_fl = G.profile_read()
            prof = (prof[0] + n, prof[1] + tot_ms, prof[2] + tot_fl) if prof else (n, tot_ms, tot_fl)
            info = G.info()
        del G

    value = float(np.median(times))
    flops = info["flops_factor"]
    out = {
        "metric": "BLR-QR factor time (s) at 131k x 65k; FP64 vs mixed at stated ||A-QR||/||A||",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-mfma+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg['m']}x{cfg['n']} {cfg['dim']}D {cfg['kernel']} kernel matrix, b={cfg['b']}, "
                        f"{cfg['rule']}, eps={cfg['tol']:g}, cap={cfg['cap']}, {args.variant} {args.precision}",
            "m": cfg["m"], "n": cfg["n"], "tile": cfg["b"], "tol": cfg["tol"], "max_rank": cfg["cap"],
            "variant": args.variant, "precision": args.precision, "config_id": args.config,
            **({"stop_after_k": args.stop_after_k} if args.stop_after_k >= 0 else {}),
        },
        "ledger_flops": flops,
        "gflops": flops / value / 1e9,
        "dense_equiv_tflops": dense_equiv_flops(cfg["m"], cfg["n"]) / value / 1e12,
        "compress_s": float(np.median(comp_times)),
        "tiles": {"dense": info["n_dense"], "lowrank": info["n_lowrank"], "fill_in": info["n_fill_in"],
                  "compress_overflow": info["compress_overflow"], "factor_overflow": info["factor_overflow"]},
        "kernel_launches": info["kernel_launches"],
    }
    if prof and prof[0] > 0:
        avg_s = prof[1] / 1e3 / prof[0]
        per_launch = prof[2] / prof[0]
        ach = per_launch / avg_s
        peak = PEAK[args.precision]
        out["roofline"] = {
            "bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": None,
            "kernel": "k_gemm<%s,128,128> (reflector-apply products)" % ("double" if args.precision == "fp64" else "float"),
            "launches": prof[0], "avg_launch_ms": avg_s * 1e3, "flops_per_launch": per_launch,
            "kernel_time_share": prof[1] / 1e3 / (value * args.steps),
        }
    if not args.no_cpu_baseline:
        tb = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed)
        print(f"[bench] cpu baseline sample done in {time.perf_counter() - tb:.1f}s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
