#!/usr/bin/env python
"""Benchmark: Householder QR factor time of a BLR kernel matrix on one MI355X.

A step = compress the synthetic kernel matrix (untimed; the factorization is
in place, so every step starts from a freshly compressed matrix resident in
HBM) and then factor it (timed with HIP events on the stream).  By default
the FP64 factor is the reported value and the mixed form (FP32 MFMA updates,
FP64 reflector generation and recompression, compressed at 1e-6) is measured
beside it; each states its Gaussian-probe estimate of ||A~ - QR|| / ||A~||.
Prints one JSON line.  Workloads (synthetic points from the seeded splitmix64 generator,
Morton sorted, kernel evaluated on the device):
  c1  2048 x 1024,     2D -log(r+1e-3),  b = 128,  adjacent boxes dense, eps 1e-8, cap 16
  c2  32768 x 16384,   3D 1/(r+1e-3),    b = 256,  gap > diameter low-rank, eps 1e-8, cap 32
  c3  131072 x 65536,  3D 1/(r+1e-3),    b = 1024, gap > diameter low-rank, eps 1e-8, cap 50
  cr  6000 x 3000,     3D 1/(r+1e-3),    b = 128,  every tile compressed, rank > b/2 dense (cap 64), eps 1e-8;
      m and n are not multiples of b
  c4  64 matrices, m log-uniform in [4096, 32768], n = m/2, 3D 1/(r+1e-3), b = 256, eps 1e-8,
      cap 64, each with a 16-RHS least-squares solve: the plain form (one factorization after
      the other) against the batched form (blr_qr_factor_batch), in FP64 and in the mixed form
      with FP64 iterative refinement of the solve
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    "c1": dict(m=2048, n=1024, b=128, dim=2, kernel="log2d", rule="adjacent", tol=1e-8, cap=16),
    "c2": dict(m=32768, n=16384, b=256, dim=3, kernel="inv_r", rule="dist_gt_diam", tol=1e-8, cap=32),
    "c3": dict(m=131072, n=65536, b=1024, dim=3, kernel="inv_r", rule="dist_gt_diam", tol=1e-8, cap=50),
    # the differentiated least-squares workload: 65536x32768, b = 512, 32 right-hand sides
    "c5": dict(m=65536, n=32768, b=512, dim=3, kernel="inv_r", rule="dist_gt_diam", tol=1e-8, cap=32),
    # compress-and-revert (non-geometric admissibility): every off-diagonal
    # tile compressed, those whose eps-rank exceeds b/2 stored dense; m and n
    # not multiples of b (ragged edge tiles, factored through the embedding)
    "cr": dict(m=6000, n=3000, b=128, dim=3, kernel="inv_r", rule="weak", tol=1e-8, cap=64),
    # batched forms: 64 independent matrices, rows log-uniform in [4096, 32768]
    # (multiples of 512), n = m/2, each followed by a 16-RHS least-squares solve
    "c4": dict(kind="batch", count=64, m_lo=4096, m_hi=32768, b=256, dim=3, kernel="inv_r",
               rule="dist_gt_diam", tol=1e-8, cap=64, nrhs=16),
    # the paper's random-BLR accuracy workload (8192x4096 row): N(0,1) dense
    # diagonal tiles, every other tile a rank-1 product, weak admissibility
    "wr": dict(m=8192, n=4096, b=128, kind="random_blr", rank=1, rule="weak", tol=1e-10, cap=128),
}
PEAK = {"fp64": 78.6e12, "mixed": 157.3e12}   # MI355X dense matrix-core peaks (FP64, FP32)
HBM_PEAK_TBS = 8.0                                # MI355X HBM3E bandwidth, TB/s

# HBM traffic per launch of the dominant kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) over the factor's launches, scaled by what the same
# counters read for a plain 1 GiB device copy (FETCH x 2.0, WRITE x 1.0); the
# commands and raw figures are in profiles/.  Valid only for the kernel source
# the counters were taken on (sha256 of csrc/gemm.hip); otherwise null.
TRAFFIC = {
    ("c3", "fp64", "block_column"): {
        "gemm_sha256": "3f4373a2f9485e0571df44419252c73c34ece5d4a830b57dd9e233db0528d6a7",
        "bytes_per_launch": 15870986701,
    },
}


def measured_traffic(config, precision, variant):
    import hashlib
    t = TRAFFIC.get((config, precision, variant))
    if not t:
        return None
    src = os.path.join(ROOT, "paper_2208_06194_amd", "csrc", "gemm.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["gemm_sha256"]:
            return None
    return t["bytes_per_launch"]


def dense_equiv_flops(m, n):
    return 2.0 * m * n * n - 2.0 / 3.0 * n ** 3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, seed, variant, limit_s=30.0):
    """The oracle (numpy FP64, untuned) timed on a bounded sample of the same
    workload: a leading block (from 4b x 2b, grown by 1.5x per side while the
    next sample's predicted time still fits in limit_s) of the same kernel
    matrix with the same tile size, rule and tolerance, factored by the same
    variant.  Scaled to the full matrix by dense-equivalent flops
    (2mn^2 - 2n^3/3)."""
    import synth
    from oracle import blockcol, blrmat, tiled
    fac = tiled.factor if variant == "tiled" else blockcol.factor
    b = cfg["b"]
    rblr = cfg.get("kind") == "random_blr"
    if not rblr:
        x, y = synth.kernel_points(seed, cfg["m"], cfg["n"], cfg["dim"])
    ms, ns = min(4 * b, cfg["m"]), min(2 * b, cfg["n"])
    spent = 0.0
    grow = lambda v, cap: min(cap, -(-(3 * v // 2) // b) * b)
    while True:
        if rblr:
            A = synth.random_blr_dense(seed, ms, ns, b, cfg["rank"])
            mask = np.ones((ms // b, ns // b), bool)
        else:
            xs, ys = x[:ms], y[:ns]
            A = blrmat.kernel_matrix(xs, ys, cfg["kernel"])
            mask = blrmat.lowrank_mask(xs, ys, b, cfg["rule"], ms // b, ns // b)
        blr = blrmat.compress(A, b, cfg["tol"], cfg["cap"], mask)
        t0 = time.perf_counter()
        fac(blr, cfg["tol"], cfg["cap"], copy=False)
        el = time.perf_counter() - t0
        spent += el
        if ms == cfg["m"] and ns == cfg["n"]:
            break
        m2, n2 = grow(ms, cfg["m"]), grow(ns, cfg["n"])
        predicted = el * dense_equiv_flops(m2, n2) / dense_equiv_flops(ms, ns)
        if spent + predicted > limit_s:
            break
        ms, ns = m2, n2
    rate = dense_equiv_flops(ms, ns) / el
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return {
        "value": dense_equiv_flops(cfg["m"], cfg["n"]) / rate, "unit": "s",
        "cores": cores, "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
        "sample": f"oracle {variant} factor of " + (f"a {ms}x{ns} random BLR matrix of the same tile size, rank and "
                  f"tolerance" if rblr else f"the leading {ms}x{ns} block (b={b}) of the same matrix") + " took "
                  f"{el:.2f} s ({rate / 1e9:.2f} GFLOP/s dense-equivalent); value extrapolated to "
                  f"{cfg['m']}x{cfg['n']} by dense-equivalent flops",
    }


def accuracy_probes(G, probes, ax):
    """Gaussian-probe estimates, from the factor of A~ and the products A~ G
    taken before the factorization:  Res = ||(A~ - Q R) G||_F / ||A~ G||_F and
    Orth = ||(Q1^T Q1 - I) G||_F / (sqrt(s) sqrt(n)), s probes."""
    import torch
    inf = G.info()
    m, n, mp = inf["m"], inf["n"], inf["m_pad"]   # Q acts on the m_pad rows of a ragged matrix's embedding
    s = probes.shape[1]
    rg = G.matmul(probes, "R")
    pad = torch.zeros((mp, s), dtype=torch.float64, device=probes.device)
    pad[:n] = rg
    qr = G.apply_qt(pad, trans=True)
    qr[:m] -= ax
    res = float(torch.linalg.norm(qr) / torch.linalg.norm(ax))
    pad.zero_()
    pad[:n] = probes
    back = G.apply_qt(G.apply_qt(pad, trans=True))
    back[:n] -= probes
    orth = float(torch.linalg.norm(back) / np.sqrt(s) / np.sqrt(n))
    return res, orth


class Phase:
    """Wall-clock plan of one measured form: warmup and timed step counts
    clamped so that the form ends by its deadline.  The first cycle (compress
    + factor) is timed and sets the estimate for the rest."""

    def __init__(self, warmup, steps, deadline):
        self.want_warmup, self.want_steps, self.deadline = warmup, steps, deadline
        self.warmup, self.steps = warmup, steps
        self.cycle = None
        self.clamped = False

    def plan_after_first(self, cycle_s, extra_s, first_was_warmup):
        """After the first cycle: how many more warmups and timed steps fit
        before the deadline (at least one timed step; extra_s is the
        once-per-form probe and solve time on the last step)."""
        self.cycle = cycle_s
        left = self.deadline - time.perf_counter() - extra_s
        fit = max(0, int(left // cycle_s))
        if first_was_warmup:
            # further warmups only when every requested timed step still fits
            more_w = max(0, min(self.want_warmup - 1, fit - self.want_steps))
            self.warmup = 1 + more_w
            self.steps = max(1, min(self.want_steps, fit - more_w))
        else:
            self.warmup = 0
            self.steps = max(1, min(self.want_steps, 1 + fit))
        self.clamped = self.warmup < self.want_warmup or self.steps < self.want_steps


def run(args, cfg, precision, tol, xd, yd, dev, phase, keep_a=False, rhs=None, x_ref=None, refine=0):
    """Compress (untimed) and factor (timed) for the phase's warmup + steps
    cycles; the last timed step also takes the accuracy probes, Q^T B and the
    least-squares solve of rhs (refined with FP64 residuals when refine > 0,
    which needs keep_a), with the solution's error against x_ref."""
    import torch
    import synth
    import paper_2208_06194_amd as P
    times, comp_times = [], []
    prof, info, acc, solve = {"fp64": (0, 0.0, 0.0), "fp32": (0, 0.0, 0.0)}, None, None, None
    x_out = None
    stream = torch.cuda.current_stream()
    probes = torch.tensor(synth.rhs(args.seed + 17, cfg["n"], args.probes), device=dev)
    step = 0
    while step < phase.warmup + phase.steps:
        torch.cuda.synchronize()
        tc = time.perf_counter()
        if cfg.get("kind") == "random_blr":
            G = P.BLRMatrix.compress_dense(xd, cfg["b"], tol, cfg["cap"], admissibility="weak",
                                           overflow="dense", seed=args.seed)
        else:
            G = P.BLRMatrix.compress_kernel(xd, yd, cfg["kernel"], cfg["b"], tol, cfg["cap"],
                                            admissibility=cfg["rule"], overflow="dense", seed=args.seed)
        torch.cuda.synchronize()
        comp_times.append(time.perf_counter() - tc)
        timed = step >= phase.warmup
        # A~ times the probes before the in-place factorization (every step:
        # which step is the last is known only after the first cycle)
        ax = G.matmul(probes, "A") if args.probes > 0 else None
        if timed:
            G.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        G.factor(args.variant, precision, stop_after_k=args.stop_after_k, keep_a=keep_a or args.adjoint)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(f"[bench] {precision} eps={tol:g} step {step} ({'timed' if timed else 'warmup'}): "
              f"compress {comp_times[-1]:.2f}s factor {ms / 1e3:.3f}s", file=sys.stderr, flush=True)
        if timed:
            times.append(ms / 1e3)
            for kk in ("fp64", "fp32"):
                n, tot_ms, tot_fl = G.profile_read(kk)
                prof[kk] = (prof[kk][0] + n, prof[kk][1] + tot_ms, prof[kk][2] + tot_fl)
            info = G.info()
        if step == 0:
            # the first cycle sets the plan of the rest of the phase; the probe
            # and solve step at the end costs about a quarter of a cycle more
            cyc = time.perf_counter() - tc
            phase.plan_after_first(cyc, 0.25 * cyc + 2.0, phase.warmup > 0)
            print(f"[bench] {precision} eps={tol:g}: cycle {cyc:.1f}s -> warmup {phase.warmup}, steps "
                  f"{phase.steps}" + (" (clamped to the time budget)" if phase.clamped else ""),
                  file=sys.stderr, flush=True)
        last = step == phase.warmup + phase.steps - 1
        if last and ax is not None and args.stop_after_k < 0:
            te = time.perf_counter()
            acc = accuracy_probes(G, probes, ax)
            print(f"[bench] {precision}: Res~ {acc[0]:.2e} Orth {acc[1]:.2e}", file=sys.stderr, flush=True)
            # Q^T B and the least-squares solve with 16 right-hand sides (untimed by the metric)
            B16 = rhs if rhs is not None else torch.tensor(synth.rhs(args.seed + 23, cfg["m"], 16), device=dev)
            B16p = torch.zeros((G.info()["m_pad"], B16.shape[1]), dtype=torch.float64, device=dev)
            B16p[:cfg["m"]] = B16
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            f0.record(stream)
            G.apply_qt(B16p)
            f1.record(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x_out = G.lstsq(B16, max_refine=refine)
            torch.cuda.synchronize()
            solve = {"nrhs": int(B16.shape[1]), "apply_qt_s": f0.elapsed_time(f1) / 1e3,
                     "lstsq_s": time.perf_counter() - t0, "max_refine": refine}
            if refine > 0:
                t0 = time.perf_counter()
                x0 = G.lstsq(B16)
                torch.cuda.synchronize()
                solve["lstsq_unrefined_s"] = time.perf_counter() - t0
            if x_ref is not None:
                nr = float(torch.linalg.norm(x_ref))
                solve["x_rel_err_vs_fp64"] = float(torch.linalg.norm(x_out - x_ref)) / nr
                if refine > 0:
                    solve["x_rel_err_vs_fp64_unrefined"] = float(torch.linalg.norm(x0 - x_ref)) / nr
            if keep_a and ax is not None:
                # the normal-equation residual of each solution against A~ itself
                # (the kept copy): eta = ||A~^T (b - A~ x)|| / (||A~||_F ||b - A~ x||)
                # per column, the largest reported; ||A~||_F from A~ times the probes
                anorm = float(torch.linalg.norm(ax)) / np.sqrt(probes.shape[1])

                def eta(x):
                    r = B16 - G.matmul(x, "A")
                    return float((torch.linalg.norm(G.matmul(r, "AT"), dim=0)
                                  / (anorm * torch.linalg.norm(r, dim=0))).max())
                solve["eta_ne"] = eta(x_out)
                if refine > 0:
                    solve["eta_ne_unrefined"] = eta(x0)
                if x_ref is not None:
                    solve["eta_ne_fp64_solution"] = eta(x_ref)
            # HBM roofline of Q^T B: the reflectors are read twice (Y^T B, then
            # B -= Y W), counted as if every tile were dense
            gi = G.info()
            b, m, q = cfg["b"], gi["m_pad"], gi["n_pad"] // cfg["b"]
            ybytes = sum((m - k * b) * b * 8 for k in range(q))
            solve["apply_qt_bytes_dense_equiv"] = 2 * ybytes
            solve["apply_qt_gbs"] = 2 * ybytes / solve["apply_qt_s"] / 1e9
            solve["apply_qt_hbm_frac"] = solve["apply_qt_gbs"] / (HBM_PEAK_TBS * 1e3)
            if args.explicit_q:
                # the explicit BLR Q~ and the paper's Orth / Res measured on it
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Qt = G.form_q()
                torch.cuda.synchronize()
                tq = time.perf_counter() - t0
                g = probes[:, :min(8, probes.shape[1])]
                qg = Qt.matmul(g, "A")
                orth_q = float(torch.linalg.norm(Qt.matmul(qg, "AT") - g) / torch.linalg.norm(g))
                res_q = float(torch.linalg.norm(Qt.matmul(G.matmul(g, "R"), "A") - ax[:, :g.shape[1]])
                              / torch.linalg.norm(ax[:, :g.shape[1]]))
                qi = Qt.info()
                solve["explicit_q"] = {"form_q_s": tq, "orth_est": orth_q, "res_est": res_q,
                                       "tiles_dense": qi["n_dense"], "tiles_lowrank": qi["n_lowrank"]}
                del Qt
                print(f"[bench] {precision}: explicit Q~ {tq:.3f}s, Orth~ {orth_q:.2e}, Res~ {res_q:.2e}",
                      file=sys.stderr, flush=True)
            if args.mgs:
                # the comparison method on the same compressed matrix: blocked
                # modified Gram-Schmidt, Q~ explicit, with the same probes
                if cfg.get("kind") == "random_blr":
                    Gm = P.BLRMatrix.compress_dense(xd, cfg["b"], tol, cfg["cap"], admissibility="weak",
                                                    overflow="dense", seed=args.seed)
                else:
                    Gm = P.BLRMatrix.compress_kernel(xd, yd, cfg["kernel"], cfg["b"], tol, cfg["cap"],
                                                     admissibility=cfg["rule"], overflow="dense", seed=args.seed)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Rm = Gm.mgs_qr()
                torch.cuda.synchronize()
                tm = time.perf_counter() - t0
                res_m = float(torch.linalg.norm(Gm.matmul(Rm.matmul(probes, "A"), "A") - ax) / torch.linalg.norm(ax))
                orth_m = float(torch.linalg.norm(Gm.matmul(Gm.matmul(probes, "A"), "AT") - probes)
                               / np.sqrt(probes.shape[1]) / np.sqrt(cfg["n"]))
                solve["mgs"] = {"factor_s": tm, "res_est": res_m, "orth_est": orth_m,
                                "note": "blocked modified Gram-Schmidt BLR-QR of the same compressed matrix "
                                        "(Q~ explicit); Gaussian-probe estimates as for the Householder factor"}
                del Gm, Rm
                print(f"[bench] {precision}: MGS {tm:.3f}s Res~ {res_m:.2e} Orth {orth_m:.2e}", file=sys.stderr,
                      flush=True)
            if args.adjoint:
                # backward pass of the least-squares solve: dL/dB and dL/dtiles
                nr = args.adjoint_rhs
                Bq = torch.tensor(synth.rhs(args.seed + 29, cfg["m"], nr), device=dev)
                Xq = G.lstsq(Bq)
                Xbar = torch.tensor(synth.rhs(args.seed + 31, cfg["n"], nr), device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                grads = G.lstsq_adjoint(Bq, Xq, Xbar)
                torch.cuda.synchronize()
                solve["adjoint"] = {"nrhs": nr, "adjoint_s": time.perf_counter() - t0}
                del grads
                print(f"[bench] {precision}: least-squares adjoint {solve['adjoint']['adjoint_s']:.3f}s "
                      f"({nr} right-hand sides)", file=sys.stderr, flush=True)
            print(f"[bench] {precision}: apply Q^T {solve['apply_qt_s']:.3f}s lstsq {solve['lstsq_s']:.3f}s "
                  f"({solve['nrhs']} right-hand sides, refine {refine})", file=sys.stderr, flush=True)
            phase.extra = time.perf_counter() - te
        del G, ax
        step += 1
    value = float(np.median(times))
    return {"value": value, "compress_s": float(np.median(comp_times)), "info": info, "tol": tol,
            "res_est": acc[0] if acc else None, "orth_est": acc[1] if acc else None, "prof": prof,
            "solve": solve, "x": x_out, "steps": phase.steps, "warmup": phase.warmup,
            "times": times}


def run_batch(args, cfg):
    """The batched-forms workload: every member compressed (untimed), then
    factored and solved for 16 right-hand sides one matrix after the other
    (plain), or as one batch (blr_qr_factor_batch, blr_lstsq_solve_batch);
    FP64 and mixed (FP32 MFMA updates, the solve refined with FP64 residuals
    against the kept A~)."""
    import torch
    import synth
    import paper_2208_06194_amd as P
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = synth.batch_rows(args.seed, cfg["count"], cfg["m_lo"], cfg["m_hi"], 2 * cfg["b"])
    seeds = [1000 * (args.seed + 1) + i for i in range(cfg["count"])]
    pts = []
    for sd, m in zip(seeds, rows):
        x, y = synth.kernel_points(sd, int(m), int(m) // 2, cfg["dim"])
        pts.append((torch.tensor(x, device=dev), torch.tensor(y, device=dev)))
    rhs = [torch.tensor(synth.rhs(sd + 7, int(m), cfg["nrhs"]), device=dev) for sd, m in zip(seeds, rows)]
    print(f"[bench] c4: {cfg['count']} members, rows {int(rows.min())}..{int(rows.max())}", file=sys.stderr,
          flush=True)

    def compress_all():
        t0 = time.perf_counter()
        Gs = [P.BLRMatrix.compress_kernel(x, y, cfg["kernel"], cfg["b"], cfg["tol"], cfg["cap"],
                                          admissibility=cfg["rule"], overflow="dense", seed=args.seed)
              for (x, y) in pts]
        torch.cuda.synchronize()
        return Gs, time.perf_counter() - t0

    out = {}
    x_ref = None
    precs = ("fp64", "mixed") if args.precision == "both" else (args.precision,)
    forms = ("plain", "batched") if args.batch_form == "both" else (args.batch_form,)
    for prec in precs:
        refine = 5 if prec == "mixed" else 0
        res_prec = {}
        x_plain = None
        for form in forms:
            Gs, tc = compress_all()
            probes, ax = None, None
            if form == "batched":
                probes = [torch.tensor(synth.rhs(args.seed + 17, G.info()["n"], 4), device=dev) for G in Gs]
                ax = [G.matmul(pr, "A") for G, pr in zip(Gs, probes)]
                Gs[0].profile(True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            if form == "plain":
                for G in Gs:
                    G.factor("block_column", prec, keep_a=refine > 0)
            else:
                P.factor_batch(Gs, precision=prec, keep_a=refine > 0)
            e1.record(stream)
            torch.cuda.synchronize()
            tf = e0.elapsed_time(e1) / 1e3
            t0 = time.perf_counter()
            if form == "plain":
                X = [G.lstsq(B, max_refine=refine) for G, B in zip(Gs, rhs)]
            else:
                X = P.lstsq_batch(Gs, rhs, max_refine=refine)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            inf = [G.info() for G in Gs]
            r = {"factor_s": tf, "lstsq_s": ts, "total_s": tf + ts, "compress_s": tc,
                 "kernel_launches": (sum(i["kernel_launches"] for i in inf) if form == "plain"
                                     else inf[0]["kernel_launches"]),
                 "factor_overflow": sum(i["factor_overflow"] for i in inf)}
            if form == "batched":
                acc = [accuracy_probes(G, pr, a) for G, pr, a in zip(Gs, probes, ax)]
                r["res_est_max"] = max(a[0] for a in acc)
                r["orth_est_max"] = max(a[1] for a in acc)
                n_g, ms_g, fl_g = Gs[0].profile_read("fp64" if prec == "fp64" else "fp32")
                if n_g > 0:
                    r["dominant_gemm"] = {"launches": n_g, "avg_launch_ms": ms_g / n_g,
                                          "tflops": fl_g / (ms_g / 1e3) / 1e12}
                r["ledger_flops"] = sum(i["flops_factor"] for i in inf)
                r["tiles"] = {"dense": sum(i["n_dense"] for i in inf), "lowrank": sum(i["n_lowrank"] for i in inf)}
                xs = [t.cpu().numpy() for t in X]
                if x_plain is not None:
                    r["identical_to_plain"] = all(np.array_equal(a, b) for a, b in zip(xs, x_plain))
                if prec == "fp64":
                    x_ref = xs
                elif x_ref is not None:
                    r["lstsq_rel_err_vs_fp64_max"] = max(
                        float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(xs, x_ref))
            if form == "plain":
                x_plain = [t.cpu().numpy() for t in X]
            res_prec[form] = r
            print(f"[bench] c4 {prec} {form}: factor {tf:.3f}s lstsq {ts:.3f}s "
                  f"(launches {r['kernel_launches']})", file=sys.stderr, flush=True)
            del Gs, X
            torch.cuda.synchronize()
        if len(forms) == 2:
            res_prec["batched_speedup_factor"] = res_prec["plain"]["factor_s"] / res_prec["batched"]["factor_s"]
            res_prec["batched_speedup_total"] = res_prec["plain"]["total_s"] / res_prec["batched"]["total_s"]
        out[prec] = res_prec
    dense_fl = float(sum(dense_equiv_flops(int(a), int(a) // 2) for a in rows))
    return out, rows, dense_fl


def roofline(prof, kernel, args, timed_s):
    """Roofline object of the dominant kernel from its HIP-event record:
    average algorithmic flops per launch / average launch duration."""
    n, tot_ms, tot_fl = prof
    if n <= 0:
        return None
    avg_s = tot_ms / 1e3 / n
    per_launch = tot_fl / n
    ach = per_launch / avg_s
    peak = PEAK["fp64" if kernel == "fp64" else "mixed"]
    ct = "double" if kernel == "fp64" else "float"
    return {
        "bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
        "frac": ach / peak,
        "traffic": measured_traffic(args.config, kernel, args.variant),
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": f"k_gemm_fast<{ct}, false, false> (128x128 MFMA tiles, untransposed: trailing updates "
                  f"and block reflectors)",
        "launches": n, "avg_launch_ms": avg_s * 1e3, "flops_per_launch": per_launch,
        "kernel_time_share": tot_ms / 1e3 / timed_s,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget", type=float, default=float(os.environ.get("BLR_BENCH_BUDGET", 450.0)),
                    help="wall-clock seconds from start to the JSON line; warmup and timed steps of every "
                         "form are clamped to fit, and the counts that ran are reported")
    ap.add_argument("--config", default=os.environ.get("BLR_BENCH_CONFIG", "c3"), choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"],
                    help="both: the FP64 factor (the reported value) and the mixed form beside it")
    ap.add_argument("--mixed-tol", type=float, default=1e-6,
                    help="compression tolerance of the mixed form's second, looser accuracy point (the first "
                         "uses the FP64 tolerance)")
    ap.add_argument("--refine", type=int, default=10,
                    help="FP64 refinement steps of the mixed form's least-squares solve")
    ap.add_argument("--variant", default="block_column", choices=["tiled", "block_column"])
    ap.add_argument("--probes", type=int, default=8, help="Gaussian probes for the Res / Orth estimates")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the least-squares adjoint (the factor keeps a copy of A~)")
    ap.add_argument("--adjoint-rhs", type=int, default=32)
    ap.add_argument("--mgs", action="store_true",
                    help="also time the blocked modified Gram-Schmidt BLR-QR of the same matrix (the paper's "
                         "comparison method) and estimate its Res and Orth")
    ap.add_argument("--explicit-q", action="store_true",
                    help="also form the explicit BLR Q~ and estimate the paper's Orth and Res on it")
    ap.add_argument("--batch-form", default="both", choices=["plain", "batched", "both"],
                    help="c4: the forms to run (both: one factorization after the other, then the batch)")
    ap.add_argument("--tune", action="store_true",
                    help="kernel-matrix configs: first run the autotuner of tile size, variant and ib on a "
                         "leading sample and report its table (the reported value keeps the config's tile size)")
    ap.add_argument("--stop-after-k", type=int, default=-1,
                    help="exploration only: factor the first K block columns (not a valid metric)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only (the factorization is single-device); --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth

    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    if cfg.get("kind") == "batch":
        res, rows, dense_fl = run_batch(args, cfg)
        p0 = "fp64" if "fp64" in res else "mixed"
        f0 = "batched" if "batched" in res[p0] else "plain"
        value = res[p0][f0]["total_s"]
        out = {
            "metric": f"batch of 64 BLR matrices: factor + 16-RHS least-squares time (s), {f0} form",
            "value": value, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": value * 1e3,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if p0 == "fp64" else "f32-mfma+f64",
            "data": "synthetic",
            "config": {"workload": f"{cfg['count']} {cfg['dim']}D {cfg['kernel']} kernel matrices, m log-uniform in "
                                   f"[{cfg['m_lo']}, {cfg['m_hi']}] (multiples of {2 * cfg['b']}), n=m/2, "
                                   f"b={cfg['b']}, {cfg['rule']}, eps={cfg['tol']:g}, cap={cfg['cap']}, "
                                   f"{cfg['nrhs']} RHS each", "config_id": args.config,
                       "rows": [int(a) for a in rows]},
            "dense_equiv_tflops": dense_fl / res[p0][f0]["factor_s"] / 1e12,
            **res,
        }
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    if cfg.get("kind") == "random_blr":
        # the dense random-BLR matrix on the device, from its seeded tile factors
        m, n, b, r = cfg["m"], cfg["n"], cfg["b"], cfg["rank"]
        p, q = m // b, n // b
        D, X, Y = synth.random_blr_tiles(args.seed, m, n, b, r)
        Xd = torch.tensor(X.reshape(p * q, b, r), device=dev)
        Yt = torch.tensor(Y.reshape(p * q, b, r), device=dev).transpose(1, 2).contiguous()
        tiles = torch.bmm(Xd, Yt)
        del Xd, Yt
        for k in range(q):
            tiles[k * q + k] = torch.tensor(D[k], device=dev)
        xd = tiles.reshape(p, q, b, b).permute(0, 2, 1, 3).reshape(m, n).contiguous()
        yd = None
        del tiles
        print(f"[bench] {args.config}: random BLR matrix ready in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)
    else:
        x, y = synth.kernel_points(args.seed, cfg["m"], cfg["n"], cfg["dim"])
        xd, yd = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
        print(f"[bench] {args.config}: points ready in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)

    tuned = None
    if args.tune and yd is not None:
        from paper_2208_06194_amd import tune
        tiles = tuple(t for t in (128, 256, 512, 1024) if cfg["b"] // 4 <= t <= cfg["b"] * 2)
        tuned = tune.tune_kernel_matrix(
            xd, yd, cfg["kernel"], cfg["tol"], cfg["cap"], admissibility=cfg["rule"],
            precision="mixed" if args.precision == "mixed" else "fp64",
            candidates=tune.default_candidates(cfg["n"], tiles=tiles, variants=(args.variant,)),
            log=lambda s: print(s, file=sys.stderr, flush=True))
        tuned["note"] = ("factor seconds of each candidate on the leading sample (median of 2), scaled to the "
                         "full size by dense-equivalent flops; the reported value keeps the config's tile size")

    # wall-clock plan: the forms share what is left of the budget after the
    # set-up, less a reserve for the CPU baseline; each form gets at least
    # one timed step
    deadline = T_START + args.budget
    cpu_reserve = 0.0 if args.no_cpu_baseline else 45.0
    both = args.precision == "both" and args.stop_after_k < 0
    shares = [("main", 0.5 if both else 1.0)]
    if both:
        shares += [("mixed_same_eps", 0.3), ("mixed_loose_eps", 0.2)]
    left = max(0.0, deadline - time.perf_counter() - cpu_reserve)
    ends, acc_t = {}, time.perf_counter()
    for name, frac in shares:
        acc_t += frac * left
        ends[name] = acc_t

    main_prec = "mixed" if args.precision == "mixed" else "fp64"
    main_tol = cfg["tol"] if main_prec == "fp64" else args.mixed_tol
    rhs16 = torch.tensor(synth.rhs(args.seed + 23, cfg["m"], 16), device=dev)
    ph = Phase(args.warmup, args.steps, ends["main"])
    r = run(args, cfg, main_prec, main_tol, xd, yd, dev, ph, rhs=rhs16)
    info = r["info"]
    value = r["value"]
    out = {
        "metric": "BLR-QR factor time (s) at 131k x 65k; FP64 vs mixed at stated ||A-QR||/||A||",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": r["warmup"],
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32-mfma+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg['m']}x{cfg['n']} random BLR (rank-{cfg['rank']} off-diagonal tiles), b={cfg['b']}, "
                         if cfg.get("kind") == "random_blr" else
                         f"{cfg['m']}x{cfg['n']} {cfg['dim']}D {cfg['kernel']} kernel matrix, b={cfg['b']}, ") +
                        f"{cfg['rule']}, eps={r['tol']:g}, cap={cfg['cap']}, {args.variant} {main_prec}",
            "m": cfg["m"], "n": cfg["n"], "tile": cfg["b"], "tol": r["tol"], "max_rank": cfg["cap"],
            "variant": args.variant, "precision": main_prec, "config_id": args.config,
            **({"stop_after_k": args.stop_after_k} if args.stop_after_k >= 0 else {}),
        },
        "timing": {"requested_steps": args.steps, "requested_warmup": args.warmup, "budget_s": args.budget,
                   "step_times_s": r["times"],
                   "note": "a step is one fresh compression (untimed) and one factorization (timed with HIP "
                           "events); warmup and steps are clamped to the wall-clock budget after the first "
                           "cycle is timed, and the counts that ran are reported"},
        "res_est": r["res_est"],
        "orth_est": r["orth_est"],
        "accuracy_note": f"Gaussian-probe estimates ({args.probes} probes) of ||A~-QR||_F/||A~||_F and "
                         "||Q1^T Q1 - I||_F/sqrt(n); A~ is the compressed matrix (||A~-A|| <= eps ||A|| per tile)",
        "solve_16rhs": r["solve"],
        "ledger_flops": info["flops_factor"],
        "gflops": info["flops_factor"] / value / 1e9,
        "dense_equiv_tflops": dense_equiv_flops(cfg["m"], cfg["n"]) / value / 1e12,
        "compress_s": r["compress_s"],
        "tiles": {"dense": info["n_dense"], "lowrank": info["n_lowrank"], "fill_in": info["n_fill_in"],
                  "compress_overflow": info["compress_overflow"], "factor_overflow": info["factor_overflow"]},
        "kernel_launches": info["kernel_launches"],
    }
    if tuned:
        out["tune"] = tuned
    # the dominant kernel of the reported value: its launches in the timed
    # factorizations of the reported form
    main_k = "fp64" if main_prec == "fp64" else "fp32"
    rf = roofline(r["prof"][main_k], main_k, args, value * r["steps"])
    if rf:
        out["roofline"] = rf
    if both:
        # the mixed form at the FP64 compression tolerance: the factor, and the
        # least-squares solve refined with FP64 residuals against the kept A~,
        # whose solution is compared with the FP64 one
        x64 = r["x"]
        mx = run(args, cfg, "mixed", cfg["tol"], xd, yd, dev, Phase(args.warmup, args.steps, ends["mixed_same_eps"]),
                 keep_a=True, rhs=rhs16, x_ref=x64, refine=args.refine)
        rfm = roofline(mx["prof"]["fp32"], "fp32", args, mx["value"] * mx["steps"])
        fp64_total = value + r["solve"]["lstsq_s"]
        mx_total = mx["value"] + mx["solve"]["lstsq_s"]
        out["mixed"] = {
            "value": mx["value"], "unit": "s", "tol": mx["tol"], "steps": mx["steps"], "warmup": mx["warmup"],
            "res_est": mx["res_est"], "orth_est": mx["orth_est"],
            "factor_speedup_vs_fp64": value / mx["value"],
            "note": "same compression tolerance as the FP64 value; the factor keeps a copy of A~ for the FP64 "
                    "refinement of the solve (the copy is inside the timed factor); products with K > 1024 add "
                    "their FP32 partial sums into FP64 every 1024 of K",
            "solve_16rhs": mx["solve"],
            "tiles": {"dense": mx["info"]["n_dense"], "lowrank": mx["info"]["n_lowrank"],
                      "fill_in": mx["info"]["n_fill_in"], "factor_overflow": mx["info"]["factor_overflow"]},
            **({"roofline": rfm} if rfm else {}),
        }
        out["same_accuracy_solve"] = {
            "fp64_factor_plus_solve_s": fp64_total,
            "mixed_factor_plus_refined_solve_s": mx_total,
            "speedup": fp64_total / mx_total,
            "refine_steps_max": args.refine,
            "x_rel_err_mixed_refined_vs_fp64": mx["solve"].get("x_rel_err_vs_fp64"),
            "x_rel_err_mixed_unrefined_vs_fp64": mx["solve"].get("x_rel_err_vs_fp64_unrefined"),
            "eta_ne_mixed_refined": mx["solve"].get("eta_ne"),
            "eta_ne_mixed_unrefined": mx["solve"].get("eta_ne_unrefined"),
            "eta_ne_fp64": mx["solve"].get("eta_ne_fp64_solution"),
            "note": "16 Gaussian right-hand sides; both solve min ||A~ x - b|| for the same A~ (same compression "
                    "tolerance and seed); the mixed solution is refined with FP64 residuals",
        }
        del x64, mx
        # a second, looser accuracy point of the mixed form (a different
        # compression tolerance, so less work: not an equal-accuracy figure)
        ml = run(args, cfg, "mixed", args.mixed_tol, xd, yd, dev,
                 Phase(args.warmup, args.steps, ends["mixed_loose_eps"]))
        out["mixed_loose_eps"] = {
            "value": ml["value"], "unit": "s", "tol": ml["tol"], "steps": ml["steps"], "warmup": ml["warmup"],
            "res_est": ml["res_est"], "orth_est": ml["orth_est"],
            "note": "a different accuracy point: compression at this looser tolerance leaves lower ranks",
            "tiles": {"dense": ml["info"]["n_dense"], "lowrank": ml["info"]["n_lowrank"],
                      "fill_in": ml["info"]["n_fill_in"], "factor_overflow": ml["info"]["factor_overflow"]},
        }
        del ml
    if not args.no_cpu_baseline:
        tb = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed, args.variant,
                                           max(5.0, min(30.0, deadline - time.perf_counter() - 5.0)))
        print(f"[bench] cpu baseline sample done in {time.perf_counter() - tb:.1f}s", file=sys.stderr, flush=True)
    out["timing"]["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
