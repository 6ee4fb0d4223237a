"""Autotuner of the launch configuration of the factorization: the tile size
b, the panel width ib and the variant (tiled, Alg. 4, or block column,
Alg. 2) for a kernel-matrix workload.

Every candidate is compressed and factored on the device through the C ABI
(the same entry points and kernels as any other call), on the leading
sample of the workload: the first ms row points and ns column points of the
Morton-ordered sets, a compact corner of the domain with the workload's
aspect ratio.  Each candidate's factor time is the median of `repeats` runs
timed with HIP events; it is extrapolated to the full size by the ratio of
dense-equivalent flops (2 m n^2 - 2 n^3 / 3) and the fastest candidate is
returned with the whole table.  A cache file (JSON) keyed by the workload's
description keeps the result, so the search runs once per workload."""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from .api import BLRMatrix


def dense_equiv_flops(m: int, n: int) -> float:
    return 2.0 * m * n * n - 2.0 / 3.0 * n ** 3


def _key(m, n, dim, kernel, tol, max_rank, admissibility, precision, sample, candidates):
    return json.dumps({"m": m, "n": n, "dim": dim, "kernel": kernel, "tol": tol, "max_rank": max_rank,
                       "admissibility": admissibility, "precision": precision, "sample": list(sample),
                       "candidates": [list(c) for c in candidates]}, sort_keys=True)


def default_candidates(n: int, tiles=(128, 256, 512, 1024), variants=("block_column", "tiled")):
    """(b, variant, ib) triples with b at most n.  ib (16 or 32) is the widest
    inner panel; panels of more than 512 rows use 16 anyway, so 32 is only a
    separate candidate where tiles are at most 256 rows."""
    out = []
    for b in tiles:
        if b > n:
            continue
        for v in variants:
            out.append((b, v, 16))
            if b <= 256:
                out.append((b, v, 32))
    return out


def sample_shape(m: int, n: int, candidates, max_tiles_per_side: int = 16):
    """Leading sample: up to max_tiles_per_side tiles of the largest candidate
    b along n (at least the whole matrix when it is smaller), rows in the
    workload's ratio, both rounded to multiples of every candidate b."""
    bmax = max(c[0] for c in candidates)
    lcm = int(np.lcm.reduce([c[0] for c in candidates]))
    ns = min(n, max_tiles_per_side * bmax)
    ns = max(lcm, ns // lcm * lcm) if n >= lcm else n
    ms = min(m, int(round(ns * m / n)))
    ms = max(ns, ms // lcm * lcm) if m >= lcm else m
    return ms, ns


def tune_kernel_matrix(x: torch.Tensor, y: torch.Tensor, kernel: str, tol: float, max_rank: int,
                       admissibility: str = "dist_gt_diam", precision: str = "fp64", candidates=None,
                       sample=None, repeats: int = 2, cache: str | None = None, log=None) -> dict:
    """x (m, d) and y (n, d): Morton-ordered device points.  Returns
    {"best": {"tile", "variant", "ib", "predicted_s"}, "table": [...],
    "sample": [ms, ns]}."""
    m, dim = x.shape
    n = y.shape[0]
    cands = list(candidates) if candidates is not None else default_candidates(n)
    if not cands:
        raise ValueError("no candidate tile size fits the matrix")
    ms, ns = sample if sample is not None else sample_shape(m, n, cands)
    key = _key(m, n, dim, kernel, tol, max_rank, admissibility, precision, (ms, ns), cands)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            return known[key]
    xs, ys = x[:ms].contiguous(), y[:ns].contiguous()
    stream = torch.cuda.current_stream()
    scale = dense_equiv_flops(m, n) / dense_equiv_flops(ms, ns)
    table = []
    for b, variant, ib in cands:
        cap = min(max_rank, b, 128)
        times = []
        for _ in range(repeats):
            G = BLRMatrix.compress_kernel(xs, ys, kernel, b, tol, cap, admissibility=admissibility)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            G.factor(variant, precision, ib=ib)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
            inf = G.info()
            del G
        t = float(np.median(times))
        row = {"tile": b, "variant": variant, "ib": ib, "max_rank": cap, "sample_s": t,
               "predicted_s": t * scale, "tiles_dense": inf["n_dense"], "tiles_lowrank": inf["n_lowrank"]}
        table.append(row)
        if log:
            log(f"[tune] b={b} {variant} ib={ib}: {t:.3f}s on {ms}x{ns} -> {t * scale:.2f}s predicted")
    best = min(table, key=lambda r: r["sample_s"])
    out = {"best": {k: best[k] for k in ("tile", "variant", "ib", "max_rank", "predicted_s")},
           "table": table, "sample": [ms, ns], "scale": scale, "timestamp": time.time()}
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = out
        with open(cache, "w") as f:
            json.dump(known, f, indent=1)
    return out
