"""Launch-shape autotuner of the batched form.

The batched form's global-memory grid (orders above 96, one workgroup per
matrix, H and Q in global memory) is bound by the memory round trips of the
double-shift chase and by the cache footprint of the matrices in flight:
more workgroups per CU hide more latency until their rows and columns no
longer fit the CU's share of L2, and large orders are better run with half
the grid.  The tuner times each (workgroups per CU, order above which half
the grid is used) candidate on a seeded sample drawn like the workload
(Gaussian Hessenberg matrices with orders uniform in [lo, hi]) and installs
the fastest whose solves all succeeded.  The paper calibrates StarPU
performance models instead (Sec. 3); this table plays that role for the
batched form.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Optional, Sequence, Tuple

import numpy as np
import torch

from . import api

CANDIDATES: Tuple[Tuple[int, int], ...] = ((1, 4095), (2, 4095), (2, 320), (2, 200), (2, 160), (2, 128),
                                           (3, 320), (3, 200), (4, 160))


def sample(lo: int, hi: int, count: int, seed: int, device) -> tuple:
    """Seeded Gaussian Hessenberg matrices (N(0,1) on and above the first
    subdiagonal) with orders uniform in [lo, hi], packed column major."""
    sizes = np.random.default_rng(seed).integers(lo, hi + 1, size=count)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    mats = [torch.randn(int(n), int(n), generator=g, dtype=torch.float64, device=device).triu(-1)
            for n in sizes]
    return [int(s) for s in sizes], api.pack(mats)


Sampler = Callable[[int, int, int, int, torch.device], tuple]


def tune(lo: int, hi: int, count: int = 0, seed: int = 7, device="cuda",
         candidates: Sequence[Tuple[int, int]] = CANDIDATES, reps: int = 1, apply: bool = True,
         sampler: Optional[Sampler] = None) -> Dict:
    """Times hqr_schur_batched on `count` sampled matrices (default: four per
    CU) for each (wg_per_cu, wide_n) candidate; returns {"wg_per_cu",
    "wide_n", "seconds": {candidate: s}} and installs the best if apply.
    `sampler(lo, hi, count, seed, device) -> (sizes, packed)` replaces the
    Gaussian sample when the workload's matrices are of another kind."""
    dev = torch.device(device)
    if count <= 0:
        count = 4 * torch.cuda.get_device_properties(dev).multi_processor_count
    sizes, packed = (sampler or sample)(lo, hi, count, seed, dev)
    prob = api.BatchedProblem(sizes, True, dev)
    prev = api.batched_launch()
    times = {}
    try:
        for wg, wide in candidates:
            api.set_batched_launch(wg, wide)
            best = float("inf")
            for _ in range(reps):
                prob.load(packed)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                prob.solve()
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            times[(wg, wide)] = best if int(prob.info.abs().max()) == 0 else float("inf")
    finally:
        api.set_batched_launch(prev["wg_per_cu"], prev["wide_n"])
    wg, wide = min(times, key=times.get)
    if apply:
        api.set_batched_launch(wg, wide)
    return {"wg_per_cu": wg, "wide_n": wide, "seconds": {f"{a},{b}": t for (a, b), t in times.items()}}


# Per-bucket AED window and shift count of the batched form (orders above
# 96).  (0, 0) is double-shift Francis; the others are (nw, ns) pairs with the
# window held in LDS (nw <= 64) and ns candidates used as shifts per step.
TABLE_CANDIDATES: Tuple[Tuple[int, int], ...] = ((0, 0), (24, 12), (32, 16), (32, 32), (48, 24), (48, 48),
                                                 (64, 32), (64, 64))
BUCKETS: Tuple[Tuple[int, int], ...] = ((97, 128), (129, 192), (193, 256))


def tune_table(buckets: Sequence[Tuple[int, int]] = BUCKETS, count: int = 0, seed: int = 11, device="cuda",
               candidates: Sequence[Tuple[int, int]] = TABLE_CANDIDATES, reps: int = 1,
               apply: bool = True, sampler: Optional[Sampler] = None) -> Dict:
    """Times hqr_schur_batched on a seeded sample of each size bucket (orders
    uniform in the bucket, `count` matrices, default two per CU) for every
    (nw, ns) candidate and keeps the fastest whose solves all succeeded; the
    last bucket also takes every larger order.  Returns {"upper", "nw", "ns",
    "seconds": {bucket: {candidate: s}}} and installs the table if apply.
    `sampler` as for tune()."""
    dev = torch.device(device)
    if count <= 0:
        count = 2 * torch.cuda.get_device_properties(dev).multi_processor_count
    prev = api.batched_table()
    chosen_nw, chosen_ns, upper, secs = [], [], [], {}
    try:
        for bi, (lo, hi) in enumerate(buckets):
            sizes, packed = (sampler or sample)(lo, hi, count, seed + bi, dev)
            prob = api.BatchedProblem(sizes, True, dev)
            times = {}
            for nw, ns in candidates:
                api.set_batched_table([4095], [nw], [ns])
                best = float("inf")
                for _ in range(reps):
                    prob.load(packed)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    prob.solve()
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                times[(nw, ns)] = best if int(prob.info.abs().max()) == 0 else float("inf")
            nw, ns = min(times, key=times.get)
            chosen_nw.append(nw)
            chosen_ns.append(ns)
            upper.append(hi if bi + 1 < len(buckets) else 4095)
            secs[f"{lo}-{hi}"] = {f"{a},{b}": t for (a, b), t in times.items()}
    finally:
        api.set_batched_table(prev["upper"], prev["nw"], prev["ns"])
    if apply:
        api.set_batched_table(upper, chosen_nw, chosen_ns)
    return {"upper": upper, "nw": chosen_nw, "ns": chosen_ns, "seconds": secs}
