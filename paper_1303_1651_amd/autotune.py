"""Autotuner for the tier thresholds and tile shapes of the library.

For a workload (a pair of device CSR operands standing for a family of
products) it times the library's own passes under candidate tuning blocks
(LDS table size, staging size, register-merge thresholds, dense-window
ratio) with the plan's HIP-event timing, keeps the fastest, and caches the
choice in a JSON file keyed by a signature of the operand shapes.  It only
calls the library; every pass it times runs in the HIP kernels.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import Batch, DeviceCSR, Plan, check

DEFAULT_GRID = {
    "table_slots": [512, 1024, 2048],
    "stage_slots": [512, 1024, 2048],
    "merge_max_nnz": [32, 64, 128],
    "merge_lists": [4, 8],
    "dense_ratio": [2.0],
}


def signature(A: DeviceCSR, B: DeviceCSR, sizer: str) -> str:
    """Operand family: sizer, log2 of the rows, mean row lengths of A and B
    (rounded), so that products of the same kind share a tuning."""
    import math
    ra = A.nnz / max(A.rows, 1)
    rb = B.nnz / max(B.rows, 1)
    return "%s:r%d:a%.0f:b%.0f" % (sizer, int(math.log2(max(A.rows, 1))), ra, rb)


def _time(A, B, sizer, model, tuning, reps, cutoff=None):
    """Best row-kernel time over `reps` products; stops after the first one
    slower than `cutoff` ms (a candidate far behind the best so far)."""
    best = None
    for _ in range(reps):
        plan = Plan(A, B, sizer, model, tuning=tuning, timing=True)
        dev = A.row_ptr.device
        if sizer == "exact":
            rp, nnz = plan.symbolic()
            cap = nnz
        else:
            rp = torch.empty(A.rows + 1, dtype=torch.int64, device=dev)
            cap = max(int(plan.info["c_capacity_hint"]), 1)
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        code, got = plan.numeric(rp, col, val, capacity=cap)
        if code == 6:
            col = torch.empty(got, dtype=torch.int32, device=dev)
            val = torch.empty(got, dtype=torch.float64, device=dev)
            code, got = plan.numeric(rp, col, val, capacity=got)
        check(code, "spgemm_numeric")
        ms = plan.info["tile_ms_total"]
        plan.close()
        best = ms if best is None else min(best, ms)
        if cutoff is not None and best > cutoff:
            break
    return best


def autotune(A: DeviceCSR, B: DeviceCSR, sizer: str = "exact", model=None, grid: dict | None = None,
             reps: int = 2, cache: str | None = None, log=None) -> dict:
    """Returns the fastest tuning block (a dict for Plan/spgemm's `tuning`)
    over the candidate grid, timing the row kernels of every pass."""
    key = signature(A, B, sizer)
    if cache and os.path.exists(cache):
        stored = json.load(open(cache))
        if key in stored:
            return stored[key]["tuning"]
    grid = grid or DEFAULT_GRID
    names = list(grid)
    results = []
    # the library's defaults first: a candidate more than twice as slow as
    # the best so far is not timed again
    lead = _time(A, B, sizer, model, {}, 1)
    for values in itertools.product(*[grid[n] for n in names]):
        t = dict(zip(names, values))
        if 12 * (t.get("table_slots", 1024) + t.get("stage_slots", 1024)) > 147456:
            continue
        ms = _time(A, B, sizer, model, t, reps, cutoff=2.0 * lead)
        lead = min(lead, ms)
        results.append((ms, t))
        if log:
            log("%8.3f ms  %s" % (ms, t))
    if not results:
        return {}   # no candidate fits the LDS budget: the library's defaults
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    if cache:
        stored = json.load(open(cache)) if os.path.exists(cache) else {}
        stored[key] = {"tuning": best, "ms": best_ms, "candidates": len(results)}
        json.dump(stored, open(cache, "w"), indent=1, sort_keys=True)
    return best


BATCH_GRID = {
    "table_slots": [512, 1024, 2048],
    "stage_slots": [512, 1024],
    "merge_max_nnz": [32, 64],
    "dense_ratio": [1.0, 2.0, 4.0],
}


def autotune_batch(As, Bs, sizer: str = "exact", model=None, grid: dict | None = None, reps: int = 3,
                   log=None) -> tuple[dict, list]:
    """Tuning block for a batch of products: every candidate of the grid
    builds the batch (its first run captures the launches) and its graph
    replays are timed (best of `reps`); returns the fastest candidate and
    every (ms, candidate) pair.  Pass a sample of a large batch: the choice
    carries over to batches of the same kind."""
    grid = grid or BATCH_GRID
    names = list(grid)
    results = []
    for values in itertools.product(*[grid[n] for n in names]):
        t = dict(zip(names, values))
        if 12 * (t.get("table_slots", 1024) + t.get("stage_slots", 1024)) > 147456:
            continue
        b = Batch(As, Bs, sizer, model=model, tuning=t)
        b.run()
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        b.close()
        results.append((best, t))
        if log:
            log("%8.3f ms  %s" % (best, t))
    results.sort(key=lambda r: r[0])
    return results[0][1], results
