"""Throughput of C = A * B (FP64 CSR) on one MI355X.

Workload (the roofline study configuration): the five-point Laplacian on a
2048 x 2048 grid squared (N = 4,194,304), plus a random N = 2^21 matrix with
exactly 16 distinct uniform columns per row and values U(-1, 1) times an
independent matrix drawn the same way.  One step is one full product of each
(plan with features, sizing and tiling, then the numeric pass writing C).

Metric: GFLOP/s with the paper's flop count (Section III: twice the number of
multiplications), and achieved HBM GB/s against a minimum-traffic model
|A| + |B| + |C|, |X| = 12 nnz(X) + 8 (rows(X) + 1) (int32 columns, FP64
values, int64 row pointers), as a fraction of the 8 TB/s HBM3E peak.

Prints ONE JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def model_bytes(A, B, nnz_c):
    return 12 * A.nnz + 8 * (A.rows + 1) + 12 * B.nnz + 8 * (B.rows + 1) + 12 * nnz_c + 8 * (A.rows + 1)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_workloads():
    import synth
    S = synth.stencil(2048)
    R1 = synth.random_fixed(1 << 21, 16, 1)
    R2 = synth.random_fixed(1 << 21, 16, 2)
    return [("stencil5_2048sq", S, S), ("random16_2pow21", R1, R2)]


def train_sizer(P, torch, seed_base=1001):
    """Trains the row-size network on the GPU with the library's kernels.
    Training rows: power-law matrices (seeds disjoint from any evaluation
    seed), small stencils and small fixed-length random matrices; labels are
    the exact row sizes from the symbolic pass."""
    import numpy as np
    import synth
    feats, labels = [], []
    mats = [synth.zipf_matrix(1 << 18, seed_base + i) for i in range(4)]
    pairs = [(M, M) for M in mats]
    for g in (64, 96, 128):
        S = synth.stencil(g)
        pairs.append((S, S))
    for pts, dim, g in ((9, 2, 96), (27, 3, 24)):
        S = synth.stencil(g, dim, pts)
        pairs.append((S, S))
    for k in (4, 8, 16, 32):
        pairs.append((synth.random_fixed(1 << 16, k, seed_base + 40 + k), synth.random_fixed(1 << 16, k, seed_base + 80 + k)))
    for A, B in pairs:
        dA = P.DeviceCSR.from_host(A)
        dB = dA if B is A else P.DeviceCSR.from_host(B)
        f1, f2, f3 = P.row_features(dA, dB)
        plan = P.Plan(dA, dB, "exact")
        rp, nnz = plan.symbolic()
        plan.close()
        feats.append((f1, f2, f3))
        labels.append((rp[1:] - rp[:-1]).to(torch.int32))
    f1 = torch.cat([f[0] for f in feats])
    f2 = torch.cat([f[1] for f in feats])
    f3 = torch.cat([f[2] for f in feats])
    lab = torch.cat(labels)
    # shuffle once so mini-batches mix the sources (permutation from a seed)
    g = torch.Generator(device="cpu").manual_seed(seed_base)
    perm = torch.randperm(f1.numel(), generator=g).to(f1.device)
    f1, f2, f3, lab = f1[perm].contiguous(), f2[perm].contiguous(), f3[perm].contiguous(), lab[perm].contiguous()
    mu, sd = P.feature_stats(f1, f2, f3)
    theta0 = synth.mlp_init(seed_base)
    model, curve = P.train_model(theta0, mu, sd, f1, f2, f3, lab, epochs=20, batch_size=32768, lr=3e-3)
    return model, {"train_rows": int(f1.numel()), "loss_first": float(curve[0]), "loss_last": float(curve[-1])}


def run_product(P, torch, dA, dB, sizer, model, timing=True):
    plan = P.Plan(dA, dB, sizer, model, timing=timing)
    dev = dA.row_ptr.device
    if sizer == "exact":
        rp, nnz = plan.symbolic()
        cap = nnz
    else:
        rp = torch.empty(dA.rows + 1, dtype=torch.int64, device=dev)
        cap = max(int(plan.info["c_capacity_hint"]), 1)
    col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    code, got = plan.numeric(rp, col, val, capacity=cap)
    if code == 6:
        col = torch.empty(got, dtype=torch.int32, device=dev)
        val = torch.empty(got, dtype=torch.float64, device=dev)
        code, got = plan.numeric(rp, col, val, capacity=got)
    P.check(code, "spgemm_numeric")
    info = dict(plan.info)
    plan.close()
    return got, info, (rp, col, val)


def cpu_baseline(workloads, budget_s=12.0):
    """The oracle (single-threaded C Gustavson) on a bounded sample: the whole
    stencil square and as many leading rows of the random product as fit the
    budget.  Reported in GFLOP/s with the same flop convention."""
    import numpy as np
    import oracle
    flops = 0
    t_tot = 0.0
    parts = []
    for name, A, B in workloads:
        f1, ub, mx = oracle.features(A, B)
        rows = A.rows
        if name.startswith("stencil"):
            r1 = rows
        else:
            # about a quarter of the budget per random sample
            r1 = min(rows, 1 << 18)
        t0 = time.perf_counter()
        oracle.spgemm(A, B, 0, r1)
        dt = time.perf_counter() - t0
        flops += 2 * int(ub[:r1].sum())
        t_tot += dt
        parts.append("%s rows 0..%d (%.2f s)" % (name, r1, dt))
    return {"value": flops / t_tot / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "; ".join(parts) + "; single-threaded C oracle, one run each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sizer", default="learned", choices=["learned", "upper_bound", "exact"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--compare", action="store_true", help="also time the other sizers")
    ap.add_argument("--workload", default="all", choices=["all", "stencil", "random"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the product runs on a single MI355X and "
              "multi-GPU row sharding is not built (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1303_1651_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    log("generating inputs")
    workloads = make_workloads()
    if args.workload != "all":
        workloads = [w for w in workloads if w[0].startswith(args.workload)]
    dev = []
    for name, A, B in workloads:
        dA = P.DeviceCSR.from_host(A)
        dB = dA if B is A else P.DeviceCSR.from_host(B)
        dev.append((name, A, B, dA, dB))

    model = None
    train_info = None
    if args.sizer == "learned" or args.compare:
        log("training the row-size network on the GPU")
        t0 = time.time()
        model, train_info = train_sizer(P, torch)
        train_info["seconds"] = round(time.time() - t0, 2)

    def step(sizer):
        per = []
        for name, A, B, dA, dB in dev:
            got, info, _ = run_product(P, torch, dA, dB, sizer, model)
            per.append((name, got, info))
        return per

    log("warmup")
    for _ in range(args.warmup):
        step(args.sizer)
    torch.cuda.synchronize()
    log("timed steps")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    per_step = []
    torch.cuda.synchronize()
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        per_step.append(step(args.sizer))
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps

    flops_step = 0
    bytes_step = 0
    tile_ms_step = 0.0
    details = {}
    for i, (name, A, B, dA, dB) in enumerate(dev):
        got = per_step[-1][i][1]
        mults = per_step[-1][i][2]["multiplications"]
        mb = model_bytes(A, B, got)
        tms = sum(s[i][2]["tile_ms_total"] for s in per_step) / args.steps
        flops_step += 2 * mults
        bytes_step += mb
        tile_ms_step += tms
        details[name] = {"nnz_c": got, "multiplications": mults, "model_bytes": mb,
                         "tile_kernel_ms": round(tms, 4),
                         "tile_kernel_GBps": round(mb / tms / 1e6, 1),
                         "tile_kernel_frac_hbm": round(mb / tms / 1e6 / HBM_PEAK_GBS, 4),
                         "tiers": {k: per_step[-1][i][2][k] for k in ("rows_merge", "rows_hash", "rows_global", "rows_empty")},
                         "overflow_rows": per_step[-1][i][2]["overflow_rows"]}
    gflops = flops_step / (ms * 1e-3) / 1e9

    if args.compare:
        for other in ("exact", "upper_bound", "learned"):
            if other == args.sizer:
                continue
            for _ in range(args.warmup):
                step(other)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            outs = [step(other) for _ in range(args.steps)]
            e1.record()
            torch.cuda.synchronize()
            oms = e0.elapsed_time(e1) / args.steps
            for i, (name, A, B, dA, dB) in enumerate(dev):
                tms = sum(s[i][2]["tile_ms_total"] for s in outs) / args.steps
                details[name]["tile_kernel_ms_" + other] = round(tms, 4)
            details["step_ms_" + other] = round(oms, 4)

    achieved = bytes_step / (tile_ms_step * 1e-3) / 1e9
    out = {
        "metric": "SpGEMM GFLOP/s & HBM GB/s vs roofline; learned-sized vs plain two-pass",
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "5-point Laplacian 2048x2048 squared + random 2^21 x 16/row A*B (FP64 CSR)",
                   "sizer": args.sizer, "products_per_step": len(dev)},
        "gbps_model": round(bytes_step / (ms * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "wall_ms_per_step": round(wall * 1e3 / args.steps, 3),
        "workloads": details,
    }
    if train_info:
        out["sizer_training"] = train_info
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline([(n, A, B) for n, A, B, _, _ in dev])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
