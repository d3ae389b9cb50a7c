"""Throughput of C = A * B (FP64 CSR) on one MI355X.

Default workload (the roofline study): the five-point Laplacian on a
2048 x 2048 grid squared (N = 4,194,304), and a random N = 2^21 matrix with
exactly 16 distinct uniform columns per row and values U(-1, 1) times an
independent matrix drawn the same way.  One step is one full product of
each on the plain two-pass path (plan, symbolic pass, scan, numeric pass);
inputs are resident in HBM before the timed region.  Before timing, the
library's autotuner picks each product's tier thresholds and tile shapes,
once per sizer the line times (kept only when that whole product beats the
default tuning; both times are reported; --no-autotune times the defaults).  Other workloads:
--workload zipf (power-law rows, N = 2^20, the learned-sizer study), st9,
st27, batched.

Metric: GFLOP/s with the paper's flop count (Section III: twice the number
of multiplications).  The roofline object is for the step's dominant kernel
(the numeric wave-tile pass of the random product): algorithmic bytes per
launch (|A| + |B| + |C| with |X| = 12 nnz(X) + 8 (rows(X) + 1): int32
columns, FP64 values, int64 row pointers) over its average launch time,
measured with HIP events on the stream the kernel runs on, against the
8 TB/s HBM3E peak.  `traffic` comes from the committed rocprofv3 counter
summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel's reading)
when that summary was taken on the current kernel source, else null.

Prints ONE JSON line.  Only one GPU is used: --gpus above 1 exits.
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
KERNEL_SRC = os.path.join(ROOT, "paper_1303_1651_amd", "csrc", "spgemm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_wave_tile_numeric_random16.json")


def model_bytes(A, B, nnz_c):
    return 12 * A.nnz + 8 * (A.rows + 1) + 12 * B.nnz + 8 * (B.rows + 1) + 12 * nnz_c + 8 * (A.rows + 1)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_sha1():
    return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()


def make_workloads(name):
    import synth
    if name == "roofline":
        S = synth.stencil(2048)
        return [("stencil5_2048sq", S, S),
                ("random16_2pow21", synth.random_fixed(1 << 21, 16, 1), synth.random_fixed(1 << 21, 16, 2))]
    if name == "stencil":
        S = synth.stencil(2048)
        return [("stencil5_2048sq", S, S)]
    if name == "random":
        return [("random16_2pow21", synth.random_fixed(1 << 21, 16, 1), synth.random_fixed(1 << 21, 16, 2))]
    if name == "zipf":
        Z = synth.zipf_matrix(1 << 20, 3)
        return [("zipf2_2pow20", Z, Z)]
    if name == "st9":
        S = synth.stencil(2048, 2, 9)
        return [("stencil9_2048sq", S, S)]
    if name == "st27":
        S = synth.stencil(160, 3, 27)
        return [("stencil27_160cube", S, S)]
    raise ValueError(name)


# Source matrices of the row-size network per workload family: smaller
# instances of the same kind, with seeds disjoint from every evaluation seed.
# The network sees only (nnz(A_i), UB_i, longest B row), and rows of
# different families can share those features while their sizes differ (an
# interior 27-point row and a power-law row of 27 entries whose products all
# land on distinct columns), so it is trained per family.
SIZER_FAMILIES = {"roofline": ("stencil", "random"), "stencil": ("stencil",), "st9": ("stencil",),
                  "st27": ("stencil",), "random": ("random",), "zipf": ("zipf",)}


def sizer_sources(family, seed_base):
    import synth
    if family == "zipf":
        # four matrices of 2^20 rows: 2^22 rows of symbolic-pass output
        return [(synth.zipf_matrix(1 << 20, seed_base + i),) * 2 for i in range(4)]
    if family == "stencil":
        out = [(synth.stencil(g),) * 2 for g in (64, 96, 128)]
        out += [(synth.stencil(g, dim, pts),) * 2 for pts, dim, g in ((9, 2, 64), (9, 2, 96), (27, 3, 16), (27, 3, 24))]
        return out
    return [(synth.random_fixed(1 << 16, k, seed_base + 40 + k), synth.random_fixed(1 << 16, k, seed_base + 80 + k))
            for k in (4, 8, 16, 32)]


def train_sizer(P, torch, workload, seed_base=1001):
    """Trains the row-size network on the GPU with the library's kernels, on
    the workload's family; labels are the exact row sizes from the symbolic
    pass.  The power-law family trains on every row of its four sources
    (2^22 rows); the others draw the same number of rows from every source
    (with replacement, from a seeded generator), so that rare row shapes
    weigh as much as common ones."""
    pairs = []
    for fam in SIZER_FAMILIES[workload]:
        for A, B in sizer_sources(fam, seed_base):
            dA = P.DeviceCSR.from_host(A)
            pairs.append((dA, dA if B is A else P.DeviceCSR.from_host(B)))
    every_row = SIZER_FAMILIES[workload] == ("zipf",)
    model, facts = P.fit_model(pairs, seed=seed_base, per_source=None if every_row else 1 << 16,
                               epochs=10 if every_row else 30, batch_size=16384 if every_row else 8192)
    del pairs
    facts["families"] = list(SIZER_FAMILIES[workload])
    return model, facts


class Product:
    """One product on the device with its output buffers allocated once."""

    def __init__(self, P, torch, name, A, B, dA, dB):
        self.P, self.torch = P, torch
        self.name, self.A, self.B, self.dA, self.dB = name, A, B, dA, dB
        self.out = {}
        self.tuning = {}   # sizer -> the autotuner's choice, when it beat the defaults

    def run(self, sizer, model, tuning=None):
        P, torch = self.P, self.torch
        if tuning is None:
            tuning = self.tuning.get(sizer)
        plan = P.Plan(self.dA, self.dB, sizer, model, timing=True, tuning=tuning)
        dev = self.dA.row_ptr.device
        sym_ms = 0.0
        if sizer == "exact":
            rp, nnz = plan.symbolic(self.out.get("rp"))
            sym_ms = plan.info["tile_ms"]
            cap = nnz
        else:
            rp = self.out.get("rp")
            if rp is None:
                rp = torch.empty(self.dA.rows + 1, dtype=torch.int64, device=dev)
            cap = max(int(plan.info["c_capacity_hint"]), 1)
        self.out["rp"] = rp
        col, val = self.out.get("col"), self.out.get("val")
        if col is None or col.numel() < cap:
            col = torch.empty(cap, dtype=torch.int32, device=dev)
            val = torch.empty(cap, dtype=torch.float64, device=dev)
            self.out["col"], self.out["val"] = col, val
        code, got = plan.numeric(rp, col, val, capacity=cap)
        if code == 6:
            col = torch.empty(got, dtype=torch.int32, device=dev)
            val = torch.empty(got, dtype=torch.float64, device=dev)
            self.out["col"], self.out["val"] = col, val
            code, got = plan.numeric(rp, col, val, capacity=got)
        P.check(code, "spgemm_numeric")
        info = dict(plan.info)
        info["symbolic_ms"] = sym_ms
        info["numeric_ms"] = info["tile_ms"]
        plan.close()
        return got, info


def time_steps(torch, products, sizer, model, steps, warmup):
    for _ in range(warmup):
        for p in products:
            p.run(sizer, model)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    per = []
    torch.cuda.synchronize()
    e0.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        per.append([p.run(sizer, model) for p in products])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall * 1e3 / steps, per


def _best_of(fn, min_runs=5, min_seconds=2.0, max_seconds=6.0):
    """The paper's protocol (Section III): repeat until more than two
    seconds have passed and at least five runs were made, keep the best (a
    cap bounds the time of slow samples); returns (best, median, runs)."""
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
        el = time.perf_counter() - t_start
        if (len(times) >= min_runs and el > min_seconds) or el > max_seconds:
            break
    times.sort()
    return times[0], times[len(times) // 2], len(times)


def cpu_baseline(workloads, random_rows=1 << 17):
    """The oracle (single-threaded C Gustavson) on a bounded sample: the whole
    stencil square and the leading rows of the random product, on one host
    core with the paper's protocol; and the same oracle run row-parallel on
    every core the box gives the job (disjoint row ranges on threads; the C
    calls release the interpreter lock), on eight times as many random rows.
    Reported in GFLOP/s with the same flop convention."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    cores = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))

    one = {"flops": 0, "best": 0.0, "median": 0.0}
    par = {"flops": 0, "best": 0.0}
    parts = []
    with cf.ThreadPoolExecutor(cores) as ex:
        for name, A, B in workloads:
            _, ub, _ = oracle.features(A, B)
            stencil = not name.startswith("random")
            r1 = A.rows if stencil else min(A.rows, random_rows)
            best, med, runs = _best_of(lambda: oracle.spgemm(A, B, 0, r1))
            one["flops"] += 2 * int(ub[:r1].sum())
            one["best"] += best
            one["median"] += med
            rp = A.rows if stencil else min(A.rows, 8 * random_rows)
            bounds = np.linspace(0, rp, 4 * cores + 1).astype(np.int64)

            def all_cores():
                list(ex.map(lambda k: oracle.spgemm(A, B, int(bounds[k]), int(bounds[k + 1])), range(4 * cores)))
            pbest, _, pruns = _best_of(all_cores)
            par["flops"] += 2 * int(ub[:rp].sum())
            par["best"] += pbest
            parts.append("%s rows 0..%d on one core (best of %d: %.3f s, median %.3f s) and rows 0..%d on %d "
                         "threads (best of %d: %.3f s)" % (name, r1, runs, best, med, rp, cores, pruns, pbest))
    return {"value": round(one["flops"] / one["best"] / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "median_value": round(one["flops"] / one["median"] / 1e9, 4),
            "all_cores": {"value": round(par["flops"] / par["best"] / 1e9, 4), "unit": "GFLOP/s", "cores": cores},
            "sample": "; ".join(parts) + "; single-threaded C oracle, each timing the best of at least five runs "
                      "over more than two seconds (the paper's protocol, Section III)"}


def measure_bmax(torch, nbytes=1 << 31, reps=10):
    """STREAM-style copy on the device (the paper's b_max, Section III): the
    best of `reps` device-to-device copies of `nbytes`, counting the bytes
    read and written."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * nbytes / (best * 1e-3) / 1e9


def time_product(torch, p, sizer, model, steps, tuning=None, numeric=False):
    """Whole-product time of one workload alone (plan, passes, host round
    trips), CUDA events around `steps` products; with numeric=True also the
    numeric pass's kernel time (the library's HIP events)."""
    p.run(sizer, model, tuning)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    num = []
    e0.record()
    for _ in range(steps):
        num.append(p.run(sizer, model, tuning)[1]["numeric_ms"])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return (ms, sum(num) / len(num)) if numeric else ms


# The storing-strategy study of Section IV-B: random matrices of 0.1 % fill,
# the dense window (MinMax) against the sorted table (Sort) as N grows.
FILL_NS = [4096, 8192, 16384, 24576, 32768, 38912, 49152, 65536, 98304, 131072, 163840, 196608]


def run_fill(P, torch, args):
    """Every product of the sweep three ways on the plain two-pass path: the
    library's default choice, every row in the workgroup tier with a dense
    window of its column region (MinMax), and every row there with a hashed
    table whose runs are sorted on the way out (Sort).  Reports the numeric
    pass and the whole product of each, and where the dense window starts to
    win (as N and as the ratio of a row's column region to its entries, the
    quantity the dense-window rule compares)."""
    import synth
    forced = {"dense_window": {"merge_max_nnz": -1, "table_slots": -1, "dense_ratio": 1e9},
              "sorted_table": {"merge_max_nnz": -1, "table_slots": -1, "dense_ratio": 1e-9}}
    out = []
    for n in FILL_NS:
        if n > args.fill_max:
            break
        A = synth.random_fill(n, 0.001, 11)
        B = synth.random_fill(n, 0.001, 12)
        dA, dB = P.DeviceCSR.from_host(A), P.DeviceCSR.from_host(B)
        prod = Product(P, torch, "fill%d" % n, A, B, dA, dB)
        got, info = prod.run("exact", None)
        row = {"n": n, "row_entries": int(A.row_ptr[1]), "nnz_c": got, "multiplications": info["multiplications"],
               "region_over_entries": round(n / max(got / n, 1e-9), 2)}
        for label, tuning in (("default", None), ("dense_window", forced["dense_window"]),
                              ("sorted_table", forced["sorted_table"])):
            ms, num = time_product(torch, prod, "exact", None, args.steps, tuning, numeric=True)
            row["product_ms_" + label] = round(ms, 4)
            row["numeric_ms_" + label] = round(num, 4)
            row["gflops_" + label] = round(2 * info["multiplications"] / (ms * 1e-3) / 1e9, 3)
        log("fill n=%d: numeric dense %.3f ms, sorted %.3f ms, default %.3f ms" % (
            n, row["numeric_ms_dense_window"], row["numeric_ms_sorted_table"], row["numeric_ms_default"]))
        out.append(row)
        del prod, dA, dB
        torch.cuda.empty_cache()
    # break-even: first N from which the dense window's numeric pass is faster
    cross = None
    for a, b in zip(out, out[1:]):
        da = a["numeric_ms_dense_window"] - a["numeric_ms_sorted_table"]
        db = b["numeric_ms_dense_window"] - b["numeric_ms_sorted_table"]
        if da > 0 >= db or da < 0 <= db:
            t = da / (da - db)
            cross = {"n": round(a["n"] + t * (b["n"] - a["n"])),
                     "region_over_entries": round(a["region_over_entries"] + t * (b["region_over_entries"] -
                                                                                  a["region_over_entries"]), 2),
                     "dense_wins_above": db <= 0}
            break
    return out, cross


def compute_only_ms(P, torch, p, steps):
    """The pure computation kernel (every row accumulated, nothing stored;
    Section IV-A) on a product whose rows all merge in registers: its kernel
    time (HIP events of the library), or None for other products."""
    plan = P.Plan(p.dA, p.dB, "exact", timing=True)
    try:
        ms = []
        for _ in range(steps + 1):
            plan.compute_only()
            ms.append(plan.info["tile_ms"])
        return sum(ms[1:]) / steps
    except P.SpgemmError:
        return None
    finally:
        plan.close()


def misprediction(P, torch, p, model, margin=0.05, slack=2):
    """How the learned sizes compare with the exact ones on this product:
    rows whose prediction falls below nnz(C_i), and rows whose capacity
    (the prediction with the default margin and slack, clamped to [longest
    selected B row, multiplication count]) does; those are the rows a
    learned one pass must place elsewhere or compute again."""
    f1, f2, f3 = P.row_features(p.dA, p.dB)
    plan = P.Plan(p.dA, p.dB, "exact")
    rp, _ = plan.symbolic()
    plan.close()
    exact = (rp[1:] - rp[:-1]).to(torch.float64)
    pred = model.predict(f1, f2, f3).to(torch.float64)
    cap = torch.ceil(pred * (1.0 + margin)) + slack
    cap = torch.minimum(torch.maximum(cap, f3.to(torch.float64)), f2.to(torch.float64))
    n = max(int(exact.numel()), 1)
    return {"rows_predicted_below_exact": round(float((pred < exact).sum()) / n, 6),
            "rows_capacity_below_exact": round(float((cap < exact).sum()) / n, 6),
            "capacity_over_nnz": round(float(cap.sum()) / max(float(exact.sum()), 1.0), 4)}


def traffic_from_profile(launch_bytes_alg):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or was taken on other kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_sha1") != kernel_source_sha1():
        return None
    return int(d["traffic_bytes_per_launch"])


def calibrate_copy(torch, nbytes=1 << 30):
    """A plain device copy of known size, for scaling the HBM counters."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    return nbytes


def pmc_summary(fetch_csv, write_csv, kernel_substr, copy_bytes, out_json, command):
    """Writes the traffic summary from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE; counter_collection.csv files): per-dispatch KiB of the
    kernel, scaled by what the same counters read for the largest device copy
    dispatch of the run (copy_bytes each way: the 2 GiB copies of the b_max
    measurement)."""
    import csv

    def rows(path, counter):
        return [(r["Kernel_Name"], float(r["Counter_Value"]))
                for r in csv.DictReader(open(path)) if r.get("Counter_Name", "") == counter]

    def mean_of(rs, sub):
        v = [x for n, x in rs if sub in n]
        return sum(v) / len(v) if v else None

    def copy_of(rs):
        v = [x for n, x in rs if "copyBuffer" in n or "copy" in n.lower()]
        return max(v) if v else None

    f = rows(fetch_csv, "FETCH_SIZE")
    w = rows(write_csv, "WRITE_SIZE")
    fk, wk = mean_of(f, kernel_substr), mean_of(w, kernel_substr)
    fc, wc = copy_of(f), copy_of(w)
    if None in (fk, wk, fc, wc):
        raise SystemExit("kernel %r or the calibration copy is missing from the counter files" % kernel_substr)
    ff = (copy_bytes / 1024.0) / fc
    wf = (copy_bytes / 1024.0) / wc
    traffic = (fk * ff + wk * wf) * 1024.0
    d = {"kernel": kernel_substr, "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
         "copy_bytes": copy_bytes, "copy_fetch_kib": fc, "copy_write_kib": wc,
         "fetch_factor": ff, "write_factor": wf, "traffic_bytes_per_launch": traffic,
         "source_sha1": kernel_source_sha1(), "command": command}
    json.dump(d, open(out_json, "w"), indent=1)
    print(json.dumps(d))


def stats_summary(stats_csv, out_txt, command, top=16):
    """Text summary of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["command: " + command, "",
             "%-64s %6s %14s %12s %7s" % ("kernel", "calls", "total_ms", "avg_ms", "pct")]
    for r in rows[:top]:
        lines.append("%-64s %6s %14.3f %12.4f %7.2f" % (r["Name"][:64], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e6, float(r["Percentage"])))
    open(out_txt, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def run_batched(P, torch, args):
    """The batched launch against a per-instance loop, both doing the same
    work per step: the numeric pass of every instance.  The batch replays its
    captured launches (the value copies and the numeric pass of the whole
    concatenation; with the exact sizer the counts of its first run are
    kept, with the one-pass sizers the whole one pass is replayed).  The loop
    calls spgemm_numeric on every instance's plan, built (and, exact sizer,
    counted by its symbolic pass) before the timed region: one call and one
    host round trip per instance.  The batch runs with the default tuning
    and with the autotuner's choice for a 256-instance sample of the same
    kind (seed disjoint from the batch's)."""
    import numpy as np
    import synth
    from paper_1303_1651_amd.autotune import autotune_batch
    log("generating %d instances, N log-uniform in [%d, %d]" % (args.batch_count, args.batch_lo, args.batch_hi))
    insts = []
    for k0 in range(0, args.batch_count, 256):
        part = synth.batch_mix(min(256, args.batch_count - k0), 7 + k0, lo=args.batch_lo, hi=args.batch_hi)
        insts += part
        log("  %d instances" % len(insts))

    def upload(items):
        As, Bs = [], []
        for it in items:
            dA = P.DeviceCSR.from_host(it.A)
            As.append(dA)
            Bs.append(dA if it.B is it.A else P.DeviceCSR.from_host(it.B))
        return As, Bs

    As, Bs = upload(insts)
    mults = 0
    for it in insts:
        # Section III count: sum over k of nnz(A column k) * nnz(B row k)
        acol = np.bincount(np.asarray(it.A.col), minlength=it.A.cols)
        mults += int(np.dot(acol.astype(np.int64), np.diff(np.asarray(it.B.row_ptr)).astype(np.int64)))
    sizer = args.batch_sizer

    def time_batch(tuning):
        b = P.Batch(As, Bs, sizer, tuning=tuning)
        b.run()
        for _ in range(args.warmup):
            b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            b.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        nnz_c, graph = int(b.nnz.sum()), b.uses_graph()
        b.close()
        del b
        torch.cuda.empty_cache()
        return ms, nnz_c, graph

    log("batched launch, default tuning")
    ms_default, nnz_c, graph = time_batch(None)
    log("autotuning on a 256-instance sample")
    sample = synth.batch_mix(256, 99991, lo=args.batch_lo, hi=args.batch_hi)
    sA, sB = upload(sample)
    tuned, cand = autotune_batch(sA, sB, sizer, reps=2, log=lambda m: log("  " + m))
    del sA, sB
    torch.cuda.empty_cache()
    log("batched launch, tuned: %s" % tuned)
    ms_tuned, _, _ = time_batch(tuned)

    log("per-instance loop: plans")
    dev = As[0].row_ptr.device
    plans, rps, caps = [], [], []
    scratch_max = 0
    for a, b in zip(As, Bs):
        pl = P.Plan(a, b, sizer, alloc_scratch=False)
        scratch_max = max(scratch_max, int(pl.info["scratch_bytes"]))
        plans.append(pl)
    shared = torch.empty(max(scratch_max, 1), dtype=torch.uint8, device=dev) if scratch_max else None
    for pl in plans:
        pl.scratch = shared
        if sizer == "exact":
            rp, nnz = pl.symbolic()
            rps.append(rp)
            caps.append(nnz)
        else:
            rps.append(torch.empty(pl.A.rows + 1, dtype=torch.int64, device=dev))
            caps.append(max(int(pl.info["c_capacity_hint"]), 1))
    cmax = max(max(caps), 1)
    col = torch.empty(cmax, dtype=torch.int32, device=dev)
    val = torch.empty(cmax, dtype=torch.float64, device=dev)

    def loop():
        for pl, rp, cap in zip(plans, rps, caps):
            code, _ = pl.numeric(rp, col, val, capacity=cap)
            P.check(code, "spgemm_numeric")
    loop()
    torch.cuda.synchronize()
    log("per-instance loop: timed")
    t0 = time.perf_counter()
    loop_steps = max(1, min(args.steps, 3))
    for _ in range(loop_steps):
        loop()
    torch.cuda.synchronize()
    lms = (time.perf_counter() - t0) * 1e3 / loop_steps
    for pl in plans:
        pl.close()
    best = min(ms_default, ms_tuned)
    return {"instances": len(insts), "rows": int(sum(it.A.rows for it in insts)), "multiplications": mults,
            "nnz_c": nnz_c, "sizer": sizer,
            "batched_ms": round(best, 3), "batched_ms_default_tuning": round(ms_default, 3),
            "batched_ms_tuned": round(ms_tuned, 3), "tuning": tuned, "tuning_candidates": len(cand),
            "loop_ms": round(lms, 3), "loop_steps": loop_steps, "speedup_over_loop": round(lms / best, 2),
            "batched_gflops": round(2 * mults / (best * 1e-3) / 1e9, 3),
            "loop_gflops": round(2 * mults / (lms * 1e-3) / 1e9, 3), "graph_replay": graph,
            "work_per_step": "both sides: the numeric pass of every instance (plans, and the exact sizer's "
                             "counts, made before the timed region)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sizer", default="exact", choices=["learned", "upper_bound", "exact"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other sizers")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default tuning block instead of the autotuner's choice")
    ap.add_argument("--workload", default="roofline",
                    choices=["roofline", "stencil", "random", "zipf", "st9", "st27", "batched", "fill"])
    ap.add_argument("--fill-max", type=int, default=196608, help="largest N of the 0.1%%-fill sweep")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-lo", type=int, default=256)
    ap.add_argument("--batch-hi", type=int, default=65536)
    ap.add_argument("--batch-sizer", default="exact", choices=["learned", "upper_bound", "exact"])
    ap.add_argument("--calibrate", action="store_true", help="also run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="write the traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-command", default="")
    ap.add_argument("--pmc-kernel", default="k_wt<1,", help="kernel name substring of the counter summary")
    ap.add_argument("--stats-summary", nargs=2, metavar=("KERNEL_STATS_CSV", "OUT_TXT"),
                    help="write a text summary of a rocprofv3 --stats run and exit (command: --pmc-command)")
    args = ap.parse_args()
    if args.stats_summary:
        stats_summary(args.stats_summary[0], args.stats_summary[1], args.pmc_command)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_kernel, 2 << 30, args.pmc_summary[2],
                    args.pmc_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the product runs on a single MI355X and "
              "multi-GPU row sharding is not built (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1303_1651_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.workload == "fill":
        rows, cross = run_fill(P, torch, args)
        ref = next((r for r in rows if r["n"] == 38912), rows[-1])
        print(json.dumps({"metric": "SpGEMM GFLOP/s on 0.1%-fill random products, dense window vs sorted table",
                          "value": ref["gflops_default"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": 1, "ms_per_step": ref["product_ms_default"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "random N x N, ceil(0.001 N) distinct columns per row, U(-1, 1), "
                                                 "C = A * B, N swept %d..%d; value at N = %d" % (
                                                     rows[0]["n"], rows[-1]["n"], ref["n"])},
                          "sweep": rows, "break_even": cross}), flush=True)
        return

    if args.workload == "batched":
        res = run_batched(P, torch, args)
        print(json.dumps({"metric": "SpGEMM GFLOP/s, batched launch vs per-instance loop", "value": res["batched_gflops"],
                          "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": res["batched_ms"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "batched: %d products, N log-uniform [%d, %d], half 5-point stencils, "
                                                 "half random 4-32/row; numeric pass of every instance per step, "
                                                 "batched replay vs per-instance loop" % (
                                                     args.batch_count, args.batch_lo, args.batch_hi)},
                          "batched": res}), flush=True)
        return

    log("generating inputs")
    workloads = make_workloads(args.workload)
    products = []
    for name, A, B in workloads:
        dA = P.DeviceCSR.from_host(A)
        dB = dA if B is A else P.DeviceCSR.from_host(B)
        products.append(Product(P, torch, name, A, B, dA, dB))
    if args.calibrate:
        calibrate_copy(torch)

    model = None
    train_info = None
    need_model = args.sizer == "learned" or not args.no_compare
    if need_model:
        log("training the row-size network on the GPU")
        t0 = time.time()
        model, train_info = train_sizer(P, torch, args.workload)
        train_info["seconds"] = round(time.time() - t0, 2)

    tuned = {}
    if not args.no_autotune:
        # thresholds and tile shapes picked per workload and sizer by the
        # library's autotuner (row-kernel time of that sizer's passes over its
        # candidate grid), kept when the whole product is faster than with the
        # defaults: a one-pass product lays rows out by other capacities than
        # the exact one, so its best tiles differ
        from paper_1303_1651_amd.autotune import autotune
        log("autotuning")
        sizers = [args.sizer] + ([] if args.no_compare else
                                 [s for s in ("exact", "upper_bound", "learned") if s != args.sizer])
        for p in products:
            tuned[p.name] = {}
            for sizer in sizers:
                t0 = time.time()
                cand = autotune(p.dA, p.dB, sizer, model if sizer == "learned" else None, reps=2)
                d_ms = time_product(torch, p, sizer, model, args.steps, tuning={})
                t_ms = time_product(torch, p, sizer, model, args.steps, tuning=cand)
                keep = t_ms < d_ms
                if keep:
                    p.tuning[sizer] = cand
                tuned[p.name][sizer] = {"candidate": cand, "kept": keep, "product_ms_default_tuning": round(d_ms, 4),
                                        "product_ms_candidate": round(t_ms, 4),
                                        "seconds": round(time.time() - t0, 2)}
                log("  %s %s: default %.3f ms, tuned %.3f ms (%s)" % (p.name, sizer, d_ms, t_ms,
                                                                     "kept" if keep else "dropped"))

    log("timed steps (%s)" % args.sizer)
    ms, wall_ms, per = time_steps(torch, products, args.sizer, model, args.steps, args.warmup)

    details = {}
    flops_step = 0
    dominant = None
    for i, p in enumerate(products):
        got, info = per[-1][i]
        mults = info["multiplications"]
        mb = model_bytes(p.A, p.B, got)
        num_ms = sum(s[i][1]["numeric_ms"] for s in per) / len(per)
        sym_ms = sum(s[i][1]["symbolic_ms"] for s in per) / len(per)
        flops_step += 2 * mults
        details[p.name] = {"nnz_c": got, "multiplications": mults, "model_bytes": mb,
                           "numeric_pass_ms": round(num_ms, 4), "symbolic_pass_ms": round(sym_ms, 4),
                           "numeric_pass_GBps": round(mb / num_ms / 1e6, 1),
                           "tiers": {k: info[k] for k in ("rows_merge", "rows_hash", "rows_global", "rows_empty")},
                           "overflow_rows": info["overflow_rows"],
                           "capacity_over_nnz": round(info["c_capacity_hint"] / max(got, 1), 3)}
        if dominant is None or num_ms > dominant[1]:
            dominant = (p.name, num_ms, mb, info)
    gflops = flops_step / (ms * 1e-3) / 1e9

    if not args.no_compare:
        for other in ("exact", "upper_bound", "learned"):
            if other == args.sizer:
                continue
            oms, _, oper = time_steps(torch, products, other, model, args.steps, args.warmup)
            details["step_ms_" + other] = round(oms, 4)
            for i, p in enumerate(products):
                details[p.name]["numeric_pass_ms_" + other] = round(
                    sum(s[i][1]["numeric_ms"] for s in oper) / len(oper), 4)
                details[p.name]["overflow_rows_" + other] = oper[-1][i][1]["overflow_rows"]
                details[p.name]["capacity_over_nnz_" + other] = round(
                    oper[-1][i][1]["c_capacity_hint"] / max(oper[-1][i][0], 1), 3)
        details["step_ms_" + args.sizer] = round(ms, 4)
        # a right-hand operand given by columns (Section IV-A converts it to
        # rows first): the transpose kernels turn B's CSC arrays (the CSR of
        # B^T) into B by rows before the same product
        conv = 0.0
        for p in products:
            b_csc = P.transpose(p.dB)
            P.transpose(b_csc)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                P.transpose(b_csc)
            e1.record()
            torch.cuda.synchronize()
            tms = e0.elapsed_time(e1) / args.steps
            details[p.name]["csc_to_csr_ms"] = round(tms, 4)
            conv += tms
            del b_csc
        details["step_ms_exact_csc_operand"] = round(details["step_ms_exact"] + conv, 4)

    whole = {}
    if not args.no_compare:
        log("whole-product times, compute-only kernel, learned sizes against exact ones")
        for p in products:
            d = details[p.name]
            mb = d["model_bytes"]
            w = {"model_bytes": mb}
            for sz in ("exact", "upper_bound", "learned"):
                ms_p = time_product(torch, p, sz, model, args.steps)
                w["product_ms_" + sz] = round(ms_p, 4)
                w["GBps_" + sz] = round(mb / (ms_p * 1e-3) / 1e9, 1)
            co = compute_only_ms(P, torch, p, args.steps)
            if co is not None:
                # Section IV-B measures storing as what the complete kernel
                # adds to the pure computation kernel
                d["compute_only_ms"] = round(co, 4)
                d["compute_only_over_numeric_pass"] = round(co / d["numeric_pass_ms"], 3)
                d["compute_only_over_product"] = round(co / w["product_ms_exact"], 3)
            d["learned_sizes"] = misprediction(P, torch, p, model)
            whole[p.name] = w
    log("device copy bandwidth (b_max)")
    bmax = measure_bmax(torch)
    for w in whole.values():
        for sz in ("exact", "upper_bound", "learned"):
            gbps = w["GBps_" + sz]
            w["frac_8TBps_" + sz] = round(gbps / HBM_PEAK_GBS, 4)
            w["frac_bmax_" + sz] = round(gbps / bmax, 4)

    name, dms, dbytes, dinfo = dominant
    achieved = dbytes / (dms * 1e-3) / 1e9
    traffic = traffic_from_profile(dbytes) if name.startswith("random16") and args.sizer == "exact" else None
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
        "config": {"workload": {"roofline": "5-point Laplacian 2048x2048 squared + random 2^21 x 16/row times an "
                                            "independent one (FP64 CSR), one full product of each per step",
                                "stencil": "5-point Laplacian 2048x2048 squared",
                                "random": "random 2^21 x 16/row times an independent one",
                                "zipf": "power-law rows Zipf(2) clipped to [1, 4096], N = 2^20, squared",
                                "st9": "9-point stencil 2048x2048 squared",
                                "st27": "27-point stencil 160^3 squared"}[args.workload],
                   "sizer": args.sizer, "products_per_step": len(products)},
        "roofline": {"bound": "hbm", "kernel": "numeric pass of %s (%s sizer)" % (name, args.sizer),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": dbytes, "launch_ms": round(dms, 4),
                     "b_max_measured": round(bmax, 1), "frac_of_b_max": round(achieved / bmax, 4)},
        "whole_product_roofline": {"note": "model bytes |A| + |B| + |C| over the whole product's time (plan, "
                                           "passes and host round trips), against 8 TB/s and against b_max, the "
                                           "device copy bandwidth measured in this run (the paper's b_max)",
                                   **whole},
        "wall_ms_per_step": round(wall_ms, 3),
        "workloads": details,
    }
    if tuned:
        out["autotuning"] = tuned
    if train_info:
        out["sizer_training"] = train_info
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline([(p.name, p.A, p.B) for p in products])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
