"""Host logic of bench.py (no GPU): the model-bytes count, the counter
summaries and their calibration, the source check of the stored traffic,
and the refusal of more than one GPU."""
import csv
import importlib.util
import json
import os
import subprocess
import sys
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_model_bytes_counts_int32_columns_fp64_values_int64_row_pointers():
    b = _bench()
    A = SimpleNamespace(nnz=10, rows=4)
    B = SimpleNamespace(nnz=7, rows=5)
    # A: 10 * 12 + 5 * 8; B: 7 * 12 + 6 * 8; C (A's rows): 9 * 12 + 5 * 8
    assert b.model_bytes(A, B, 9) == 160 + 132 + 148


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_pmc_summary_scales_each_counter_by_the_largest_copy(tmp_path):
    b = _bench()
    copy = 1 << 30
    fetch, write, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "s.json"
    # the copy reads half its bytes by FETCH_SIZE (factor 2) and all by WRITE_SIZE
    _counter_csv(fetch, "FETCH_SIZE", [("void spg::k_wt<1, 4>(...)", 1000.0), ("void spg::k_wt<1, 4>(...)", 3000.0),
                                       ("__amd_rocclr_copyBuffer", copy / 1024 / 2), ("__amd_rocclr_copyBuffer", 10.0),
                                       ("void spg::k_scan<int>(...)", 77.0)])
    _counter_csv(write, "WRITE_SIZE", [("void spg::k_wt<1, 4>(...)", 500.0), ("__amd_rocclr_copyBuffer", copy / 1024)])
    b.pmc_summary(str(fetch), str(write), "k_wt<1,", copy, str(out), "cmd")
    d = json.load(open(out))
    assert d["fetch_kib_per_launch"] == 2000.0   # mean over the kernel's dispatches
    assert abs(d["fetch_factor"] - 2.0) < 1e-12 and abs(d["write_factor"] - 1.0) < 1e-12
    assert abs(d["traffic_bytes_per_launch"] - (2000.0 * 2 + 500.0) * 1024) < 1e-6
    assert d["source_sha1"] == b.kernel_source_sha1() and d["command"] == "cmd"


def test_stored_traffic_is_used_only_for_the_same_kernel_source(tmp_path, monkeypatch):
    b = _bench()
    f = tmp_path / "t.json"
    json.dump({"traffic_bytes_per_launch": 123.0, "source_sha1": b.kernel_source_sha1()}, open(f, "w"))
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.traffic_from_profile(1) == 123
    json.dump({"traffic_bytes_per_launch": 123.0, "source_sha1": "other"}, open(f, "w"))
    assert b.traffic_from_profile(1) is None
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert b.traffic_from_profile(1) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""
