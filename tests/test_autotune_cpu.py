"""Host logic of the autotuner (no GPU): the candidate it returns, the
pruning of slow candidates and its cache, with the row-kernel timing
replaced by a table of times."""
import json
from types import SimpleNamespace

import pytest

autotune_mod = pytest.importorskip("paper_1303_1651_amd.autotune")


def _fake_operands():
    A = SimpleNamespace(nnz=4096, rows=1024)
    return A, A


def _install(monkeypatch, times):
    calls = []

    def fake_time(A, B, sizer, model, tuning, reps, cutoff=None):
        calls.append((dict(tuning), reps, cutoff))
        return times(tuning)

    monkeypatch.setattr(autotune_mod, "_time", fake_time)
    return calls


def test_returns_the_fastest_candidate(monkeypatch):
    grid = {"table_slots": [512, 1024, 2048], "stage_slots": [512, 1024]}
    speed = {(512, 512): 3.0, (512, 1024): 2.5, (1024, 512): 1.5, (1024, 1024): 2.0, (2048, 512): 4.0,
             (2048, 1024): 1.75}
    calls = _install(monkeypatch, lambda t: 2.2 if not t else speed[(t["table_slots"], t["stage_slots"])])
    A, B = _fake_operands()
    best = autotune_mod.autotune(A, B, "exact", grid=grid, reps=2)
    assert best == {"table_slots": 1024, "stage_slots": 512}
    # the defaults first, timed once
    assert calls[0] == ({}, 1, None)
    assert len(calls) == 1 + 6


def test_cutoff_follows_the_best_so_far(monkeypatch):
    grid = {"table_slots": [512, 1024, 2048]}
    speed = {512: 9.0, 1024: 1.0, 2048: 5.0}
    calls = _install(monkeypatch, lambda t: 4.0 if not t else speed[t["table_slots"]])
    A, B = _fake_operands()
    autotune_mod.autotune(A, B, "exact", grid=grid, reps=3)
    # every candidate is timed with a cutoff of twice the best time seen before it
    cutoffs = [c for _, _, c in calls[1:]]
    assert cutoffs == [8.0, 8.0, 2.0]


def test_candidates_over_the_lds_budget_are_skipped(monkeypatch):
    # 12 * (4096 + 8192) bytes is the budget exactly; 12 * (8192 + 8192) exceeds it
    grid = {"table_slots": [4096, 8192], "stage_slots": [8192]}
    calls = _install(monkeypatch, lambda t: 1.0)
    A, B = _fake_operands()
    assert autotune_mod.autotune(A, B, "exact", grid=grid, reps=1) == {"table_slots": 4096, "stage_slots": 8192}
    assert [c[0] for c in calls] == [{}, {"table_slots": 4096, "stage_slots": 8192}]
    # nothing fits: the library's defaults
    calls.clear()
    assert autotune_mod.autotune(A, B, "exact", grid={"table_slots": [8192], "stage_slots": [8192]}, reps=1) == {}
    assert [c[0] for c in calls] == [{}]


def test_cache_is_keyed_by_the_operand_family(monkeypatch, tmp_path):
    grid = {"table_slots": [512, 1024]}
    _install(monkeypatch, lambda t: {512: 2.0, 1024: 1.0}.get(t.get("table_slots"), 3.0))
    A, B = _fake_operands()
    cache = str(tmp_path / "tune.json")
    best = autotune_mod.autotune(A, B, "exact", grid=grid, reps=1, cache=cache)
    stored = json.load(open(cache))
    key = autotune_mod.signature(A, B, "exact")
    assert stored[key]["tuning"] == best == {"table_slots": 1024}
    # a second call reads the cache and times nothing
    calls = _install(monkeypatch, lambda t: 0.0)
    assert autotune_mod.autotune(A, B, "exact", grid=grid, reps=1, cache=cache) == best
    assert calls == []
