"""CPU checks of the autotuner's stored picks: the committed tuned.json holds
both workloads for gfx950 with values from the search grid, and apply()
hands exactly those values to a context."""
import json
import os

import pytest

from paper_2103_15217_amd import autotune


def test_committed_picks_are_from_the_grid():
    assert os.path.exists(autotune.CACHE)
    cache = json.load(open(autotune.CACHE))
    for workload in ("single", "batch"):
        entry = cache[f"gfx950/{workload}"]
        assert set(entry["params"]) == set(autotune.GRID)
        for k, v in entry["params"].items():
            assert v in autotune.GRID[k], (workload, k, v)
        assert entry["ms"] <= entry["default_ms"]


class _FakeCtx:
    def __init__(self):
        self.params = {}

    def set_param(self, name, value):
        self.params[name] = value


def test_apply_loads_the_workload_entry(tmp_path, monkeypatch):
    cache = {"gfx950/single": {"params": {"lr_k1_log2": 5, "query_block": 128}},
             "gfx950/batch": {"params": {"lr_per_wave1": 64}}}
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps(cache))
    monkeypatch.setattr(autotune, "CACHE", str(path))
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    ctx = _FakeCtx()
    assert autotune.apply(ctx, "single") == {"lr_k1_log2": 5, "query_block": 128}
    assert ctx.params == {"lr_k1_log2": 5, "query_block": 128}
    ctx = _FakeCtx()
    autotune.apply(ctx, "batch")
    assert ctx.params == {"lr_per_wave1": 64}
    monkeypatch.setattr(autotune, "arch", lambda: "gfx942")
    ctx = _FakeCtx()
    assert autotune.apply(ctx, "single") is None and ctx.params == {}


@pytest.mark.parametrize("workload", ["single", "batch"])
def test_missing_cache_means_library_defaults(tmp_path, monkeypatch, workload):
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "absent.json"))
    ctx = _FakeCtx()
    assert autotune.apply(ctx, workload) is None and ctx.params == {}


def test_coordinate_search_finds_a_separable_minimum():
    grid = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": [0, 1]}
    target = {"a": 3, "b": 10, "c": 1}
    calls = []

    def cost(p):
        calls.append(dict(p))
        return 100.0 + sum(abs(grid[k].index(p[k]) - grid[k].index(target[k])) for k in grid)
    best, ms, default, table = autotune.coordinate_search(cost, grid, {"a": 1, "b": 30, "c": 0},
                                                          log=lambda m: None)
    assert best == target and ms == 100.0 and default == 105.0
    assert len(table) == len(calls) - 2          # the winner and the start timed again at the end


def test_coordinate_search_drops_a_pick_that_does_not_hold_up():
    # a trial that looks fast once but not when timed again is not kept
    grid = {"a": [1, 2]}
    seen = {}

    def cost(p):
        seen[p["a"]] = seen.get(p["a"], 0) + 1
        return 50.0 if (p["a"] == 2 and seen[2] == 1) else 100.0
    best, ms, default, _ = autotune.coordinate_search(cost, grid, {"a": 1}, log=lambda m: None)
    assert best == {"a": 1} and ms == default == 100.0


def test_bucket_choice():
    assert autotune.bucket_for(1, [12, 16, 20, 24]) == 12
    assert autotune.bucket_for(1 << 12, [12, 16, 20, 24]) == 12
    assert autotune.bucket_for(1 << 14, [12, 16, 20, 24]) == 16      # tie: the larger bucket
    assert autotune.bucket_for((1 << 14) - 100, [12, 16, 20, 24]) == 12
    assert autotune.bucket_for(3 << 20, [12, 16, 20, 24]) == 20
    assert autotune.bucket_for(1 << 30, [12, 16, 20, 24]) == 24
    assert autotune.bucket_for(1 << 10, [27]) == 27
    assert autotune.bucket_for(5, []) is None


def test_apply_by_size_picks_the_nearest_bucket(tmp_path, monkeypatch):
    cache = {"gfx950/single/2^12": {"params": {"lr_k1_log2": 3}},
             "gfx950/single/2^24": {"params": {"lr_k1_log2": 5}},
             "gfx950/batch": {"params": {"lr_per_wave1": 64}, "log2n": 27}}
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps(cache))
    monkeypatch.setattr(autotune, "CACHE", str(path))
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    assert autotune.stored_buckets(cache, "gfx950", "single") == {12: {"lr_k1_log2": 3}, 24: {"lr_k1_log2": 5}}
    assert autotune.stored_buckets(cache, "gfx950", "batch") == {27: {"lr_per_wave1": 64}}
    ctx = _FakeCtx()
    assert autotune.apply(ctx, "single", size=3000) == {"lr_k1_log2": 3}
    assert autotune.apply(ctx, "single", size=1 << 23) == {"lr_k1_log2": 5}
    assert autotune.apply(ctx, "single") == {"lr_k1_log2": 5}        # no size: the largest bucket
    assert autotune.apply(ctx, "batch", size=100) == {"lr_per_wave1": 64}
    # the same parameters again are not sent to the context a second time
    calls = []
    ctx2 = _FakeCtx()
    ctx2.set_param = lambda k, v: calls.append((k, v))
    autotune.apply(ctx2, "single", size=1 << 24)
    autotune.apply(ctx2, "single", size=1 << 25)
    assert calls == [("lr_k1_log2", 5)]
