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
