"""Launch-shape autotuner for the list ranking inside et_tree_build.

Times et_tree_build on a seeded tree for a grid of context parameters
(``et_ctx_set_param``), one parameter at a time around the current best
(coordinate descent), and stores the winner in ``tuned.json`` next to this
file, keyed by GPU architecture. ``apply(ctx)`` loads it into a context.
Results of the library never depend on these parameters; only speed does.

    python -m paper_2103_15217_amd.autotune --log2n 24 [--write]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

GRID = {
    "lr_k1_log2": [3, 4, 5, 6],
    "lr_per_wave1": [64, 128, 256, 512, 1024],
    "lr_kn_log2": [2, 3, 4, 5],
    "lr_per_waven": [64, 128, 256, 512],
}
DEFAULT = {"lr_k1_log2": 4, "lr_per_wave1": 256, "lr_kn_log2": 3, "lr_per_waven": 128}


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def apply(ctx):
    """Load the tuned parameters of this GPU's architecture into ``ctx``."""
    if not os.path.exists(CACHE):
        return None
    entry = json.load(open(CACHE)).get(arch())
    if not entry:
        return None
    for k, v in entry["params"].items():
        ctx.set_param(k, v)
    return entry["params"]


def time_build(et, ctx, d_parent, reps):
    import torch
    for _ in range(2):
        et.et_tree_build(d_parent, ctx=ctx).free()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        et.et_tree_build(d_parent, ctx=ctx).free()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(log2n=24, grasps=(None, 1000, 1), reps=5, rounds=2, log=print):
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import gen
    import paper_2103_15217_amd as et
    n = 1 << log2n
    trees = [torch.from_numpy(gen.random_tree(n, g, seed=11 + i)).cuda() for i, g in enumerate(grasps)]
    ctx = et.Context()

    def cost(params):
        for k, v in params.items():
            ctx.set_param(k, v)
        return sum(time_build(et, ctx, t, reps) for t in trees)

    best = dict(DEFAULT)
    best_ms = cost(best)
    log(f"default {best} -> {best_ms:.3f} ms")
    table = [(dict(best), best_ms)]
    for _ in range(rounds):
        improved = False
        for name, values in GRID.items():
            for v in values:
                if v == best[name]:
                    continue
                trial = dict(best, **{name: v})
                ms = cost(trial)
                table.append((trial, ms))
                log(f"  {name}={v}: {ms:.3f} ms")
                if ms < best_ms * 0.995:
                    best, best_ms, improved = trial, ms, True
        if not improved:
            break
    ctx.check()
    log(f"best {best} -> {best_ms:.3f} ms (sum over {len(trees)} trees of 2^{log2n} nodes)")
    return best, best_ms, table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--write", action="store_true", help=f"store the winner in {CACHE}")
    a = ap.parse_args()
    t0 = time.time()
    best, ms, table = tune(a.log2n, reps=a.reps, log=lambda m: print(m, flush=True))
    out = {"arch": arch(), "params": best, "ms_sum_3_trees": ms, "log2n": a.log2n,
           "default_ms": table[0][1], "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    if a.write:
        cache = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
        cache[out["arch"]] = {"params": best, "ms_sum_3_trees": ms, "default_ms": table[0][1],
                              "log2n": a.log2n}
        json.dump(cache, open(CACHE, "w"), indent=1)


if __name__ == "__main__":
    main()
