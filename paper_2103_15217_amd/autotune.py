"""Launch-shape autotuner.

Times a workload for a grid of context parameters (``et_ctx_set_param``),
one parameter at a time around the current best (coordinate descent), and
stores the winner in ``tuned.json`` next to this file, keyed by GPU
architecture, workload and log2-size bucket (the size the workload was
tuned at: nodes of a tree, nodes of a whole batch). ``apply(ctx, workload,
size)`` loads the entry of the stored bucket nearest to ``size`` (in log2)
into a context. Results of the library never depend on these parameters;
only speed does.

Parameters: list-ranking splitter spacing and sublists per wavefront
(level 1 and upper levels), the range-minimum block size of the bridge and
RMQ-LCA tables, and the workgroup size of the LCA query kernels.

Workloads:
  single  three trees of 2^log2n nodes (grasp n, 1000, 1), each built and
          queried with 2^log2n uniform pairs, plus bridges on a planted
          sparse graph of 2^graph_log2n vertices and 8x as many edges
  batch   a forest of trees of log-uniform size (batched build and batched
          queries) plus one batched bridge call over many graphs: at
          log2n >= 26 the 4096-tree forest of 2^6..2^18-node trees and 1024
          graphs of 2^6..2^14 vertices; below, 16 trees of
          2^(log2n-6)..2^(log2n-3) nodes (about 2^log2n in all) and 16
          graphs of a quarter of that size

    python -m paper_2103_15217_amd.autotune --workload single --log2n 20 [--write]
"""
import argparse
import json
import math
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
    "rmq_block_log2": [5, 6],
    "query_block": [64, 128, 256, 512, 1024],
}
DEFAULT = {"lr_k1_log2": 4, "lr_per_wave1": 256, "lr_kn_log2": 3, "lr_per_waven": 128, "rmq_block_log2": 5,
           "query_block": 256}


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(workload, bucket=None):
    k = f"{arch()}/{workload}"
    return k if bucket is None else f"{k}/2^{int(bucket)}"


_cache = {"path": None, "mtime": None, "data": {}}


def _read(path=None):
    path = path or CACHE
    if not os.path.exists(path):
        return {}
    m = os.path.getmtime(path)
    if _cache["path"] != path or _cache["mtime"] != m:
        _cache.update(path=path, mtime=m, data=json.load(open(path)))
    return _cache["data"]


def stored_buckets(cache, arch_name, workload):
    """{log2 size: params} of one workload; an entry without a bucket in its
    key counts at the size it was tuned at (its log2n)."""
    out = {}
    prefix = f"{arch_name}/{workload}"
    for k, entry in cache.items():
        if k == prefix:
            out.setdefault(int(entry.get("log2n", 24)), dict(entry["params"]))
        elif k.startswith(prefix + "/2^"):
            out[int(k[len(prefix) + 3:])] = dict(entry["params"])
    return out


def bucket_for(size, buckets):
    """The stored bucket nearest to ``size`` in log2 (ties go to the larger)."""
    if not buckets:
        return None
    lg = math.log2(max(int(size), 1))
    return min(buckets, key=lambda b: (abs(b - lg), -b))


def load(workload, size=None):
    """The stored parameters of this GPU and workload for ``size`` (the
    largest stored bucket when None), or None."""
    cache = _read()
    if not cache:
        return None
    buckets = stored_buckets(cache, arch(), workload)
    if not buckets:
        return None
    b = max(buckets) if size is None else bucket_for(size, list(buckets))
    return dict(buckets[b])


def apply(ctx, workload="single", size=None):
    """Load the tuned parameters of this GPU, workload and size into ``ctx``
    (skipped when the context already holds them); returns them (None when
    nothing is stored)."""
    params = load(workload, size)
    if params and getattr(ctx, "_tuned_params", None) != params:
        for k, v in params.items():
            ctx.set_param(k, v)
        try:
            ctx._tuned_params = dict(params)
        except AttributeError:
            pass
    return params


def _best_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def single_workload(et, ctx, log2n, graph_log2n):
    """Callables of the single-instance workload (built once, timed many times)."""
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import gen
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    n = 1 << log2n
    trees = [d(gen.random_tree(n, g, seed=11 + i)) for i, g in enumerate((None, 1000, 1))]
    qx, qy = [d(a) for a in gen.random_queries(n, n, seed=11)]
    gn = 1 << graph_log2n
    rp, col, _ = gen.planted_bridge_graph(n=gn, m=8 * gn, chains=max(1, gn >> 10), max_chain=512, seed=11)
    drp, dcol = d(rp), d(col)

    def trees_and_queries():
        for p in trees:
            t = et.et_tree_build(p, ctx=ctx)
            t.lca(qx, qy)
            t.free()

    def bridges():
        et.et_bridges(drp, dcol, ctx=ctx, count=False)

    def rmq_engine():
        t = et.et_tree_build(trees[0], ctx=ctx).rmq_build(trees[0])
        t.lca_rmq(qx, qy)
        t.free()

    return [trees_and_queries, bridges, rmq_engine]


def batch_workload(et, ctx, log2n):
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import gen
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    if log2n >= 26:
        trees, tlo, thi, graphs, glo, ghi = 4096, 6, 18, 1024, 6, 14
    else:
        trees, tlo, thi = 16, max(log2n - 6, 4), max(log2n - 3, 5)
        graphs, glo, ghi = 16, max(log2n - 8, 6), max(log2n - 5, 7)
    b = gen.forest_batch(trees, seed=12, log2_min=tlo, log2_max=thi)
    parent, offs = d(b["parent"]), torch.from_numpy(b["offsets"].astype(np.int64)).cuda()
    qt, qx, qy = d(b["qtree"]), d(b["qx"]), d(b["qy"])
    rng = np.random.default_rng(12)
    gl = []
    for t in range(graphs):
        n = int(2 ** rng.uniform(glo, ghi))
        chains = max(1, n // 512)
        rp, col, _ = gen.planted_bridge_graph(n=n, m=4 * n, chains=chains, max_chain=max(2, n // (8 * chains)),
                                              seed=1000 + t)
        gl.append((rp, col))
    rows = d(np.concatenate([g[0] for g in gl]))
    cols = d(np.concatenate([g[1] for g in gl]))
    slots = [len(g[1]) for g in gl]
    voff = torch.from_numpy(np.cumsum([0] + [len(g[0]) - 1 for g in gl]).astype(np.int64)).cuda()
    soff = torch.from_numpy(np.cumsum([0] + slots).astype(np.int64)).cuda()

    def forest():
        t = et.et_tree_build_batch(parent, offs, ctx=ctx)
        t.lca_batch(qt, qx, qy)
        t.free()

    def graph_batch():
        et.et_bridges_batch(row_ptr=rows, col=cols, voff=voff, soff=soff, slots=slots, ctx=ctx, counts=False)

    return [forest, graph_batch]


def coordinate_search(cost, grid=None, start=None, rounds=2, log=print):
    """Coordinate descent over ``grid`` from ``start``: each round tries every
    other value of every parameter with the rest held, and keeps a trial
    that is at least 0.5 % faster. The winner is then timed once more
    against ``start``; if it is not faster there, ``start`` is kept, so a
    pick that only won through noise is dropped. Returns (best, its cost,
    the start's cost, [(params, cost)] of every trial)."""
    grid = GRID if grid is None else grid
    start = dict(DEFAULT if start is None else start)
    best = dict(start)
    best_ms = cost(best)
    log(f"default {best} -> {best_ms:.3f} ms")
    table = [(dict(best), best_ms)]
    for _ in range(rounds):
        improved = False
        for name, values in grid.items():
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
    final, default = cost(best), cost(start)
    if final >= default:
        best, final = dict(start), default
    return best, final, default, table


def tune(workload="single", log2n=24, graph_log2n=22, reps=3, rounds=2, log=print):
    import paper_2103_15217_amd as et
    ctx = et.Context()
    if workload == "single":
        parts = single_workload(et, ctx, log2n, graph_log2n)
    else:
        parts = batch_workload(et, ctx, log2n)

    def cost(params):
        for k, v in params.items():
            ctx.set_param(k, v)
        return sum(_best_ms(f, reps) for f in parts)

    best, final, default, table = coordinate_search(cost, rounds=rounds, log=log)
    ctx.check()
    log(f"best {best} -> {final:.3f} ms (default {default:.3f} ms)")
    return best, final, default, table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["single", "batch"], default="single")
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--graph-log2n", type=int, default=None, help="default: log2n - 2")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--write", action="store_true", help=f"store the winner in {CACHE}")
    ap.add_argument("--out", default=CACHE, help="the file --write updates")
    a = ap.parse_args()
    t0 = time.time()
    if a.graph_log2n is None:
        a.graph_log2n = max(a.log2n - 2, 8)
    best, ms, default, table = tune(a.workload, a.log2n, a.graph_log2n, reps=a.reps,
                                   log=lambda m: print(m, flush=True))
    out = {"key": key(a.workload, a.log2n), "params": best, "ms": ms, "default_ms": default, "trials": len(table),
           "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    if a.write:
        cache = json.load(open(a.out)) if os.path.exists(a.out) else {}
        cache[out["key"]] = {"params": best, "ms": ms, "default_ms": default,
                             "workload": a.workload, "log2n": a.log2n, "graph_log2n": a.graph_log2n}
        json.dump(cache, open(a.out, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
