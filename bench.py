"""Benchmark of the Euler-tour hot path on one MI355X.

One step = the whole path over one batch of synthetic input:
  for each grasp g in {n, 1000, 1}: et_tree_build of a 2^24-node grasp tree
  (grouping, successor, list ranking, depth / preorder / size, Inlabel
  tables) and et_lca over 2^24 uniform query pairs; then et_bridges on a
  2^22-vertex, ~2^25-edge sparse graph with 4096 planted bridge chains.
Inputs are generated on the host, copied to HBM before timing, and stay
resident. W untimed warmup steps, then K timed steps between two device
synchronisations. Prints one JSON line.

value = (sum over the three trees of (nodes + queries) + graph edges) per
second of step time. Per-component rates, per-kernel times (HIP events on
the library's stream, from three untimed steps in which every launch is
bracketed), the roofline of the dominant kernel (whose launches alone carry
events during the timed steps, so its durations come from the timed region
while the events add nothing measurable to the step) and the CPU oracle on
a bounded sample are reported beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LCA queries/s + tour nodes/s at 2^24; bridges edges/s; batched vs plain p99"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit for the kernels that can dominate a step.
# (bytes per unit, what a unit is, how many units one launch processes)
ALG_BYTES = {
    # list ranking: read the successor (4 B) and write the rank (4 B) of every half-edge
    "k_walk1<true>": (8, "half-edge", lambda w: 2 * w["n"]),
    "k_walk1<false>": (8, "half-edge", lambda w: 2 * (w["graph_n"] - 1)),
    # LCA: 12 B streamed (x, y, out) + 4 gathers of 16-B records per query
    "k_lca": (76, "query", lambda w: w["q"]),
    # first hooking round: row pointers (8 B) and up to two columns (8 B) per vertex
    "k_hook_sample": (16, "vertex", lambda w: w["graph_n"]),
    # path tops: 16-B record, parent and the parent's gathered inlabel read; about half the
    # nodes are tops and write an 8-B head entry and a 4-B parent-path label
    "k_head": (30, "node", lambda w: w["n"]),
    # successor: parent and child read per grouped position, succ(2c+1) and (at the first
    # child) succ(2p) written
    "k_succ": (14, "node", lambda w: w["n"]),
    # ascendant into the node record: inlabel read, label ascendant gathered, 4 B written
    "k_asc": (12, "node", lambda w: w["n"]),
    # node statistics: the 8-B records of 2c and 2c+1 and their two 8-B sublist offsets
    # read; rank pair (8 B), pre, size, inlabel (4 B each) and the 16-B node record written
    "k_node": (68, "node", lambda w: w["n"]),
    # non-forest min/max: column (4 B) + gathered preorder (4 B) per slot
    "k_minmax": (8, "CSR slot", lambda w: w["graph_nnz"]),
    # radix passes: key + value read and written
    "k_downsweep<false>": (16, "key", lambda w: w["n"]),
    "k_downsweep<true>": (12, "key", lambda w: w["n"]),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log2n", type=int, default=24, help="tree size (2^k nodes and queries)")
    ap.add_argument("--graph-log2n", type=int, default=22)
    ap.add_argument("--graph-log2m", type=int, default=25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4096-tree batched vs plain comparison")
    ap.add_argument("--only-small-batches", action="store_true",
                    help="of the batch components run only the one-launch sweeps (small trees, small graphs)")
    ap.add_argument("--batch-trees", type=int, default=4096)
    ap.add_argument("--batch-graphs", type=int, default=1024)
    ap.add_argument("--no-serve", action="store_true", help="skip the served vs plain trace replay")
    ap.add_argument("--no-engines", action="store_true",
                    help="skip the Inlabel vs RMQ query engine comparison (and the scale-free tree)")
    ap.add_argument("--no-ck", action="store_true",
                    help="skip the Chaitanya-Kothapalli and hybrid bridge comparison")
    ap.add_argument("--no-edges", action="store_true",
                    help="skip the edge-list (DCEL construction) build comparison")
    ap.add_argument("--no-naive", action="store_true",
                    help="skip the naive (climbing) LCA comparison and its depth and q:n sweeps")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the same step with its independent jobs on two streams")
    ap.add_argument("--no-lists", action="store_true",
                    help="skip the plain vs weighted list ranking of the tours and of a random list")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0,
                    help="device-memory budget of the continuous-batching server (GiB)")
    ap.add_argument("--serve-sweep", default="1000,4000,8000",
                    help="extra arrival rates (jobs/s) replayed for 2 s each to show where each path saturates; "
                         "empty to skip")
    ap.add_argument("--protocol-seeds", type=int, default=5,
                    help="instances of the paper's measurement protocol (0 to skip)")
    ap.add_argument("--protocol-runs", type=int, default=5, help="timed runs per instance (after one warm-up)")
    ap.add_argument("--default-params", action="store_true",
                    help="run with the library's default launch shapes instead of the autotuned ones")
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="do not bracket kernels with events during the timed steps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy of MIB MiB (int32 negate: reads and writes MIB MiB) "
                         "five times, to calibrate HBM byte counters against a known size")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(this path runs on a single MI355X; it has no multi-GPU sharding)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    import paper_2103_15217_amd as et

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    n = 1 << args.log2n
    q = n
    grasps = [None, 1000, 1]
    t0 = time.time()
    trees, queries = [], []
    for i, g in enumerate(grasps):
        trees.append(gen.random_tree(n, g, seed=args.seed + i))
    qx, qy = gen.random_queries(n, q, seed=args.seed)
    log(f"trees generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    gn, gm = 1 << args.graph_log2n, 1 << args.graph_log2m
    chains = 4096 if args.graph_log2n >= 16 else 16
    rp, col, ginfo = gen.planted_bridge_graph(n=gn, m=gm, chains=chains,
                                              max_chain=min(512, max(2, gn >> 13)), seed=args.seed)
    log(f"graph generated in {time.time() - t0:.1f}s: V={gn} m={ginfo['m']} nnz={len(col)}")

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)

    d_parent = [d(p) for p in trees]
    d_qx, d_qy = d(qx), d(qy)
    d_rp, d_col = d(rp), d(col)
    d_out = torch.empty(q, dtype=torch.int32, device=dev)
    d_mask = torch.empty(max((len(col) + 31) // 32, 1), dtype=torch.int32, device=dev)
    ctx = et.default_context()
    # launch shapes picked by the autotuner for this GPU (results never depend on them)
    from paper_2103_15217_amd import autotune
    launch = {"single": None, "batch": None}
    if not args.default_params:
        launch["single"] = autotune.apply(ctx, "single")
    bctx = et.Context()
    if not args.default_params:
        launch["batch"] = autotune.apply(bctx, "batch")
    work = {"n": n, "q": q, "graph_n": gn, "graph_nnz": len(col), "graph_m": ginfo["m"]}

    stream = torch.cuda.current_stream()
    marks = {}

    def ev(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        marks.setdefault(name, []).append(e)

    def step(record):
        for i in range(len(grasps)):
            if record:
                ev(f"build{i}.start")
            t = et.et_tree_build(d_parent[i], ctx=ctx)
            if record:
                ev(f"build{i}.end")
            t.lca(d_qx, d_qy, out=d_out)
            if record:
                ev(f"lca{i}.end")
            t.free()
        if record:
            ev("bridges.start")
        et.et_bridges(d_rp, d_col, mask=d_mask, ctx=ctx, count=False)
        if record:
            ev("bridges.end")

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    ctx.check()
    ctx.profile_read()
    kernels, dom = {}, None
    prof_steps = 3
    if not args.no_kernel_times:
        # per-kernel breakdown from separate, untimed steps: bracketing every
        # launch with events costs several percent of the step
        ctx.profile(True)
        for _ in range(prof_steps):
            step(False)
        torch.cuda.synchronize()
        kernels = ctx.profile_read()
        busy = {k: v[1] for k, v in kernels.items() if not k.startswith("phase:")}
        dom = max(busy, key=busy.get) if busy else None
        # in the timed steps only the dominant kernel's launches carry events
        ctx.profile(True, only=dom)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        step(True)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    timed = ctx.profile_read() if not args.no_kernel_times else {}
    ctx.profile(False)
    ctx.check()
    ms_per_step = total_ms / args.steps

    def span(a, b):
        return sum(x.elapsed_time(y) for x, y in zip(marks[a], marks[b])) / args.steps

    build_ms = [span(f"build{i}.start", f"build{i}.end") for i in range(len(grasps))]
    lca_ms = [span(f"build{i}.end", f"lca{i}.end") for i in range(len(grasps))]
    bridges_ms = span("bridges.start", "bridges.end")
    elements = len(grasps) * (n + q) + ginfo["m"]
    gname = ["n", "1000", "1"]
    components = {
        "lca_preprocess_nodes_per_s": {gname[i]: n / (build_ms[i] * 1e-3) for i in range(3)},
        "lca_queries_per_s": {gname[i]: q / (lca_ms[i] * 1e-3) for i in range(3)},
        "lca_total_queries_per_s": {gname[i]: q / ((build_ms[i] + lca_ms[i]) * 1e-3) for i in range(3)},
        "bridges_edges_per_s": ginfo["m"] / (bridges_ms * 1e-3),
        "ms": {"build": dict(zip(gname, build_ms)), "lca": dict(zip(gname, lca_ms)), "bridges": bridges_ms},
    }
    if "phase:tour" in kernels:
        tour_ms = kernels["phase:tour"][1] / kernels["phase:tour"][0]
        components["tour_nodes_per_s"] = n / (tour_ms * 1e-3)

    # dominant kernel and its roofline; its launch durations are the ones
    # timed inside the timed steps
    per_step = {k: (v[0] / prof_steps, v[1] / prof_steps, v[1] / v[0]) for k, v in kernels.items()
                if not k.startswith("phase:")}
    roofline = None
    if dom and dom in timed:
        launches = timed[dom][0] / args.steps
        avg_ms = timed[dom][1] / timed[dom][0]
        roofline = kernel_roofline(dom, avg_ms, launches, work, launch["single"])
    # list ranking and LCA queries, and the largest kernels of the build and
    # of the bridges, from the profiled steps
    kernel_rooflines = {}
    for k in ("k_walk1<true>", "k_lca", "k_node", "k_head", "k_succ", "k_asc", "k_minmax"):
        if k in kernels and kernels[k][0] > 0:
            kernel_rooflines[k] = kernel_roofline(k, kernels[k][1] / kernels[k][0], kernels[k][0] / prof_steps,
                                                  work, launch["single"])

    result = {
        "metric": METRIC,
        "value": elements / (ms_per_step * 1e-3),
        "unit": "elements/s (tree nodes + LCA queries + graph edges)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": (f"3 grasp trees (g=n,1000,1) of 2^{args.log2n} nodes, each built and queried with "
                         f"2^{args.log2n} uniform LCA pairs; bridges on a {gn}-vertex {ginfo['m']}-edge graph "
                         f"with {chains} planted chains"),
            "tree_nodes": n, "queries_per_tree": q, "grasps": ["n", 1000, 1],
            "graph_vertices": gn, "graph_edges": ginfo["m"], "graph_csr_slots": len(col),
            "seed": args.seed,
        },
        "launch_params": launch,
        "components": components,
        "kernels_ms_per_step": {k: round(v[1], 4) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1][1])},
        "roofline": roofline,
        "kernel_rooflines": kernel_rooflines,
    }

    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")
    if not args.no_concurrent:
        log("the step's independent jobs on two streams")
        result["components"]["concurrent_step"] = concurrent_step(args, et, d_parent, d_qx, d_qy, d_rp, d_col,
                                                                  ms_per_step, elements)
    if not args.no_batch and not args.only_small_batches:
        log("batched forest: generating")
        result["components"]["batched"] = batched_vs_plain(args, et, bctx, d, dev)
    if not args.no_batch:
        log("small-tree batches: one fused launch vs the multi-kernel batch")
        result["components"]["small_batches"] = small_batches(args, et, bctx, d, dev)
    if not args.no_batch:
        log("small-graph batches: one fused launch vs the multi-kernel batch")
        result["components"]["small_graph_batches"] = small_graph_batches(args, et, bctx, d)
    if not args.no_batch and not args.only_small_batches:
        log("batched graphs: generating")
        result["components"]["bridges_batched"] = bridges_batched_vs_plain(args, et, bctx, d)
    if not args.no_engines:
        log("query engines: Inlabel vs RMQ, scale-free tree")
        result["components"]["query_engines"] = query_engines(args, et, ctx, d, d_parent, d_qx, d_qy, grasps)
    if not args.no_ck:
        log("bridges: CK and hybrid")
        result["components"]["bridges_methods"] = bridges_methods(et, ctx, d_rp, d_col, d_mask, ginfo["m"])
    if not args.no_edges:
        log("edge-list build")
        result["components"]["edge_list_build"] = edges_vs_parent(args, et, ctx, d, trees, d_parent, grasps)
    if not args.no_naive:
        log("naive LCA: levels and climbing queries")
        result["components"]["naive_lca"] = naive_vs_inlabel(args, et, ctx, d, d_parent, d_qx, d_qy, grasps)
    if not args.no_lists:
        log("list ranking: plain and weighted")
        result["components"]["list_ranking"] = list_ranking(args, et, ctx, d, d_parent)
    if not args.no_serve:
        log("serving: generating the job pool")
        result["components"]["serving"] = serving(args, dev)
    if args.protocol_seeds > 0:
        log(f"protocol: {args.protocol_seeds} instances x {args.protocol_runs} runs")
        result["components"]["protocol"] = protocol(args, et, ctx, d, grasps,
                                                    (d_parent, d_qx, d_qy, d_rp, d_col))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the sample")
        result["cpu_baseline"], result["parity"] = cpu_baseline(trees[0], qx, qy, rp, col, ginfo, et, d, ctx,
                                                                d_parent[0], d_qx, d_qy, d_rp, d_col)
    print(json.dumps(result), flush=True)


def _gpu_ms(fn, reps=3):
    """Best-of-reps GPU time of fn() on the current stream (after one warm-up call)."""
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


def _kernel_breakdown(ctx, fn, top=8):
    """Per-kernel GPU time (ms, summed over launches) of one profiled call
    of fn(): the ``top`` largest, plus their share of the call's kernel time."""
    import torch
    ctx.profile_read()
    ctx.profile(True)
    fn()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    ks = sorted(((k, v[1]) for k, v in prof.items() if not k.startswith("phase:")), key=lambda kv: -kv[1])
    total = sum(v for _, v in ks)
    return {"kernel_ms": {k: round(v, 4) for k, v in ks[:top]}, "kernels_total_ms": total}


def query_engines(args, et, ctx, d, d_parent, d_qx, d_qy, grasps):
    """Inlabel against the RMQ engine over the Euler tour (Section 3) on the
    three bench trees and on a 2^log2n scale-free (Barabasi-Albert) tree
    (Section 3.2, Figs. 7-8), with 2^log2n uniform queries each; the naive
    method is added on the scale-free tree, which is shallow."""
    import torch
    import gen
    res = {}
    trees = list(zip(["n", "1000", "1"], d_parent))
    n = d_parent[0].numel()
    t0 = time.time()
    trees.append(("scale_free", d(gen.ba_tree(n, seed=args.seed + 9))))
    log(f"scale-free tree generated in {time.time() - t0:.1f}s")
    out = torch.empty_like(d_qx)
    for name, par in trees:
        r = {"inlabel_build_ms": _gpu_ms(lambda: et.et_tree_build(par, ctx=ctx).free(), 2)}
        tree = et.et_tree_build(par, ctx=ctx)
        r["rmq_build_ms"] = _gpu_ms(lambda: tree.rmq_build(par), 2)
        r["inlabel_query_ms"] = _gpu_ms(lambda: tree.lca(d_qx, d_qy, out=out))
        ref = out.clone()
        r["rmq_query_ms"] = _gpu_ms(lambda: tree.lca_rmq(d_qx, d_qy, out=out))
        r["rmq_matches_inlabel"] = bool(torch.equal(out, ref))
        if name == "scale_free":
            lv = torch.empty_like(par)
            r["naive_levels_ms"] = _gpu_ms(lambda: et.et_levels(par, out=lv, ctx=ctx), 2)
            r["naive_query_ms"] = _gpu_ms(lambda: et.et_lca_naive(par, lv, d_qx, d_qy, out=out, ctx=ctx))
            r["naive_matches_inlabel"] = bool(torch.equal(out, ref))
        tree.free()
        ctx.check()
        r["queries"] = d_qx.numel()
        res[name] = r
    return res


BRIDGE_PHASES = {
    "spanning forest": ("k_check_csr", "k_hook_sample", "k_cc_compress", "k_big_component", "k_hook_rest"),
    "BFS": ("k_bfs_level", "k_bfs_slots"),
    "Euler tour": ("k_tree_deg", "k_tree_fill", "k_root_flags", "k_root_list", "k_succ_csr", "k_link_roots",
                   "k_walk1<false>", "k_walkN", "k_final_lds", "k_final_walk", "k_push_down", "k_check_reached",
                   "k_rank_fix", "k_count_used", "k_rank_of", "k_direction", "k_preorder", "k_hybrid_nodes"),
    "marking": ("k_ck_mark", "k_ck_out"),
    "low/high + test": ("k_minmax", "k_rmq_blocks", "k_sparse_level", "k_bridge_test"),
}


def bridges_methods(et, ctx, d_rp, d_col, tv_mask, m):
    """Tarjan-Vishkin against the paper's comparison methods on the bench
    graph (Section 4.2, Figs. 10-11): Chaitanya-Kothapalli marking on a BFS
    forest and the hybrid (marking on the Euler-tour-rooted connectivity
    forest). Whole-call time (best of 2) and a per-phase kernel breakdown."""
    import torch
    res = {}
    calls = {"TV": lambda: et.et_bridges(d_rp, d_col, ctx=ctx, count=False)[0],
             "CK": lambda: et.et_bridges_ck(d_rp, d_col, spanning="bfs", ctx=ctx, count=False)[0],
             "hybrid": lambda: et.et_bridges_ck(d_rp, d_col, spanning="forest", ctx=ctx, count=False)[0]}
    for name, fn in calls.items():
        ms = _gpu_ms(fn, 2)
        ctx.profile_read()
        ctx.profile(True)
        out = fn()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        phases = {ph: sum(prof[k][1] for k in ks if k in prof) for ph, ks in BRIDGE_PHASES.items()}
        res[name] = {"ms": ms, "edges_per_s": m / (ms * 1e-3), "same_mask_as_tv": bool(torch.equal(out, tv_mask)),
                     "phase_ms": {k: v for k, v in phases.items() if v > 0}}
        ctx.check()
    return res


def edges_vs_parent(args, et, ctx, d, trees, d_parent, grasps):
    """The same three 2^log2n trees given as unordered, randomly oriented
    edge lists: et_tree_build_edges (the DCEL construction of Section 2.1,
    with its lexicographic sort) against et_tree_build from the parent
    array; also checks that depth and size agree."""
    import torch
    res = {}
    names = ["n", "1000", "1"]
    for i, g in enumerate(grasps):
        parent = trees[i]
        rng = np.random.default_rng(args.seed + 40 + i)
        c = np.flatnonzero(parent >= 0).astype(np.int32)
        p = parent[c]
        flip = rng.random(c.shape[0]) < 0.5
        order = rng.permutation(c.shape[0])
        u, v = d(np.where(flip, c, p)[order]), d(np.where(flip, p, c)[order])
        n = parent.shape[0]
        root = int(np.flatnonzero(parent == -1)[0])
        edges_ms = _gpu_ms(lambda: et.et_tree_build_edges(u, v, n, root, ctx=ctx).free())
        parent_ms = _gpu_ms(lambda: et.et_tree_build(d_parent[i], ctx=ctx).free())
        te = et.et_tree_build_edges(u, v, n, root, ctx=ctx)
        tp = et.et_tree_build(d_parent[i], ctx=ctx)
        a, b = te.export(("depth", "size")), tp.export(("depth", "size"))
        same = bool(torch.equal(a["depth"], b["depth"]) and torch.equal(a["size"], b["size"]))
        te.free()
        tp.free()
        ctx.check()
        res[names[i]] = {"edges_build_ms": edges_ms, "parent_build_ms": parent_ms,
                         "edges_nodes_per_s": n / (edges_ms * 1e-3), "depth_size_agree": same}
    return res


def naive_vs_inlabel(args, et, ctx, d, d_parent, d_qx, d_qy, grasps):
    """The paper's comparison of the naive algorithm (levels by pointer
    jumping, queries by climbing) with Inlabel (Section 3.2, Figs. 4-5):
    preprocessing of the three 2^log2n bench trees, queries where climbing
    stays affordable, a depth sweep (grasp) and a q:n sweep at 2^20 nodes."""
    import torch
    import gen
    res = {"trees": {}}
    n = d_parent[0].numel()
    names = ["n", "1000", "1"]
    for i, g in enumerate(grasps):
        lv = torch.empty_like(d_parent[i])
        r = {"levels_ms": _gpu_ms(lambda: et.et_levels(d_parent[i], out=lv, ctx=ctx))}
        q = {None: n, 1000: 1 << 16}.get(g)          # a path makes every climb ~n/3 steps long
        if q:
            x, y = d_qx[:q], d_qy[:q]
            out = torch.empty_like(x)
            r["queries"] = q
            r["naive_query_ms"] = _gpu_ms(lambda: et.et_lca_naive(d_parent[i], lv, x, y, out=out, ctx=ctx))
            tree = et.et_tree_build(d_parent[i], ctx=ctx)
            ref = tree.lca(x, y)
            r["inlabel_query_ms"] = _gpu_ms(lambda: tree.lca(x, y, out=ref))
            r["naive_matches_inlabel"] = bool(torch.equal(out, ref))
            tree.free()
        r["inlabel_build_ms"] = _gpu_ms(lambda: et.et_tree_build(d_parent[i], ctx=ctx).free())
        res["trees"][names[i]] = r
        ctx.check()
    m = 1 << 20
    qx, qy = gen.random_queries(m, 1 << 24, seed=args.seed + 5)
    dqx, dqy = d(qx), d(qy)

    def both(parent, q):
        lv = torch.empty_like(parent)
        out = torch.empty(q, dtype=torch.int32, device=parent.device)
        x, y = dqx[:q], dqy[:q]

        def naive():
            et.et_levels(parent, out=lv, ctx=ctx)
            et.et_lca_naive(parent, lv, x, y, out=out, ctx=ctx)

        def inlabel():
            t = et.et_tree_build(parent, ctx=ctx)
            t.lca(x, y, out=out)
            t.free()
        return _gpu_ms(naive, 2), _gpu_ms(inlabel, 2)

    res["depth_sweep"] = []
    for g in (None, 1 << 14, 1 << 10, 1 << 8, 1 << 6):
        parent = d(gen.random_tree(m, g, seed=args.seed + 7))
        nv, il = both(parent, m)
        res["depth_sweep"].append({"n": m, "grasp": g or m, "q": m, "naive_ms": nv, "inlabel_ms": il})
        log(f"naive sweep grasp {g or m}: naive {nv:.3f} ms, inlabel {il:.3f} ms")
    parent = d(gen.random_tree(m, None, seed=args.seed + 8))
    res["q_sweep"] = []
    for lq in (10, 14, 18, 20, 22, 24):
        nv, il = both(parent, 1 << lq)
        res["q_sweep"].append({"n": m, "grasp": m, "q": 1 << lq, "naive_ms": nv, "inlabel_ms": il})
    ctx.check()
    return res


def list_ranking(args, et, ctx, d, d_parent):
    """List ranking on its own (Section 2.2): the tours of the three bench
    trees ranked plain and with weights +1 on down and -1 on up half-edges
    (the weighted sum at a down half-edge is that child's depth, checked
    against the build's depth), and one random list of 2^(log2n+1)
    elements with weights in [-2^20, 2^20)."""
    import numpy as np
    import torch
    res = {"tours": {}}
    for name, parent in zip(["n", "1000", "1"], d_parent):
        tree = et.et_tree_build(parent, ctx=ctx)
        t = tree.export(["succ", "depth"])
        head = tree.tour()[:1].clone()
        tree.free()
        succ = t["succ"]
        w = (1 - 2 * (torch.arange(succ.numel(), device=succ.device, dtype=torch.int32) & 1)).to(torch.int32)
        L = succ.numel() - 2
        r = {"elements": L}
        r["rank_ms"] = _gpu_ms(lambda: et.et_list_rank(succ, head, ctx=ctx))
        r["scan_ms"] = _gpu_ms(lambda: et.et_list_scan(succ, w, head, ctx=ctx))
        r["scan_and_rank_ms"] = _gpu_ms(lambda: et.et_list_scan(succ, w, head, rank=True, ctx=ctx))
        sums = et.et_list_scan(succ, w, head, ctx=ctx)
        down = sums[0::2]
        used = succ[0::2] != -2
        r["depth_matches_build"] = bool(torch.equal(down[used], t["depth"][used]))
        r["rank_elements_per_s"] = L / (r["rank_ms"] * 1e-3)
        r["scan_elements_per_s"] = L / (r["scan_ms"] * 1e-3)
        res["tours"][name] = r
        ctx.check()
    L = 1 << (args.log2n + 1)
    rng = np.random.default_rng(args.seed + 11)
    order = rng.permutation(L).astype(np.int32)
    succ = np.empty(L, dtype=np.int32)
    succ[order[:-1]] = order[1:]
    succ[order[-1]] = -1
    dsucc, head = d(succ), d(order[:1].copy())
    dw = d(rng.integers(-(1 << 20), 1 << 20, L, dtype=np.int32))
    r = {"elements": L}
    r["rank_ms"] = _gpu_ms(lambda: et.et_list_rank(dsucc, head, ctx=ctx))
    r["scan_ms"] = _gpu_ms(lambda: et.et_list_scan(dsucc, dw, head, ctx=ctx))
    rank = et.et_list_rank(dsucc, head, ctx=ctx)
    r["rank_is_position"] = bool(torch.equal(rank[d(order).long()],
                                             torch.arange(L, dtype=torch.int32, device=rank.device)))
    r["rank_elements_per_s"] = L / (r["rank_ms"] * 1e-3)
    r["scan_elements_per_s"] = L / (r["scan_ms"] * 1e-3)
    res["random_list"] = r
    ctx.check()
    log(f"list ranking 2^{args.log2n + 1}: rank {r['rank_ms']:.3f} ms, weighted {r['scan_ms']:.3f} ms")
    return res


def concurrent_step(args, et, d_parent, d_qx, d_qy, d_rp, d_col, seq_ms, elements):
    """The timed step's four independent jobs (the three trees, each built,
    queried and freed, and the bridges) split over two streams, each with
    its own context: the latency-bound kernels and launch gaps of one
    stream overlap the other's work. Answers are compared with the same
    jobs run one after another on one stream. The headline step stays
    sequential, so its per-kernel times are the kernels' own."""
    import torch
    from paper_2103_15217_amd import autotune
    dev = d_qx.device
    q = d_qx.numel()
    streams = [torch.cuda.Stream() for _ in range(2)]
    ctxs = []
    for st in streams:
        with torch.cuda.stream(st):
            c = et.Context()
            if not args.default_params:
                autotune.apply(c, "single")
            ctxs.append(c)
    outs = [torch.empty(q, dtype=torch.int32, device=dev) for _ in d_parent]
    mask = torch.empty(max((d_col.numel() + 31) // 32, 1), dtype=torch.int32, device=dev)
    jobs = [("tree", i) for i in range(len(d_parent))] + [("bridges", None)]

    def run(nstreams):
        main = torch.cuda.current_stream()
        for st in streams[:nstreams]:
            st.wait_stream(main)
        for j, (kind, i) in enumerate(jobs):
            st, c = streams[j % nstreams], ctxs[j % nstreams]
            with torch.cuda.stream(st):
                if kind == "tree":
                    t = et.et_tree_build(d_parent[i], ctx=c)
                    t.lca(d_qx, d_qy, out=outs[i])
                    t.free()
                else:
                    et.et_bridges(d_rp, d_col, mask=mask, ctx=c, count=False)
        for st in streams[:nstreams]:
            main.wait_stream(st)

    run(1)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs] + [mask.clone()]
    for _ in range(3):
        run(2)
    torch.cuda.synchronize()
    reps = max(5, min(args.steps, 20))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run(2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    same = all(torch.equal(a, b) for a, b in zip(ref, outs + [mask]))
    for c in ctxs:
        c.check()
        c.close()
    return {"streams": 2, "jobs_per_stream": [[f"{k}{'' if i is None else i}" for k, i in jobs[s::2]] for s in range(2)],
            "ms_per_step": ms, "sequential_ms_per_step": seq_ms, "elements_per_s": elements / (ms * 1e-3),
            "speedup_over_sequential": seq_ms / ms, "answers_equal": same}


def _small_first(b, limit):
    """The batch with its trees of at most ``limit`` nodes first (stable):
    a relabelling of tree ids, the order a batching host that sorts work by
    size class would hand over. Queries stay grouped by tree."""
    sizes = b["sizes"]
    order = np.argsort(sizes > limit, kind="stable")
    off = b["offsets"]
    qs = np.searchsorted(b["qtree"], np.arange(len(sizes) + 1))
    new_sizes = sizes[order]
    new_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    new_off[1:] = np.cumsum(new_sizes)
    qn = np.diff(qs)[order]
    parent = np.concatenate([b["parent"][off[t]:off[t + 1]] for t in order])
    qx = np.concatenate([b["qx"][qs[t]:qs[t + 1]] for t in order])
    qy = np.concatenate([b["qy"][qs[t]:qs[t + 1]] for t in order])
    qtree = np.repeat(np.arange(len(sizes), dtype=np.int32), qn)
    out = {"parent": parent, "offsets": new_off, "sizes": new_sizes, "qx": qx, "qy": qy, "qtree": qtree}
    if "grasp" in b:
        out["grasp"] = np.asarray(b["grasp"])[order]
    return out


def batched_vs_plain(args, et, ctx, d, dev):
    """4096 trees of log-uniform size in [2^6, 2^18] (grasp 1, 64 or n) with
    2^10..2^14 queries each: one batched build + one batched query launch
    versus building and querying every tree on its own, same stream."""
    import torch
    import gen
    t0 = time.time()
    b = _small_first(gen.forest_batch(args.batch_trees, seed=args.seed), et.FUSED_MAX_NODES)
    log(f"batched forest: {int(b['offsets'][-1])} nodes generated in {time.time() - t0:.1f}s")
    T = len(b["sizes"])
    d_parent = d(b["parent"])
    d_off = torch.from_numpy(b["offsets"].astype(np.int64)).to(dev)
    d_qt, d_qx, d_qy = d(b["qtree"]), d(b["qx"]), d(b["qy"])
    d_out = torch.empty_like(d_qx)
    off = b["offsets"]
    qs = np.searchsorted(b["qtree"], np.arange(T + 1))
    parts = [(d_parent[int(off[t]):int(off[t + 1])], d_qx[int(qs[t]):int(qs[t + 1])],
              d_qy[int(qs[t]):int(qs[t + 1])], d_out[int(qs[t]):int(qs[t + 1])]) for t in range(T)]
    stream = torch.cuda.current_stream()

    def batched():
        tr = et.et_tree_build_batch(d_parent, d_off, ctx=ctx)
        tr.lca_batch(d_qt, d_qx, d_qy, out=d_out)
        tr.free()

    def plain():
        for p, x, y, o in parts:
            tr = et.et_tree_build(p, ctx=ctx)
            tr.lca(x, y, out=o)
            tr.free()

    res = {}
    for name, fn, reps in (("batched", batched, 5), ("plain", plain, 1)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = {"gpu_ms": e0.elapsed_time(e1) / reps, "wall_ms": (time.perf_counter() - w0) * 1e3 / reps}
    res["breakdown"] = _kernel_breakdown(ctx, batched)
    g = et.BatchGraph(d_parent, d_off, d_qt, d_qx, d_qy, ctx=ctx)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    res["graph"] = {"gpu_ms": e0.elapsed_time(e1) / 5}
    graph_ok = bool(torch.equal(g.out, d_out))
    g.close()
    ctx.check()
    # the trees that fit one workgroup through the one-launch kernel, the
    # rest through the multi-kernel batch, in one HIP graph
    sctx = et.Context()
    if not args.default_params:
        from paper_2103_15217_amd import autotune
        autotune.apply(sctx, "batch")  # the shapes the batched path runs with
    sg = et.SplitBatchGraph(d_parent, off, qs, d_qx, d_qy, ctx=sctx)
    sg.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        sg.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    split_ms = e0.elapsed_time(e1) / 5
    split_ok = bool(torch.equal(sg.out, d_out))
    split_trees = sg.split
    sg.close()
    sctx.check()
    sctx.close()
    nodes, q = int(off[-1]), len(b["qx"])
    return {"trees": T, "nodes": nodes, "queries": q,
            "batched_ms": res["batched"]["gpu_ms"], "plain_ms": res["plain"]["gpu_ms"],
            "plain_wall_ms": res["plain"]["wall_ms"],
            "batched_nodes_per_s": nodes / (res["batched"]["gpu_ms"] * 1e-3),
            "plain_nodes_per_s": nodes / (res["plain"]["gpu_ms"] * 1e-3),
            "batched_queries_per_s": q / (res["batched"]["gpu_ms"] * 1e-3),
            "speedup": res["plain"]["gpu_ms"] / res["batched"]["gpu_ms"],
            "graph_ms": res["graph"]["gpu_ms"], "graph_matches_eager": graph_ok,
            "split_graph_ms": split_ms, "split_fused_trees": split_trees,
            "split_fused_nodes": int(off[split_trees]), "split_fused_queries": int(qs[split_trees]),
            "split_matches_batched": split_ok, **res["breakdown"]}


def _fused_tree_bytes(nodes, queries, trees):
    """Bytes the one-launch tree batch streams by design: the parents, the
    query pairs and their answers, the node and query offsets."""
    return 4 * nodes + 12 * queries + 16 * (trees + 1)


def small_batches(args, et, ctx, d, dev):
    """Batches of small trees (log-uniform sizes in [2^6, 2^12], grasp 1, 64
    or n, 2^10..2^14 queries per tree) with total size from 2^10 to 2^22
    nodes: the one-launch fused path (eager and replayed from a HIP graph)
    against the multi-kernel batched path (eager and from its HIP graph).
    The crossover is the smallest total at which the multi-kernel graph is
    faster; every fused answer is checked against the multi-kernel one."""
    import torch
    import gen
    rows = []
    stream = torch.cuda.current_stream()

    def time_fn(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for lg in range(10, 23, 2):
        target = 1 << lg
        # enough trees for the target total (mean size of log-uniform [2^6, 2^12] is about 950)
        T = max(1, int(target / 950 * 1.3) + 2)
        b = gen.forest_batch(T, seed=args.seed + lg, log2_min=6, log2_max=min(12, lg))
        keep = int(np.searchsorted(b["offsets"], target, side="right")) - 1
        keep = max(1, min(keep, T))
        qn = int(np.searchsorted(b["qtree"], keep))
        off = b["offsets"][:keep + 1]
        parent = b["parent"][:int(off[-1])]
        qt, qx, qy = b["qtree"][:qn], b["qx"][:qn], b["qy"][:qn]
        qoff = np.searchsorted(qt, np.arange(keep + 1)).astype(np.int64)
        d_parent, d_qt, d_qx, d_qy = d(parent), d(qt), d(qx), d(qy)
        d_off = torch.from_numpy(off.astype(np.int64)).to(dev)
        d_qoff = torch.from_numpy(qoff).to(dev)
        max_nodes = int(np.diff(off).max())
        d_out = torch.empty_like(d_qx)
        reps = 20 if lg <= 16 else 5

        # costliest trees first when they run 1024-lane workgroups, as FusedBatchGraph does
        d_order = torch.from_numpy(et.et.fused_order(off, qoff)).to(dev) if max_nodes > 1024 else None

        def fused():
            et.et_lca_batch_fused(d_parent, d_off, d_qoff, d_qx, d_qy, max_nodes, out=d_out, ctx=ctx, order=d_order)

        def multi():
            tr = et.et_tree_build_batch(d_parent, d_off, ctx=ctx)
            tr.lca_batch(d_qt, d_qx, d_qy)
            tr.free()

        fused_ms = time_fn(fused, reps)
        multi_ms = time_fn(multi, reps)
        fg = et.FusedBatchGraph(d_parent, d_off, d_qoff, d_qx, d_qy, max_nodes, ctx=ctx)
        fused_graph_ms = time_fn(fg.replay, reps)
        mctx = et.Context()
        mg = et.BatchGraph(d_parent, d_off, d_qt, d_qx, d_qy, ctx=mctx)
        multi_graph_ms = time_fn(mg.replay, reps)
        same = bool(torch.equal(fg.out, mg.out))
        fg.close()
        mg.close()
        mctx.close()
        ctx.check()
        nodes = int(off[-1])
        alg = _fused_tree_bytes(nodes, qn, keep)
        rows.append({"log2_target": lg, "trees": keep, "nodes": nodes, "queries": qn, "max_tree_nodes": max_nodes,
                     "fused_ms": fused_ms, "fused_graph_ms": fused_graph_ms, "multi_ms": multi_ms,
                     "multi_graph_ms": multi_graph_ms,
                     "fused_nodes_per_s": nodes / (fused_graph_ms * 1e-3),
                     "multi_nodes_per_s": nodes / (multi_graph_ms * 1e-3),
                     "fused_alg_bytes": alg, "fused_alg_GBps": alg / (fused_graph_ms * 1e-3) / 1e9,
                     "fused_frac_of_hbm": alg / (fused_graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "fused_over_multi_graph": multi_graph_ms / fused_graph_ms, "answers_equal": same})
    cross = next((r["nodes"] for r in rows if r["multi_graph_ms"] < r["fused_graph_ms"]), None)
    # tiny trees (2^4..2^10 nodes, 2^4..2^10 queries each): the 256-lane shape
    tiny = []
    for lg in (14, 18, 22):
        T = max(1, int((1 << lg) / 180 * 1.3) + 2)
        b = gen.forest_batch(T, seed=args.seed + 100 + lg, log2_min=4, log2_max=10, qlog2_min=4, qlog2_max=10)
        keep = max(1, min(int(np.searchsorted(b["offsets"], 1 << lg, side="right")) - 1, T))
        qn = int(np.searchsorted(b["qtree"], keep))
        off = b["offsets"][:keep + 1]
        d_parent, d_qt, d_qx, d_qy = d(b["parent"][:int(off[-1])]), d(b["qtree"][:qn]), d(b["qx"][:qn]), d(b["qy"][:qn])
        d_off = torch.from_numpy(off.astype(np.int64)).to(dev)
        d_qoff = torch.from_numpy(np.searchsorted(b["qtree"][:qn], np.arange(keep + 1)).astype(np.int64)).to(dev)
        max_nodes = int(np.diff(off).max())
        fg = et.FusedBatchGraph(d_parent, d_off, d_qoff, d_qx, d_qy, max_nodes, ctx=ctx)
        fused_graph_ms = time_fn(fg.replay, 10)
        mctx = et.Context()
        mg = et.BatchGraph(d_parent, d_off, d_qt, d_qx, d_qy, ctx=mctx)
        multi_graph_ms = time_fn(mg.replay, 10)
        same = bool(torch.equal(fg.out, mg.out))
        fg.close()
        mg.close()
        mctx.close()
        ctx.check()
        nodes = int(off[-1])
        alg = _fused_tree_bytes(nodes, qn, keep)
        tiny.append({"log2_target": lg, "trees": keep, "nodes": nodes, "queries": qn, "max_tree_nodes": max_nodes,
                     "fused_graph_ms": fused_graph_ms, "multi_graph_ms": multi_graph_ms,
                     "fused_trees_per_s": keep / (fused_graph_ms * 1e-3),
                     "fused_alg_bytes": alg, "fused_alg_GBps": alg / (fused_graph_ms * 1e-3) / 1e9,
                     "fused_frac_of_hbm": alg / (fused_graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "fused_over_multi_graph": multi_graph_ms / fused_graph_ms, "answers_equal": same})
    return {"sweep": rows, "crossover_nodes": cross, "tiny_trees": tiny}


def bridges_batched_vs_plain(args, et, ctx, d):
    """1024 graphs of log-uniform size in [2^6, 2^14] vertices (average
    degree 8, a few planted bridge chains each): one et_bridges_batch call
    versus one et_bridges call per graph, same stream; the per-graph masks
    of the two must agree."""
    import torch
    import gen
    t0 = time.time()
    rng = np.random.default_rng(args.seed + 17)
    graphs = []
    for t in range(args.batch_graphs):
        n = int(2 ** rng.uniform(6, 14))
        chains = max(1, n // 512)
        rp, col, _ = gen.planted_bridge_graph(n=n, m=4 * n, chains=chains, max_chain=max(2, n // (8 * chains)),
                                              seed=args.seed * 7919 + t)
        graphs.append((d(rp), d(col)))
    nv = sum(g[0].numel() - 1 for g in graphs)
    m = sum(g[1].numel() for g in graphs) // 2
    log(f"batched graphs: {len(graphs)} graphs, {nv} vertices, {m} edges in {time.time() - t0:.1f}s")
    # concatenated inputs made once, as a caller holding a batch would have them
    rows = torch.cat([g[0] for g in graphs])
    cols = torch.cat([g[1] for g in graphs])
    vs = np.concatenate([[0], np.cumsum([g[0].numel() - 1 for g in graphs])])
    ss = np.concatenate([[0], np.cumsum([g[1].numel() for g in graphs])])
    voff = torch.from_numpy(vs.astype(np.int64)).cuda()
    soff = torch.from_numpy(ss.astype(np.int64)).cuda()
    slots = np.diff(ss).tolist()
    mask_b = {}
    masks_p = [None] * len(graphs)

    def batched():
        mask_b["m"], mask_b["spans"], _ = et.et_bridges_batch(row_ptr=rows, col=cols, voff=voff, soff=soff,
                                                              slots=slots, ctx=ctx, counts=False)

    def plain():
        for i, (rp, col) in enumerate(graphs):
            masks_p[i], _ = et.et_bridges(rp, col, ctx=ctx, count=False)

    res = {}
    for name, fn, reps in (("batched", batched, 5), ("plain", plain, 1)):
        res[name] = _gpu_ms(fn, reps)
    ctx.check()
    ok = all(torch.equal(mask_b["m"][a:a + w], masks_p[i][:w]) for i, (a, w) in enumerate(mask_b["spans"]))
    res["breakdown"] = _kernel_breakdown(ctx, batched)
    g = et.BridgesBatchGraph(rows, cols, voff, soff, slots)
    res["graph"] = _gpu_ms(g.replay, 5)
    graph_ok = bool(torch.equal(g.mask, mask_b["m"]))
    g.ctx.check()
    g.close()
    return {"graphs": len(graphs), "vertices": nv, "edges": m, "batched_ms": res["batched"],
            "plain_ms": res["plain"], "graph_ms": res["graph"], "batched_edges_per_s": m / (res["batched"] * 1e-3),
            "plain_edges_per_s": m / (res["plain"] * 1e-3), "speedup": res["plain"] / res["batched"],
            "masks_equal": ok, "graph_matches_eager": graph_ok, **res["breakdown"]}


def small_graph_batches(args, et, ctx, d):
    """Batches of small graphs (log-uniform 2^3..2^10 vertices, average
    degree 4, distinct pairs: sparse, so rich in bridges) with 2^12 to 2^20
    vertices in all: the one-launch path (et_bridges_batch_fused) against
    the multi-kernel et_bridges_batch, both replayed from a HIP graph, masks
    and counts compared."""
    import torch
    import gen
    rows_out = []
    for lg in (12, 14, 16, 18, 20):
        rng = np.random.default_rng(args.seed + 31 + lg)
        graphs, nv = [], 0
        while nv < (1 << lg):
            n = int(2 ** rng.uniform(3, 10))
            rp, col = gen.random_multigraph(n, 2 * n, seed=int(rng.integers(1 << 30)), loops=False, multi=False)
            graphs.append((d(rp), d(col)))
            nv += n
        rows = torch.cat([g[0] for g in graphs])
        cols = torch.cat([g[1] for g in graphs])
        vs = [g[0].numel() - 1 for g in graphs]
        ss = [g[1].numel() for g in graphs]
        voff = torch.from_numpy(np.concatenate([[0], np.cumsum(vs)]).astype(np.int64)).cuda()
        soff = torch.from_numpy(np.concatenate([[0], np.cumsum(ss)]).astype(np.int64)).cuda()
        fg = et.BridgesFusedGraph(rows, cols, voff, soff, ss, vs, ctx=ctx)
        fused_ms = _gpu_ms(fg.replay, 10)
        mg = et.BridgesBatchGraph(rows, cols, voff, soff, ss)
        multi_ms = _gpu_ms(mg.replay, 10)
        total = sum((x + 31) // 32 for x in ss)
        same = bool(torch.equal(fg.mask[:total], mg.mask[:total]) and torch.equal(fg.counts, mg.counts))
        fg.close()
        mg.ctx.check()
        mg.close()
        ctx.check()
        m = sum(ss) // 2
        # streamed by design: row offsets, columns, the three offset arrays
        # read; one bit per slot and a count per graph written
        G = len(graphs)
        alg = 4 * (nv + G) + 4 * sum(ss) + 24 * (G + 1) + sum(ss) // 8 + 4 * G
        rows_out.append({"log2_target": lg, "graphs": len(graphs), "vertices": nv, "edges": m,
                         "fused_graph_ms": fused_ms, "multi_graph_ms": multi_ms,
                         "fused_alg_bytes": alg, "fused_alg_GBps": alg / (fused_ms * 1e-3) / 1e9,
                         "fused_frac_of_hbm": alg / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "fused_edges_per_s": m / (fused_ms * 1e-3), "multi_edges_per_s": m / (multi_ms * 1e-3),
                         "fused_over_multi_graph": multi_ms / fused_ms, "answers_equal": same})
    cross = next((r["vertices"] for r in rows_out if r["multi_graph_ms"] < r["fused_graph_ms"]), None)
    return {"sweep": rows_out, "crossover_vertices": cross}


def serving(args, dev):
    """Open-loop Poisson trace (70 % LCA jobs on trees of 2^10..2^22 nodes:
    with probability 1/2 one of the 32 most recently used trees, else a tree
    never seen before; 30 % bridge jobs on graphs of 2^12..2^20 vertices,
    average degree 8..32) replayed in real time through the plain FCFS
    per-job path and through the continuous-batching server, which admits
    jobs by the library's footprint figures within a device-memory budget."""
    from paper_2103_15217_amd import serve
    t0 = time.time()
    bases = serve.make_bases(seed=args.seed)
    graphs = serve.make_graphs(seed=args.seed)
    dinp = serve.DeviceInputs(bases, graphs, dev)
    budget = int(args.serve_budget_gib * (1 << 30))

    def replay(rate, seconds, seed):
        jobs, specs = serve.make_trace(bases, graphs, rate, seconds, seed=seed)
        dinp.prepare(jobs, specs)
        r = serve.compare(dinp, jobs, budget_bytes=budget, tuned=not args.default_params)
        r["trace_cold_fraction"] = serve.cold_fraction(jobs)
        r["distinct_trees"] = len(specs)
        dinp.release_trees()
        return r

    jobs_probe, _ = serve.make_trace(bases, graphs, args.serve_rate, args.serve_seconds, seed=args.seed)
    log(f"serving: {len(bases)} base trees, {len(graphs)} graphs, {len(jobs_probe)}-job trace "
        f"ready in {time.time() - t0:.1f}s")
    res = replay(args.serve_rate, args.serve_seconds, args.seed)
    res["rate_jobs_per_s"] = args.serve_rate
    res["trace_seconds"] = args.serve_seconds
    res["budget_bytes"] = budget
    res["p99_ratio_served_over_plain"] = res["served"]["p99_ms"] / res["plain"]["p99_ms"]
    s = res["served"]
    log(f"serving {args.serve_rate:.0f} jobs/s: plain p50/p99 {res['plain']['p50_ms']:.2f}/"
        f"{res['plain']['p99_ms']:.2f} ms, served {s['p50_ms']:.2f}/{s['p99_ms']:.2f} ms; cold "
        f"{s['cold_fraction']:.2f}, evictions {s['evictions']}, deferrals {s['deferrals']}")
    sweep = []
    for rate in [float(r) for r in args.serve_sweep.split(",") if r.strip()]:
        r = replay(rate, 2.0, args.seed + 1)
        log(f"serving sweep {rate:.0f} jobs/s: plain p99 {r['plain']['p99_ms']:.2f} ms, "
            f"served p99 {r['served']['p99_ms']:.2f} ms")
        sweep.append({"rate_jobs_per_s": rate, "jobs": r["served"]["jobs"],
                      **{f"{k}_{m}": r[k][m] for k in ("plain", "served")
                         for m in ("p50_ms", "p99_ms", "jobs_per_s", "wall_s")},
                      **{f"served_{m}": r["served"][m] for m in ("cold_fraction", "evictions", "deferrals")}})
    res["sweep"] = sweep
    return res


def kernel_roofline(kernel, avg_ms, launches, work, params):
    """Roofline figures of one kernel from its average launch time: the
    algorithmic bytes per launch over that time against 8 TB/s; the bytes
    the L2 actually requested from memory per launch (request-size counters,
    when a current summary exists) against 8 TB/s and against the measured
    read-only and copy stream rates; and its units per second against the
    measured random-access ceiling of its access pattern."""
    r = {"kernel": kernel, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
         "traffic": measured_traffic(kernel, params), "avg_launch_ms": avg_ms, "launches_per_step": launches}
    if kernel not in ALG_BYTES:
        return r
    bpu, unit, units = ALG_BYTES[kernel]
    upl = units(work)
    r.update({"achieved": bpu * upl / (avg_ms * 1e-3) / 1e9, "alg_bytes_per_unit": bpu, "unit_name": unit,
              "units_per_launch": upl})
    r["frac"] = r["achieved"] / HBM_PEAK_GBS
    if r["traffic"]:
        # what the memory side serves: a random read costs a whole 128-byte line,
        # a random store a 32-byte write (HBM and last-level-cache hits together)
        rate = r["traffic"] / (avg_ms * 1e-3) / 1e9
        r["traffic_GBps"] = rate
        r["traffic_frac"] = rate / HBM_PEAK_GBS
        r["traffic_over_alg"] = r["traffic"] / (bpu * upl)
        for name in ("read", "copy"):                      # measured stream rates (probe/ceiling.hip)
            ceil = probe_ceiling(name, 27, "GB_per_s")
            if ceil:
                r[f"{name}_stream_GBps"] = ceil
                r[f"traffic_frac_of_{name}_stream"] = rate / ceil
    # dependent walks against chase + store, the rest against independent gathers
    ceil = probe_ceiling("chase+w8" if kernel.startswith("k_walk1") else "gather")
    if ceil:
        r["units_per_s"] = upl / (avg_ms * 1e-3)
        r["random_ceiling_per_s"] = ceil
        r["random_frac"] = r["units_per_s"] / ceil
    return r


def probe_ceiling(name, log2n=25, field="elements_per_s"):
    """One figure of a probe of probe/ceiling.hip (copy, read, gather,
    scatter, dependent chase, chase with an 8-byte store) from its committed
    summary (profiles/random_access_ceiling.txt)."""
    path = os.path.join(ROOT, "profiles", "random_access_ceiling.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("{"):
            rec = json.loads(line)
            if rec.get("probe") == name and rec.get("log2n") == log2n:
                return rec[field]
    return None


def measured_traffic(kernel, params=None):
    """Bytes per launch of `kernel` that the L2 requested from memory (reads
    in 32-, 64- and 128-byte requests, writes in 32- and 64-byte requests,
    from rocprofv3's TCC_EA0 request counters), from the committed summary;
    None when none was taken, the kernel's source changed since, or it was
    taken with other launch parameters."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_2e24.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))["kernels"].get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
        return None
    if rec.get("launch_params") != params:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def cpu_baseline(parent, qx, qy, rp, col, ginfo, et, d, ctx, d_parent, d_qx, d_qy, d_rp, d_col):
    """The oracle (single-threaded C) on one sample: the grasp-n tree (tour,
    statistics, Inlabel tables, all 2^24 LCA queries) and the bridges graph.
    Also checks the GPU's outputs on that sample against it."""
    import oracle
    n, q = len(parent), len(qx)
    t0 = time.perf_counter()
    t = oracle.euler_tour(parent)
    oracle.sv_tables(parent, t["depth"], t["pre"], t["size"])
    lca_ref = oracle.lca_offline(parent, qx, qy)
    t1 = time.perf_counter()
    mask_ref, cnt_ref = oracle.bridges(rp, col)
    t2 = time.perf_counter()
    secs = t2 - t0
    elements = n + q + ginfo["m"]
    tree = et.et_tree_build(d_parent, ctx=ctx)
    got = tree.lca(d_qx, d_qy).cpu().numpy()
    tree.free()
    mask, cnt = et.et_bridges(d_rp, d_col, ctx=ctx)
    ctx.check()
    parity = {
        "lca_grasp_n_2e24": bool(np.array_equal(got, lca_ref)),
        "bridges_mask": bool(np.array_equal(mask.cpu().numpy().view(np.uint32)[: len(mask_ref)], mask_ref)),
        "bridges_count": int(cnt), "bridges_count_oracle": int(cnt_ref),
    }
    base = {"value": elements / secs, "unit": "elements/s (tree nodes + LCA queries + graph edges)",
            "cores": 1, "kind": "oracle", **host_cpu(),
            "sample": (f"grasp-n tree of {n} nodes (Euler tour, depth/preorder/size, Inlabel tables) + {q} "
                       f"offline LCA queries ({t1 - t0:.1f}s), and Tarjan bridges on the {len(rp) - 1}-vertex "
                       f"{ginfo['m']}-edge graph ({t2 - t1:.1f}s)"),
            "seconds": secs}
    return base, parity


def host_cpu():
    """The host's CPU model and logical CPU count (the oracle runs on one
    thread of it)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"host_cpu_model": model, "host_logical_cpus": os.cpu_count(), "host_cpus_usable": usable}


def protocol(args, et, ctx, d, grasps, first):
    """The paper's protocol (Section 3.3, Section 4.3): 5 instances (seeds)
    x 5 runs after one warm-up run, per component: the build of each grasp
    tree, its 2^log2n queries, and the bridges call. ``first`` holds the
    instance of ``args.seed`` already on the device."""
    import torch
    import gen
    n = 1 << args.log2n
    gn, gm = 1 << args.graph_log2n, 1 << args.graph_log2m
    chains = 4096 if args.graph_log2n >= 16 else 16
    runs = {f"build_{g}": [] for g in ("n", "1000", "1")}
    runs.update({f"lca_{g}": [] for g in ("n", "1000", "1")})
    runs["bridges"] = []
    stream = torch.cuda.current_stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        return r, (a, b)

    for k in range(args.protocol_seeds):
        seed = args.seed + k
        t0 = time.time()
        if k == 0:
            d_parent, d_qx, d_qy, d_rp, d_col = first
            m = None
        else:
            d_parent = [d(gen.random_tree(n, g, seed=seed + i)) for i, g in enumerate(grasps)]
            qx, qy = gen.random_queries(n, n, seed=seed)
            d_qx, d_qy = d(qx), d(qy)
            rp, col, _ = gen.planted_bridge_graph(n=gn, m=gm, chains=chains, max_chain=min(512, max(2, gn >> 13)),
                                                  seed=seed)
            d_rp, d_col = d(rp), d(col)
        out = torch.empty_like(d_qx)
        mask = torch.empty(max((d_col.numel() + 31) // 32, 1), dtype=torch.int32, device=d_col.device)
        pairs = {key: [] for key in runs}
        for r in range(1 + args.protocol_runs):
            for i, g in enumerate(("n", "1000", "1")):
                t, e = timed(lambda: et.et_tree_build(d_parent[i], ctx=ctx))
                _, e2 = timed(lambda: t.lca(d_qx, d_qy, out=out))
                t.free()
                if r:
                    pairs[f"build_{g}"].append(e)
                    pairs[f"lca_{g}"].append(e2)
            _, e = timed(lambda: et.et_bridges(d_rp, d_col, mask=mask, ctx=ctx, count=False))
            if r:
                pairs["bridges"].append(e)
        torch.cuda.synchronize()
        ctx.check()
        for key, evs in pairs.items():
            runs[key].extend(a.elapsed_time(b) for a, b in evs)
        log(f"protocol: instance {k} (seed {seed}) in {time.time() - t0:.1f}s")
    units = {"build": ("nodes/s", n), "lca": ("queries/s", n), "bridges": ("edges/s", None)}
    out = {"instances": args.protocol_seeds, "runs_per_instance": args.protocol_runs, "warmup_runs": 1}
    for key, ms in runs.items():
        ms = np.asarray(ms)
        unit, count = units[key.split("_")[0]]
        count = count if count is not None else gm
        rate = count / (ms * 1e-3)
        out[key] = {"ms_mean": float(ms.mean()), "ms_min": float(ms.min()), "ms_max": float(ms.max()),
                    "ms_rel_std": float(ms.std() / ms.mean()), "rate_mean": float(rate.mean()),
                    "rate_max": float(rate.max()), "unit": unit}
    return out


def end_children():
    """List and end any child process this run left (none is expected);
    names them on stderr so a leftover can be traced to its source."""
    try:
        import psutil
    except ImportError:
        return []
    kids = psutil.Process().children(recursive=True)
    for k in kids:
        try:
            log(f"ending leftover child process {k.pid}: {' '.join(k.cmdline())[:200]}")
            k.terminate()
        except psutil.Error:
            pass
    if kids:
        psutil.wait_procs(kids, timeout=5)
    return [k.pid for k in kids]


if __name__ == "__main__":
    main()
    end_children()
