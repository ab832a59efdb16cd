"""Serving loop: LCA-query and bridge jobs of mixed sizes as they arrive.

Two executors replay the same open-loop arrival trace in real time:

* ``PlainExecutor``: first come, first served, one job at a time on one
  stream; an LCA job builds its tree, answers its queries and frees it.
* ``ServedExecutor``: continuous batching. Every pass of its loop admits the
  jobs that have arrived while earlier ones are still on the GPU, as far as
  a device-memory budget allows; the trees that admitted LCA jobs need and
  that are not resident are built together with one batched build
  (``et_tree_build_batch``) and stay resident for later jobs (least
  recently used batches are evicted when the budget is short); each job's
  queries and each bridge job are launched on one of several streams (one
  library context per stream), so jobs overlap on the device; a job is done
  when the event recorded after its last launch has completed.

Latency is arrival to completion as seen by the host loop. Results do not
depend on the executor; ``results`` holds every job's output for checking.
"""
import collections
import dataclasses
import time

import numpy as np
import torch

from . import autotune, et

# device bytes per unit used for admission (tables + build scratch)
TREE_BYTES_PER_NODE = 160
BRIDGE_BYTES_PER_SLOT = 48
QUERY_BYTES = 12


@dataclasses.dataclass
class Job:
    jid: int
    kind: str            # "lca" or "bridges"
    arrival: float       # seconds after the start of the trace
    item: int            # tree or graph index in the pool
    qx: object = None    # device int32 queries (LCA)
    qy: object = None
    nq: int = 0


def make_trace(pool, rate, duration, seed=0, lca_frac=0.7, reuse=0.5, qlog2=(10, 16)):
    """Poisson arrivals at ``rate`` jobs/s for ``duration`` s. 70 % LCA jobs
    on pool trees (a tree used before is picked again with probability
    ``reuse``), 30 % bridge jobs on pool graphs; queries per LCA job
    log-uniform in [2^qlog2[0], 2^qlog2[1]]."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5e]))
    t, jobs, used = 0.0, [], []
    ntrees, ngraphs = len(pool["trees"]), len(pool["graphs"])
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        jid = len(jobs)
        if rng.random() < lca_frac:
            if used and rng.random() < reuse:
                item = used[int(rng.integers(len(used)))]
            else:
                item = int(rng.integers(ntrees))
                used.append(item)
            n = pool["tree_sizes"][item]
            nq = int(2.0 ** rng.uniform(*qlog2))
            qx = rng.integers(0, n, size=nq, dtype=np.int64).astype(np.int32)
            qy = rng.integers(0, n, size=nq, dtype=np.int64).astype(np.int32)
            jobs.append(Job(jid, "lca", t, item, qx, qy, nq))
        else:
            jobs.append(Job(jid, "bridges", t, int(rng.integers(ngraphs))))
    return jobs


def upload_trace(jobs, dev):
    for j in jobs:
        if j.kind == "lca":
            j.qx = torch.from_numpy(j.qx).to(dev)
            j.qy = torch.from_numpy(j.qy).to(dev)
    torch.cuda.synchronize()


def make_pool(seed=0, trees=48, graphs=16, tree_log2=(10, 22), graph_log2=(12, 20), deg=(8, 32)):
    """Seeded pool: trees of log-uniform size with grasp from {1, 64, n};
    sparse random graphs (distinct pairs, average degree uniform in
    ``deg``) with a few planted pendant chains so that bridges exist."""
    import gen
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x9a]))
    pool = {"trees": [], "tree_sizes": [], "graphs": [], "graph_sizes": []}
    for t in range(trees):
        n = int(2.0 ** rng.uniform(*tree_log2))
        g = [1, 64, None][int(rng.integers(3))]
        pool["trees"].append(gen.random_tree(n, g, seed=int(seed) * 7919 + t))
        pool["tree_sizes"].append(n)
    for k in range(graphs):
        n = int(2.0 ** rng.uniform(*graph_log2))
        d = float(rng.uniform(*deg))
        chains = max(1, n // 1024)
        rp, col, info = gen.planted_bridge_graph(n=n, m=int(n * d / 2), chains=chains,
                                                 max_chain=min(64, max(2, n // (4 * chains))),
                                                 seed=int(seed) * 104729 + k)
        pool["graphs"].append((rp.astype(np.int32), col))
        pool["graph_sizes"].append((n, len(col)))
    return pool


def upload_pool(pool, dev):
    d = {"trees": [torch.from_numpy(p).to(dev) for p in pool["trees"]],
         "graphs": [(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev))
                    for rp, col in pool["graphs"]],
         "tree_sizes": pool["tree_sizes"], "graph_sizes": pool["graph_sizes"]}
    torch.cuda.synchronize()
    return d


def _stats(lat, wall, njobs):
    lat = np.sort(np.asarray(lat))
    return {"jobs": njobs, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat[-1] * 1e3), "jobs_per_s": njobs / wall, "wall_s": wall}


class PlainExecutor:
    """FCFS, one job at a time, nothing kept between jobs."""

    def __init__(self, dpool, keep_results=False, tuned=True):
        self.dpool = dpool
        self.ctx = et.Context()
        if tuned:
            autotune.apply(self.ctx, "single")   # one instance per call
        self.keep = keep_results
        self.results = {}

    def run_job(self, j):
        if j.kind == "lca":
            t = et.et_tree_build(self.dpool["trees"][j.item], ctx=self.ctx)
            out = t.lca(j.qx, j.qy)
            t.free()
        else:
            rp, col = self.dpool["graphs"][j.item]
            out, _ = et.et_bridges(rp, col, ctx=self.ctx, count=False)
        return out

    def run(self, jobs):
        lat = []
        t0 = time.perf_counter()
        for j in jobs:
            while time.perf_counter() - t0 < j.arrival:
                pass
            out = self.run_job(j)
            torch.cuda.current_stream().synchronize()
            lat.append(time.perf_counter() - t0 - j.arrival)
            if self.keep:
                self.results[j.jid] = out.cpu()
        wall = time.perf_counter() - t0
        self.ctx.check()
        return _stats(lat, wall, len(jobs))


class ServedExecutor:
    """Continuous batching with a resident-tree cache and memory admission."""

    def __init__(self, dpool, streams=4, budget_bytes=8 << 30, keep_results=False, max_batch=64,
                 bridge_batch=True, tuned=True):
        self.dpool = dpool
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.ctxs = []
        for st in self.streams:
            with torch.cuda.stream(st):
                self.ctxs.append(et.Context())
                if tuned:
                    autotune.apply(self.ctxs[-1], "batch")   # batched builds, queries and bridge calls
        self.build_ctx, self.build_stream = self.ctxs[0], self.streams[0]
        self.budget = budget_bytes
        self.keep = keep_results
        self.max_batch = max_batch
        self.bridge_batch = bridge_batch  # waiting bridge jobs go out as one et_bridges_batch call
        self.results = {}
        # resident batches: bid -> {"tree": Tree, "items": [...], "bytes": b, "ready": event, "pins": k}
        self.batches = collections.OrderedDict()
        self.where = {}       # tree item -> (bid, local index)
        self.resident = 0
        self.next_bid = 0
        self.rr = 0
        self.active = 0       # jobs launched and not yet retired

    # ---------------------------------------------------------------- memory
    def _evict_for(self, need):
        for bid in list(self.batches):
            if self.resident + need <= self.budget:
                return True
            b = self.batches[bid]
            if b["pins"] > 0:
                continue
            with torch.cuda.stream(self.build_stream):
                b["tree"].free()
            for it in b["items"]:
                self.where.pop(it, None)
            self.resident -= b["bytes"]
            del self.batches[bid]
        return self.resident + need <= self.budget

    def _admit(self, need):
        """Make room for ``need`` bytes by evicting idle resident batches; when
        even that is not enough, admit only if nothing else is on the device
        (so an oversized job still runs and the queue always drains)."""
        return self._evict_for(need) or self.active == 0

    def _build(self, items):
        """One batched build, on the build stream, of the longest prefix of
        ``items`` that fits the memory budget."""
        sizes = [self.dpool["tree_sizes"][i] for i in items]
        take, need = 0, 0
        while take < len(items) and self._evict_for(need + sizes[take] * TREE_BYTES_PER_NODE):
            need += sizes[take] * TREE_BYTES_PER_NODE
            take += 1
        if take == 0:
            if not self._admit(sizes[0] * TREE_BYTES_PER_NODE):
                return None
            take, need = 1, sizes[0] * TREE_BYTES_PER_NODE
        items, sizes = items[:take], sizes[:take]
        with torch.cuda.stream(self.build_stream):
            parts = [self.dpool["trees"][i] for i in items]
            parent = torch.cat(parts) if len(parts) > 1 else parts[0]
            offs = torch.tensor(np.concatenate([[0], np.cumsum(sizes)]), dtype=torch.int64,
                                device=parent.device)
            tree = et.et_tree_build_batch(parent, offs, ctx=self.build_ctx)
            ready = torch.cuda.Event()
            ready.record(self.build_stream)
        bid = self.next_bid
        self.next_bid += 1
        self.batches[bid] = {"tree": tree, "items": list(items), "bytes": need, "ready": ready, "pins": 0,
                             "keep": (parent, offs)}
        for k, it in enumerate(items):
            self.where[it] = (bid, k)
        self.resident += need
        return bid

    def _launch_bridges(self, bjobs, inflight):
        """All waiting bridge jobs that fit the memory budget in one batched
        call (each graph's result is its word-aligned slice of the batch
        mask); returns the jobs left for the next pass."""
        need, take = 0, 0
        for j in bjobs[: self.max_batch]:
            b = self.dpool["graph_sizes"][j.item][1] * BRIDGE_BYTES_PER_SLOT
            if not self._evict_for(need + b):
                break
            need += b
            take += 1
        if take == 0:
            if not self._admit(self.dpool["graph_sizes"][bjobs[0].item][1] * BRIDGE_BYTES_PER_SLOT):
                return bjobs
            take = 1
        batch, rest = bjobs[:take], bjobs[take:]
        st = self.streams[self.rr % len(self.streams)]
        ctx = self.ctxs[self.rr % len(self.ctxs)]
        self.rr += 1
        with torch.cuda.stream(st):
            mask, spans, _ = et.et_bridges_batch([self.dpool["graphs"][j.item] for j in batch], ctx=ctx,
                                                 counts=False)
            ev = torch.cuda.Event()
            ev.record(st)
        for j, (start, words) in zip(batch, spans):
            # a graph without slots gets the one zero word et_bridges returns for it
            out = mask[start:start + words] if words else torch.zeros(1, dtype=mask.dtype, device=mask.device)
            inflight.append((j, ev, None, out))
        self.active += len(batch)
        return rest

    # ---------------------------------------------------------------- loop
    def run(self, jobs):
        lat = {}
        t0 = time.perf_counter()
        pending = collections.deque(jobs)
        ready = collections.deque()
        inflight = []  # (job, event, bid or None, output)
        while pending or ready or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            # retire finished jobs
            still = []
            for j, ev, bid, out in inflight:
                if ev.query():
                    lat[j.jid] = time.perf_counter() - t0 - j.arrival
                    if bid is not None:
                        self.batches[bid]["pins"] -= 1
                        self.batches.move_to_end(bid)
                    if self.keep:
                        self.results[j.jid] = out.cpu()
                else:
                    still.append((j, ev, bid, out))
            inflight = still
            self.active = len(inflight)
            if not ready:
                if not inflight and pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 2e-4)))
                continue
            # admit: build every missing tree of the waiting LCA jobs in one batch
            missing = []
            for j in ready:
                if j.kind == "lca" and j.item not in self.where and j.item not in missing:
                    missing.append(j.item)
                    if len(missing) >= self.max_batch:
                        break
            if missing:
                self._build(missing)
            nxt = collections.deque()
            bjobs = []
            for j in ready:
                st = self.streams[self.rr % len(self.streams)]
                ctx = self.ctxs[self.rr % len(self.ctxs)]
                if j.kind == "lca":
                    loc = self.where.get(j.item)
                    if loc is None:
                        nxt.append(j)        # not built yet (memory or batch limit): next pass
                        continue
                    bid, k = loc
                    b = self.batches[bid]
                    self.rr += 1
                    with torch.cuda.stream(st):
                        st.wait_event(b["ready"])
                        qt = torch.full((j.nq,), k, dtype=torch.int32, device=j.qx.device)
                        out = b["tree"].lca_batch(qt, j.qx, j.qy)
                        ev = torch.cuda.Event()
                        ev.record(st)
                    b["pins"] += 1
                    self.batches.move_to_end(bid)
                    inflight.append((j, ev, bid, out))
                    self.active += 1
                elif self.bridge_batch:
                    bjobs.append(j)
                else:
                    n, nnz = self.dpool["graph_sizes"][j.item]
                    if not self._admit(nnz * BRIDGE_BYTES_PER_SLOT):
                        nxt.append(j)
                        continue
                    self.rr += 1
                    rp, col = self.dpool["graphs"][j.item]
                    with torch.cuda.stream(st):
                        out, _ = et.et_bridges(rp, col, ctx=ctx, count=False)
                        ev = torch.cuda.Event()
                        ev.record(st)
                    inflight.append((j, ev, None, out))
                    self.active += 1
            if bjobs:
                nxt.extend(self._launch_bridges(bjobs, inflight))
            ready = nxt
        wall = time.perf_counter() - t0
        torch.cuda.synchronize()
        for c in self.ctxs:
            c.check()
        return _stats([lat[j.jid] for j in jobs], wall, len(jobs))

    def close(self):
        torch.cuda.synchronize()
        for b in self.batches.values():
            b["tree"].free()
        self.batches.clear()
        self.where.clear()
        self.resident = 0


def compare(dpool, jobs, streams=4, budget_bytes=8 << 30, tuned=True):
    """Replay ``jobs`` through the plain and the served executor."""
    plain = PlainExecutor(dpool, tuned=tuned)
    p = plain.run(jobs)
    served = ServedExecutor(dpool, streams=streams, budget_bytes=budget_bytes, tuned=tuned)
    s = served.run(jobs)
    served.close()
    return {"plain": p, "served": s}


def main():
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="served vs plain on an open-loop Poisson trace")
    ap.add_argument("--rates", default="2000", help="comma-separated arrival rates (jobs/s)")
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--streams", type=int, default=4)
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    t0 = time.time()
    pool = make_pool(seed=a.seed)
    dpool = upload_pool(pool, dev)
    print(f"[serve] pool ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    for rate in [float(r) for r in a.rates.split(",")]:
        jobs = make_trace(pool, rate, a.duration, seed=a.seed)
        upload_trace(jobs, dev)
        res = compare(dpool, jobs, streams=a.streams)
        print(json.dumps({"rate": rate, **res}), flush=True)


if __name__ == "__main__":
    main()
