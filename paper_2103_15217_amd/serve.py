"""Serving loop: LCA-query and bridge jobs of mixed sizes as they arrive
(the online, batched query setting of Section 3.3, with the bridge problem
of Section 4 as a second job kind).

Trace. An open-loop Poisson stream of jobs. 70 % are LCA jobs: a tree and a
batch of query pairs; with probability ``reuse`` the tree is one that an
earlier job used (drawn from the ``hot`` most recently used trees), else it
is a tree never seen before. New trees are distinct labellings of a pool of
base shapes: tree k is base b_k relabelled by i -> (a_k i + c_k) mod n with
a_k coprime to n, so its tour, ranks and tables are its own and it has to be
built. 30 % are bridge jobs on a pool of sparse random graphs with planted
bridge chains.

Two executors replay a trace in real time:

* ``PlainExecutor``: first come, first served, one job at a time on one
  stream; an LCA job builds its tree, answers its queries and frees it.
* ``ServedExecutor``: continuous batching. A host ``Scheduler`` admits jobs
  while earlier ones are still on the device, as far as a device-memory
  budget allows. The bytes come from the library (``et.tree_footprint``,
  ``et.bridges_footprint``): resident trees hold their tables until evicted;
  a build holds its scratch and input copy until it completes; a query or
  bridge launch holds its buffers until it completes. Trees that waiting
  LCA jobs need and that are not resident are built together by one batched
  build and stay resident for later jobs; idle resident batches are evicted
  least recently used first when memory is short; a batch with queries in
  flight is pinned. A job that does not fit waits (a deferral), except that
  a job too large for the budget runs alone when nothing else is on the
  device, so the queue always drains. Jobs may be cancelled, and a job that
  is not started before its deadline times out.

The scheduler talks to a backend: ``GpuBackend`` runs the library on
several streams (builds on one; queries and bridge batches spread over all
of them); ``MockBackend`` runs nothing, advances a simulated clock by a cost
model and checks the memory invariants, so admission, eviction, pinning,
cancellation and timeouts are tested on the CPU.
"""
import collections
import dataclasses
import math
import time

import numpy as np

from . import et

# ------------------------------------------------------------------ trace


@dataclasses.dataclass
class Job:
    jid: int
    kind: str              # "lca" or "bridges"
    arrival: float         # seconds after the start of the trace
    key: int               # tree key (lca) or graph index (bridges)
    n: int = 0             # nodes of the tree / vertices of the graph
    nnz: int = 0           # CSR slots of the graph
    qx: object = None      # queries (host int32 arrays, device tensors after upload)
    qy: object = None
    nq: int = 0
    deadline: float = math.inf   # latest start time (seconds after the trace start)
    cancel_at: float = math.inf  # the client withdraws the job at this time


@dataclasses.dataclass
class TreeSpec:
    base: int
    n: int
    a: int      # relabel multiplier, coprime to n
    c: int      # relabel offset


def make_bases(seed=0, count=32, tree_log2=(10, 22)):
    """Base tree shapes: log-uniform sizes, grasp drawn from {1, 64, n}."""
    import gen
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x9a]))
    bases = []
    for b in range(count):
        n = int(2.0 ** rng.uniform(*tree_log2))
        g = [1, 64, None][int(rng.integers(3))]
        bases.append(gen.random_tree(n, g, seed=int(seed) * 7919 + b))
    return bases


def make_graphs(seed=0, count=16, graph_log2=(12, 20), deg=(8, 32)):
    """Sparse random graphs (distinct pairs, average degree uniform in
    ``deg``) with n/1024 planted pendant or bridging chains."""
    import gen
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x6a]))
    graphs = []
    for k in range(count):
        n = int(2.0 ** rng.uniform(*graph_log2))
        d = float(rng.uniform(*deg))
        chains = max(1, n // 1024)
        rp, col, _ = gen.planted_bridge_graph(n=n, m=int(n * d / 2), chains=chains,
                                              max_chain=min(64, max(2, n // (4 * chains))),
                                              seed=int(seed) * 104729 + k)
        graphs.append((rp.astype(np.int32), col))
    return graphs


def relabel(parent, a, c):
    """The tree ``parent`` with node i renamed (a i + c) mod n (host)."""
    n = parent.shape[0]
    pi = (a * np.arange(n, dtype=np.int64) + c) % n
    out = np.empty(n, dtype=np.int32)
    out[pi] = np.where(parent >= 0, (a * parent.astype(np.int64) + c) % n, -1)
    return out


def _coprime(rng, n):
    while True:
        a = int(rng.integers(1, max(n, 2)))
        if math.gcd(a, n) == 1:
            return a


def make_trace(bases, graphs, rate, duration, seed=0, lca_frac=0.7, reuse=0.5, hot=32, qlog2=(10, 16),
               timeout=None):
    """Poisson arrivals at ``rate`` jobs/s for ``duration`` s; returns
    (jobs, tree specs by key). ``timeout``: each job's deadline is its
    arrival plus this many seconds."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5e]))
    t, jobs, specs = 0.0, [], []
    recent = collections.OrderedDict()   # tree keys, most recently used last
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        jid = len(jobs)
        if rng.random() < lca_frac:
            if recent and rng.random() < reuse:
                keys = list(recent)[-hot:]
                key = keys[int(rng.integers(len(keys)))]
            else:
                key = len(specs)
                b = int(rng.integers(len(bases)))
                n = bases[b].shape[0]
                specs.append(TreeSpec(b, n, _coprime(rng, n), int(rng.integers(n))))
            recent[key] = True
            recent.move_to_end(key)
            n = specs[key].n
            nq = int(2.0 ** rng.uniform(*qlog2))
            qx = rng.integers(0, n, size=nq, dtype=np.int64).astype(np.int32)
            qy = rng.integers(0, n, size=nq, dtype=np.int64).astype(np.int32)
            jobs.append(Job(jid, "lca", t, key, n=n, qx=qx, qy=qy, nq=nq))
        else:
            g = int(rng.integers(len(graphs)))
            rp, col = graphs[g]
            jobs.append(Job(jid, "bridges", t, g, n=rp.shape[0] - 1, nnz=col.shape[0]))
        if timeout is not None:
            jobs[-1].deadline = t + timeout
    return jobs, specs


def cold_fraction(jobs):
    """Share of LCA jobs whose tree no earlier job used (a lower bound on the
    share that needs a build: evicted trees are built again)."""
    seen, cold, lca = set(), 0, 0
    for j in jobs:
        if j.kind == "lca":
            lca += 1
            cold += j.key not in seen
            seen.add(j.key)
    return cold / max(lca, 1)


# ------------------------------------------------------------------ device inputs

class DeviceInputs:
    """Base trees, graphs, every trace tree's parent array (relabelled on the
    device from its base) and every job's queries, resident before a replay."""

    def __init__(self, bases, graphs, dev):
        import torch
        self.dev = dev
        self.bases = [torch.from_numpy(np.ascontiguousarray(p)).to(dev) for p in bases]
        self.graphs = [(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)) for rp, col in graphs]
        self.graph_sizes = [(rp.shape[0] - 1, col.shape[0]) for rp, col in graphs]
        self.trees = {}

    def tree(self, spec):
        import torch
        p = self.bases[spec.base]
        n = spec.n
        i = torch.arange(n, dtype=torch.int64, device=self.dev)
        pi = (spec.a * i + spec.c) % n
        np_ = torch.where(p >= 0, (spec.a * p.long() + spec.c) % n, torch.full_like(i, -1))
        out = torch.empty(n, dtype=torch.int32, device=self.dev)
        out[pi] = np_.int()
        return out

    def prepare(self, jobs, specs):
        import torch
        for j in jobs:
            if j.kind == "lca":
                if j.key not in self.trees:
                    self.trees[j.key] = self.tree(specs[j.key])
                if not torch.is_tensor(j.qx):
                    j.qx = torch.from_numpy(j.qx).to(self.dev)
                    j.qy = torch.from_numpy(j.qy).to(self.dev)
        torch.cuda.synchronize()

    def release_trees(self):
        self.trees = {}


def _stats(lat, wall, njobs):
    lat = np.sort(np.asarray(lat)) if len(lat) else np.zeros(1)
    return {"jobs": njobs, "completed": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat[-1] * 1e3), "jobs_per_s": len(lat) / wall, "wall_s": wall}


# ------------------------------------------------------------------ plain path

class PlainExecutor:
    """FCFS, one job at a time, nothing kept between jobs."""

    def __init__(self, dinp, keep_results=False, tuned=True):
        from . import autotune
        self.dinp = dinp
        self.ctx = et.Context()
        self.tuned = tuned
        self.autotune = autotune
        self.keep = keep_results
        self.results = {}

    def run_job(self, j):
        if j.kind == "lca":
            if self.tuned:
                self.autotune.apply(self.ctx, "single", size=j.n)
            t = et.et_tree_build(self.dinp.trees[j.key], ctx=self.ctx)
            out = t.lca(j.qx, j.qy)
            t.free()
        else:
            rp, col = self.dinp.graphs[j.key]
            if self.tuned:
                self.autotune.apply(self.ctx, "single", size=j.n)
            out, _ = et.et_bridges(rp, col, ctx=self.ctx, count=False)
        return out

    def run(self, jobs):
        import torch
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


# ------------------------------------------------------------------ scheduler

class Scheduler:
    """Admission by device-memory footprint, resident-tree cache, batching.

    Bytes in use = tables of resident tree batches + reservations of work in
    flight. Invariant: in use <= budget, except while a single job too large
    for the budget runs with nothing else in flight."""

    def __init__(self, backend, budget_bytes, max_batch=64, keep_results=False):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.keep = keep_results
        self.results = {}
        self.status = {}                          # jid -> "done" | "timeout" | "cancelled"
        self.latency = {}
        self.batches = collections.OrderedDict()  # bid -> batch record (LRU order: least recent first)
        self.where = {}                           # tree key -> (bid, index in the batch)
        self.resident = 0                         # table bytes of resident batches
        self.reserved = 0                         # bytes of work in flight
        self.inflight = []                        # work records
        self.next_bid = 0
        self.stats = collections.Counter()
        self.peak_used = 0
        self.deferred_jobs = set()
        self.cold_jobs = set()
        if hasattr(backend, "sched"):
            backend.sched = self

    # -------------------------------------------------------------- memory
    def used(self):
        return self.resident + self.reserved

    def _note(self):
        """After every launch: track the peak and check the invariant (over
        the budget only while one launch runs alone)."""
        self.peak_used = max(self.peak_used, self.used())
        if self.used() > self.budget and len(self.inflight) > 1:
            self.stats["over_budget"] += 1

    def _evict_until(self, need):
        """Evict idle resident batches, least recently used first, until
        ``need`` more bytes fit; True if they fit."""
        for bid in list(self.batches):
            if self.used() + need <= self.budget:
                return True
            b = self.batches[bid]
            if b["pins"] > 0 or not b["built"]:
                continue
            self.be.free(b["handle"])
            for key in b["keys"]:
                self.where.pop(key, None)
            self.resident -= b["bytes"]
            del self.batches[bid]
            self.stats["evictions"] += 1
            self.stats["evicted_trees"] += len(b["keys"])
        return self.used() + need <= self.budget

    def _fits(self, need):
        return self._evict_until(need)

    def _room(self):
        """Bytes that could be made free: the budget left plus every idle
        resident batch (what eviction could release)."""
        idle = sum(b["bytes"] for b in self.batches.values() if b["pins"] == 0 and b["built"])
        return self.budget - self.used() + idle

    def _alone_ok(self):
        """An oversized job may run when nothing else is in flight."""
        return not self.inflight

    # -------------------------------------------------------------- launches
    def _launch_build(self, keys, sizes):
        table, scratch = self.be.tree_cost(sizes)
        handle, token, io = self.be.build(keys, sizes)
        bid = self.next_bid
        self.next_bid += 1
        self.batches[bid] = {"handle": handle, "keys": list(keys), "bytes": table, "pins": 0, "built": False}
        for k, key in enumerate(keys):
            self.where[key] = (bid, k)
        self.resident += table
        self.reserved += scratch + io
        self.inflight.append({"kind": "build", "token": token, "bytes": scratch + io, "bid": bid, "jobs": []})
        self.stats["builds"] += 1
        self.stats["trees_built"] += len(keys)
        self._note()
        return bid

    def _launch_lca(self, j):
        bid, k = self.where[j.key]
        b = self.batches[bid]
        io = self.be.lca_bytes(j)
        token, out = self.be.lca(b["handle"], k, j)
        b["pins"] += 1
        self.batches.move_to_end(bid)
        self.reserved += io
        self.inflight.append({"kind": "lca", "token": token, "bytes": io, "bid": bid, "jobs": [(j, out)]})
        self._note()

    def _launch_bridges(self, jobs, need):
        token, outs = self.be.bridges(jobs)
        self.reserved += need
        self.inflight.append({"kind": "bridges", "token": token, "bytes": need, "bid": None,
                              "jobs": list(zip(jobs, outs))})
        self._note()

    # -------------------------------------------------------------- one pass
    def _retire(self, now):
        still = []
        for w in self.inflight:
            if not self.be.done(w["token"]):
                still.append(w)
                continue
            self.reserved -= w["bytes"]
            if w["kind"] == "build":
                self.batches[w["bid"]]["built"] = True
            if w["kind"] == "lca":
                self.batches[w["bid"]]["pins"] -= 1
            t = self.be.now()
            for j, out in w["jobs"]:
                if self.status.get(j.jid) == "cancelled":
                    continue
                self.status[j.jid] = "done"
                self.latency[j.jid] = t - j.arrival
                if self.keep:
                    self.results[j.jid] = self.be.fetch(out)
        self.inflight = still

    def _drop(self, ready, now):
        keep = collections.deque()
        for j in ready:
            if now >= j.cancel_at:
                self.status[j.jid] = "cancelled"
                self.stats["cancelled"] += 1
            elif now > j.deadline:
                self.status[j.jid] = "timeout"
                self.stats["timeouts"] += 1
            else:
                keep.append(j)
        # a job withdrawn while running: its result is discarded
        for w in self.inflight:
            for j, _ in w["jobs"]:
                if now >= j.cancel_at and self.status.get(j.jid) is None:
                    self.status[j.jid] = "cancelled"
                    self.stats["cancelled"] += 1
        return keep

    def _admit(self, ready):
        nxt = collections.deque()
        # 1. trees that waiting LCA jobs need and that are not resident: one batched build
        missing, sizes = [], []
        for j in ready:
            if j.kind == "lca" and j.key not in self.where and j.key not in missing:
                missing.append(j.key)
                sizes.append(j.n)
                if len(missing) >= self.max_batch:
                    break
        short = set()     # trees that could not be built for lack of memory
        if missing:
            room, take = self._room(), len(missing)

            def need(k):
                table, scratch = self.be.tree_cost(sizes[:k])
                return table + scratch + self.be.build_io_bytes(sizes[:k])

            while take > 0 and need(take) > room:
                take -= 1
            if take > 0 and not self._fits(need(take)):
                take = 0
            if take == 0 and self._alone_ok():
                take = 1
                self.stats["oversized"] += 1
            if take > 0:
                self._launch_build(missing[:take], sizes[:take])
            short = set(missing[take:])
        # 2. LCA jobs on resident trees (ready or being built) and bridge jobs
        bjobs = []
        for j in ready:
            if j.kind == "lca":
                if j.key not in self.where:
                    if j.key in short:
                        self.deferred_jobs.add(j.jid)
                        self.stats["deferrals"] += 1
                    nxt.append(j)
                    continue
                bid = self.where[j.key][0]
                if not self.batches[bid]["built"] or j.key in missing:
                    self.cold_jobs.add(j.jid)
                need = self.be.lca_bytes(j)
                self.batches[bid]["pins"] += 1  # no eviction of this batch while making room
                ok = self._fits(need) or self._alone_ok()
                self.batches[bid]["pins"] -= 1
                if not ok:
                    self.deferred_jobs.add(j.jid)
                    self.stats["deferrals"] += 1
                    nxt.append(j)
                    continue
                self._launch_lca(j)
            else:
                bjobs.append(j)
        # 3. waiting bridge jobs: the longest prefix that fits, as one batch
        if bjobs:
            room, take = self._room(), min(len(bjobs), self.max_batch)
            while take > 0 and self.be.bridges_bytes(bjobs[:take]) > room:
                take -= 1
            if take > 0 and not self._fits(self.be.bridges_bytes(bjobs[:take])):
                take = 0
            if take == 0 and self._alone_ok():
                take = 1
                self.stats["oversized"] += 1
            if take > 0:
                self._launch_bridges(bjobs[:take], self.be.bridges_bytes(bjobs[:take]))
            for k, j in enumerate(bjobs[take:]):
                if take + k < self.max_batch:   # past the batch limit it waits for its turn, not for memory
                    self.deferred_jobs.add(j.jid)
                    self.stats["deferrals"] += 1
                nxt.append(j)
        return nxt

    def run(self, jobs):
        jobs = sorted(jobs, key=lambda j: j.arrival)
        pending = collections.deque(jobs)
        ready = collections.deque()
        self.be.start()
        while True:
            now = self.be.now()
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            self._retire(now)
            ready = self._drop(ready, now)
            if not (pending or ready or self.inflight):
                break
            if ready:
                before = (len(ready), len(self.inflight))
                ready = self._admit(ready)
                if (len(ready), len(self.inflight)) != before:
                    continue
            # nothing could start: wait for an arrival, a completion or a deadline
            nxt = pending[0].arrival if pending else math.inf
            for j in ready:
                nxt = min(nxt, j.cancel_at, j.deadline)
            self.be.wait(nxt)
        wall = self.be.now()
        self.be.finish()
        done = [j for j in jobs if self.status.get(j.jid) == "done"]
        lca = [j for j in jobs if j.kind == "lca" and self.status.get(j.jid) == "done"]
        st = _stats([self.latency[j.jid] for j in done], wall, len(jobs))
        st.update({
            "cold_fraction": len([j for j in lca if j.jid in self.cold_jobs]) / max(len(lca), 1),
            "builds": self.stats["builds"], "trees_built": self.stats["trees_built"],
            "evictions": self.stats["evictions"], "evicted_trees": self.stats["evicted_trees"],
            "deferrals": self.stats["deferrals"], "deferred_jobs": len(self.deferred_jobs),
            "oversized": self.stats["oversized"], "timeouts": self.stats["timeouts"],
            "cancelled": self.stats["cancelled"], "budget_bytes": self.budget, "peak_used_bytes": self.peak_used,
            "over_budget": self.stats["over_budget"],
        })
        st.update(self.be.report())
        return st

    def close(self):
        for b in self.batches.values():
            self.be.free(b["handle"])
        self.batches.clear()
        self.where.clear()
        self.resident = 0


# ------------------------------------------------------------------ backends

class GpuBackend:
    """The library on several HIP streams (one context per stream). Trees are
    built on stream 0 with context 0; their queries run on any stream after
    the build's event (LCA queries take no scratch and only read the tables);
    bridge batches run on the stream of their own context. A batch of one
    tree or one graph goes through the single-instance calls (et_tree_build,
    et_lca, et_bridges), which skip the batch's concatenation and splitting."""

    def __init__(self, dinp, streams=4, tuned=True):
        import torch
        from . import autotune
        self.torch = torch
        self.dinp = dinp
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.ctxs = []
        for st in self.streams:
            with torch.cuda.stream(st):
                self.ctxs.append(et.Context())
        self.tuned = tuned
        self.autotune = autotune
        self.rr = 0
        self.t0 = None
        self.sched = None       # the scheduler driving this backend (set by it)
        self.calls = collections.Counter()   # library calls made, by kind

    def start(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def wait(self, until):
        # spin rather than sleep (a sleep of the OS's granularity would add its
        # length to the latency of every job that finishes meanwhile), and
        # return as soon as a launch in flight completes, at an arrival or a
        # deadline, or after 50 us at the latest
        end = self.t0 + min(until, self.now() + 5e-5)
        events = [w["token"][0] for w in self.sched.inflight] if self.sched else []
        while time.perf_counter() < end:
            if any(e.query() for e in events):
                return

    def finish(self):
        self.torch.cuda.synchronize()
        for c in self.ctxs:
            c.check()

    def report(self):
        pools = [c.pool_stats() for c in self.ctxs]
        return {"pool_held_bytes": sum(p["held"] for p in pools), "pool_peak_live_bytes": max(p["peak_live"] for p in pools),
                "calls": dict(self.calls)}

    # sizes, from the library
    def tree_cost(self, sizes):
        if len(sizes) == 1:
            return et.tree_footprint(sizes[0], 0, ctx=self.ctxs[0])
        return et.tree_footprint(sum(sizes), len(sizes), ctx=self.ctxs[0])

    def build_io_bytes(self, sizes):
        return 4 * sum(sizes) + 8 * (len(sizes) + 1)   # the concatenated parent array and offsets

    @staticmethod
    def lca_bytes(j):
        return 16 * j.nq    # tree ids and answers beside the resident query pairs

    def bridges_bytes(self, jobs):
        n = sum(j.n for j in jobs)
        nnz = sum(j.nnz for j in jobs)
        words = sum((j.nnz + 31) // 32 for j in jobs)
        if len(jobs) == 1:   # et_bridges on the resident CSR: its scratch and the mask
            return et.bridges_footprint(n, nnz, 0, ctx=self.ctxs[0]) + 4 * max(words, 1)
        scratch = et.bridges_footprint(n, nnz, len(jobs), ctx=self.ctxs[0])
        return scratch + 4 * (n + len(jobs) + nnz + words) + 16 * (len(jobs) + 1)

    # launches
    def build(self, keys, sizes):
        torch = self.torch
        st, ctx = self.streams[0], self.ctxs[0]
        parts = [self.dinp.trees[k] for k in keys]
        with torch.cuda.stream(st):
            if len(parts) == 1:
                if self.tuned:
                    self.autotune.apply(ctx, "single", size=sizes[0])
                parent, keep = parts[0], ()
                tree = et.et_tree_build(parent, ctx=ctx)
                self.calls["et_tree_build"] += 1
            else:
                if self.tuned:
                    self.autotune.apply(ctx, "batch", size=sum(sizes))
                parent = torch.cat(parts)
                # offsets go up from pinned memory without waiting for the stream
                h_offs = torch.tensor(np.concatenate([[0], np.cumsum(sizes)]), dtype=torch.int64).pin_memory()
                offs = h_offs.to(parent.device, non_blocking=True)
                keep = (offs, h_offs)
                tree = et.et_tree_build_batch(parent, offs, ctx=ctx)
                self.calls["et_tree_build_batch"] += 1
            ev = torch.cuda.Event()
            ev.record(st)
        # the inputs stay referenced until the build has completed
        return (tree, ev), (ev, (parent,) + keep), self.build_io_bytes(sizes)

    def lca(self, handle, k, j):
        torch = self.torch
        tree, ready = handle
        st = self.streams[self.rr % len(self.streams)]
        self.rr += 1
        with torch.cuda.stream(st):
            st.wait_event(ready)
            if tree.batch:
                qt = torch.full((j.nq,), k, dtype=torch.int32, device=j.qx.device)
                out = tree.lca_batch(qt, j.qx, j.qy)
            else:
                qt = None
                out = tree.lca(j.qx, j.qy)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, qt), out

    def bridges(self, jobs):
        torch = self.torch
        i = self.rr % len(self.streams)
        self.rr += 1
        st, ctx = self.streams[i], self.ctxs[i]
        with torch.cuda.stream(st):
            if len(jobs) == 1:
                if self.tuned:
                    self.autotune.apply(ctx, "single", size=jobs[0].n)
                mask, _ = et.et_bridges(*self.dinp.graphs[jobs[0].key], ctx=ctx, count=False)
                spans = [(0, mask.numel())]
                self.calls["et_bridges"] += 1
            else:
                if self.tuned:
                    self.autotune.apply(ctx, "batch", size=sum(j.n for j in jobs))
                mask, spans, _ = et.et_bridges_batch([self.dinp.graphs[j.key] for j in jobs], ctx=ctx,
                                                     counts=False)
                self.calls["et_bridges_batch"] += 1
            ev = torch.cuda.Event()
            ev.record(st)
        outs = []
        for start, words in spans:
            # a graph without slots gets the one zero word et_bridges returns for it
            outs.append(mask[start:start + words] if words else torch.zeros(1, dtype=mask.dtype, device=mask.device))
        return (ev, mask), outs

    def done(self, token):
        return token[0].query()

    def free(self, handle):
        tree, ready = handle
        # the tree's queries have all completed (its pins are zero); freeing
        # on the build stream orders the reuse of its blocks behind them
        with self.torch.cuda.stream(self.streams[0]):
            tree.free()

    def fetch(self, out):
        return out.cpu()


class MockBackend:
    """No device: a simulated clock and a cost model. Every launch occupies
    one of ``streams`` simulated queues for its modelled time; the clock
    jumps to the next event when the scheduler waits. Byte figures come from
    the library's footprint functions (host-only calls); freeing a batch that
    has queries in flight, or querying a freed one, raises."""

    def __init__(self, streams=4, build_s_per_node=2e-10, build_s=60e-6, lca_s_per_q=4e-11,
                 lca_s=8e-6, bridges_s_per_slot=2e-10, bridges_s=120e-6):
        self.streams = [0.0] * streams
        self.rr = 0
        self.t = 0.0
        self.cost = dict(bn=build_s_per_node, b0=build_s, q=lca_s_per_q, q0=lca_s, e=bridges_s_per_slot,
                         e0=bridges_s)
        self.live = {}          # handle id -> table bytes of a resident batch
        self.pinned = collections.Counter()
        self.next_handle = 0
        self.sched = None       # the scheduler driving this backend (set by it)
        self.log = []

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait(self, until):
        nxt = [w["token"] for w in self.sched.inflight] if self.sched else []
        nxt = [x for x in nxt if x > self.t]
        target = min([until] + nxt)
        if math.isinf(target):
            raise RuntimeError("scheduler waits with nothing pending")
        self.t = max(self.t + 1e-9, target)   # always forward: a deadline reached now expires

    def finish(self):
        pass

    def report(self):
        return {}

    def tree_cost(self, sizes):
        if len(sizes) == 1:
            return et.tree_footprint(sizes[0], 0)
        return et.tree_footprint(sum(sizes), len(sizes))

    @staticmethod
    def build_io_bytes(sizes):
        return 4 * sum(sizes) + 8 * (len(sizes) + 1)

    @staticmethod
    def lca_bytes(j):
        return 16 * j.nq

    def bridges_bytes(self, jobs):
        n = sum(j.n for j in jobs)
        nnz = sum(j.nnz for j in jobs)
        words = sum((j.nnz + 31) // 32 for j in jobs)
        return et.bridges_footprint(n, nnz, len(jobs)) + 4 * (n + len(jobs) + nnz + words) + 16 * (len(jobs) + 1)

    def _queue(self, dur, stream=None):
        i = self.rr % len(self.streams) if stream is None else stream
        if stream is None:
            self.rr += 1
        start = max(self.t, self.streams[i])
        self.streams[i] = start + dur
        return start + dur

    def build(self, keys, sizes):
        n = sum(sizes)
        h = self.next_handle
        self.next_handle += 1
        self.live[h] = keys
        done = self._queue(self.cost["b0"] + self.cost["bn"] * n, stream=0)
        self.log.append(("build", self.t, tuple(keys)))
        return h, done, 0

    def lca(self, handle, k, j):
        if handle not in self.live:
            raise AssertionError("query on a freed tree batch")
        self.pinned[handle] += 1
        done = self._queue(self.cost["q0"] + self.cost["q"] * j.nq)
        self.log.append(("lca", self.t, j.jid))
        return done, ("lca", handle, j.jid, done)

    def bridges(self, jobs):
        nnz = sum(j.nnz for j in jobs)
        done = self._queue(self.cost["e0"] + self.cost["e"] * nnz)
        self.log.append(("bridges", self.t, tuple(j.jid for j in jobs)))
        return done, [("bridges", None, j.jid, done) for j in jobs]

    def done(self, token):
        return token <= self.t

    def free(self, handle):
        # every query on the batch must have completed in simulated time
        s = self.sched
        if s is not None:
            for w in s.inflight:
                for j, out in w["jobs"]:
                    if w["kind"] == "lca" and out[1] == handle:
                        raise AssertionError("evicted a batch with queries in flight")
        self.live.pop(handle, None)
        self.log.append(("free", self.t, handle))

    def fetch(self, out):
        return out


class ServedExecutor:
    """Continuous batching on the GPU: the scheduler over a GpuBackend."""

    def __init__(self, dinp, streams=4, budget_bytes=8 << 30, keep_results=False, max_batch=64, tuned=True):
        self.backend = GpuBackend(dinp, streams=streams, tuned=tuned)
        self.sched = Scheduler(self.backend, budget_bytes, max_batch=max_batch, keep_results=keep_results)

    @property
    def results(self):
        return self.sched.results

    def run(self, jobs):
        return self.sched.run(jobs)

    def close(self):
        import torch
        torch.cuda.synchronize()
        self.sched.close()


def compare(dinp, jobs, streams=4, budget_bytes=8 << 30, tuned=True):
    """Replay ``jobs`` through the plain and the served executor."""
    plain = PlainExecutor(dinp, tuned=tuned)
    p = plain.run(jobs)
    served = ServedExecutor(dinp, streams=streams, budget_bytes=budget_bytes, tuned=tuned)
    s = served.run(jobs)
    served.close()
    return {"plain": p, "served": s}
