"""The serving scheduler on the CPU: a mock backend with a simulated clock
runs nothing and checks that no tree batch is freed while queries on it are
in flight; byte figures come from the library's host-only footprint
functions. Covered: the trace's share of never-seen trees, admission under a
binding memory budget (evictions and deferrals happen, the budget is never
exceeded except by one oversized job running alone), pins, cancellation
before and after start, timeouts, and every job finishing exactly once."""
import math

import numpy as np

import paper_2103_15217_amd.et as et
from paper_2103_15217_amd import serve


def _bases(count=12, lo=10, hi=18, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(2 ** rng.uniform(lo, hi))
        p = np.empty(n, dtype=np.int32)
        p[0] = -1
        p[1:] = (rng.random(n - 1) * np.arange(1, n)).astype(np.int32)
        out.append(p)
    return out


def _graphs(count=6, lo=10, hi=16, seed=1):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(2 ** rng.uniform(lo, hi))
        nnz = 16 * n
        out.append((np.zeros(n + 1, dtype=np.int32), np.zeros(nnz, dtype=np.int32)))
    return out


def _run(jobs, budget, streams=4, max_batch=16, **cost):
    be = serve.MockBackend(streams=streams, **cost)
    sched = serve.Scheduler(be, budget, max_batch=max_batch, keep_results=True)
    st = sched.run(jobs)
    return sched, be, st


def test_trace_half_of_lca_jobs_need_a_new_tree():
    jobs, specs = serve.make_trace(_bases(), _graphs(), rate=2000, duration=4.0, seed=3)
    lca = [j for j in jobs if j.kind == "lca"]
    assert abs(len(lca) / len(jobs) - 0.7) < 0.03
    assert abs(serve.cold_fraction(jobs) - 0.5) < 0.03
    # every new tree is a new key with its own relabelling
    assert len(specs) == len({j.key for j in lca})
    assert len({(s.base, s.a, s.c) for s in specs}) == len(specs)


def test_relabelled_tree_is_the_same_shape(oracle_mod):
    base = _bases(1, 8, 9, seed=5)[0]
    n = base.shape[0]
    rng = np.random.default_rng(0)
    a, c = serve._coprime(rng, n), int(rng.integers(n))
    t = serve.relabel(base, a, c)
    pi = (a * np.arange(n, dtype=np.int64) + c) % n
    assert sorted(pi.tolist()) == list(range(n))
    assert np.array_equal(t[pi], np.where(base >= 0, pi[np.maximum(base, 0)], -1))
    # LCA commutes with the renaming
    x, y = rng.integers(0, n, 500).astype(np.int32), rng.integers(0, n, 500).astype(np.int32)
    want = pi[oracle_mod.lca_offline(base, x, y)]
    got = oracle_mod.lca_offline(t, pi[x].astype(np.int32), pi[y].astype(np.int32))
    assert np.array_equal(got, want)


def test_footprints_come_from_the_library():
    be = serve.MockBackend()
    for sizes in ([1000], [5000, 70000, 3], [1 << 20]):
        if len(sizes) == 1:
            assert be.tree_cost(sizes) == et.tree_footprint(sizes[0])
        else:
            assert be.tree_cost(sizes) == et.tree_footprint(sum(sizes), len(sizes))
    # tables: exactly the 256-byte pool blocks of succ, rank (8 B/node each),
    # pre, size (4 B), records (16 B), head table (8 B per label + 2) and the root scalar
    for n in (1, 2, 1000, 12345, 1 << 20):
        blocks = [8 * n, 8 * n, 4 * n, 4 * n, 16 * n, 8 * (n + 2), 64]
        assert et.tree_footprint(n)[0] == sum((b + 255) // 256 * 256 for b in blocks)
    prev = (0, 0)
    for k in range(1, 25):
        cur = et.tree_footprint(1 << k)
        assert cur[0] >= prev[0] and cur[1] >= prev[1]
        prev = cur
    assert et.bridges_footprint(1 << 20, 1 << 24) > et.bridges_footprint(1 << 16, 1 << 20) > 0
    assert et.bridges_footprint(1, 0) == 0


def test_binding_budget_evicts_and_defers_but_never_overshoots():
    bases = _bases(16, 12, 18)
    jobs, _ = serve.make_trace(bases, _graphs(), rate=2000, duration=2.0, seed=7)
    big = max(et.tree_footprint(b.shape[0]) for b in bases)
    budget = 3 * sum(big)
    sched, be, st = _run(jobs, budget, bridges_s=1e-3, build_s=3e-4)
    assert st["completed"] == len(jobs)
    assert all(sched.status[j.jid] == "done" for j in jobs)
    assert st["evictions"] > 0 and st["deferrals"] > 0
    assert st["over_budget"] == 0 and st["oversized"] == 0
    assert st["peak_used_bytes"] <= budget
    assert serve.cold_fraction(jobs) - 1e-9 <= st["cold_fraction"] <= 1.0   # evicted trees are built again
    # with room for everything nothing is evicted or deferred
    sched2, _, st2 = _run(jobs, 1 << 50, bridges_s=1e-3, build_s=3e-4)
    assert st2["evictions"] == 0 and st2["deferrals"] == 0
    # cold = first use, plus jobs that arrive while their tree's first build still runs
    assert serve.cold_fraction(jobs) - 1e-9 <= st2["cold_fraction"] < serve.cold_fraction(jobs) + 0.05


def test_pinned_batches_survive_long_queries():
    # slow queries keep batches pinned while new trees keep arriving
    jobs, _ = serve.make_trace(_bases(10, 12, 16), _graphs(), rate=4000, duration=0.5, seed=9, lca_frac=1.0)
    budget = 6 * sum(et.tree_footprint(1 << 16))
    sched, be, st = _run(jobs, budget, lca_s_per_q=2e-7)   # MockBackend.free raises on a pinned batch
    assert st["completed"] == len(jobs) and st["evictions"] > 0 and st["over_budget"] == 0


def test_oversized_job_runs_alone():
    bases = _bases(3, 16, 17)
    jobs, _ = serve.make_trace(bases, _graphs(), rate=500, duration=0.2, seed=2)
    budget = sum(et.tree_footprint(1 << 15)) // 2   # smaller than any tree's build
    sched, be, st = _run(jobs, budget)
    assert st["completed"] == len(jobs)
    assert st["oversized"] > 0 and st["over_budget"] == 0
    # launches never overlap: each starts after the previous one has finished
    starts = [e for e in be.log if e[0] in ("build", "lca", "bridges")]
    assert len(starts) >= len(jobs)


def test_cancellation_before_and_after_start():
    jobs, _ = serve.make_trace(_bases(), _graphs(), rate=3000, duration=0.3, seed=4)
    # a long queue: slow bridges on one stream
    for j in jobs[10:20]:
        j.cancel_at = j.arrival          # withdrawn at once: never starts
    running = jobs[3]
    running.cancel_at = running.arrival + 1e-7   # withdrawn while (or after) it runs
    sched, be, st = _run(jobs, 1 << 50, streams=1, bridges_s=2e-3, build_s=1e-3)
    launched = set()
    for kind, _, ids in be.log:
        if kind == "lca":
            launched.add(ids)
        elif kind == "bridges":
            launched.update(ids)
    for j in jobs[10:20]:
        assert sched.status[j.jid] == "cancelled" and j.jid not in sched.results
        assert j.jid not in launched
    assert sched.status[running.jid] in ("cancelled", "done")
    if sched.status[running.jid] == "cancelled":
        assert running.jid not in sched.results
    others = [j for j in jobs if j.jid not in {x.jid for x in jobs[10:20]} | {running.jid}]
    assert all(sched.status[j.jid] == "done" for j in others)
    assert st["cancelled"] >= 10


def test_timeouts_drop_jobs_that_cannot_start():
    # a budget that lets about one launch run at a time: jobs wait for memory past their deadlines
    bases = _bases()
    jobs, _ = serve.make_trace(bases, _graphs(), rate=5000, duration=0.2, seed=6, timeout=2e-3)
    budget = 2 * max(sum(et.tree_footprint(b.shape[0])) for b in bases)
    sched, be, st = _run(jobs, budget, streams=1, bridges_s=3e-3, build_s=2e-3)
    assert st["timeouts"] > 0
    starts = {}
    for kind, t, ids in be.log:
        for jid in (ids if isinstance(ids, tuple) and kind == "bridges" else (ids,) if kind == "lca" else ()):
            starts.setdefault(jid, t)
    for j in jobs:
        s = sched.status[j.jid]
        assert s in ("done", "timeout")
        if j.jid in starts:
            assert starts[j.jid] <= j.deadline + 1e-12   # nothing starts after its deadline
    assert st["completed"] + st["timeouts"] == len(jobs)


def test_every_job_finishes_once_under_pressure():
    jobs, _ = serve.make_trace(_bases(20, 10, 17), _graphs(), rate=20000, duration=0.2, seed=8)
    budget = 4 * sum(et.tree_footprint(1 << 17))
    sched, be, st = _run(jobs, budget, max_batch=5)
    assert sorted(sched.results) == [j.jid for j in jobs]
    assert st["over_budget"] == 0 and math.isfinite(st["p99_ms"])
