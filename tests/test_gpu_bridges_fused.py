"""GPU parity of the one-launch graph batch (et_bridges_batch_fused): each
graph's mask words and bridge count must equal the Tarjan DFS oracle's for
that graph alone, bit for bit, and the multi-kernel et_bridges_batch on the
same batch."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2103_15217_amd as et
    assert torch.cuda.is_available()
    return et


def _dev(a, dtype=np.int32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _empty_graph(n):
    return np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32)


def run_fused(lib, graphs, ctx=None, **bounds):
    dg = [(_dev(rp), _dev(col)) for rp, col in graphs]
    mask, spans, counts = lib.et_bridges_batch_fused(dg, ctx=ctx, **bounds)
    return mask.cpu().numpy().view(np.uint32), spans, counts.cpu().numpy()


def check(lib, oracle_mod, graphs, ctx=None, **bounds):
    ctx = ctx or lib.default_context()
    mask, spans, counts = run_fused(lib, graphs, ctx=ctx, **bounds)
    ctx.check()
    bad = []
    for t, ((rp, col), (start, words)) in enumerate(zip(graphs, spans)):
        ref_mask, ref_cnt = oracle_mod.bridges(rp, col)
        if words != len(ref_mask) or not np.array_equal(mask[start:start + words], ref_mask) or counts[t] != ref_cnt:
            bad.append(t)
    assert not bad, bad[:10]
    return mask, spans, counts


def test_tiny_multigraphs(lib, oracle_mod):
    rng = np.random.default_rng(78)
    graphs = []
    for seed in range(400):
        kind = int(rng.integers(10))
        if kind == 0:
            graphs.append(_empty_graph(0))                       # no vertex at all
        elif kind == 1:
            graphs.append(_empty_graph(int(rng.integers(1, 5))))  # vertices, no edge
        else:
            n = int(rng.integers(1, 30))
            graphs.append(gen.random_multigraph(n, int(rng.integers(0, 45)), seed=seed, loops=True, multi=True))
    check(lib, oracle_mod, graphs)


@pytest.mark.parametrize("T,seed", [(1, 0), (17, 1), (300, 2)])
def test_planted_and_random_graphs(lib, oracle_mod, T, seed):
    rng = np.random.default_rng(seed)
    graphs = []
    for t in range(T):
        n = int(2 ** rng.uniform(3, 10))
        deg = int(rng.integers(2, 8))
        if rng.random() < 0.5:
            graphs.append(gen.random_multigraph(n, n * deg // 2, seed=1000 * seed + t, loops=True, multi=True))
        else:
            chains = max(1, n // 64)
            rp, col, _ = gen.planted_bridge_graph(n=n, m=n * deg // 2, chains=chains,
                                                  max_chain=max(2, n // (8 * chains)), seed=1000 * seed + t)
            graphs.append((rp, col))
    check(lib, oracle_mod, graphs)


def test_special_graphs_at_the_limits(lib, oracle_mod):
    graphs = [gen.tree_graph(gen.path_tree(1024)),            # every edge a bridge, the deepest tour
              gen.tree_graph(gen.path_tree(1024, seed=4)),
              gen.tree_graph(gen.star_tree(1024, root=511)),  # one row of 1023 slots
              gen.tree_graph(gen.random_tree(1024, None, seed=5)),
              gen.cycle_graph(1024),                           # no bridge
              gen.complete_graph(64),                          # 4032 slots, no bridge
              gen.random_multigraph(1024, 4096, seed=6, loops=True, multi=True),   # 8192 slots
              gen.planted_bridge_graph(n=1024, m=4000, chains=16, max_chain=8, seed=7)[:2]]
    graphs = [(rp, col) for rp, col in graphs]
    assert max(len(c) for _, c in graphs) <= 8192
    check(lib, oracle_mod, graphs, max_vertices=1024, max_slots=8192)


def test_equals_multi_kernel_batch(lib):
    rng = np.random.default_rng(9)
    graphs = []
    for t in range(500):
        n = int(2 ** rng.uniform(3, 10))
        rp, col, _ = gen.planted_bridge_graph(n=n, m=n * 3, chains=max(1, n // 128), max_chain=4, seed=t)
        graphs.append((rp, col))
    ctx = lib.default_context()
    mask, spans, counts = run_fused(lib, graphs, ctx=ctx)
    m2, s2, c2 = lib.et_bridges_batch([(_dev(rp), _dev(col)) for rp, col in graphs], ctx=ctx)
    ctx.check()
    assert spans == s2
    assert np.array_equal(mask[:sum(w for _, w in spans)], m2.cpu().numpy().view(np.uint32)[:sum(w for _, w in s2)])
    assert np.array_equal(counts, c2.cpu().numpy())


def test_graph_replays(lib):
    """The work counter resets itself after every launch: a captured call
    replayed with eager calls in between gives the eager answer each time."""
    import torch
    rng = np.random.default_rng(10)
    graphs = [gen.random_multigraph(int(rng.integers(2, 400)), int(rng.integers(1, 900)), seed=t) for t in range(300)]
    small = [gen.cycle_graph(5), gen.tree_graph(gen.random_tree(9, None, seed=1))]
    ctx = lib.Context()
    try:
        want, spans, want_c = run_fused(lib, graphs, ctx=ctx)
        want_small = run_fused(lib, small, ctx=ctx)[0]
        dg = [(_dev(rp), _dev(col)) for rp, col in graphs]
        rp = torch.cat([g[0] for g in dg])
        col = torch.cat([g[1] for g in dg])
        vs = [len(r) - 1 for r, _ in graphs]
        ss = [len(c) for _, c in graphs]
        voff = _dev(np.concatenate([[0], np.cumsum(vs)]), np.int64)
        soff = _dev(np.concatenate([[0], np.cumsum(ss)]), np.int64)
        mask = torch.zeros(len(want), dtype=torch.int32, device="cuda")
        moff = _dev(np.concatenate([[0], np.cumsum([(x + 31) // 32 for x in ss])]), np.int64)
        kw = dict(row_ptr=rp, col=col, voff=voff, soff=soff, slots=ss, vertices=vs, moff=moff, mask=mask, ctx=ctx)
        out = {}
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            lib.et_bridges_batch_fused(**kw)   # warm-up outside capture (moff upload, attributes)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out["mask"], _, out["counts"] = lib.et_bridges_batch_fused(**kw)
        for _ in range(3):
            mask.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(mask.cpu().numpy().view(np.uint32), want)
            assert np.array_equal(out["counts"].cpu().numpy(), want_c)
            assert np.array_equal(run_fused(lib, small, ctx=ctx)[0], want_small)
        ctx.check()
    finally:
        ctx.close()


def test_malformed_graphs_are_flagged_and_others_answered(lib, oracle_mod):
    good = [gen.cycle_graph(6), gen.tree_graph(gen.random_tree(20, None, seed=1))]
    asym = (np.array([0, 1, 1], dtype=np.int32), np.array([1], dtype=np.int32))       # 0 -> 1 without 1 -> 0
    unsorted = (np.array([0, 2, 3, 4], dtype=np.int32), np.array([2, 1, 0, 0], dtype=np.int32))
    graphs = [good[0], asym, good[1], unsorted]
    ctx = lib.default_context()
    mask, spans, counts = run_fused(lib, graphs, ctx=ctx)
    assert ctx.status_bits() != 0
    for t in (0, 2):
        ref_mask, ref_cnt = oracle_mod.bridges(*graphs[t])
        start, words = spans[t]
        assert np.array_equal(mask[start:start + words], ref_mask) and counts[t] == ref_cnt
    for t in (1, 3):
        start, words = spans[t]
        assert (mask[start:start + words] == 0).all() and counts[t] == 0
    # a graph beyond the stated bound (the batch as a whole within it) is flagged, not read past
    big = gen.cycle_graph(300)
    graphs = [big, gen.cycle_graph(10)]
    mask, spans, counts = run_fused(lib, graphs, ctx=ctx, max_vertices=200, max_slots=1000)
    assert ctx.status_bits() != 0
    assert counts[0] == 0 and counts[1] == 0


def test_host_argument_errors(lib):
    g = [(_dev(np.array([0, 1, 2], dtype=np.int32)), _dev(np.array([1, 0], dtype=np.int32)))]
    with pytest.raises(lib.EtError) as e:
        lib.et_bridges_batch_fused(g, max_vertices=2000)
    assert e.value.code == lib.et.ET_ESIZE
    with pytest.raises(lib.EtError) as e:
        lib.et_bridges_batch_fused(g, max_vertices=1, max_slots=2)   # 2 vertices cannot be one graph of <= 1
    assert e.value.code == lib.et.ET_EINVAL


def test_graph_order_changes_nothing_but_the_order(lib):
    """Graphs handed out in another order (a random permutation, or the
    costliest first as BridgesFusedGraph does) give the same masks and
    counts; an entry out of range is flagged and only the graph it
    displaces goes unanswered."""
    import torch
    rng = np.random.default_rng(61)
    graphs = [gen.random_multigraph(int(rng.integers(2, 600)), int(rng.integers(1, 1500)), seed=t, loops=True,
                                    multi=True) for t in range(200)]
    ctx = lib.default_context()
    want, spans, want_c = run_fused(lib, graphs, ctx=ctx)
    ctx.check()
    dg = [(_dev(rp), _dev(col)) for rp, col in graphs]
    rows = torch.cat([g[0] for g in dg])
    cols = torch.cat([g[1] for g in dg])
    vs = [len(r) - 1 for r, _ in graphs]
    ss = [len(c) for _, c in graphs]
    voff = _dev(np.concatenate([[0], np.cumsum(vs)]), np.int64)
    soff = _dev(np.concatenate([[0], np.cumsum(ss)]), np.int64)
    kw = dict(row_ptr=rows, col=cols, voff=voff, soff=soff, slots=ss, vertices=vs, ctx=ctx)
    T = len(graphs)
    for order in (rng.permutation(T).astype(np.int32), lib.fused_graph_order(ss, vs)):
        assert sorted(order.tolist()) == list(range(T))
        mask, _, counts = lib.et_bridges_batch_fused(order=_dev(order), **kw)
        ctx.check()
        assert np.array_equal(mask.cpu().numpy().view(np.uint32), want)
        assert np.array_equal(counts.cpu().numpy(), want_c)
    g = lib.BridgesFusedGraph(rows, cols, voff, soff, ss, vs)
    assert g.order is not None
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(g.mask.cpu().numpy().view(np.uint32), want)
    g.close()
    # graph 0's slot names no graph: flagged, graph 0's words untouched, the rest answered
    bad = np.arange(T, dtype=np.int32)
    bad[0] = T
    total = sum((x + 31) // 32 for x in ss)
    mask = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    lib.et_bridges_batch_fused(order=_dev(bad), mask=mask, **kw)
    assert ctx.status_bits() != 0
    got = mask.cpu().numpy().view(np.uint32)
    w0 = (ss[0] + 31) // 32
    assert (got[:w0] == np.uint32(0xfffffff9)).all()
    assert np.array_equal(got[w0:], want[w0:])
