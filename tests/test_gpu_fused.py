"""GPU parity of the one-launch small-tree batch (et_lca_batch_fused): every
tree's depth, preorder and subtree size and every query answer must equal
the oracle run on that tree alone (bit-exact), and the multi-kernel batched
path on the same batch."""
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


def _qoff(qtree, T):
    return np.searchsorted(qtree, np.arange(T + 1)).astype(np.int64)


def _batch_from_trees(parents, qcounts, seed):
    """Concatenate explicit trees with uniform queries per tree."""
    offsets = np.zeros(len(parents) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in parents])
    qx, qy, qt = [], [], []
    for t, (p, q) in enumerate(zip(parents, qcounts)):
        x, y = gen.random_queries(len(p), q, seed=seed * 7919 + t)
        qx.append(x)
        qy.append(y)
        qt.append(np.full(q, t, dtype=np.int32))
    return {"parent": np.concatenate(parents).astype(np.int32), "offsets": offsets,
            "sizes": np.diff(offsets), "qx": np.concatenate(qx).astype(np.int32),
            "qy": np.concatenate(qy).astype(np.int32), "qtree": np.concatenate(qt).astype(np.int32)}


def run_fused(lib, batch, max_nodes, ctx=None):
    T = len(batch["sizes"])
    out, st = lib.et_lca_batch_fused(_dev(batch["parent"]), _dev(batch["offsets"], np.int64),
                                     _dev(_qoff(batch["qtree"], T), np.int64), _dev(batch["qx"]),
                                     _dev(batch["qy"]), max_nodes, stats=True, ctx=ctx)
    return out.cpu().numpy(), {k: v.cpu().numpy() for k, v in st.items()}


def check_against_oracle(oracle_mod, batch, out, st):
    off = batch["offsets"]
    T = len(batch["sizes"])
    qoff = _qoff(batch["qtree"], T)
    bad = []
    for t in range(T):
        a, b = int(off[t]), int(off[t + 1])
        p = batch["parent"][a:b]
        ref = oracle_mod.euler_tour(p)
        for k in ("depth", "pre", "size"):
            if not np.array_equal(st[k][a:b], ref[k]):
                bad.append((t, k))
        qa, qb = int(qoff[t]), int(qoff[t + 1])
        if qb > qa and not np.array_equal(out[qa:qb], oracle_mod.lca_offline(p, batch["qx"][qa:qb],
                                                                           batch["qy"][qa:qb])):
            bad.append((t, "lca"))
    assert not bad, bad[:10]


@pytest.mark.parametrize("T,lo,hi,seed", [(1, 6, 6, 0), (37, 6, 12, 1), (500, 6, 12, 2), (300, 2, 8, 3),
                                          (64, 11, 12, 4), (700, 4, 10, 5)])
def test_random_batches(lib, oracle_mod, T, lo, hi, seed):
    batch = gen.forest_batch(T, seed=seed, log2_min=lo, log2_max=hi, qlog2_min=0, qlog2_max=10)
    max_nodes = int(batch["sizes"].max())
    ctx = lib.default_context()
    out, st = run_fused(lib, batch, max_nodes)
    ctx.check()
    check_against_oracle(oracle_mod, batch, out, st)


def test_shapes_and_edge_sizes(lib, oracle_mod):
    parents = [np.array([-1], dtype=np.int32),                 # one node
               np.array([1, -1], dtype=np.int32),              # two nodes, root 1
               gen.path_tree(4096, seed=3),                    # deepest: a path at the size limit
               gen.star_tree(4096, root=4095),                 # widest
               gen.heap_binary_tree(4095),
               gen.caterpillar_tree(300, 3, seed=5),
               gen.random_tree(4096, 1, seed=6), gen.random_tree(4096, None, seed=7),
               gen.random_tree(65, 1000, seed=8), gen.random_tree(63, None, seed=9),
               gen.path_tree(4096)]                            # ids in tour order (no relabel)
    batch = _batch_from_trees(parents, [1, 5, 3000, 2000, 100, 0, 4096, 4096, 64, 63, 50], seed=1)
    ctx = lib.default_context()
    out, st = run_fused(lib, batch, 4096)
    ctx.check()
    check_against_oracle(oracle_mod, batch, out, st)


def test_bound_not_multiple_of_64_and_many_tiny_trees(lib, oracle_mod):
    rng = np.random.default_rng(11)
    sizes = rng.integers(1, 101, size=3000)
    parents = [gen.random_tree(int(s), None, seed=1000 + i) for i, s in enumerate(sizes)]
    batch = _batch_from_trees(parents, [int(x) for x in rng.integers(0, 20, size=len(sizes))], seed=2)
    ctx = lib.default_context()
    out, st = run_fused(lib, batch, 100)
    ctx.check()
    check_against_oracle(oracle_mod, batch, out, st)


def test_equals_multi_kernel_batch(lib):
    batch = gen.forest_batch(800, seed=5, log2_min=6, log2_max=12, qlog2_min=4, qlog2_max=10)
    ctx = lib.default_context()
    out, st = run_fused(lib, batch, 4096)
    tree = lib.et_tree_build_batch(_dev(batch["parent"]), _dev(batch["offsets"], np.int64), ctx=ctx)
    ref = {k: v.cpu().numpy() for k, v in tree.export().items()}
    want = tree.lca_batch(_dev(batch["qtree"]), _dev(batch["qx"]), _dev(batch["qy"])).cpu().numpy()
    ctx.check()
    tree.free()
    assert np.array_equal(out, want)
    for k in ("depth", "pre", "size"):
        assert np.array_equal(st[k], ref[k]), k


@pytest.mark.parametrize("log2_max,bound", [(12, 4096), (10, 1024)])  # the 1024- and the 256-lane shape
def test_repeated_calls_and_graph_replays(lib, log2_max, bound):
    """The work counter resets itself at the end of every launch: calls in a
    row with different grids, and replays of a captured graph, all agree."""
    import torch
    big = gen.forest_batch(600, seed=21, log2_min=6, log2_max=log2_max, qlog2_min=4, qlog2_max=9)
    small = gen.forest_batch(3, seed=22, log2_min=6, log2_max=8, qlog2_min=4, qlog2_max=6)
    ctx = lib.Context()
    try:
        first = [run_fused(lib, b, bound, ctx=ctx)[0] for b in (big, small, big)]
        ctx.check()
        assert np.array_equal(first[0], first[2])
        T = len(big["sizes"])
        args = (_dev(big["parent"]), _dev(big["offsets"], np.int64), _dev(_qoff(big["qtree"], T), np.int64),
                _dev(big["qx"]), _dev(big["qy"]))
        out = torch.full((len(big["qx"]),), -7, dtype=torch.int32, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            lib.et_lca_batch_fused(*args, bound, out=out, ctx=ctx)  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lib.et_lca_batch_fused(*args, bound, out=out, ctx=ctx)
        for _ in range(4):
            out.fill_(-7)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), first[0])
            # eager work between replays
            assert np.array_equal(run_fused(lib, small, bound, ctx=ctx)[0], first[1])
        ctx.check()
    finally:
        ctx.close()


def test_malformed_trees_are_flagged_and_others_answered(lib, oracle_mod):
    good = [gen.random_tree(200, None, seed=31), gen.random_tree(50, 1, seed=32)]
    two_roots = np.array([-1, 0, -1, 2], dtype=np.int32)
    cycle = np.array([-1, 2, 1, 0], dtype=np.int32)        # 1 and 2 point at each other
    self_parent = np.array([-1, 1, 0], dtype=np.int32)
    parents = [good[0], two_roots, good[1], cycle, self_parent]
    batch = _batch_from_trees(parents, [30, 4, 30, 4, 3], seed=3)
    ctx = lib.default_context()
    out, _ = run_fused(lib, batch, 256)
    bits = ctx.status_bits()
    assert bits != 0
    qoff = _qoff(batch["qtree"], len(parents))
    for t in (1, 3, 4):
        assert (out[qoff[t]:qoff[t + 1]] == -1).all()
    off = batch["offsets"]
    for t in (0, 2):
        p = batch["parent"][off[t]:off[t + 1]]
        qa, qb = qoff[t], qoff[t + 1]
        assert np.array_equal(out[qa:qb], oracle_mod.lca_offline(p, batch["qx"][qa:qb], batch["qy"][qa:qb]))
    # a tree larger than the stated bound (the batch as a whole within it) is
    # flagged on the device and not read past; the other tree is answered
    batch = _batch_from_trees([gen.random_tree(300, None, seed=33), gen.random_tree(10, None, seed=34)],
                              [10, 10], seed=4)
    out, _ = run_fused(lib, batch, 256)
    assert ctx.status_bits() != 0
    assert (out[:10] == -1).all()
    p = batch["parent"][300:]
    assert np.array_equal(out[10:], oracle_mod.lca_offline(p, batch["qx"][10:], batch["qy"][10:]))


def test_host_argument_errors(lib):
    import torch
    z64 = torch.zeros(2, dtype=torch.int64, device="cuda")
    z32 = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(lib.EtError) as e:
        lib.et_lca_batch_fused(z32, z64, z64, z32, z32, 5000)
    assert e.value.code == lib.et.ET_ESIZE
    big = torch.zeros(300, dtype=torch.int32, device="cuda")
    with pytest.raises(lib.EtError) as e:
        lib.et_lca_batch_fused(big, z64, z64, z32, z32, 100)  # 300 nodes cannot be one tree of <= 100
    assert e.value.code == lib.et.ET_EINVAL


@pytest.mark.parametrize("n_small,n_large,seed", [(300, 20, 41), (40, 0, 42), (0, 6, 43)])
def test_split_batch_graph(lib, oracle_mod, n_small, n_large, seed):
    """Trees that fit one workgroup first (one-launch kernel), larger ones
    after (multi-kernel batch), captured in one HIP graph: every answer
    equals the multi-kernel batch's on the same batch and, tree by tree on a
    sample, the oracle's; replays with eager work between them agree."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.concatenate([rng.integers(1, lib.et.FUSED_MAX_NODES + 1, size=n_small),
                            rng.integers(lib.et.FUSED_MAX_NODES + 1, 20000, size=n_large)]).astype(int)
    parents = [gen.random_tree(int(s), [None, 1, 64][i % 3], seed=1000 * seed + i) for i, s in enumerate(sizes)]
    batch = _batch_from_trees(parents, [int(x) for x in rng.integers(0, 400, size=len(sizes))], seed=seed)
    T = len(sizes)
    qoff = _qoff(batch["qtree"], T)
    d_parent, d_qx, d_qy = _dev(batch["parent"]), _dev(batch["qx"]), _dev(batch["qy"])
    ctx = lib.Context()
    g = lib.SplitBatchGraph(d_parent, batch["offsets"], qoff, d_qx, d_qy, ctx=ctx)
    try:
        assert g.split == n_small
        tree = lib.et_tree_build_batch(d_parent, _dev(batch["offsets"], np.int64))
        want = tree.lca_batch(_dev(batch["qtree"]), d_qx, d_qy).cpu().numpy()
        tree.free()
        lib.default_context().check()
        small = gen.forest_batch(5, seed=seed, log2_min=4, log2_max=8, qlog2_min=2, qlog2_max=6)
        first_small = run_fused(lib, small, 256)[0]
        for _ in range(3):
            g.out.fill_(-7)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(g.out.cpu().numpy(), want)
            assert np.array_equal(run_fused(lib, small, 256)[0], first_small)  # eager work in between
        ctx.check()
        off = batch["offsets"]
        sample = sorted(set(range(0, T, 7)) | set(range(n_small, T)))
        for t in sample:
            qa, qb = int(qoff[t]), int(qoff[t + 1])
            if qb > qa:
                p = batch["parent"][int(off[t]):int(off[t + 1])]
                assert np.array_equal(want[qa:qb], oracle_mod.lca_offline(p, batch["qx"][qa:qb], batch["qy"][qa:qb])), t
    finally:
        g.close()
        ctx.close()


def test_split_batch_graph_rejects_bad_offsets(lib):
    z = _dev(np.zeros(4, dtype=np.int32))
    with pytest.raises(ValueError):
        lib.SplitBatchGraph(_dev(np.array([-1, 0, 0], dtype=np.int32)), [0, 2], [0, 4], z, z)  # 3 nodes, offsets say 2
    with pytest.raises(ValueError):
        lib.SplitBatchGraph(_dev(np.array([-1, 0], dtype=np.int32)), [0, 2], [0, 2, 4], z, z)  # qoffsets too long


def test_split_batch_graph_at_the_size_bound(lib, oracle_mod):
    """Trees of exactly FUSED_MAX_NODES nodes go through the one-launch
    kernel, one node more through the multi-kernel batch; a tree of the
    bound after a larger one stays with the larger ones (the split is the
    leading run of small trees)."""
    bound = lib.et.FUSED_MAX_NODES
    parents = [gen.path_tree(bound, seed=1), gen.random_tree(1, None, seed=2), gen.star_tree(bound, root=7),
               gen.random_tree(bound + 1, None, seed=3), gen.random_tree(bound, 64, seed=4)]
    batch = _batch_from_trees(parents, [50, 1, 60, 70, 80], seed=9)
    T = len(parents)
    qoff = _qoff(batch["qtree"], T)
    ctx = lib.Context()
    g = lib.SplitBatchGraph(_dev(batch["parent"]), batch["offsets"], qoff, _dev(batch["qx"]), _dev(batch["qy"]),
                            ctx=ctx)
    try:
        assert g.split == 3
        out = g.replay().cpu().numpy()
        ctx.check()
        off = batch["offsets"]
        for t in range(T):
            qa, qb = int(qoff[t]), int(qoff[t + 1])
            p = batch["parent"][int(off[t]):int(off[t + 1])]
            assert np.array_equal(out[qa:qb], oracle_mod.lca_offline(p, batch["qx"][qa:qb], batch["qy"][qa:qb])), t
    finally:
        g.close()
        ctx.close()


def test_tree_order_changes_nothing_but_the_order(lib, oracle_mod):
    """Trees handed out in another order (a random permutation, or costliest
    first as FusedBatchGraph does for 1024-lane workgroups) give the same
    answers and statistics; an entry out of range is flagged and only the
    tree it displaces goes unanswered."""
    import torch
    batch = gen.forest_batch(400, seed=51, log2_min=6, log2_max=12, qlog2_min=2, qlog2_max=8)
    T = len(batch["sizes"])
    qoff = _qoff(batch["qtree"], T)
    args = (_dev(batch["parent"]), _dev(batch["offsets"], np.int64), _dev(qoff, np.int64), _dev(batch["qx"]),
            _dev(batch["qy"]))
    ctx = lib.default_context()
    want, st = lib.et_lca_batch_fused(*args, 4096, stats=True)
    want = want.cpu().numpy()
    rng = np.random.default_rng(52)
    for order in (rng.permutation(T).astype(np.int32), lib.fused_order(batch["offsets"], qoff)):
        assert sorted(order.tolist()) == list(range(T))
        got, st2 = lib.et_lca_batch_fused(*args, 4096, stats=True, order=_dev(order))
        ctx.check()
        assert np.array_equal(got.cpu().numpy(), want)
        for k in ("depth", "pre", "size"):
            assert torch.equal(st[k], st2[k]), k
    g = lib.FusedBatchGraph(*args, 4096)
    assert g.order is not None
    assert np.array_equal(g.replay().cpu().numpy(), want)
    g.close()
    check_against_oracle(oracle_mod, batch, want, {k: v.cpu().numpy() for k, v in st.items()})
    # tree 0's slot names no tree: flagged, tree 0 unanswered, the rest answered
    bad = np.arange(T, dtype=np.int32)
    bad[0] = T
    out = torch.full((len(batch["qx"]),), -7, dtype=torch.int32, device="cuda")
    lib.et_lca_batch_fused(*args, 4096, out=out, order=_dev(bad))
    assert ctx.status_bits() != 0
    got = out.cpu().numpy()
    assert (got[:qoff[1]] == -7).all()
    assert np.array_equal(got[qoff[1]:], want[qoff[1]:])
