"""GPU parity of the batched forest path (et_tree_build_batch / et_lca_batch):
every tree of a batch must get exactly the per-tree statistics and LCA
answers of the oracle run on that tree alone (bit-exact)."""
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


def check_batch(lib, oracle_mod, batch, trees_to_check=None, ctx=None, workers=1):
    ctx = ctx or lib.default_context()
    T = len(batch["sizes"])
    tree = lib.et_tree_build_batch(_dev(batch["parent"]), _dev(batch["offsets"], np.int64), ctx=ctx)
    got = {k: v.cpu().numpy() for k, v in tree.export().items()}
    out = tree.lca_batch(_dev(batch["qtree"]), _dev(batch["qx"]), _dev(batch["qy"])).cpu().numpy()
    ctx.check()
    tree.free()
    off = batch["offsets"]
    qstart = np.searchsorted(batch["qtree"], np.arange(T + 1))

    def one(t):
        """None when tree t matches the oracle run on it alone, else what differs."""
        a, b = int(off[t]), int(off[t + 1])
        p = batch["parent"][a:b]
        ref = oracle_mod.euler_tour(p)
        for k in ("depth", "pre", "size"):
            if not np.array_equal(got[k][a:b], ref[k]):
                return (t, k)
        qa, qb = int(qstart[t]), int(qstart[t + 1])
        if qb > qa:
            want = oracle_mod.lca_offline(p, batch["qx"][qa:qb], batch["qy"][qa:qb])
            if not np.array_equal(out[qa:qb], want):
                return (t, "lca")
        return None

    trees = range(T) if trees_to_check is None else trees_to_check
    if workers > 1:
        # the oracle is C behind ctypes, which releases the GIL during the calls
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            bad = [r for r in ex.map(one, trees) if r is not None]
    else:
        bad = [r for r in map(one, trees) if r is not None]
    assert not bad, bad[:10]


def test_small_mixed_batch(lib, oracle_mod):
    batch = gen.forest_batch(200, seed=1, log2_min=0, log2_max=12, qlog2_min=0, qlog2_max=9)
    check_batch(lib, oracle_mod, batch)


def test_single_node_trees(lib, oracle_mod):
    # trees of 1 and 2 nodes between larger ones
    parents = [np.array([-1], np.int32), gen.random_tree(50, None, seed=1), np.array([-1], np.int32),
               np.array([1, -1], np.int32), gen.random_tree(3000, 1, seed=2), np.array([-1], np.int32)]
    sizes = np.array([len(p) for p in parents])
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    qx, qy, qt = [], [], []
    for t, p in enumerate(parents):
        x, y = gen.random_queries(len(p), 64, seed=t)
        qx.append(x)
        qy.append(y)
        qt.append(np.full(64, t, np.int32))
    batch = {"parent": np.concatenate(parents), "offsets": offsets, "sizes": sizes,
             "qx": np.concatenate(qx), "qy": np.concatenate(qy), "qtree": np.concatenate(qt)}
    check_batch(lib, oracle_mod, batch)


def test_batch_of_one_equals_single_build(lib):
    parent = gen.random_tree(100000, 7, seed=3)
    qx, qy = gen.random_queries(100000, 50000, seed=3)
    single = lib.et_tree_build(_dev(parent))
    a = single.lca(_dev(qx), _dev(qy)).cpu().numpy()
    single.free()
    batch = lib.et_tree_build_batch(_dev(parent), _dev([0, 100000], np.int64))
    b = batch.lca_batch(_dev(np.zeros(50000)), _dev(qx), _dev(qy)).cpu().numpy()
    batch.free()
    lib.default_context().check()
    assert np.array_equal(a, b)


def test_malformed_batches_flagged(lib):
    parents = np.concatenate([gen.random_tree(100, None, seed=1), gen.random_tree(100, None, seed=2)])
    bad = parents.copy()
    bad[np.nonzero(bad[100:] >= 0)[0][0] + 100] = -1          # second root in tree 1
    for p in (bad,):
        ctx = lib.Context()
        t = lib.et_tree_build_batch(_dev(p), _dev([0, 100, 200], np.int64), ctx=ctx)
        with pytest.raises(lib.EtError):
            ctx.check()
        t.free()
        ctx.close()
    ctx = lib.Context()
    t = lib.et_tree_build_batch(_dev(parents), _dev([0, 100, 200], np.int64), ctx=ctx)
    ctx.check()
    out = t.lca_batch(_dev([0, 1, 2, 1]), _dev([3, 100, 0, -1]), _dev([4, 5, 0, 0])).cpu().numpy()
    assert out[0] >= 0 and out[1] == -1 and out[2] == -1 and out[3] == -1
    with pytest.raises(lib.EtError):
        ctx.check()
    t.free()
    ctx.close()


def test_full_size_4096_trees(lib, oracle_mod, bench_ctx):
    # 4096 trees, sizes log-uniform in [2^6, 2^18], grasp from {1, 64, n},
    # 2^10..2^14 queries each (about 1.26e8 nodes and 2.3e7 queries): every
    # tree's depth, preorder, size and LCA answers against the oracle run on
    # that tree alone
    import os
    import time
    t0 = time.time()
    batch = gen.forest_batch(4096, seed=0)
    print(f"\n[batch] {int(batch['offsets'][-1])} nodes, {len(batch['qx'])} queries, "
          f"generated in {time.time() - t0:.1f}s", flush=True)
    check_batch(lib, oracle_mod, batch, ctx=bench_ctx("batch"), workers=min(16, os.cpu_count() or 1))
    print(f"[batch] all 4096 trees compared in {time.time() - t0:.1f}s", flush=True)
