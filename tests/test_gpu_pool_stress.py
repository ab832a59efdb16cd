"""One context, many calls of every kind and size in a seeded random order:
each result must still equal the oracle's. The context's scratch pool hands
blocks of earlier calls to later ones (best fit, grown on demand), so this
checks that no call reads scratch it did not initialise and that trees
outlive the scratch of the calls that follow them."""
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _np(t):
    return t.cpu().numpy()


def test_mixed_calls_share_one_pool(lib, oracle_mod):
    rng = np.random.default_rng(2024)
    ctx = lib.Context()
    kept = []                                            # trees kept alive across later calls
    for it in range(200):
        kind = ["tree", "lca_kept", "bridges", "list", "edges", "naive", "rmq", "batch"][int(rng.integers(8))]
        n = int(2 ** rng.uniform(0, 17))
        seed = int(rng.integers(1 << 30))
        if kind == "lca_kept" and kept:
            parent, tree = kept[int(rng.integers(len(kept)))]
            qx, qy = gen.random_queries(len(parent), 3000, seed=seed)
            got = _np(tree.lca(_dev(qx), _dev(qy)))
            assert np.array_equal(got, oracle_mod.lca_offline(parent, qx, qy)), (it, kind)
        elif kind in ("tree", "lca_kept"):
            parent = gen.random_tree(n, [None, 3, 1][seed % 3], seed=seed)
            tree = lib.et_tree_build(_dev(parent), ctx=ctx)
            ref = oracle_mod.euler_tour(parent)
            got = tree.export(("depth", "pre", "size"))
            for k in ("depth", "pre", "size"):
                assert np.array_equal(_np(got[k]), ref[k]), (it, kind, k)
            if len(kept) < 4 and rng.random() < 0.5:
                kept.append((parent, tree))
            else:
                tree.free()
        elif kind == "bridges":
            rp, col = gen.random_multigraph(n, int(1.5 * n), seed=seed, loops=True, multi=True)
            mask, cnt = lib.et_bridges(_dev(rp), _dev(col), ctx=ctx)
            ref_mask, ref_cnt = oracle_mod.bridges(rp, col)
            assert np.array_equal(_np(mask).view(np.uint32)[: len(ref_mask)], ref_mask), (it, kind)
            assert cnt == ref_cnt
        elif kind == "list":
            parent = gen.random_tree(n, None, seed=seed)
            succ, head = oracle_mod.tree_succ(parent)
            heads = np.array([head if head >= 0 else -1], dtype=np.int32)
            if head < 0:
                continue
            got = _np(lib.et_list_rank(_dev(succ), _dev(heads), ctx=ctx))
            assert np.array_equal(got, oracle_mod.list_rank(succ, heads)), (it, kind)
        elif kind == "edges":
            parent = gen.random_tree(n, None, seed=seed)
            c = np.flatnonzero(parent >= 0).astype(np.int32)
            root = int(rng.integers(n))
            tree = lib.et_tree_build_edges(_dev(parent[c]), _dev(c), n, root, ctx=ctx)
            ref = oracle_mod.euler_tour_edges(n, parent[c], c, root)
            got = tree.export(("depth", "pre", "size"))
            for k in ("depth", "pre", "size"):
                assert np.array_equal(_np(got[k]), ref[k]), (it, kind, k)
            tree.free()
        elif kind == "naive":
            parent = gen.random_tree(n, None, seed=seed)
            lv = lib.et_levels(_dev(parent), ctx=ctx)
            assert np.array_equal(_np(lv), oracle_mod.euler_tour(parent)["depth"]), (it, kind)
        elif kind == "rmq":
            parent = gen.ba_tree(n, seed=seed)
            d_parent = _dev(parent)
            tree = lib.et_tree_build(d_parent, ctx=ctx).rmq_build(d_parent)
            qx, qy = gen.random_queries(n, 3000, seed=seed)
            got = _np(tree.lca_rmq(_dev(qx), _dev(qy)))
            assert np.array_equal(got, oracle_mod.lca_offline(parent, qx, qy)), (it, kind)
            tree.free()
        else:
            b = gen.forest_batch(int(rng.integers(1, 40)), seed=seed, log2_min=0, log2_max=12, qlog2_min=4,
                                 qlog2_max=8)
            import torch
            offs = torch.from_numpy(b["offsets"].astype(np.int64)).cuda()
            tree = lib.et_tree_build_batch(_dev(b["parent"]), offs, ctx=ctx)
            got = _np(tree.lca_batch(_dev(b["qtree"]), _dev(b["qx"]), _dev(b["qy"])))
            off = b["offsets"]
            for t in range(len(b["sizes"])):
                sel = b["qtree"] == t
                p = b["parent"][off[t]:off[t + 1]]
                assert np.array_equal(got[sel], oracle_mod.lca_offline(p, b["qx"][sel], b["qy"][sel])), (it, t)
            tree.free()
        ctx.check()
    for _, tree in kept:
        tree.free()
    ctx.close()
