"""GPU parity: Euler tour, node statistics, Inlabel tables and LCA queries of
the HIP library against the CPU oracle, element by element (all integer
work, so the bar is bit-exact equality)."""
import json
import os

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


def build_and_compare(lib, oracle_mod, parent, queries=None, check_tables=True, ctx=None):
    """Build on the GPU and compare every exported table with the oracle."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    n = parent.shape[0]
    ctx = ctx or lib.default_context()
    tree = lib.et_tree_build(_dev(parent), ctx=ctx)
    got = {k: _np(v) for k, v in tree.export().items()}
    ctx.check()
    ref = oracle_mod.euler_tour(parent)
    succ_ref, _ = oracle_mod.tree_succ(parent)
    assert np.array_equal(got["succ"], succ_ref), "tour successor"
    assert np.array_equal(got["rank"], ref["rank"]), "tour rank"
    assert np.array_equal(got["depth"], ref["depth"]), "depth"
    assert np.array_equal(got["pre"], ref["pre"]), "preorder"
    assert np.array_equal(got["size"], ref["size"]), "subtree size"
    if check_tables:
        T = oracle_mod.sv_tables(parent, ref["depth"], ref["pre"], ref["size"])
        assert np.array_equal(got["inlabel"].view(np.uint32), T["inlabel"]), "inlabel"
        assert np.array_equal(got["asc"].view(np.uint32), T["asc"]), "ascendant"
    if queries is not None:
        qx, qy = queries
        out = _np(tree.lca(_dev(qx), _dev(qy)))
        ctx.check()
        assert np.array_equal(out, oracle_mod.lca_offline(parent, qx, qy)), "lca"
    tree.free()
    return ref


def test_fig1_worked_example(lib, oracle_mod):
    with open(os.path.join(os.path.dirname(__file__), "golden", "fig1_fig2.json")) as f:
        fig = json.load(f)
    parent = np.full(6, -1, dtype=np.int32)
    for p, c in fig["tree_edges_parent_child"]:
        parent[c] = p
    qx, qy = [a.ravel() for a in np.meshgrid(np.arange(6), np.arange(6))]
    build_and_compare(lib, oracle_mod, parent, (qx, qy))
    # the tour itself, against the figure
    tree = lib.et_tree_build(_dev(parent))
    rank = _np(tree.export()["rank"])
    order = np.argsort(np.where(rank < 0, 1 << 30, rank))[:10]
    pairs = [[int(parent[e >> 1]), int(e >> 1)] if e % 2 == 0 else [int(e >> 1), int(parent[e >> 1])]
             for e in order]
    assert pairs == fig["fig1_tour_in_order"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 65, 1000, 4097])
@pytest.mark.parametrize("grasp", [None, 1, 3])
def test_small_trees_all_pairs(lib, oracle_mod, n, grasp):
    parent = gen.random_tree(n, grasp, seed=n * 7 + (grasp or 0))
    if n <= 65:
        qx, qy = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n))]
    else:
        qx, qy = gen.random_queries(n, 4 * n, seed=n)
    build_and_compare(lib, oracle_mod, parent, (qx, qy))


@pytest.mark.parametrize("n,grasp,seed", [(1 << 16, None, 0), (1 << 16, None, 1), (300007, None, 2),
                                          (300007, 1, 3), (300007, 1000, 4), (1 << 20, 64, 5)])
def test_medium_trees(lib, oracle_mod, n, grasp, seed):
    # 2^16 is the parity configuration; 300007 is ragged against every tile size
    parent = gen.random_tree(n, grasp, seed=seed)
    qx, qy = gen.random_queries(n, n, seed=seed)
    build_and_compare(lib, oracle_mod, parent, (qx, qy))


@pytest.mark.parametrize("kind", ["path", "path_relabel", "star", "star_mid", "caterpillar", "heap"])
def test_special_shapes(lib, oracle_mod, kind):
    n = 200003
    parent = {
        "path": lambda: gen.path_tree(n),
        "path_relabel": lambda: gen.path_tree(n, seed=3),
        "star": lambda: gen.star_tree(n, 0),
        "star_mid": lambda: gen.star_tree(n, n // 2),
        "caterpillar": lambda: gen.caterpillar_tree(20000, 9, seed=4),
        "heap": lambda: gen.heap_binary_tree(n),
    }[kind]()
    qx, qy = gen.random_queries(len(parent), 100000, seed=5)
    build_and_compare(lib, oracle_mod, parent, (qx, qy))


def test_repeat_is_deterministic(lib):
    parent = gen.random_tree(123457, None, seed=8)
    outs = []
    for _ in range(3):
        t = lib.et_tree_build(_dev(parent))
        outs.append({k: _np(v) for k, v in t.export().items()})
        t.free()
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k


def test_lca_batches_equal_one_batch(lib, oracle_mod):
    n = 50000
    parent = gen.random_tree(n, 10, seed=9)
    qx, qy = gen.random_queries(n, 30001, seed=9)
    t = lib.et_tree_build(_dev(parent))
    whole = _np(t.lca(_dev(qx), _dev(qy)))
    parts = np.concatenate([_np(t.lca(_dev(qx[i:i + 777]), _dev(qy[i:i + 777])))
                            for i in range(0, len(qx), 777)])
    assert np.array_equal(whole, parts)
    empty = _np(t.lca(_dev(qx[:0]), _dev(qy[:0])))
    assert empty.shape == (0,)
    t.free()


@pytest.mark.parametrize("bad", ["two_roots", "no_root", "cycle", "out_of_range", "self_parent"])
def test_malformed_parent_sets_status(lib, bad):
    n = 5000
    p = gen.random_tree(n, None, seed=1).copy()
    root = int(np.nonzero(p == -1)[0][0])
    other = (root + 1) % n
    if bad == "two_roots":
        p[other] = -1
    elif bad == "no_root":
        p[root] = other
    elif bad == "cycle":
        a, b = [int(v) for v in np.nonzero(p >= 0)[0][:2]]
        p[a], p[b] = b, a
    elif bad == "out_of_range":
        p[other] = n + 5
    elif bad == "self_parent":
        p[other] = other
    ctx = lib.Context()
    t = lib.et_tree_build(_dev(p), ctx=ctx)
    with pytest.raises(lib.EtError):
        ctx.check()
    # the tree is still queryable without faulting
    qx, qy = gen.random_queries(n, 1000, seed=2)
    t.lca(_dev(qx), _dev(qy))
    ctx.status_bits()
    t.free()
    ctx.close()


def test_bad_queries_flagged(lib):
    n = 1000
    parent = gen.random_tree(n, None, seed=3)
    ctx = lib.Context()
    t = lib.et_tree_build(_dev(parent), ctx=ctx)
    ctx.check()
    out = _np(t.lca(_dev([0, n, -1, 5]), _dev([1, 2, 3, n + 7])))
    assert out[1] == -1 and out[2] == -1 and out[3] == -1 and out[0] >= 0
    with pytest.raises(lib.EtError):
        ctx.check()
    t.free()
    ctx.close()


@pytest.mark.parametrize("grasp", [None, 1000, 1])
def test_full_size_2e24(lib, oracle_mod, bench_ctx, grasp):
    # the 2^24-node configuration (grasp n, 1000, 1) with 2^24 uniform
    # queries, in the launch configuration the benchmark times
    import time
    n = 1 << 24
    t0 = time.time()
    parent = gen.random_tree(n, grasp, seed=0)
    qx, qy = gen.random_queries(n, n, seed=0)
    print(f"\n[full-size grasp={grasp}] inputs {time.time() - t0:.1f}s", flush=True)
    ctx = bench_ctx("single")
    build_and_compare(lib, oracle_mod, parent, (qx, qy), check_tables=True, ctx=ctx)
    print(f"[full-size grasp={grasp}] compared in {time.time() - t0:.1f}s", flush=True)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 4097, (1 << 17) + 11])
@pytest.mark.parametrize("grasp", [None, 1])
def test_tour_array(lib, oracle_mod, n, grasp):
    parent = gen.random_tree(n, grasp, seed=n + 3)
    tree = lib.et_tree_build(_dev(parent))
    got = _np(tree.tour())
    tree.free()
    lib.default_context().check()
    assert np.array_equal(got, oracle_mod.euler_tour(parent)["tour"])


def test_tour_array_full_size(lib, bench_ctx):
    # 2^24 nodes: the tour is the inverse of the exported rank
    import torch
    n = 1 << 24
    parent = gen.random_tree(n, 1000, seed=9)
    ctx = bench_ctx("single")
    tree = lib.et_tree_build(_dev(parent), ctx=ctx)
    tour = tree.tour()
    rank = tree.export(("rank",))["rank"]
    ctx.check()
    L = 2 * (n - 1)
    assert tour.numel() == L
    assert torch.equal(rank[tour.long()], torch.arange(L, dtype=torch.int32, device=tour.device))
    tree.free()


def test_tour_array_rejected_for_batches(lib):
    import torch
    b = gen.forest_batch(5, seed=2, log2_min=2, log2_max=6)
    offs = torch.from_numpy(b["offsets"].astype(np.int64)).cuda()
    tree = lib.et_tree_build_batch(_dev(b["parent"]), offs)
    with pytest.raises(lib.EtError):
        tree.tour()
    tree.free()
