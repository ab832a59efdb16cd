"""GPU parity of the RMQ query engine (range minima over the Euler tour,
the alternative to Inlabel in Section 3) and of both engines on the
scale-free trees of Section 3.2: answers equal the oracle's LCAs bit for
bit."""
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


def both_engines(lib, oracle_mod, parent, qx, qy, ctx=None):
    ctx = ctx or lib.default_context()
    d_parent = _dev(parent)
    tree = lib.et_tree_build(d_parent, ctx=ctx).rmq_build(d_parent)
    rmq = _np(tree.lca_rmq(_dev(qx), _dev(qy)))
    sv = _np(tree.lca(_dev(qx), _dev(qy)))
    tree.free()
    ctx.check()
    ref = oracle_mod.lca_offline(parent, qx, qy)
    assert np.array_equal(rmq, ref), "rmq engine"
    assert np.array_equal(sv, ref), "inlabel engine"


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 100])
@pytest.mark.parametrize("grasp", [None, 2, 1])
def test_small_trees_all_pairs(lib, oracle_mod, n, grasp):
    parent = gen.random_tree(n, grasp, seed=n + 7)
    xs, ys = np.meshgrid(np.arange(n), np.arange(n))
    both_engines(lib, oracle_mod, parent, xs.ravel().astype(np.int32), ys.ravel().astype(np.int32))


@pytest.mark.parametrize("grasp", [None, 64, 1])
def test_medium_trees(lib, oracle_mod, grasp):
    n = (1 << 16) + 37
    parent = gen.random_tree(n, grasp, seed=5)
    qx, qy = gen.random_queries(n, 1 << 16, seed=5)
    both_engines(lib, oracle_mod, parent, qx, qy)


@pytest.mark.parametrize("kind", ["star", "path", "heap", "caterpillar"])
def test_special_shapes(lib, oracle_mod, kind):
    n = 1 << 13
    parent = {"star": lambda: gen.star_tree(n, root=9), "path": lambda: gen.path_tree(n, seed=6),
              "heap": lambda: gen.heap_binary_tree(n - 1),
              "caterpillar": lambda: gen.caterpillar_tree(700, 9, seed=6)}[kind]()
    qx, qy = gen.random_queries(parent.shape[0], 1 << 14, seed=6)
    both_engines(lib, oracle_mod, parent, qx, qy)


@pytest.mark.parametrize("n", [1 << 12, (1 << 18) + 5])
def test_scale_free_trees(lib, oracle_mod, n):
    parent = gen.ba_tree(n, seed=n)
    qx, qy = gen.random_queries(n, 1 << 16, seed=n)
    both_engines(lib, oracle_mod, parent, qx, qy)


@pytest.mark.parametrize("grasp", [None, 1000, 1])
def test_full_size_2e24(lib, oracle_mod, bench_ctx, grasp):
    n = 1 << 24
    print(f"[rmq] n=2^24 grasp={grasp}", flush=True)
    parent = gen.random_tree(n, grasp, seed=31)
    qx, qy = gen.random_queries(n, 1 << 24, seed=31)
    ctx = bench_ctx("single")
    d_parent = _dev(parent)
    tree = lib.et_tree_build(d_parent, ctx=ctx).rmq_build(d_parent)
    dqx, dqy = _dev(qx), _dev(qy)
    rmq = tree.lca_rmq(dqx, dqy)
    sv = tree.lca(dqx, dqy)
    import torch
    assert torch.equal(rmq, sv)                          # all 2^24 queries: the two engines agree
    rmq = _np(rmq)
    tree.free()
    ctx.check()
    k = 1 << 20                                          # and a sample against the oracle
    assert np.array_equal(rmq[:k], oracle_mod.lca_offline(parent, qx[:k], qy[:k]))


def test_full_size_scale_free(lib, oracle_mod, bench_ctx):
    n = 1 << 24
    parent = gen.ba_tree(n, seed=24)
    qx, qy = gen.random_queries(n, 1 << 20, seed=24)
    both_engines(lib, oracle_mod, parent, qx, qy, ctx=bench_ctx("single"))


def test_rejected_uses(lib):
    n = 100
    parent = gen.random_tree(n, None, seed=1)
    tree = lib.et_tree_build(_dev(parent))
    with pytest.raises(lib.EtError):                     # tables not built yet
        tree.lca_rmq(_dev([1]), _dev([2]))
    tree.free()
    c = np.flatnonzero(parent >= 0)
    et = lib.et_tree_build_edges(_dev(parent[c]), _dev(c), n, int(np.flatnonzero(parent == -1)[0]))
    with pytest.raises(lib.EtError):                     # edge-built trees number half-edges by edge
        et.rmq_build(_dev(parent))
    et.free()
    lib.default_context().check()
