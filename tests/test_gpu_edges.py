"""GPU parity of the edge-list build (Section 2.1, the DCEL construction):
tour successor, ranks, parent, depth, preorder and subtree size against the
oracle's construction from the same edges, and LCA answers against the
offline oracle; bit-exact throughout."""
import json
import os

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def shuffled_edges(parent, seed):
    """The tree's edges in random order with random orientation."""
    rng = np.random.default_rng(seed)
    c = np.flatnonzero(parent >= 0).astype(np.int32)
    p = parent[c].astype(np.int32)
    flip = rng.random(c.shape[0]) < 0.5
    u, v = np.where(flip, c, p), np.where(flip, p, c)
    order = rng.permutation(c.shape[0])
    return u[order], v[order]


def compare(lib, oracle_mod, n, u, v, root, queries=None, ctx=None):
    import torch
    ctx = ctx or lib.default_context()
    par = torch.empty(n, dtype=torch.int32, device="cuda")
    tree = lib.et_tree_build_edges(_dev(u), _dev(v), n, root, parent_out=par, ctx=ctx)
    got = {k: _np(t) for k, t in tree.export().items()}
    got_parent = _np(par)
    ctx.check()
    ref = oracle_mod.euler_tour_edges(n, u, v, root)
    L = 2 * (n - 1)
    assert np.array_equal(got["succ"][:L], ref["succ"]), "tour successor"
    assert np.array_equal(got["rank"][:L], ref["rank"]), "tour rank"
    assert np.array_equal(_np(tree.tour()), ref["tour"]), "tour array"
    for k in ("depth", "pre", "size"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(got_parent, ref["parent"]), "parent"
    if queries is not None:
        qx, qy = queries
        out = _np(tree.lca(_dev(qx), _dev(qy)))
        ctx.check()
        assert np.array_equal(out, oracle_mod.lca_offline(ref["parent"], qx, qy)), "lca"
    tree.free()


def test_fig1_edges(lib, oracle_mod):
    fig = json.load(open(os.path.join(HERE, "golden", "fig1_fig2.json")))
    E = np.array(fig["tree_edges_parent_child"], dtype=np.int32)
    compare(lib, oracle_mod, 6, E[:, 0], E[:, 1], fig["root"])


@pytest.mark.parametrize("n", [1, 2, 3, 10, 100])
def test_small_trees_every_root(lib, oracle_mod, n):
    parent = gen.random_tree(n, None, seed=n)
    u, v = shuffled_edges(parent, n)
    xs, ys = np.meshgrid(np.arange(n), np.arange(n))
    q = (xs.ravel().astype(np.int32), ys.ravel().astype(np.int32))
    for root in sorted(set([0, n - 1, n // 2])):
        compare(lib, oracle_mod, n, u, v, root, q)


@pytest.mark.parametrize("grasp", [None, 64, 1])
@pytest.mark.parametrize("seed", [0, 1])
def test_medium_trees(lib, oracle_mod, grasp, seed):
    n = (1 << 16) + 37
    parent = gen.random_tree(n, grasp, seed=seed)
    u, v = shuffled_edges(parent, seed)
    root = int(np.random.default_rng(seed).integers(n))
    compare(lib, oracle_mod, n, u, v, root, gen.random_queries(n, 1 << 14, seed=seed))


@pytest.mark.parametrize("kind", ["star", "path", "heap"])
def test_special_shapes(lib, oracle_mod, kind):
    n = 1 << 13
    parent = {"star": lambda: gen.star_tree(n, root=5), "path": lambda: gen.path_tree(n, seed=2),
              "heap": lambda: gen.heap_binary_tree(n - 1)}[kind]()
    m = parent.shape[0]
    u, v = shuffled_edges(parent, 3)
    compare(lib, oracle_mod, m, u, v, 7 % m, gen.random_queries(m, 4096, seed=3))


@pytest.mark.parametrize("grasp", [None, 1000, 1])
def test_full_size_2e24(lib, oracle_mod, bench_ctx, grasp):
    n = 1 << 24
    print(f"[edges] n=2^24 grasp={grasp}", flush=True)
    parent = gen.random_tree(n, grasp, seed=21)
    u, v = shuffled_edges(parent, 21)
    compare(lib, oracle_mod, n, u, v, 12345, gen.random_queries(n, 1 << 20, seed=21), ctx=bench_ctx("single"))


@pytest.mark.parametrize("bad", ["cycle", "self_loop", "out_of_range", "repeated"])
def test_malformed_edges_flagged(lib, bad):
    n = 1000
    parent = gen.random_tree(n, None, seed=4)
    u, v = shuffled_edges(parent, 4)
    u, v = u.copy(), v.copy()
    if bad == "cycle":                 # a path whose last edge is replaced by (0, 2): cycle 0-1-2, node n-1 cut off
        u = np.arange(0, n - 1, dtype=np.int32)
        v = np.arange(1, n, dtype=np.int32)
        u[-1], v[-1] = 0, 2
    elif bad == "self_loop":
        v[0] = u[0]
    elif bad == "out_of_range":
        v[0] = n + 3
    else:
        u[1], v[1] = u[0], v[0]
    ctx = lib.default_context()
    tree = lib.et_tree_build_edges(_dev(u), _dev(v), n, 0)
    with pytest.raises(lib.EtError):
        ctx.check()
    tree.free()
