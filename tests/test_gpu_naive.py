"""GPU parity of the naive LCA algorithm (Section 3.1, "The Naive
Algorithm"): levels by pointer jumping must equal the oracle's depths and
the climbing queries the oracle's LCAs, bit for bit."""
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


def run_naive(lib, parent, qx=None, qy=None):
    ctx = lib.default_context()
    d_parent = _dev(parent)
    level = lib.et_levels(d_parent)
    out = None
    if qx is not None:
        out = _np(lib.et_lca_naive(d_parent, level, _dev(qx), _dev(qy)))
    lv = _np(level)
    ctx.check()
    return lv, out


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64])
@pytest.mark.parametrize("grasp", [None, 2, 1])
def test_small_trees_all_pairs(lib, oracle_mod, n, grasp):
    parent = gen.random_tree(n, grasp, seed=n)
    xs, ys = np.meshgrid(np.arange(n), np.arange(n))
    qx, qy = xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)
    lv, out = run_naive(lib, parent, qx, qy)
    assert np.array_equal(lv, oracle_mod.euler_tour(parent)["depth"])
    assert np.array_equal(out, oracle_mod.lca_offline(parent, qx, qy))


@pytest.mark.parametrize("grasp", [None, 64, 1])
@pytest.mark.parametrize("seed", [0, 1])
def test_medium_trees(lib, oracle_mod, grasp, seed):
    n = (1 << 16) + 37                                   # several workgroups and a ragged tail
    parent = gen.random_tree(n, grasp, seed=seed)
    qx, qy = gen.random_queries(n, 1 << 14, seed=seed)
    lv, out = run_naive(lib, parent, qx, qy)
    assert np.array_equal(lv, oracle_mod.euler_tour(parent)["depth"])
    assert np.array_equal(out, oracle_mod.lca_offline(parent, qx, qy))


@pytest.mark.parametrize("kind", ["path", "star", "heap", "caterpillar"])
def test_special_shapes(lib, oracle_mod, kind):
    n = 1 << 14
    parent = {"path": lambda: gen.path_tree(n, seed=3), "star": lambda: gen.star_tree(n, root=777),
              "heap": lambda: gen.heap_binary_tree(n - 1),
              "caterpillar": lambda: gen.caterpillar_tree(1000, 5, seed=4)}[kind]()
    m = parent.shape[0]
    qx, qy = gen.random_queries(m, 4096, seed=5)
    lv, out = run_naive(lib, parent, qx, qy)
    assert np.array_equal(lv, oracle_mod.euler_tour(parent)["depth"])
    assert np.array_equal(out, oracle_mod.lca_offline(parent, qx, qy))


def test_agrees_with_inlabel_queries(lib):
    n = 1 << 18
    parent = gen.random_tree(n, None, seed=9)
    qx, qy = gen.random_queries(n, 1 << 18, seed=9)
    _, naive = run_naive(lib, parent, qx, qy)
    tree = lib.et_tree_build(_dev(parent))
    sv = _np(tree.lca(_dev(qx), _dev(qy)))
    tree.free()
    lib.default_context().check()
    assert np.array_equal(naive, sv)


@pytest.mark.parametrize("grasp", [None, 1000, 1])
def test_full_size_levels(lib, oracle_mod, grasp):
    n = 1 << 24
    parent = gen.random_tree(n, grasp, seed=11)
    print(f"[naive] levels n=2^24 grasp={grasp}", flush=True)
    if grasp == 1:
        lv, _ = run_naive(lib, parent)                   # climbing a 2^24-node path is out of reach
    else:
        q = (1 << 20) if grasp is None else (1 << 14)
        qx, qy = gen.random_queries(n, q, seed=12)
        lv, out = run_naive(lib, parent, qx, qy)
        assert np.array_equal(out, oracle_mod.lca_offline(parent, qx, qy))
    assert np.array_equal(lv, oracle_mod.euler_tour(parent)["depth"])


@pytest.mark.parametrize("bad", ["cycle", "two_roots", "no_root", "out_of_range"])
def test_malformed_parent_flagged(lib, bad):
    parent = gen.random_tree(1000, None, seed=2).copy()
    root = int(np.flatnonzero(parent == -1)[0])
    other = (root + 1) % 1000
    if bad == "cycle":
        a, b = [v for v in range(1000) if v != root][:2]
        parent[a], parent[b] = b, a                      # a 2-cycle cut off from the root
    elif bad == "two_roots":
        parent[other] = -1
    elif bad == "no_root":
        parent[root] = other
    else:
        parent[other] = 5000
    ctx = lib.default_context()
    lib.et_levels(_dev(parent))
    with pytest.raises(lib.EtError):
        ctx.check()


def test_bad_queries_and_levels_flagged(lib, oracle_mod):
    n = 4096
    parent = gen.random_tree(n, 8, seed=6)
    ctx = lib.default_context()
    d_parent = _dev(parent)
    level = lib.et_levels(d_parent)
    ctx.check()
    out = _np(lib.et_lca_naive(d_parent, level, _dev([0, n, -1]), _dev([1, 0, 2])))
    assert out[1] == -1 and out[2] == -1
    with pytest.raises(lib.EtError):
        ctx.check()
    import torch
    qx, qy = np.arange(64, dtype=np.int32), np.arange(64, 128, dtype=np.int32)
    truth = oracle_mod.lca_offline(parent, qx, qy)
    for wrong in (torch.zeros_like(level), torch.full_like(level, n)):   # levels that do not fit the tree
        out = _np(lib.et_lca_naive(d_parent, wrong, _dev(qx), _dev(qy)))
        # every climb stays bounded: a query either fails (-1, flagged) or, when the
        # lock-step climb happens to meet, still lands on the true LCA
        assert np.all((out == -1) | (out == truth)) and np.any(out == -1)
        with pytest.raises(lib.EtError):
            ctx.check()
