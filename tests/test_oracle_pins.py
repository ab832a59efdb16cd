"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library. Each test checks the oracle against
something other than itself: the paper's worked example (Section 2,
Figures 1 and 2), the paper's own DCEL construction run as written
(Section 2.1), brute-force definitions on tiny inputs, closed forms, a
library routine (networkx) and structural invariants.
"""
import json
import os

import networkx as nx
import numpy as np
import pytest

import gen
from tests import _brute as brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_fig2.json")


def _fig():
    with open(GOLDEN) as f:
        return json.load(f)


def _fig_parent(fig):
    n = 1 + max(max(e) for e in fig["tree_edges_parent_child"])
    parent = np.full(n, -1, dtype=np.int32)
    for p, c in fig["tree_edges_parent_child"]:
        parent[c] = p
    return parent


def _half_edge_pair(parent, e):
    c = e >> 1
    return (int(parent[c]), c) if e % 2 == 0 else (c, int(parent[c]))


def paper_dcel_tour(parent, head_edge, edges=None):
    """The construction of Section 2.1 run as written: array A of twin
    half-edges side by side, its lexicographically sorted copy B, first[x],
    twin = neighbour in A, next = neighbour in B (wrapping to first[x] at
    the end of x's run), succ = next(twin(e)), list split at ``head_edge``.
    ``edges`` is the input collection of undirected edges (default: the
    tree edges in child-id order). Returns the tour as a list of (x, y)
    pairs."""
    if edges is None:
        edges = [(int(parent[c]), c) for c in range(len(parent)) if parent[c] >= 0]
    A = []
    for x, y in edges:
        A += [(x, y), (y, x)]
    order = sorted(range(len(A)), key=lambda i: A[i])
    B = [A[i] for i in order]
    pos_in_B = {A[i]: b for b, i in enumerate(order)}
    first = {}
    for b, (x, _) in enumerate(B):
        first.setdefault(x, b)

    def twin(e):
        i = A.index(e)
        return A[i ^ 1]

    def nxt(e):
        b = pos_in_B[e]
        if b + 1 < len(B) and B[b + 1][0] == e[0]:
            return B[b + 1]
        return B[first[e[0]]]

    tour = [head_edge]
    while True:
        s = nxt(twin(tour[-1]))
        if s == head_edge:
            break
        tour.append(s)
    return tour, A, B, first, twin, nxt


# --------------------------------------------------------------- worked example

def test_fig1_tour_from_oracle(oracle_mod):
    fig = _fig()
    parent = _fig_parent(fig)
    t = oracle_mod.euler_tour(parent)
    pairs = [list(_half_edge_pair(parent, int(e))) for e in t["tour"]]
    assert pairs == fig["fig1_tour_in_order"]
    assert t["root"] == fig["root"]


def test_fig2_dcel_arrays_and_worked_succ():
    fig = _fig()
    parent = _fig_parent(fig)
    edges = [tuple(e) for e in fig["tree_edges_parent_child"]]
    tour, A, B, first, twin, nxt = paper_dcel_tour(parent, (0, 2), edges)
    assert [list(e) for e in A] == fig["fig2_A"]
    assert [list(e) for e in B] == fig["fig2_B"]
    assert {str(k): v for k, v in first.items()} == fig["fig2_first_B_index_of_vertex"]
    for cyc in fig["fig2_next_cycles"]:
        cyc = [tuple(e) for e in cyc]
        for i, e in enumerate(cyc):
            assert nxt(e) == cyc[(i + 1) % len(cyc)]
    ex = fig["worked_succ_example"]
    numbered = [tuple(e) for e in fig["fig1_tour_in_order"]]
    e6 = numbered[ex["edge_number"] - 1]
    assert twin(e6) == numbered[ex["twin_edge_number"] - 1]
    assert nxt(twin(e6)) == numbered[ex["succ_edge_number"] - 1]
    assert [list(e) for e in tour] == fig["fig1_tour_in_order"]


@pytest.mark.parametrize("seed", range(8))
def test_paper_dcel_tour_equals_oracle_when_parents_precede_children(oracle_mod, seed):
    # with parent id < child id (trees in generation order) the paper's
    # cyclic-after-parent child order is ascending order, so the paper's
    # construction and the oracle's DFS give the same tour
    n = 3 + seed * 5
    parent = gen.random_tree(n, [None, 1, 2, 3][seed % 4], seed=seed, relabel=False)
    t = oracle_mod.euler_tour(parent)
    root = t["root"]
    first_child = min(c for c in range(n) if parent[c] == root)
    tour, *_ = paper_dcel_tour(parent, (root, first_child))
    assert tour == [_half_edge_pair(parent, int(e)) for e in t["tour"]]


# --------------------------------------------------------------- tree statistics

@pytest.mark.parametrize("seed", range(40))
def test_tree_stats_match_definitions(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 41))
    grasp = [None, 1, 2, 5][seed % 4]
    parent = gen.random_tree(n, grasp, seed=seed)
    t = oracle_mod.euler_tour(parent)
    assert np.array_equal(t["depth"], brute.depth(parent))
    assert np.array_equal(t["size"], brute.subtree_size(parent))
    assert np.array_equal(t["pre"], brute.preorder(parent))


@pytest.mark.parametrize("n,grasp,seed", [(1, None, 0), (2, None, 1), (2000, None, 2),
                                          (2000, 1, 3), (2000, 7, 4), (4095, None, 5)])
def test_tour_invariants(oracle_mod, n, grasp, seed):
    parent = gen.random_tree(n, grasp, seed=seed)
    t = oracle_mod.euler_tour(parent)
    tour, rank, pre, size, depth = t["tour"], t["rank"], t["pre"], t["size"], t["depth"]
    root = t["root"]
    L = 2 * (n - 1)
    assert tour.shape[0] == L
    # every tree edge once in each direction; the root's ids never appear
    assert np.array_equal(np.sort(tour), np.setdiff1d(np.arange(2 * n), [2 * root, 2 * root + 1]))
    assert np.array_equal(rank[tour], np.arange(L))
    assert rank[2 * root] == -1 and rank[2 * root + 1] == -1
    nonroot = np.nonzero(parent >= 0)[0]
    # the half-edge going down precedes its twin (Section 2 footnote)
    assert np.all(rank[2 * nonroot] < rank[2 * nonroot + 1])
    assert np.array_equal(np.sort(pre), np.arange(n))
    assert size[root] == n and depth[root] == 0 and pre[root] == 0
    p = parent[nonroot]
    assert np.all(depth[nonroot] == depth[p] + 1)
    assert np.all((pre[nonroot] > pre[p]) & (pre[nonroot] < pre[p] + size[p]))
    child_sum = np.bincount(p, weights=size[nonroot], minlength=n)
    assert np.array_equal(size, 1 + child_sum.astype(np.int64))
    # subtree = interval of the tour: 2 * (size - 1) half-edges inside
    assert np.all(rank[2 * nonroot + 1] - rank[2 * nonroot] == 2 * size[nonroot] - 1)
    # children are visited in ascending id order
    order = np.lexsort((nonroot, p))
    same = p[order][1:] == p[order][:-1]
    assert np.all(pre[nonroot[order]][1:][same] > pre[nonroot[order]][:-1][same])


@pytest.mark.parametrize("seed", range(5))
def test_tour_matches_networkx_dfs(oracle_mod, seed):
    parent = gen.random_tree(300, [None, 3][seed % 2], seed=seed)
    t = oracle_mod.euler_tour(parent)
    G = nx.Graph()
    G.add_nodes_from(range(len(parent)))
    # insertion order of the adjacency = ascending neighbour id
    for v in range(len(parent)):
        for c in sorted(np.nonzero(parent == v)[0].tolist()):
            G.add_edge(v, int(c))
    # networkx reports a 'reverse' step as (parent, child); the tour walks it
    # from the child back up to the parent
    seq = [(u, v) if d == "forward" else (v, u)
           for u, v, d in nx.dfs_labeled_edges(G, source=t["root"])
           if d in ("forward", "reverse") and u != v]
    assert seq == [_half_edge_pair(parent, int(e)) for e in t["tour"]]


def test_generator_mean_depth(oracle_mod):
    # Section 3.2: mean depth about ln n for unbounded grasp, about
    # n / (grasp + 1) otherwise
    n = 1 << 18
    d = oracle_mod.euler_tour(gen.random_tree(n, None, seed=3))["depth"].mean()
    harmonic = np.sum(1.0 / np.arange(1, n + 1))
    assert abs(d - (harmonic - 1)) < 0.05 * harmonic  # 0-based ids: E[depth of i] = H_i
    assert abs(d - np.log(n)) < 0.1 * np.log(n)
    for g in (16, 1000):
        d = oracle_mod.euler_tour(gen.random_tree(n, g, seed=4))["depth"].mean()
        assert abs(d - n / (g + 1)) < 0.05 * n / (g + 1)
    d = oracle_mod.euler_tour(gen.random_tree(n, 1, seed=5))["depth"].mean()
    assert d == (n - 1) / 2


def test_oracle_rejects_non_trees(oracle_mod):
    bad = [np.array([-1, -1, 0], np.int32),           # two roots
           np.array([1, 2, 0], np.int32),             # no root
           np.array([-1, 2, 1, 0], np.int32),         # cycle 1-2 beside the root
           np.array([-1, 7, 0], np.int32),            # id out of range
           np.array([-1, 1], np.int32)]               # self parent
    for p in bad:
        with pytest.raises(oracle_mod.OracleInputError):
            oracle_mod.euler_tour(p)


# --------------------------------------------------------------- list ranking

@pytest.mark.parametrize("seed", range(10))
def test_list_rank_vs_pointer_jumping(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 3000))
    nlists = int(rng.integers(1, min(L, 9) + 1))
    unused = rng.random(L) < 0.1
    ids = rng.permutation(np.nonzero(~unused)[0])
    if ids.shape[0] < nlists:
        ids = rng.permutation(L)
        unused[:] = False
    cuts = np.sort(rng.choice(np.arange(1, ids.shape[0]), size=nlists - 1, replace=False)) if nlists > 1 else []
    succ = np.full(L, -2, dtype=np.int32)
    heads = []
    for part in np.split(ids, cuts):
        succ[part[:-1]] = part[1:]
        succ[part[-1]] = -1
        heads.append(int(part[0]))
    r = oracle_mod.list_rank(succ, np.array(heads, np.int32))
    assert np.array_equal(r, brute.list_rank_pointer_jumping(succ, heads))


def _random_lists(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 3000))
    nlists = int(rng.integers(1, min(L, 9) + 1))
    unused = rng.random(L) < 0.1
    ids = rng.permutation(np.nonzero(~unused)[0])
    if ids.shape[0] < nlists:
        ids = rng.permutation(L)
    cuts = np.sort(rng.choice(np.arange(1, ids.shape[0]), size=nlists - 1, replace=False)) if nlists > 1 else []
    succ = np.full(L, -2, dtype=np.int32)
    heads = []
    for part in np.split(ids, cuts):
        succ[part[:-1]] = part[1:]
        succ[part[-1]] = -1
        heads.append(int(part[0]))
    return succ, np.array(heads, np.int32), rng


@pytest.mark.parametrize("seed", range(6))
def test_list_scan_unit_weights_are_ranks_plus_one(oracle_mod, seed):
    succ, heads, _ = _random_lists(100 + seed)
    s, r = oracle_mod.list_scan(succ, np.ones_like(succ), heads)
    used = succ != -2
    assert np.array_equal(s[used], r[used] + 1)
    assert np.array_equal(r, brute.list_rank_pointer_jumping(succ, list(heads)))
    assert not s[~used].any()


@pytest.mark.parametrize("seed", range(6))
def test_list_scan_random_weights_by_walking(oracle_mod, seed):
    # weights anywhere in int32, sums wrapping modulo 2^32: each list walked in Python
    succ, heads, rng = _random_lists(200 + seed)
    w = rng.integers(-(1 << 31), 1 << 31, size=succ.shape[0]).astype(np.int32)
    s, _ = oracle_mod.list_scan(succ, w, heads)
    want = np.zeros_like(succ)
    for h in heads:
        acc, e = 0, int(h)
        while e != -1:
            acc = (acc + int(w[e])) % (1 << 32)
            want[e] = acc - (1 << 32) if acc >= (1 << 31) else acc
            e = int(succ[e])
    assert np.array_equal(s, want)


@pytest.mark.parametrize("seed", range(4))
def test_list_scan_by_doubling_and_cumsum(oracle_mod, seed):
    # another route to the same sums: every element finds its list's tail by
    # pointer doubling, elements are ordered by (tail, pointer-jumping rank),
    # and the weights are summed by numpy's cumsum within each list
    succ, heads, rng = _random_lists(300 + seed)
    w = rng.integers(-(1 << 31), 1 << 31, size=succ.shape[0]).astype(np.int32)
    s, r = oracle_mod.list_scan(succ, w, heads)
    used = np.flatnonzero(succ != -2)
    tail = np.where(succ == -1, np.arange(succ.shape[0]), succ).astype(np.int64)
    for _ in range(int(np.ceil(np.log2(max(2, succ.shape[0])))) + 1):
        tail = np.where(tail >= 0, tail[np.maximum(tail, 0)], tail)
    rank = brute.list_rank_pointer_jumping(succ, list(heads))
    order = used[np.lexsort((rank[used], tail[used]))]
    csum = np.cumsum(w[order].astype(np.int64))
    starts = np.flatnonzero(np.r_[True, tail[order][1:] != tail[order][:-1]])
    base = np.repeat(np.r_[0, csum][starts], np.diff(np.r_[starts, order.shape[0]]))
    want = np.zeros_like(succ)
    want[order] = ((csum - base) % (1 << 32)).astype(np.uint32).view(np.int32)
    assert np.array_equal(s, want)
    assert np.array_equal(r, rank)


@pytest.mark.parametrize("grasp", [None, 5, 1])
def test_list_scan_of_tour_weights_gives_depth(oracle_mod, grasp):
    # +1 on every down half-edge, -1 on every up one: the sum at 2c is the
    # depth of c (Section 2), which the DFS tour computes on its own
    parent = gen.random_tree(5000, grasp, seed=7)
    succ, head = oracle_mod.tree_succ(parent)
    w = np.where(np.arange(succ.shape[0]) % 2 == 0, 1, -1).astype(np.int32)
    s, _ = oracle_mod.list_scan(succ, w, np.array([head], np.int32))
    depth = oracle_mod.euler_tour(parent)["depth"]
    c = np.flatnonzero(parent >= 0)
    assert np.array_equal(s[2 * c], depth[c])
    assert np.array_equal(s[2 * c + 1], depth[c] - 1)


def test_list_rank_rejects_bad_lists(oracle_mod):
    with pytest.raises(oracle_mod.OracleInputError):   # cycle reachable from the head
        oracle_mod.list_rank(np.array([1, 2, 1], np.int32), np.array([0], np.int32))
    with pytest.raises(oracle_mod.OracleInputError):   # element not on any list
        oracle_mod.list_rank(np.array([-1, -1], np.int32), np.array([0], np.int32))


# --------------------------------------------------------------- LCA

@pytest.mark.parametrize("seed", range(30))
def test_lca_bruteforce_all_pairs(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 30))
    parent = gen.random_tree(n, [None, 1, 3][seed % 3], seed=seed)
    qx, qy = [a.ravel().astype(np.int32) for a in np.meshgrid(np.arange(n), np.arange(n))]
    expect = np.array([brute.lca(parent, int(x), int(y)) for x, y in zip(qx, qy)])
    depth = oracle_mod.euler_tour(parent)["depth"]
    assert np.array_equal(oracle_mod.lca_climb(parent, depth, qx, qy), expect)
    assert np.array_equal(oracle_mod.lca_offline(parent, qx, qy), expect)


def test_lca_networkx(oracle_mod):
    parent = gen.random_tree(400, None, seed=11)
    qx, qy = gen.random_queries(400, 3000, seed=11)
    G = nx.DiGraph()
    G.add_nodes_from(range(400))
    G.add_edges_from((int(parent[c]), c) for c in range(400) if parent[c] >= 0)
    ref = dict(nx.tree_all_pairs_lowest_common_ancestor(G, pairs=list(zip(qx.tolist(), qy.tolist()))))
    expect = np.array([ref[(int(x), int(y))] for x, y in zip(qx, qy)])
    assert np.array_equal(oracle_mod.lca_offline(parent, qx, qy), expect)


def test_lca_closed_forms(oracle_mod):
    # path: the LCA is the endpoint nearer the root
    n = 5000
    parent = gen.path_tree(n)
    qx, qy = gen.random_queries(n, 20000, seed=1)
    assert np.array_equal(oracle_mod.lca_offline(parent, qx, qy), np.minimum(qx, qy))
    # star: distinct leaves meet at the root
    parent = gen.star_tree(n, root=17)
    out = oracle_mod.lca_offline(parent, qx, qy)
    assert np.array_equal(out, np.where(qx == qy, qx, 17))
    # heap-shaped binary tree, 1-based heap labels h = v + 1: the LCA label
    # is the longest common binary prefix of the two labels
    n = (1 << 12) - 1 + 777
    parent = gen.heap_binary_tree(n)
    hx, hy = qx.astype(np.int64) % n + 1, qy.astype(np.int64) % n + 1
    bx = np.floor(np.log2(hx)).astype(np.int64)
    by = np.floor(np.log2(hy)).astype(np.int64)
    ax = hx >> np.maximum(bx - by, 0)
    ay = hy >> np.maximum(by - bx, 0)
    diff = ax ^ ay
    shift = np.where(diff > 0, np.floor(np.log2(np.maximum(diff, 1))).astype(np.int64) + 1, 0)
    expect = (ax >> shift) - 1
    out = oracle_mod.lca_offline(parent, (hx - 1).astype(np.int32), (hy - 1).astype(np.int32))
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("grasp", [None, 64, 1])
def test_lca_climb_agrees_with_offline(oracle_mod, grasp):
    n = 1 << 14
    parent = gen.random_tree(n, grasp, seed=9)
    qx, qy = gen.random_queries(n, n, seed=9)
    depth = oracle_mod.euler_tour(parent)["depth"]
    assert np.array_equal(oracle_mod.lca_climb(parent, depth, qx, qy),
                          oracle_mod.lca_offline(parent, qx, qy))


# --------------------------------------------------------------- Schieber-Vishkin tables

def _ctz(x):
    return (x & -x).bit_length() - 1


def _msb(x):
    return x.bit_length() - 1


def sv_query(T, depth, x, y):
    """Schieber-Vishkin query (Section 3.1) on the oracle's tables."""
    inl, asc, hp, hd = T["inlabel"], T["asc"], T["head_parent"], T["head_depth"]
    a, b = int(inl[x]), int(inl[y])
    if a == b:
        return x if depth[x] <= depth[y] else y
    i = max(_ctz(a), _ctz(b), _msb(a ^ b))
    common = int(asc[x]) & int(asc[y]) & ~((1 << i) - 1)
    j = _ctz(common)

    def lift(v, lab, A):
        if _ctz(lab) == j:
            return v, int(depth[v])
        k = _msb(A & ((1 << j) - 1))
        w = ((lab >> (k + 1)) << (k + 1)) | (1 << k)
        return int(hp[w]), int(hd[w])

    xv, xd = lift(x, a, int(asc[x]))
    yv, yd = lift(y, b, int(asc[y]))
    return xv if xd <= yd else yv


@pytest.mark.parametrize("seed", range(60))
def test_sv_tables_and_query(oracle_mod, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 48))
    parent = gen.random_tree(n, [None, 1, 2, 5][seed % 4], seed=seed)
    t = oracle_mod.euler_tour(parent)
    T = oracle_mod.sv_tables(parent, t["depth"], t["pre"], t["size"])
    inl = T["inlabel"].astype(np.int64)
    pre, size = t["pre"].astype(np.int64), t["size"].astype(np.int64)
    # closed form of the inlabel: keep the bits of j above the highest bit
    # in which p-1 and j differ (p = pre+1, j = pre+size)
    p, j = pre + 1, pre + size
    k = np.array([_msb(int(a) ^ int(b)) for a, b in zip(p - 1, j)])
    assert np.array_equal(inl, (j >> k) << k)
    # path partition: nodes sharing a label form one vertical path
    for lab in np.unique(inl):
        nodes = np.nonzero(inl == lab)[0]
        tops = [v for v in nodes if parent[v] < 0 or inl[parent[v]] != lab]
        assert len(tops) == 1
        d = t["depth"][nodes]
        assert sorted(d.tolist()) == list(range(d.min(), d.min() + len(nodes)))
        for v in nodes:
            if v != tops[0]:
                assert inl[parent[v]] == lab
    # inorder property: a descendant's label lies in the ancestor label's subtree of B
    for v in range(n):
        for a in brute.ancestors(parent, v):
            h = _ctz(int(inl[a]))
            assert abs(int(inl[v]) - int(inl[a])) < (1 << h)
            assert _ctz(int(inl[v])) <= h
    # ascendant by walking to the root
    for v in range(n):
        acc = 0
        for a in brute.ancestors(parent, v):
            acc |= 1 << _ctz(int(inl[a]))
        assert int(T["asc"][v]) == acc
    # query formula against brute force on all pairs
    for x in range(n):
        for y in range(n):
            assert sv_query(T, t["depth"], x, y) == brute.lca(parent, x, y)


# --------------------------------------------------------------- bridges

@pytest.mark.parametrize("seed", range(60))
def test_bridges_bruteforce_multigraphs(oracle_mod, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(1, 11))
    m = int(rng.integers(0, 15))
    row_ptr, col = gen.random_multigraph(n, m, seed=seed, loops=True, multi=True)
    mask, cnt = oracle_mod.bridges(row_ptr, col)
    flags, bcnt = brute.bridge_slots(row_ptr, col)
    assert np.array_equal(oracle_mod.mask_to_bool(mask, len(col)), flags)
    assert cnt == bcnt


def test_bridges_networkx_simple_graphs(oracle_mod):
    for seed in range(6):
        n = 300
        row_ptr, col = gen.random_multigraph(n, 330 + 40 * seed, seed=seed, loops=False, multi=False)
        G = nx.Graph()
        G.add_nodes_from(range(n))
        src = np.repeat(np.arange(n), np.diff(row_ptr))
        G.add_edges_from(zip(src.tolist(), col.tolist()))
        ref = {frozenset(e) for e in nx.bridges(G)}
        flags = oracle_mod.mask_to_bool(oracle_mod.bridges(row_ptr, col)[0], len(col))
        got = {frozenset((int(a), int(b))) for a, b, f in zip(src, col, flags) if f}
        assert got == ref


def test_bridges_special_graphs(oracle_mod):
    parent = gen.random_tree(500, None, seed=1)
    rp, col = gen.tree_graph(parent)
    mask, cnt = oracle_mod.bridges(rp, col)
    assert cnt == 499 and oracle_mod.mask_to_bool(mask, len(col)).all()
    for crp, ccol in (gen.cycle_graph(400), gen.complete_graph(30)):
        mask, cnt = oracle_mod.bridges(crp, ccol)
        assert cnt == 0 and not oracle_mod.mask_to_bool(mask, len(ccol)).any()
    # every edge doubled: no bridges at all
    src = np.repeat(np.arange(500), np.diff(rp))
    rp2, col2 = gen.csr_from_pairs(500, np.concatenate([src, src]), np.concatenate([col, col]))
    mask, cnt = oracle_mod.bridges(rp2, col2)
    assert cnt == 0


def test_bridges_planted_chains(oracle_mod):
    rp, col, info = gen.planted_bridge_graph(n=1 << 15, m=1 << 18, chains=64, max_chain=40, seed=2)
    mask, cnt = oracle_mod.bridges(rp, col)
    flags = oracle_mod.mask_to_bool(mask, len(col))
    src = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    bridge_pairs = {(int(a), int(b)) for a, b, f in zip(src, col, flags) if f}
    for a, b in info["chain_edges"]:
        assert (int(a), int(b)) in bridge_pairs and (int(b), int(a)) in bridge_pairs
    assert cnt >= len(info["chain_edges"])


# --------------------------------------------------------------- tour from an edge list (Section 2.1)

def _half_edge_pairs(eu, ev):
    src = np.empty(2 * len(eu), dtype=np.int64)
    dst = np.empty(2 * len(eu), dtype=np.int64)
    src[0::2], dst[0::2] = eu, ev
    src[1::2], dst[1::2] = ev, eu
    return src, dst


def test_fig1_tour_from_edge_list(oracle_mod):
    fig = _fig()
    E = np.array(fig["tree_edges_parent_child"])
    t = oracle_mod.euler_tour_edges(6, E[:, 0], E[:, 1], fig["root"])
    src, dst = _half_edge_pairs(E[:, 0], E[:, 1])
    pairs = [[int(src[h]), int(dst[h])] for h in t["tour"]]
    assert pairs == fig["fig1_tour_in_order"]
    # the worked example: succ of tour edge 6 is tour edge 7, through the twin of edge 6 (tour edge 1)
    ex = fig["worked_succ_example"]
    e6 = int(t["tour"][ex["edge_number"] - 1])
    assert int(t["tour"][ex["twin_edge_number"] - 1]) == e6 ^ 1
    assert int(t["succ"][e6]) == int(t["tour"][ex["succ_edge_number"] - 1])


@pytest.mark.parametrize("seed", range(30))
def test_edge_list_tour_is_the_cyclic_dfs(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    parent = gen.random_tree(n, [None, 1, 2, 4][seed % 4], seed=seed)
    edges = [(int(parent[c]), c) for c in range(n) if parent[c] >= 0]
    flip = rng.random(len(edges)) < 0.5                  # input orientation and order are arbitrary
    edges = [(y, x) if f else (x, y) for (x, y), f in zip(edges, flip)]
    edges = [edges[i] for i in rng.permutation(len(edges))]
    root = int(rng.integers(n))
    eu = np.array([e[0] for e in edges], dtype=np.int32)
    ev = np.array([e[1] for e in edges], dtype=np.int32)
    t = oracle_mod.euler_tour_edges(n, eu, ev, root)
    tour, par, dep, pre, size = brute.cyclic_dfs_tour(n, edges, root)
    src, dst = _half_edge_pairs(eu, ev)
    assert [(int(src[h]), int(dst[h])) for h in t["tour"]] == tour
    assert list(t["parent"]) == par and list(t["depth"]) == dep
    assert list(t["pre"]) == pre and list(t["size"]) == size
    assert all(t["rank"][t["tour"]] == np.arange(len(t["tour"])))


@pytest.mark.parametrize("seed", range(6))
def test_edge_list_tour_matches_ascending_oracle_when_order_agrees(oracle_mod, seed):
    # rooted at 0 with every parent id below its children's, the cyclic order
    # after the parent is ascending order: both constructions give one tour
    n = 5 + 7 * seed
    parent = gen.random_tree(n, [None, 1, 3][seed % 3], seed=seed, relabel=False)
    eu = parent[1:].astype(np.int32)
    ev = np.arange(1, n, dtype=np.int32)
    t = oracle_mod.euler_tour_edges(n, eu, ev, 0)
    ref = oracle_mod.euler_tour(parent)
    src, dst = _half_edge_pairs(eu, ev)
    assert [(int(src[h]), int(dst[h])) for h in t["tour"]] == \
        [_half_edge_pair(parent, int(e)) for e in ref["tour"]]
    for k in ("depth", "pre", "size"):
        assert np.array_equal(t[k], ref[k]), k
    assert np.array_equal(t["parent"], parent)


@pytest.mark.parametrize("bad", ["cycle", "self_loop", "out_of_range", "too_few", "isolated_root"])
def test_edge_list_malformed(oracle_mod, bad):
    eu, ev, n, root = [0, 1, 2], [1, 2, 3], 4, 0
    if bad == "cycle":
        eu, ev = [0, 1, 2], [1, 2, 0]                      # 3 edges on 4 nodes: node 3 cut off
    elif bad == "self_loop":
        eu, ev = [0, 1, 2], [1, 2, 2]
    elif bad == "out_of_range":
        ev = [1, 2, 4]
    elif bad == "too_few":
        eu, ev = [0, 1], [1, 2]
    else:
        eu, ev, root = [1, 1, 2], [2, 3, 3], 0            # root 0 has no edge (and 1-2-3 is a cycle)
    with pytest.raises(oracle_mod.OracleInputError):
        oracle_mod.euler_tour_edges(n, np.array(eu), np.array(ev), root)


def test_edge_list_single_node(oracle_mod):
    t = oracle_mod.euler_tour_edges(1, np.zeros(0, np.int32), np.zeros(0, np.int32), 0)
    assert t["tour"].shape[0] == 0
    assert list(t["parent"]) == [-1] and list(t["size"]) == [1] and list(t["pre"]) == [0]


# --------------------------------------------------------------- scale-free generator (Section 3.2)

def test_ba_tree_degree_distribution():
    # preferential attachment with one edge per node: P(deg = k) = 4 / (k (k+1) (k+2))
    n = 1 << 20
    p = gen.ba_tree(n, seed=3, relabel=False)
    assert p[0] == -1 and np.all(p[1:] >= 0) and np.all(p[1:] < np.arange(1, n))
    deg = np.bincount(p[1:], minlength=n) + (np.arange(n) > 0)
    for k in (1, 2, 3, 4, 8):
        expect = 4.0 / (k * (k + 1) * (k + 2))
        assert abs(np.mean(deg == k) - expect) < 5 * np.sqrt(expect / n) + 1e-4, k


def test_ba_tree_small_cases_and_relabel(oracle_mod):
    assert list(gen.ba_tree(1, seed=0)) == [-1]
    assert sorted(gen.ba_tree(2, seed=0).tolist()) == [-1, 0] or sorted(gen.ba_tree(2, seed=0).tolist()) == [-1, 1]
    p = gen.ba_tree(5000, seed=4)
    t = oracle_mod.euler_tour(p)                         # a valid tree: the oracle accepts it
    assert t["size"][t["root"]] == 5000
