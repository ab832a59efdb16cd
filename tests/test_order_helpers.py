"""Host logic: the costliest-first orders handed to the one-launch batch
kernels (a permutation of the trees or graphs, by descending cost, equal
costs in storage order)."""
import numpy as np

import paper_2103_15217_amd as et


def _check_perm_by_cost(order, cost):
    assert order.dtype == np.int32
    assert np.array_equal(np.sort(order), np.arange(len(cost)))
    c = cost[order]
    assert np.all(c[:-1] >= c[1:])
    for i in range(len(order) - 1):  # equal costs keep their storage order
        if c[i] == c[i + 1]:
            assert order[i] < order[i + 1]


def test_fused_order_small_example():
    # costs: 10 nodes + 0 queries; 2 nodes + 400 // 4; 100 nodes + 4 // 4
    order = et.fused_order([0, 10, 12, 112], [0, 0, 400, 404])
    assert order.tolist() == [1, 2, 0]


def test_fused_order_is_a_descending_permutation():
    rng = np.random.default_rng(5)
    for T in (1, 2, 7, 300):
        sizes = rng.integers(1, 4097, T)
        sizes[rng.integers(0, T, T // 3)] = 64  # some ties
        qs = rng.integers(0, 20000, T)
        off = np.concatenate([[0], np.cumsum(sizes)])
        qoff = np.concatenate([[0], np.cumsum(qs)])
        _check_perm_by_cost(et.fused_order(off, qoff), sizes + qs // 4)


def test_fused_graph_order():
    assert et.fused_graph_order([5, 20, 3], [10, 1, 2]).tolist() == [0, 1, 2]
    assert et.fused_graph_order([4, 4, 9], [1, 1, 0]).tolist() == [2, 0, 1]
    rng = np.random.default_rng(6)
    slots = rng.integers(0, 8193, 500)
    verts = rng.integers(1, 1025, 500)
    _check_perm_by_cost(et.fused_graph_order(slots, verts), slots + 2 * verts)


def test_orders_of_empty_batches():
    assert et.fused_order([0], [0]).tolist() == []
    assert et.fused_order([0], [0]).dtype == np.int32
    assert et.fused_graph_order([], []).tolist() == []
