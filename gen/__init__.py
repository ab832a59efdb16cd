"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random instances; it holds none of the Euler-tour,
LCA or bridge arithmetic. Every generator takes an explicit seed and uses
``numpy.random.default_rng`` (PCG64), so an instance is a pure function of
its arguments.

Trees follow the paper's LCA datasets (Section 3.2): node ``i >= 1`` picks its
parent uniformly among the ``grasp`` nodes that precede it (grasp = n gives
the shallow random recursive tree, grasp = 1 a path), and the node ids are
then mapped through a random permutation so ids carry no structure. The
scale-free trees of the same section come from preferential attachment
(``ba_tree``). Queries are uniform pairs over the node ids.

Graphs stand in for the bridge datasets of Section 4.2 (Table 1), which are
public downloads and not used here: sparse, low-diameter random blobs joined
by planted chains whose edges are bridges by construction.
"""
from .trees import (random_tree, random_queries, path_tree, star_tree,
                    heap_binary_tree, caterpillar_tree, forest_batch, ba_tree)
from .graphs import (planted_bridge_graph, random_multigraph, csr_from_pairs,
                     cycle_graph, complete_graph, tree_graph)

__all__ = [
    "random_tree", "random_queries", "path_tree", "star_tree",
    "heap_binary_tree", "caterpillar_tree", "forest_batch", "ba_tree",
    "planted_bridge_graph", "random_multigraph", "csr_from_pairs",
    "cycle_graph", "complete_graph", "tree_graph",
]
