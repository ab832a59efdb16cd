"""MI355X (gfx950) Euler-tour library: list ranking, Euler tour of a rooted
tree with depth / preorder / subtree size, Inlabel LCA queries, and
Tarjan-Vishkin bridges, after Polak, Siwiec and Stobierski, "Euler Meets
GPU: Practical Graph Algorithms with Theoretical Guarantees".

The work runs in the hand-written HIP kernels of ``libet.so``; the C ABI is
``include/et.h`` and :mod:`paper_2103_15217_amd.et` is its thin binding.
"""
from .et import (BatchGraph, BridgesBatchGraph, BridgesFusedGraph, Context, FusedBatchGraph, EtError, SplitBatchGraph, Tree, default_context, et_bridges,
                 et_bridges_batch, et_bridges_batch_fused, et_bridges_ck, et_lca, et_lca_batch, et_lca_batch_fused, et_lca_naive, fused_order, fused_graph_order,
                 et_levels, et_list_rank, et_list_scan, et_tree_build, et_tree_build_batch, et_tree_build_edges,
                 tree_footprint, bridges_footprint, version, LIB_PATH, FUSED_MAX_NODES, FUSED_MAX_VERTICES,
                 FUSED_MAX_SLOTS)

__all__ = ["BatchGraph", "BridgesBatchGraph", "BridgesFusedGraph", "Context", "FusedBatchGraph", "EtError", "SplitBatchGraph", "Tree", "default_context", "et_bridges",
           "et_bridges_batch", "et_bridges_batch_fused", "et_bridges_ck", "et_lca", "et_lca_batch", "et_lca_batch_fused", "et_lca_naive", "fused_order", "fused_graph_order", "et_levels",
           "et_list_rank", "et_list_scan", "et_tree_build", "et_tree_build_batch", "et_tree_build_edges",
           "tree_footprint", "bridges_footprint", "version", "LIB_PATH", "FUSED_MAX_NODES", "FUSED_MAX_VERTICES",
           "FUSED_MAX_SLOTS"]
