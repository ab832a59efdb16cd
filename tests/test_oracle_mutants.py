"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it with gcc, points the oracle wrapper at the mutant and runs the pin
battery of test_oracle_pins.py; at least one pin must fail. The committed
oracle itself is untouched.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "et_oracle.c")

MUTANTS = {
    # children visited in descending id order
    "child_order": ("for (int32_t v = 0; v < n; ++v)\n        if (parent[v] >= 0) cidx[fill[parent[v]]++] = v;",
                    "for (int32_t v = n - 1; v >= 0; --v)\n        if (parent[v] >= 0) cidx[fill[parent[v]]++] = v;"),
    # preorder numbered from 1
    "pre_base": ("int32_t visited = 0;    /* next preorder number */",
                 "int32_t visited = 1;    /* next preorder number */"),
    # subtree size without the node itself
    "size_self": ("int32_t s = 1;\n            for (int32_t k = cptr[u]",
                  "int32_t s = 0;\n            for (int32_t k = cptr[u]"),
    # depth not incremented
    "depth": ("d[c] = d[u] + 1;", "d[c] = d[u];"),
    # ranks reported off by one
    "rank_origin": ("if (rank) rank[2 * c] = (int32_t)pos;", "if (rank) rank[2 * c] = (int32_t)pos + 1;"),
    # offline LCA unites in the wrong direction (the parent's set under the child's)
    "lca_union": ("up[a] = b;\n            anc[b] = p;", "up[b] = a;\n            anc[b] = p;"),
    # climbing LCA reports the meeting point's parent
    "lca_climb": ("while (x != y) { x = parent[x]; y = parent[y]; }\n        out[i] = x;",
                  "while (x != y) { x = parent[x]; y = parent[y]; }\n        out[i] = parent[x] >= 0 ? parent[x] : x;"),
    # offline LCA answers a query when the other end is not finished yet
    "lca_done": ("if (done[other]) out[i] = anc[dsu_find(up, other)];",
                 "if (!done[other]) out[i] = anc[dsu_find(up, other)];"),
    # inlabel = the interval's largest member instead of the most trailing zeros
    "inlabel": ("for (int t = 31; t >= 0 && !best; --t) {", "for (int t = 0; t >= 0 && !best; --t) {"),
    # ascendant without the node's own level
    "asc_own": ("asc[v] = (parent[v] < 0) ? own : (asc[parent[v]] | own);",
                "asc[v] = (parent[v] < 0) ? own : asc[parent[v]];"),
    # head table stores the top's depth instead of its parent's
    "head_depth": ("head_depth[inlabel[v]] = depth[v] - 1;", "head_depth[inlabel[v]] = depth[v];"),
    # every copy of the parent edge skipped (parallel edges then look like bridges)
    "bridge_multi": ("if (w == par[u] && back_slot[u] == -1) { back_slot[u] = k; continue; }",
                     "if (w == par[u]) { back_slot[u] = k; continue; }"),
    # non-strict bridge comparison
    "bridge_cmp": ("if (low[u] > disc[p]) {", "if (low[u] >= disc[p]) {"),
    # next() wraps to the end of the source's run instead of its start
    "dcel_wrap": ("succ[e] = (k + 1 < first[x + 1]) ? B[k + 1] : B[first[x]];",
                  "succ[e] = (k + 1 < first[x + 1]) ? B[k + 1] : B[first[x + 1] - 1];"),
    # successor taken as next(e) instead of next(twin(e))
    "dcel_no_twin": ("const int32_t t = (int32_t)(e ^ 1);", "const int32_t t = (int32_t)e;"),
    # a half-edge counted as going down when it follows its twin
    "dcel_direction": ("if (rank[e] < rank[tw]) {                          /* down into dst[e] */",
                       "if (rank[e] > rank[tw]) {                          /* down into dst[e] */"),
    # list ranks start at 1
    "list_rank_origin": ("int32_t r = 0;\n        while (e != -1) {", "int32_t r = 1;\n        while (e != -1) {"),
    # only the first list of a multi-list input is walked
    "list_rank_heads": ("for (int32_t h = 0; h < nheads; ++h) {", "for (int32_t h = 0; h < nheads && h < 1; ++h) {"),
    # list scan exclusive instead of inclusive
    "list_scan_excl": ("acc += (uint32_t)weight[e];\n            sum[e] = (int32_t)acc;",
                       "sum[e] = (int32_t)acc;\n            acc += (uint32_t)weight[e];"),
    # low values not passed up from a finished child
    "bridge_low_up": ("if (low[u] < low[p]) low[p] = low[u];", "(void)low[p];"),
    # only the parent-to-child slot of a bridge marked
    "bridge_one_slot": ("mask[b >> 5] |= 1u << (b & 31);", "(void)b;"),
    # head table records the path top instead of its parent
    "head_parent": ("head_parent[inlabel[v]] = p;", "head_parent[inlabel[v]] = v;"),
    # inlabel interval taken as (pre, pre + size] without its first member
    "inlabel_lo": ("if (m >= lo && m != 0) best = m;", "if (m > lo && m != 0) best = m;"),
    # the edge-list tour cut after the root's first half-edge instead of before it
    "dcel_cut": ("if (succ[e] == head) { succ[e] = -1; break; }", "if (e == head) { succ[e] = -1; break; }"),
    # the lexicographic order of B built by source only (the target sort dropped)
    "dcel_sort": ("for (int64_t h = 0; h < L; ++h) tmp[cnt[dst[h]]++] = (int32_t)h;",
                  "for (int64_t h = 0; h < L; ++h) tmp[h] = (int32_t)h;"),
}


def battery(mod):
    """Run the pins against the current oracle library; return the first failure."""
    checks = [
        lambda: pins.test_fig1_tour_from_oracle(mod),
        *[lambda s=s: pins.test_paper_dcel_tour_equals_oracle_when_parents_precede_children(mod, s)
          for s in range(8)],
        *[lambda s=s: pins.test_tree_stats_match_definitions(mod, s) for s in range(40)],
        lambda: pins.test_tour_invariants(mod, 2000, None, 2),
        lambda: pins.test_tour_matches_networkx_dfs(mod, 0),
        *[lambda s=s: pins.test_list_rank_vs_pointer_jumping(mod, s) for s in range(4)],
        *[lambda s=s: pins.test_list_scan_unit_weights_are_ranks_plus_one(mod, s) for s in range(2)],
        *[lambda g=g: pins.test_list_scan_of_tour_weights_gives_depth(mod, g) for g in (None, 1)],
        *[lambda s=s: pins.test_lca_bruteforce_all_pairs(mod, s) for s in range(12)],
        lambda: pins.test_lca_closed_forms(mod),
        *[lambda s=s: pins.test_sv_tables_and_query(mod, s) for s in range(20)],
        *[lambda s=s: pins.test_bridges_bruteforce_multigraphs(mod, s) for s in range(40)],
        lambda: pins.test_bridges_special_graphs(mod),
        lambda: pins.test_fig1_tour_from_edge_list(mod),
        *[lambda s=s: pins.test_edge_list_tour_is_the_cyclic_dfs(mod, s) for s in range(12)],
        *[lambda s=s: pins.test_edge_list_tour_matches_ascending_oracle_when_order_agrees(mod, s)
          for s in range(3)],
    ]
    for chk in checks:
        try:
            chk()
        except (AssertionError, oracle.OracleInputError, RuntimeError, IndexError, ValueError) as e:
            return e
    return None


@pytest.fixture(scope="module")
def builddir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def test_unmodified_oracle_passes_battery(oracle_mod):
    assert battery(oracle_mod) is None


@pytest.mark.timeout(120)
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(oracle_mod, builddir, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    path_c = os.path.join(builddir, f"{name}.c")
    path_so = os.path.join(builddir, f"{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", path_c, "-o", path_so])
    prev = oracle.use_library(path_so)
    try:
        failure = battery(oracle)
    finally:
        oracle.use_library(prev)
    assert failure is not None, f"planted mistake '{name}' passed every pin"
