"""GPU parity of the comparison bridge methods (Section 4.1):
Chaitanya-Kothapalli marking on a BFS forest and the hybrid (marking on the
connectivity forest rooted by the Euler tour). The bridge set is unique, so
both must give the oracle's per-slot mask and count bit for bit."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
SPANNING = ["bfs", "forest"]


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2103_15217_amd as et
    assert torch.cuda.is_available()
    return et


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def compare(lib, oracle_mod, row_ptr, col, spanning, ctx=None):
    ctx = ctx or lib.default_context()
    mask, cnt = lib.et_bridges_ck(_dev(row_ptr), _dev(col), spanning=spanning, ctx=ctx)
    ctx.check()
    ref_mask, ref_cnt = oracle_mod.bridges(row_ptr, col)
    got = mask.cpu().numpy().view(np.uint32)[: len(ref_mask)]
    assert np.array_equal(got, ref_mask), "bridge mask"
    assert cnt == ref_cnt
    return cnt


@pytest.mark.parametrize("spanning", SPANNING)
def test_tiny_multigraphs(lib, oracle_mod, spanning):
    for seed in range(200):
        rng = np.random.default_rng(2000 + seed)
        n = int(rng.integers(1, 14))
        m = int(rng.integers(0, 20))
        rp, col = gen.random_multigraph(n, m, seed=seed, loops=True, multi=True)
        compare(lib, oracle_mod, rp, col, spanning)


@pytest.mark.parametrize("spanning", SPANNING)
@pytest.mark.parametrize("kind", ["tree", "path", "cycle", "complete", "doubled_tree", "empty", "isolated"])
def test_special_graphs(lib, oracle_mod, spanning, kind):
    if kind == "tree":
        rp, col = gen.tree_graph(gen.random_tree(100003, None, seed=1))
    elif kind == "path":
        rp, col = gen.tree_graph(gen.path_tree(20001, seed=2))
    elif kind == "cycle":
        rp, col = gen.cycle_graph(20000)
    elif kind == "complete":
        rp, col = gen.complete_graph(300)
    elif kind == "doubled_tree":
        p = gen.random_tree(20000, None, seed=3)
        c = np.nonzero(p >= 0)[0]
        rp, col = gen.csr_from_pairs(20000, np.concatenate([c, c]), np.concatenate([p[c], p[c]]))
    elif kind == "empty":
        rp, col = gen.csr_from_pairs(1000, np.array([], np.int64), np.array([], np.int64))
    else:
        rp, col = gen.csr_from_pairs(1000, np.array([3, 7, 7]), np.array([4, 8, 9]))
    compare(lib, oracle_mod, rp, col, spanning)


@pytest.mark.parametrize("spanning", SPANNING)
@pytest.mark.parametrize("seed", range(2))
def test_random_sparse(lib, oracle_mod, spanning, seed):
    n = 200000
    rp, col = gen.random_multigraph(n, int(1.2 * n), seed=seed, loops=True, multi=True)
    compare(lib, oracle_mod, rp, col, spanning)


@pytest.mark.parametrize("spanning", SPANNING)
def test_planted_medium(lib, oracle_mod, spanning):
    rp, col, info = gen.planted_bridge_graph(n=1 << 18, m=1 << 21, chains=256, max_chain=64, seed=4)
    assert compare(lib, oracle_mod, rp, col, spanning) >= len(info["chain_edges"])


@pytest.mark.parametrize("spanning", SPANNING)
def test_full_size_planted(lib, oracle_mod, bench_ctx, spanning):
    import time
    t0 = time.time()
    rp, col, info = gen.planted_bridge_graph(seed=0)
    print(f"\n[bridges {spanning}] graph {time.time() - t0:.1f}s", flush=True)
    cnt = compare(lib, oracle_mod, rp, col, spanning, ctx=bench_ctx("single"))
    print(f"[bridges {spanning}] compared in {time.time() - t0:.1f}s, {cnt} bridges", flush=True)


def test_spanning_argument_checked(lib):
    with pytest.raises(KeyError):
        lib.et_bridges_ck(_dev([0, 0]), _dev([]), spanning="dfs")
