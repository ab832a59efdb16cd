"""GPU parity: et_list_rank against the oracle's list walk (bit-exact)."""
import numpy as np
import pytest

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


def random_lists(L, nlists, unused_frac, seed):
    rng = np.random.default_rng(seed)
    unused = rng.random(L) < unused_frac
    ids = rng.permutation(np.nonzero(~unused)[0])
    nlists = max(1, min(nlists, ids.shape[0]))
    cuts = np.sort(rng.choice(np.arange(1, ids.shape[0]), size=nlists - 1, replace=False)) if nlists > 1 else []
    succ = np.full(L, -2, dtype=np.int32)
    heads = []
    for part in np.split(ids, cuts):
        succ[part[:-1]] = part[1:]
        succ[part[-1]] = -1
        heads.append(int(part[0]))
    return succ, np.array(heads, dtype=np.int32)


@pytest.mark.parametrize("L,nlists,unused,seed", [
    (1, 1, 0.0, 0), (2, 1, 0.0, 1), (15, 3, 0.2, 2), (4096, 1, 0.0, 3), (4097, 7, 0.1, 4),
    (100003, 1, 0.0, 5), (100003, 1000, 0.3, 6), (1 << 20, 1, 0.0, 7), (1 << 20, 20000, 0.05, 8),
    (3_000_001, 3, 0.0, 9)])
def test_random_lists(lib, oracle_mod, L, nlists, unused, seed):
    succ, heads = random_lists(L, nlists, unused, seed)
    ctx = lib.default_context()
    got = lib.et_list_rank(_dev(succ), _dev(heads)).cpu().numpy()
    ctx.check()
    assert np.array_equal(got, oracle_mod.list_rank(succ, heads))


def test_sequential_list(lib, oracle_mod):
    # ids in list order: every sublist is a run of consecutive ids
    L = 1 << 21
    succ = np.arange(1, L + 1, dtype=np.int32)
    succ[-1] = -1
    got = lib.et_list_rank(_dev(succ), _dev([0])).cpu().numpy()
    lib.default_context().check()
    assert np.array_equal(got, np.arange(L))


def test_reverse_list(lib):
    L = 999_999
    succ = np.arange(-1, L - 1, dtype=np.int32)
    got = lib.et_list_rank(_dev(succ), _dev([L - 1])).cpu().numpy()
    lib.default_context().check()
    assert np.array_equal(got, np.arange(L - 1, -1, -1))


def test_many_heads_single_elements(lib, oracle_mod):
    L = 50000
    succ = np.full(L, -1, dtype=np.int32)
    heads = np.arange(L, dtype=np.int32)
    got = lib.et_list_rank(_dev(succ), _dev(heads)).cpu().numpy()
    lib.default_context().check()
    assert np.array_equal(got, np.zeros(L, dtype=np.int32))


@pytest.mark.parametrize("bad", ["cycle", "unreached", "out_of_range", "bad_head"])
def test_malformed_lists_set_status(lib, bad):
    L = 10000
    succ, heads = random_lists(L, 1, 0.0, 11)
    if bad == "cycle":
        # element after the head points back to the head: the rest is cut off
        succ[succ[heads[0]]] = heads[0]
    elif bad == "unreached":
        succ, heads = random_lists(L, 2, 0.0, 12)
        heads = heads[:1]
    elif bad == "out_of_range":
        succ[heads[0]] = L + 10
    elif bad == "bad_head":
        heads = np.array([L + 3], dtype=np.int32)
    ctx = lib.Context()
    lib.et_list_rank(_dev(succ), _dev(heads), ctx=ctx)
    with pytest.raises(lib.EtError):
        ctx.check()
    ctx.close()


@pytest.mark.parametrize("L,nlists,unused,seed", [
    (1, 1, 0.0, 20), (15, 3, 0.2, 21), (4097, 7, 0.1, 22), (100003, 1000, 0.3, 23), (1 << 20, 1, 0.0, 24),
    (1 << 20, 20000, 0.05, 25), (1 << 25, 3, 0.01, 26)])
def test_list_scan_random_weights(lib, oracle_mod, L, nlists, unused, seed):
    # weights over all of int32: sums wrap modulo 2^32 on both sides
    succ, heads = random_lists(L, nlists, unused, seed)
    w = np.random.default_rng(seed).integers(-(1 << 31), 1 << 31, size=L).astype(np.int32)
    ctx = lib.default_context()
    s, r = lib.et_list_scan(_dev(succ), _dev(w), _dev(heads), rank=True)
    s_only = lib.et_list_scan(_dev(succ), _dev(w), _dev(heads))  # the sums-only records
    ctx.check()
    ref_s, ref_r = oracle_mod.list_scan(succ, w, heads)
    assert np.array_equal(s.cpu().numpy(), ref_s)
    assert np.array_equal(r.cpu().numpy(), ref_r)
    assert np.array_equal(s_only.cpu().numpy(), ref_s)


@pytest.mark.parametrize("grasp", [None, 1000, 1])
def test_list_scan_tour_weights_give_depth_2e24(lib, oracle_mod, bench_ctx, grasp):
    # +1 on down half-edges and -1 on up ones along the 2^24-node tour: the
    # sum at 2c is depth(c) (Section 2)
    import gen
    n = 1 << 24
    parent = gen.random_tree(n, grasp, seed=41)
    succ, head = oracle_mod.tree_succ(parent)
    w = np.where(np.arange(2 * n) % 2 == 0, 1, -1).astype(np.int32)
    ctx = bench_ctx("single")
    s = lib.et_list_scan(_dev(succ), _dev(w), _dev([head]), ctx=ctx).cpu().numpy()
    ctx.check()
    depth = oracle_mod.euler_tour(parent)["depth"]
    c = np.flatnonzero(parent >= 0)
    assert np.array_equal(s[2 * c], depth[c])
    assert np.array_equal(s[2 * c + 1], depth[c] - 1)


def test_list_scan_malformed_list_flagged(lib):
    succ, heads = random_lists(10000, 1, 0.0, 30)
    succ[succ[heads[0]]] = heads[0]
    ctx = lib.Context()
    lib.et_list_scan(_dev(succ), _dev(np.ones(10000, np.int32)), _dev(heads), ctx=ctx)
    with pytest.raises(lib.EtError):
        ctx.check()
    ctx.close()
