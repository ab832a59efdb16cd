"""GPU test of et_list_rank_noalloc (list ranking with the library's fixed
per-GPU scratch, for callers that cannot allocate): called through the C ABI
and compared bit-exactly with et_list_rank, the allocating entry point, on
two calls in a row, the second with a smaller input; neither the context's
pool nor torch's allocator grows during the calls."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lists(L, nlists, unused_frac, seed):
    # seeded random lists over a random subset of [0, L): unused slots -2
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


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2103_15217_amd as et
    assert torch.cuda.is_available()
    return et


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _noalloc(et, ctx, succ_t, heads_t, rank_t, length=None, n_heads=None):
    """One et_list_rank_noalloc call through the C ABI (raw pointers)."""
    import torch
    L = succ_t.numel() if length is None else length
    H = heads_t.numel() if n_heads is None else n_heads
    return et.et._lib.et_list_rank_noalloc(
        ctx.handle, ctypes.c_void_p(succ_t.data_ptr()), L, ctypes.c_void_p(heads_t.data_ptr()), H,
        ctypes.c_void_p(rank_t.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _pool_held(et, ctx):
    held, live, peak = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert et.et._lib.et_ctx_pool_stats(ctx.handle, ctypes.byref(held), ctypes.byref(live),
                                        ctypes.byref(peak), 0) == 0
    return held.value


@pytest.mark.parametrize("first,second", [
    ((1 << 20, 1 << 16, 0.0, 11), (300_001, 37, 0.1, 12)),   # the maximum, then a ragged smaller one
    ((500_000, 1, 0.2, 13), (4097, 7, 0.0, 14)),
    ((65_536, 1000, 0.05, 15), (1, 1, 0.0, 16)),
])
def test_noalloc_matches_allocating_call(lib, first, second):
    import torch
    ctx = lib.Context()
    try:
        for (L, nlists, unused, seed) in (first, second):
            succ, heads = _lists(L, nlists, unused, seed)
            s_t, h_t = _dev(succ), _dev(heads)
            want = lib.et_list_rank(s_t, h_t, ctx=ctx)
            ctx.check()
            got = torch.full((L,), 12345, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            held = _pool_held(lib, ctx)
            torch_bytes = torch.cuda.memory_allocated()
            assert _noalloc(lib, ctx, s_t, h_t, got) == 0
            ctx.check()
            assert _pool_held(lib, ctx) == held, "the non-allocating call took pool memory"
            assert torch.cuda.memory_allocated() == torch_bytes
            assert torch.equal(got, want), (L, nlists, seed)
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(lib):
    import torch
    ctx = lib.Context()
    try:
        s_t = _dev([1, -1])
        h_t = _dev([0])
        r_t = torch.empty(2, dtype=torch.int32, device="cuda")
        # host-side size checks: ET_ESIZE (-5), nothing enqueued
        assert _noalloc(lib, ctx, s_t, h_t, r_t, length=lib.et.NOALLOC_MAX_LEN + 1) == lib.et.ET_ESIZE
        assert _noalloc(lib, ctx, s_t, h_t, r_t, n_heads=lib.et.NOALLOC_MAX_HEADS + 1) == lib.et.ET_ESIZE
        # the smallest launch shapes still fit at the maximum sizes
        ctx.set_param("lr_k1_log2", 1)
        ctx.set_param("lr_kn_log2", 1)
        succ, heads = _lists(1 << 20, 1 << 16, 0.0, 21)
        s_t, h_t = _dev(succ), _dev(heads)
        got = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
        assert _noalloc(lib, ctx, s_t, h_t, got) == 0
        ctx.check()
        want = lib.et_list_rank(s_t, h_t, ctx=ctx)
        ctx.check()
        assert torch.equal(got, want)
    finally:
        ctx.close()
