"""The path at the largest sizes the boundary accepts.

et_tree_build takes n < 2^30 nodes (2n - 2 half-edges just under 2^31) and
et_bridges nnz < 2^31 CSR slots. These cases run at or next to those limits
and check every output against closed forms or against properties that
determine the result at any size (the oracle would take minutes here):

* a relabelled path of 2^30 - 1 nodes: depth = preorder = position on the
  path, size = n - position; LCA = the endpoint nearer the root;
* a star of 2^29 nodes with a random root: children in ascending id order,
  so preorder is the child's rank plus one; LCA = the root unless x = y;
* a random recursive tree of 2^28 nodes (Section 3.2 generator): depth
  recurrence, preorder a permutation with nested intervals, size recurrence,
  ascending sibling order on sampled parents, and sampled LCA queries by
  climbing;
* a graph of a 2^29-vertex cycle and a (2^29 - 1)-vertex path (n = 2^30 - 1
  vertices, nnz = 2^31 - 4 slots), relabelled: exactly the path edges are
  bridges;
* one list of 2^31 - 2^20 - 1 elements (the longest et_list_rank and
  et_list_scan accept) visiting e_i = i * a mod L: rank(e_i) = i, and the
  weighted sums equal a cumulative sum taken in list order by torch.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[maxsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2103_15217_amd as et
    return et


@pytest.fixture
def ctx(lib):
    c = lib.Context()
    yield c
    c.close()
    torch.cuda.empty_cache()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def random_pairs(n, q, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, n, size=q, dtype=np.int64).astype(np.int32),
            rng.integers(0, n, size=q, dtype=np.int64).astype(np.int32))


def test_path_at_the_node_limit(lib, ctx):
    n = (1 << 30) - 1
    rng = np.random.default_rng(30)
    perm = rng.permutation(n).astype(np.int32)          # node at position i gets id perm[i]
    parent = np.empty(n, dtype=np.int32)
    parent[perm[1:]] = perm[:-1]
    parent[perm[0]] = -1
    pos = np.empty(n, dtype=np.int32)
    pos[perm] = np.arange(n, dtype=np.int32)
    del perm
    log(f"path n={n} generated")
    d_parent = dev(parent)
    del parent
    tree = lib.et_tree_build(d_parent, ctx=ctx)
    ctx.check()
    log("built")
    out = tree.export(("depth", "pre", "size"))
    depth = host(out.pop("depth"))
    assert np.array_equal(depth, pos)
    del depth
    pre = host(out.pop("pre"))
    assert np.array_equal(pre, pos)
    del pre
    size = host(out.pop("size"))
    assert np.array_equal(size, n - pos)
    del size
    qx, qy = random_pairs(n, 1 << 20, 31)
    got = host(tree.lca(dev(qx), dev(qy)))
    ctx.check()
    assert np.array_equal(got, np.where(pos[qx] <= pos[qy], qx, qy))
    tree.free()
    log("path checked")


def test_lists_at_the_length_limit(lib, ctx):
    import math
    L = (1 << 31) - (1 << 20) - 1
    a = 1_000_003
    assert math.gcd(a, L) == 1
    i = torch.arange(L, dtype=torch.int64, device="cuda")
    order = (i * a) % L                                   # element at list position i
    succ = torch.empty(L, dtype=torch.int32, device="cuda")
    succ[order[:-1]] = order[1:].to(torch.int32)
    succ[order[-1]] = -1
    head = order[:1].to(torch.int32)
    pos = i.to(torch.int32)
    del i
    log(f"list L={L} generated")
    torch.cuda.empty_cache()                               # leave the library's pool room
    rank = lib.et_list_rank(succ, head, ctx=ctx)
    ctx.check()
    assert torch.equal(rank[order], pos)
    log("ranks checked")
    e = torch.arange(L, dtype=torch.int64, device="cuda")
    w = (((e * 2654435761) >> 13) % 65536 - 32768).to(torch.int32)   # weight of element e, in [-2^15, 2^15)
    del e
    torch.cuda.empty_cache()                               # leave the library's pool room
    s = lib.et_list_scan(succ, w, head, ctx=ctx)
    ctx.check()
    want = torch.cumsum(w[order].to(torch.int64), 0)
    want = ((want + (1 << 31)) % (1 << 32) - (1 << 31)).to(torch.int32)
    assert torch.equal(s[order], want)
    del s
    log("sums checked")
    torch.cuda.empty_cache()                               # leave the library's pool room
    s, r = lib.et_list_scan(succ, w, head, rank=True, ctx=ctx)
    ctx.check()
    assert torch.equal(r, rank)
    assert torch.equal(s[order], want)
    log("sums with ranks checked")


def test_star_with_random_root(lib, ctx):
    n = 1 << 29
    root = int(np.random.default_rng(29).integers(n))
    parent = np.full(n, root, dtype=np.int32)
    parent[root] = -1
    tree = lib.et_tree_build(dev(parent), ctx=ctx)
    ctx.check()
    log(f"star n={n} root={root} built")
    ids = np.arange(n, dtype=np.int32)
    out = tree.export(("depth", "pre", "size"))
    depth, pre, size = host(out["depth"]), host(out["pre"]), host(out["size"])
    del out
    exp_pre = np.where(ids < root, ids + 1, ids)
    exp_pre[root] = 0
    assert np.array_equal(pre, exp_pre)
    assert depth[root] == 0 and size[root] == n
    others = ids != root
    assert np.all(depth[others] == 1) and np.all(size[others] == 1)
    qx, qy = random_pairs(n, 1 << 20, 28)
    qy[:1000] = qx[:1000]
    got = host(tree.lca(dev(qx), dev(qy)))
    ctx.check()
    assert np.array_equal(got, np.where(qx == qy, qx, root))
    tree.free()
    log("star checked")


def test_random_recursive_tree_properties(lib, ctx):
    import gen
    n = 1 << 28
    parent = gen.random_tree(n, None, seed=28)
    log(f"random tree n={n} generated")
    tree = lib.et_tree_build(dev(parent), ctx=ctx)
    ctx.check()
    out = tree.export(("depth", "pre", "size"))
    depth, pre, size = host(out["depth"]), host(out["pre"]), host(out["size"])
    del out
    log("built and exported")
    root = int(np.flatnonzero(parent == -1)[0])
    assert depth[root] == 0 and pre[root] == 0 and size[root] == n
    c = np.flatnonzero(parent >= 0)
    p = parent[c]
    assert np.array_equal(depth[c], depth[p] + 1)
    seen = np.zeros(n, dtype=bool)
    seen[pre] = True
    assert seen.all()                                   # preorder is a permutation
    del seen
    assert np.all(pre[c] > pre[p])
    assert np.all(pre[c].astype(np.int64) + size[c] <= pre[p].astype(np.int64) + size[p])
    child_sum = np.bincount(p, weights=size[c].astype(np.float64), minlength=n)
    assert np.array_equal(size.astype(np.float64), child_sum + 1.0)   # exact in float64
    del child_sum, c, p
    log("recurrences hold")
    # children of sampled parents tile the parent's interval in ascending id order
    rng = np.random.default_rng(7)
    parents = np.unique(parent[rng.integers(0, n, size=24)])
    for q in parents[parents >= 0]:
        ch = np.flatnonzero(parent == q)
        expect = pre[q] + 1 + np.concatenate(([0], np.cumsum(size[ch][:-1], dtype=np.int64)))
        assert np.array_equal(pre[ch], expect), f"sibling order of {q}"
    log("sibling order holds on sampled parents")
    # sampled LCA queries by climbing with the (verified) depths
    qx, qy = random_pairs(n, 1 << 16, 27)
    got = host(tree.lca(dev(qx), dev(qy)))
    ctx.check()
    x, y = qx.astype(np.int64), qy.astype(np.int64)
    for _ in range(n):
        dx, dy = depth[x], depth[y]
        if not np.any(x != y):
            break
        up_x = (x != y) & (dx >= dy)
        up_y = (x != y) & (dy > dx)
        x = np.where(up_x, parent[x], x)
        y = np.where(up_y, parent[y], y)
    assert np.array_equal(got, x.astype(np.int32))
    tree.free()
    log("sampled LCA checked")


def cycle_and_path_csr(c, p, seed):
    """CSR of a c-vertex cycle (original ids 0..c-1) and a p-vertex path
    (original ids c..c+p-1), relabelled by a seeded permutation; rows sorted.
    Returns row_ptr, col and a per-new-id flag marking path vertices."""
    V = c + p
    perm = np.random.default_rng(seed).permutation(V).astype(np.int32)
    nb1 = np.empty(V, dtype=np.int32)                   # neighbours in original ids (-1 = none)
    nb2 = np.empty(V, dtype=np.int32)
    i = np.arange(c, dtype=np.int32)
    nb1[:c] = np.where(i == 0, c - 1, i - 1)
    nb2[:c] = np.where(i == c - 1, 0, i + 1)
    j = np.arange(p, dtype=np.int32)
    nb1[c:] = np.where(j == 0, -1, c + j - 1)
    nb2[c:] = np.where(j == p - 1, -1, c + j + 1)
    del i, j
    a = np.where(nb1 >= 0, perm[np.maximum(nb1, 0)], -1)
    b = np.where(nb2 >= 0, perm[np.maximum(nb2, 0)], -1)
    del nb1, nb2
    deg = (a >= 0).astype(np.int64) + (b >= 0)
    lo = np.where((a >= 0) & ((b < 0) | (a < b)), a, b)   # smaller existing neighbour first
    hi = np.where(lo == a, b, a)
    del a, b
    deg_new = np.empty(V, dtype=np.int64)
    deg_new[perm] = deg
    row_ptr = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(deg_new, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    start = row_ptr[:-1][perm]                          # row start of each original vertex
    one = deg >= 1
    col[start[one]] = lo[one]
    two = deg == 2
    col[start[two] + 1] = hi[two]
    is_path = np.zeros(V, dtype=bool)
    is_path[perm[c:]] = True
    return row_ptr.astype(np.int32), col, is_path, deg_new


def test_bridges_at_the_slot_limit(lib, ctx):
    c, p = 1 << 29, (1 << 29) - 1                     # n = 2^30 - 1 vertices
    row_ptr, col, is_path, deg = cycle_and_path_csr(c, p, seed=31)
    nnz = col.shape[0]
    assert nnz == (1 << 31) - 4                       # 2c + 2(p - 1) slots
    log(f"cycle + path graph: V={c + p} nnz={nnz}")
    d_rp, d_col = dev(row_ptr), dev(col)
    del row_ptr, col
    mask, count = lib.et_bridges(d_rp, d_col, ctx=ctx)
    ctx.check()
    log("bridges done")
    assert count == p - 1
    expect = np.packbits(np.repeat(is_path, deg), bitorder="little")
    got = host(mask).view(np.uint8)
    full = nnz // 8
    assert np.array_equal(got[:full], expect[:full])
    tail = (1 << (nnz % 8)) - 1                        # bits of the last, partial byte
    assert (int(got[full]) & tail) == (int(expect[full]) & tail)
    log("bridge mask checked")


def test_vertex_limit_rejected(lib, ctx):
    import ctypes
    row_ptr = torch.zeros((1 << 30) + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(1, dtype=torch.int32, device="cuda")
    mask = torch.zeros(1, dtype=torch.int32, device="cuda")
    # the binding refuses the size before the call ...
    with pytest.raises(ValueError):
        lib.et_bridges(row_ptr, col, ctx=ctx)
    # ... and the C ABI itself returns ET_EINVAL for n = 2^30 vertices
    P = ctypes.c_void_p
    rc = lib.et._lib.et_bridges(ctx.handle, P(row_ptr.data_ptr()), P(col.data_ptr()), 1 << 30, 0,
                                P(mask.data_ptr()), None, P(torch.cuda.current_stream().cuda_stream))
    assert rc == lib.et.ET_EINVAL
