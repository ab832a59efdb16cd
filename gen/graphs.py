"""Seeded undirected graph generators, returned as symmetric CSR.

A graph is ``(row_ptr int64[n+1], col int32[nnz])``: every undirected edge
{u, w} appears as slot (u, w) in row u and slot (w, u) in row w, rows are
sorted ascending, parallel edges repeat a column, and a self-loop {u, u}
gives two (u, u) slots in row u.
"""
import numpy as np


def csr_from_pairs(n, u, w):
    """Symmetric CSR with sorted rows from undirected pairs ``(u[i], w[i])``."""
    u = np.asarray(u, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    src = np.concatenate([u, w])
    dst = np.concatenate([w, u])
    key = np.sort(src * np.int64(n) + dst)
    src = key // n
    col = (key - src * n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, col


def cycle_graph(n):
    v = np.arange(n, dtype=np.int64)
    return csr_from_pairs(n, v, (v + 1) % n)


def complete_graph(n):
    a, b = np.triu_indices(n, k=1)
    return csr_from_pairs(n, a, b)


def tree_graph(parent):
    """The undirected graph of a tree given as a parent array."""
    parent = np.asarray(parent, dtype=np.int64)
    c = np.nonzero(parent >= 0)[0]
    return csr_from_pairs(parent.shape[0], c, parent[c])


def random_multigraph(n, m, seed=0, loops=True, multi=True):
    """``m`` uniform random pairs on ``n`` vertices; with ``loops`` and
    ``multi`` the result may hold self-loops and parallel edges."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x6d]))
    u = rng.integers(0, n, size=m)
    w = rng.integers(0, n, size=m)
    if not loops:
        keep = u != w
        u, w = u[keep], w[keep]
    if not multi:
        lo, hi = np.minimum(u, w), np.maximum(u, w)
        key = np.unique(lo * n + hi)
        u, w = key // n, key % n
    return csr_from_pairs(n, u, w)


def planted_bridge_graph(n=1 << 22, m=1 << 25, chains=4096, max_chain=512,
                         seed=0, relabel=True):
    """Sparse random graph whose blobs are joined by planted chains.

    ``chains + 1`` blobs of near-equal size each get a random recursive
    spanning tree plus uniform distinct extra pairs, so that blob edges fill
    ``m`` minus the chain edges (average degree ``2m/n``). Chain ``k`` has a
    uniform length in ``[1, max_chain]`` edges and joins a uniform vertex of
    blob ``k + 1`` to a uniform vertex of a uniform earlier blob, so blobs
    and chains form a tree and every chain edge is a bridge. All ids then go
    through a seeded permutation.

    Returns ``(row_ptr, col, info)`` where ``info["chain_edges"]`` is an
    ``(E, 2)`` array of the planted bridge pairs (after relabelling) and
    ``info["m"]`` the realised number of undirected edges.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xb6]))
    clen = rng.integers(1, max_chain + 1, size=chains).astype(np.int64)
    n_chain_vertices = int((clen - 1).sum())
    nblobs = chains + 1
    nb = n - n_chain_vertices
    if nb < 2 * nblobs:
        raise ValueError("too few vertices for the requested chains")
    size = np.full(nblobs, nb // nblobs, dtype=np.int64)
    size[rng.permutation(nblobs)[: nb - int(size.sum())]] += 1
    start = np.zeros(nblobs + 1, dtype=np.int64)
    np.cumsum(size, out=start[1:])
    blob_of_vertex = np.repeat(np.arange(nblobs), size)

    # blob spanning trees: local vertex i >= 1 picks a parent in [0, i)
    local = np.arange(nb, dtype=np.int64) - start[blob_of_vertex]
    nonroot = local > 0
    child = np.nonzero(nonroot)[0]
    tparent = start[blob_of_vertex[child]] + np.floor(
        rng.random(child.shape[0]) * local[child]).astype(np.int64)
    tu, tw = child, tparent

    # extra distinct pairs inside each blob
    mb = m - int(clen.sum())
    share = np.floor(mb * size / nb).astype(np.int64)
    share[: mb - int(share.sum())] += 1
    extra = np.maximum(share - (size - 1), 0)
    extra = np.minimum(extra, size * (size - 1) // 2 - (size - 1))
    draw = (extra * 1.15 + 16).astype(np.int64)
    bid = np.repeat(np.arange(nblobs), draw)
    su = start[bid] + np.floor(rng.random(bid.shape[0]) * size[bid]).astype(np.int64)
    sw = start[bid] + np.floor(rng.random(bid.shape[0]) * size[bid]).astype(np.int64)
    keep = su != sw
    su, sw, bid = su[keep], sw[keep], bid[keep]
    lo, hi = np.minimum(su, sw), np.maximum(su, sw)
    key, first = np.unique(lo * n + hi, return_index=True)
    bid = bid[first]
    tkey = np.minimum(tu, tw) * n + np.maximum(tu, tw)
    fresh = ~np.isin(key, tkey, assume_unique=False)
    key, bid = key[fresh], bid[fresh]
    prio = (bid << 32) | rng.integers(0, 1 << 32, size=key.shape[0], dtype=np.int64)
    order = np.argsort(prio)
    key, bid = key[order], bid[order]
    gstart = np.searchsorted(bid, np.arange(nblobs))
    rank_in_blob = np.arange(key.shape[0]) - gstart[bid]
    key = key[rank_in_blob < extra[bid]]
    eu, ew = key // n, key % n

    # planted chains: blob k+1 -> uniform earlier blob
    target = np.floor(rng.random(chains) * np.arange(1, chains + 1)).astype(np.int64)
    a_end = start[np.arange(1, chains + 1)] + np.floor(
        rng.random(chains) * size[1:]).astype(np.int64)
    b_end = start[target] + np.floor(rng.random(chains) * size[target]).astype(np.int64)
    istart = nb + np.concatenate([[0], np.cumsum(clen - 1)[:-1]])
    k = np.repeat(np.arange(chains), clen)
    j = np.arange(k.shape[0]) - np.repeat(np.cumsum(clen) - clen, clen)
    cu = np.where(j == 0, a_end[k], istart[k] + j - 1)
    cw = np.where(j == clen[k] - 1, b_end[k], istart[k] + j)
    assert int(istart[-1] + clen[-1] - 1) == n

    u = np.concatenate([tu, eu, cu])
    w = np.concatenate([tw, ew, cw])
    chain_edges = np.stack([cu, cw], axis=1)
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        u, w = perm[u], perm[w]
        chain_edges = perm[chain_edges]
    row_ptr, col = csr_from_pairs(n, u, w)
    return row_ptr, col, {"chain_edges": chain_edges, "m": int(u.shape[0]),
                          "blobs": nblobs, "chain_lengths": clen}
