"""Brute-force definitions used to pin the oracle on tiny inputs.

Each function restates a definition from the paper in the most direct
(quadratic or worse) way, independently of how the oracle computes it.
"""
from collections import deque

import numpy as np


def ancestors(parent, v):
    """Root path of v as a list [v, parent(v), ..., root]."""
    out = [v]
    while parent[v] >= 0:
        v = int(parent[v])
        out.append(v)
    return out


def lca(parent, x, y):
    """LCA by ancestor-set intersection (Section 3: the deepest node that
    is an ancestor of both)."""
    ax = set(ancestors(parent, x))
    for u in ancestors(parent, y):
        if u in ax:
            return u
    raise AssertionError("no common ancestor")


def depth(parent):
    return np.array([len(ancestors(parent, v)) - 1 for v in range(len(parent))], dtype=np.int64)


def subtree_size(parent):
    """size(v) = number of nodes having v on their root path."""
    n = len(parent)
    size = np.zeros(n, dtype=np.int64)
    for u in range(n):
        for a in ancestors(parent, u):
            size[a] += 1
    return size


def preorder(parent):
    """0-based preorder with children in ascending id: u precedes v iff u's
    root path (read from the root down) is lexicographically smaller."""
    n = len(parent)
    keys = [tuple(reversed(ancestors(parent, v))) for v in range(n)]
    order = sorted(range(n), key=lambda v: keys[v])
    pre = np.empty(n, dtype=np.int64)
    pre[order] = np.arange(n)
    return pre


def list_rank_pointer_jumping(succ, heads):
    """Wyllie pointer jumping: a different algorithm from walking. Computes
    the distance to the tail, then rank = (list length - 1) - that."""
    succ = np.asarray(succ, dtype=np.int64)
    L = succ.shape[0]
    used = succ != -2
    nxt = np.where(used, succ, -1)
    dist = np.where(used & (nxt >= 0), 1, 0).astype(np.int64)
    while True:
        live = nxt >= 0
        if not live.any():
            break
        j = nxt[live]
        dist[live] += dist[j]
        nxt[live] = nxt[j]
    # dist is the number of steps to the tail; the head has the largest
    rank = np.full(L, -1, dtype=np.int64)
    for h in heads:
        # members of h's list: follow it once to get its tail
        e = int(h)
        while succ[e] >= 0:
            e = int(succ[e])
        tail = e
        total = dist[h]
        # every element whose walk ends at this tail belongs to h's list
        members = [int(h)]
        e = int(h)
        while succ[e] >= 0:
            e = int(succ[e])
            members.append(e)
        assert members[-1] == tail
        for m in members:
            rank[m] = total - dist[m]
    return rank


def edge_pairs(row_ptr, col):
    """Undirected edges of a symmetric CSR as a list of (u, w, slot_uw,
    slot_wu): the k-th (u, w) slot in row u is paired with the k-th (w, u)
    slot in row w; a self-loop pairs consecutive (u, u) slots."""
    n = len(row_ptr) - 1
    seen = {}
    pairs = []
    for u in range(n):
        for k in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            w = int(col[k])
            key = (u, w)
            seen.setdefault(key, []).append(k)
    used = set()
    for (u, w), slots in seen.items():
        if u < w:
            back = seen.get((w, u), [])
            assert len(back) == len(slots), "CSR not symmetric"
            for a, b in zip(slots, back):
                pairs.append((u, w, a, b))
        elif u == w:
            assert len(slots) % 2 == 0
            for i in range(0, len(slots), 2):
                pairs.append((u, u, slots[i], slots[i + 1]))
    return pairs


def connected(n, edges, s, t):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = [False] * n
    seen[s] = True
    dq = deque([s])
    while dq:
        u = dq.popleft()
        if u == t:
            return True
        for w in adj[u]:
            if not seen[w]:
                seen[w] = True
                dq.append(w)
    return seen[t]


def bridge_slots(row_ptr, col):
    """Slot-level bridge flags by definition (Section 4): an edge is a
    bridge iff deleting it disconnects its endpoints."""
    n = len(row_ptr) - 1
    nnz = len(col)
    pairs = edge_pairs(row_ptr, col)
    flags = np.zeros(nnz, dtype=bool)
    count = 0
    for i, (u, w, a, b) in enumerate(pairs):
        if u == w:
            continue
        rest = [(p[0], p[1]) for j, p in enumerate(pairs) if j != i]
        if not connected(n, rest, u, w):
            flags[a] = flags[b] = True
            count += 1
    return flags, count


def cyclic_dfs_tour(n, edges, root):
    """Depth-first traversal of the tree given by undirected ``edges`` in
    the child order that the DCEL's next() produces (Section 2.1): at a node
    entered from p the neighbours are taken in ascending id order starting
    after p and wrapping around; at the root they start from the smallest.
    Written as a plain recursive DFS over sorted adjacency lists, with no
    half-edge arrays. Returns the tour as (x, y) pairs and parent, depth,
    preorder and subtree size lists."""
    import sys
    adj = [[] for _ in range(n)]
    for x, y in edges:
        adj[x].append(y)
        adj[y].append(x)
    for a in adj:
        a.sort()
    tour, parent = [], [-1] * n
    depth, pre, size = [0] * n, [0] * n, [1] * n
    counter = [0]
    sys.setrecursionlimit(max(1000, 4 * n + 100))

    def visit(x, p, d):
        pre[x] = counter[0]
        counter[0] += 1
        depth[x] = d
        nb = adj[x]
        if p < 0:
            order = nb
        else:
            k = nb.index(p)
            order = nb[k + 1:] + nb[:k]
        for c in order:
            parent[c] = x
            tour.append((x, c))
            visit(c, x, d + 1)
            size[x] += size[c]
            tour.append((c, x))

    visit(root, -1, 0)
    return tour, parent, depth, pre, size
