"""Seeded tree and query generators (paper Section 3.2, LCA datasets).

A tree is an int32 parent array: ``parent[v]`` is the parent id of ``v`` and
``parent[root] == -1``.
"""
import numpy as np


def _relabel(parent_seq, rng):
    """Map the ids of a tree given in generation order through a random
    permutation (Section 3.2: ids must not leak the generation order)."""
    n = parent_seq.shape[0]
    perm = rng.permutation(n).astype(np.int64)
    out = np.empty(n, dtype=np.int32)
    has_parent = parent_seq >= 0
    out[perm[has_parent]] = perm[parent_seq[has_parent]].astype(np.int32)
    out[perm[~has_parent]] = -1
    return out


def random_tree(n, grasp=None, seed=0, relabel=True):
    """Grasp tree of Section 3.2, 0-based: node 0 is the root and node
    ``i >= 1`` takes a parent uniformly from ``[max(0, i - grasp), i)``.

    ``grasp=None`` (or ``grasp >= n``) is the unbounded case, the random
    recursive tree with expected average depth about ln n; ``grasp=1`` is a
    path. With ``relabel`` the ids go through a seeded permutation.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    g = n if grasp is None else max(1, min(int(grasp), n))
    seq = np.empty(n, dtype=np.int64)
    seq[0] = -1
    if n > 1:
        i = np.arange(1, n, dtype=np.int64)
        lo = np.maximum(i - g, 0)
        seq[1:] = rng.integers(lo, i)
    if not relabel:
        return seq.astype(np.int32)
    return _relabel(seq, rng)


def random_queries(n, q, seed=0):
    """``q`` query pairs drawn uniformly from ``[n] x [n]`` (Section 3.2);
    ``x == y`` pairs occur and are valid queries."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x51]))
    qx = rng.integers(0, n, size=int(q), dtype=np.int64).astype(np.int32)
    qy = rng.integers(0, n, size=int(q), dtype=np.int64).astype(np.int32)
    return qx, qy


def path_tree(n, seed=None):
    """Path 0-1-2-...-(n-1) rooted at 0 (grasp 1); relabelled if ``seed``."""
    seq = np.arange(-1, n - 1, dtype=np.int64)
    if seed is None:
        return seq.astype(np.int32)
    return _relabel(seq, np.random.default_rng(seed))


def star_tree(n, root=0):
    """Every node hangs directly below ``root``."""
    p = np.full(n, root, dtype=np.int32)
    p[root] = -1
    return p


def heap_binary_tree(n):
    """Heap-shaped binary tree: node ``v`` (0-based) has parent
    ``(v - 1) // 2``; perfect when ``n + 1`` is a power of two."""
    v = np.arange(n, dtype=np.int64)
    p = (v - 1) // 2
    p[0] = -1
    return p.astype(np.int32)


def caterpillar_tree(spine, legs, seed=None):
    """A path of ``spine`` nodes, each with ``legs`` leaves attached."""
    n = spine * (1 + legs)
    seq = np.empty(n, dtype=np.int64)
    seq[:spine] = np.arange(-1, spine - 1)
    leaf = np.arange(spine, n)
    seq[spine:] = (leaf - spine) // max(legs, 1)
    if seed is None:
        return seq.astype(np.int32)
    return _relabel(seq, np.random.default_rng(seed))


def forest_batch(num_trees, seed=0, log2_min=6, log2_max=18,
                 qlog2_min=10, qlog2_max=14, grasps=(1, 64, None)):
    """Batch of independent trees of uneven size.

    Sizes are log-uniform on ``[2**log2_min, 2**log2_max]``, the grasp of
    each tree is drawn from ``grasps`` (``None`` = unbounded) and each tree
    gets a log-uniform number of uniform queries. Returns a dict with the
    concatenated local parent arrays (ids 0-based within each tree), the
    node offsets ``[T+1]``, the concatenated local queries and their tree ids.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xF0]))
    sizes = np.floor(2.0 ** rng.uniform(log2_min, log2_max, size=num_trees)).astype(np.int64)
    gidx = rng.integers(0, len(grasps), size=num_trees)
    qcount = np.floor(2.0 ** rng.uniform(qlog2_min, qlog2_max, size=num_trees)).astype(np.int64)
    offsets = np.zeros(num_trees + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    parents, qx, qy, qt = [], [], [], []
    for t in range(num_trees):
        g = grasps[gidx[t]]
        parents.append(random_tree(int(sizes[t]), g, seed=int(seed) * 1000003 + t))
        x, y = random_queries(int(sizes[t]), int(qcount[t]), seed=int(seed) * 1000003 + t)
        qx.append(x)
        qy.append(y)
        qt.append(np.full(int(qcount[t]), t, dtype=np.int32))
    return {
        "parent": np.concatenate(parents).astype(np.int32),
        "offsets": offsets,
        "sizes": sizes,
        "grasp": [grasps[i] for i in gidx],
        "qx": np.concatenate(qx), "qy": np.concatenate(qy),
        "qtree": np.concatenate(qt),
    }


def ba_tree(n, seed=0, relabel=True):
    """Scale-free tree by preferential attachment (Barabasi-Albert with one
    edge per new node; the paper's Section 3.2 scale-free LCA workload):
    nodes 0 and 1 start joined; node i >= 2 attaches to an existing node
    chosen with probability proportional to its degree, i.e. to one end of
    a uniformly chosen earlier edge. Returns a parent array rooted at node 0
    (ids then go through a seeded permutation with ``relabel``).

    Edge k (k = 1..i-1) joins node k and its parent, so a uniform choice
    among the 2(i-1) edge ends is: r even -> node r/2 + 1, r odd -> the
    parent of node (r-1)/2 + 1. The second case refers to an earlier
    parent, resolved below by pointer jumping over the whole array."""
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xBA]))
    seq = np.full(n, -1, dtype=np.int64)
    if n >= 2:
        seq[1] = 0
    if n >= 3:
        i = np.arange(2, n, dtype=np.int64)
        r = rng.integers(0, 2 * (i - 1))
        k = r // 2 + 1
        direct = (r % 2) == 0
        target = np.where(direct, k, -1)       # parent known now
        ref = np.where(direct, -1, k)          # parent = parent of node ref
        seq[2:] = target
        refs = np.full(n, -1, dtype=np.int64)
        refs[2:] = ref
        todo = np.flatnonzero(refs >= 0)
        while todo.size:
            a = refs[todo]
            pa = seq[a]
            done = pa >= 0
            seq[todo[done]] = pa[done]
            # not known yet: node a also copies a parent, so look where a looks
            refs[todo[~done]] = refs[a[~done]]
            todo = todo[~done]
    if not relabel:
        return seq.astype(np.int32)
    return _relabel(seq, rng)
