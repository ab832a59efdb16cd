"""Thin Python binding of ``libet.so`` (the C ABI in ``include/et.h``).

Argument marshalling only: every step runs in the HIP kernels of the
library. Tensors must be contiguous int32 / uint32 device tensors on the
context's device; the HIP stream is torch's current stream. If the library
is not built this module raises on import: there is no CPU fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libet.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2103_15217_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback")

_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_SIG = {
    "et_version": ([], ctypes.c_int),
    "et_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "et_ctx_create": ([ctypes.POINTER(_P)], ctypes.c_int),
    "et_ctx_destroy": ([_P], None),
    "et_ctx_status": ([_P, _P], ctypes.c_int),
    "et_ctx_status_bits": ([_P, _P, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "et_ctx_profile": ([_P, ctypes.c_int], ctypes.c_int),
    "et_ctx_profile_only": ([_P, ctypes.c_char_p], ctypes.c_int),
    "et_ctx_set_param": ([_P, ctypes.c_char_p, _i64], ctypes.c_int),
    "et_ctx_profile_read": ([_P, _P, ctypes.c_char_p, _i32], ctypes.c_int),
    "et_list_rank": ([_P, _P, _i32, _P, _i32, _P, _P], ctypes.c_int),
    "et_list_scan": ([_P, _P, _P, _i32, _P, _i32, _P, _P, _P], ctypes.c_int),
    "et_list_rank_noalloc": ([_P, _P, _i32, _P, _i32, _P, _P], ctypes.c_int),
    "et_lca_batch_fused": ([_P, _P, _P, _i32, _i64, _i32, _P, _P, _P, _i64, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "et_bridges_batch_fused": ([_P, _P, _P, _P, _P, _P, _i32, _i32, _i32, _i32, _i32, _P, _i64, _P, _P, _P],
                               ctypes.c_int),
    "et_tree_build": ([_P, _P, _i32, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "et_tree_size": ([_P], _i32),
    "et_tree_batch_size": ([_P], _i32),
    "et_tree_build_batch": ([_P, _P, _P, _i32, _i64, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "et_lca_batch": ([_P, _P, _P, _P, _i64, _P, _P], ctypes.c_int),
    "et_tree_export": ([_P, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "et_tree_free": ([_P, _P], None),
    "et_tree_export_tour": ([_P, _P, _P], ctypes.c_int),
    "et_lca": ([_P, _P, _P, _i64, _P, _P], ctypes.c_int),
    "et_bridges": ([_P, _P, _P, _i32, _i32, _P, ctypes.POINTER(_i64), _P], ctypes.c_int),
    "et_bridges_count": ([_P, _P, _P], ctypes.c_int),
    "et_bridges_batch": ([_P, _P, _P, _P, _P, _i32, _i32, _i32, _P, _i64, _P, _P], ctypes.c_int),
    "et_bridges_ck": ([_P, _P, _P, _i32, _i32, _i32, _P, ctypes.POINTER(_i64), _P], ctypes.c_int),
    "et_levels": ([_P, _P, _i32, _P, _P], ctypes.c_int),
    "et_tree_build_edges": ([_P, _P, _P, _i32, _i32, _P, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "et_tree_rmq_build": ([_P, _P, _P], ctypes.c_int),
    "et_lca_rmq": ([_P, _P, _P, _i64, _P, _P], ctypes.c_int),
    "et_lca_naive": ([_P, _P, _P, _i32, _P, _P, _i64, _P, _P], ctypes.c_int),
    "et_tree_footprint": ([_P, _i64, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], ctypes.c_int),
    "et_bridges_footprint": ([_P, _i32, _i32, _i32, ctypes.POINTER(_i64)], ctypes.c_int),
    "et_tree_bytes": ([_P, ctypes.POINTER(_i64)], ctypes.c_int),
    "et_ctx_pool_stats": ([_P, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int],
                          ctypes.c_int),
}
for _name, (_args, _res) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

ET_OK, ET_EINVAL, ET_ENOMEM, ET_EHIP, ET_EINPUT, ET_ESIZE = 0, -1, -2, -3, -4, -5
FUSED_MAX_NODES = 4096  # trees of et_lca_batch_fused (et.h)
FUSED_MAX_VERTICES, FUSED_MAX_SLOTS = 1024, 8192  # graphs of et_bridges_batch_fused (et.h)
# limits of et_list_rank_noalloc (et.h)
NOALLOC_MAX_LEN = 1 << 20
NOALLOC_MAX_HEADS = 1 << 16

STATUS_BITS = {
    1 << 0: "bad parent", 1 << 1: "root count", 1 << 2: "unreached element",
    1 << 3: "bad successor", 1 << 4: "bad head", 1 << 5: "walk bound exceeded",
    1 << 6: "bad query", 1 << 7: "bad CSR", 1 << 8: "table index out of range",
    1 << 9: "output buffer too small",
}


class EtError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {_lib.et_strerror(code).decode()} ({code})")


def _check(rc, what):
    if rc != ET_OK:
        raise EtError(rc, what)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


INT32_MAX = (1 << 31) - 1
NODE_MAX = (1 << 30) - 1          # nodes of a tree, vertices of a graph (et.h)
LIST_MAX = INT32_MAX - (1 << 20)  # elements of one et_list_rank / et_list_scan call


def _i32(value, name, limit=INT32_MAX):
    """A size that goes to an int32 argument of the C ABI: ctypes would
    truncate a larger one silently (2^32 + 5 becomes 5), so refuse it here."""
    value = int(value)
    if value < 0 or value > limit:
        raise ValueError(f"{name} = {value} is outside the library's range [0, {limit}]")
    return value


def version():
    return _lib.et_version()


class Context:
    """An ``et_ctx``: scratch pool and device status word on the current device."""

    def __init__(self):
        h = _P()
        _check(_lib.et_ctx_create(ctypes.byref(h)), "et_ctx_create")
        self._h = h
        self.device = torch.cuda.current_device()

    @property
    def handle(self):
        return self._h

    def status_bits(self):
        bits = ctypes.c_uint32(0)
        _check(_lib.et_ctx_status_bits(self._h, _stream(), ctypes.byref(bits)), "et_ctx_status_bits")
        return int(bits.value)

    def check(self):
        """Wait for the stream and raise EtError(ET_EINPUT) if a kernel flagged bad input."""
        bits = self.status_bits()
        if bits:
            names = [v for k, v in STATUS_BITS.items() if bits & k]
            raise EtError(ET_EINPUT, "device status: " + ", ".join(names))

    def set_param(self, name, value):
        """Set a tunable launch parameter (see et_ctx_set_param in et.h)."""
        _check(_lib.et_ctx_set_param(self._h, name.encode(), int(value)), f"et_ctx_set_param({name})")

    def profile(self, enable=True, only=None):
        """Bracket every later kernel launch on this context with HIP events
        (only the launches of kernel ``only`` when given)."""
        _check(_lib.et_ctx_profile_only(self._h, only.encode() if only else None), "et_ctx_profile_only")
        _check(_lib.et_ctx_profile(self._h, 1 if enable else 0), "et_ctx_profile")

    def profile_read(self):
        """Wait for the stream; return {kernel: (launches, total_ms, max_ms)}
        over the launches timed since the previous read."""
        import json
        size = 1 << 16
        while True:
            buf = ctypes.create_string_buffer(size)
            rc = _lib.et_ctx_profile_read(self._h, _stream(), buf, size)
            if rc == ET_EINVAL and size < (1 << 24):
                size *= 4
                continue
            _check(rc, "et_ctx_profile_read")
            return {k: tuple(v) for k, v in json.loads(buf.value.decode()).items()}

    def pool_stats(self, reset_peak=False):
        """Device bytes of this context's scratch pool: ``held`` (allocated
        from the device, cached blocks included), ``live`` (handed out now:
        resident trees' tables and running calls' scratch) and ``peak_live``
        (the most live since the last reset)."""
        held, live, peak = _i64(0), _i64(0), _i64(0)
        _check(_lib.et_ctx_pool_stats(self._h, ctypes.byref(held), ctypes.byref(live), ctypes.byref(peak),
                                      1 if reset_peak else 0), "et_ctx_pool_stats")
        return {"held": held.value, "live": live.value, "peak_live": peak.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.et_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = None


def default_context():
    global _default
    if _default is None:
        _default = Context()
    return _default


# ------------------------------------------------------------------ footprints (host only)

def tree_footprint(n_total, n_trees=0, ctx=None):
    """(table bytes, scratch bytes) of et_tree_build on one tree of ``n_total``
    nodes (``n_trees`` = 0) or of et_tree_build_batch on ``n_trees`` trees with
    ``n_total`` nodes in all: the tables the tree keeps (exact) and an upper
    bound on the scratch the build takes. Launch shapes from ``ctx`` (library
    defaults when None). No device call: this works without a GPU."""
    tb, sb = _i64(0), _i64(0)
    _check(_lib.et_tree_footprint(ctx.handle if ctx else None, int(n_total), _i32(n_trees, "number of trees"),
                                  ctypes.byref(tb), ctypes.byref(sb)), "et_tree_footprint")
    return tb.value, sb.value


def bridges_footprint(n_total, nnz_total, n_graphs=0, ctx=None):
    """Upper bound on the scratch bytes of et_bridges on one graph
    (``n_graphs`` = 0) or of et_bridges_batch on ``n_graphs`` graphs, from
    their vertex and CSR-slot totals. No device call."""
    sb = _i64(0)
    _check(_lib.et_bridges_footprint(ctx.handle if ctx else None, _i32(n_total, "vertex count", NODE_MAX),
                                     _i32(nnz_total, "CSR slot count"), _i32(n_graphs, "number of graphs"),
                                     ctypes.byref(sb)), "et_bridges_footprint")
    return sb.value


# ------------------------------------------------------------------ list ranking

def et_list_rank(succ, heads, rank=None, ctx=None):
    """Rank of every element of the lists starting at ``heads`` (head = 0);
    ``succ[e] == -1`` ends a list and ``-2`` marks an unused slot (rank -1)."""
    ctx = ctx or default_context()
    succ = _dev(succ, torch.int32, "succ")
    heads = _dev(heads, torch.int32, "heads")
    L = _i32(succ.numel(), "list length", LIST_MAX)
    H = _i32(heads.numel(), "number of list heads")
    if rank is None:
        rank = torch.empty_like(succ)
    _check(_lib.et_list_rank(ctx.handle, _ptr(succ), L, _ptr(heads), H,
                             _ptr(rank), _stream()), "et_list_rank")
    return rank


def et_list_rank_noalloc(succ, heads, rank, ctx=None):
    """``et_list_rank`` with its scratch in the library's fixed per-GPU array:
    the call allocates nothing, so ``rank`` must be given. Lists of at most
    ``NOALLOC_MAX_LEN`` elements and ``NOALLOC_MAX_HEADS`` heads; calls that
    overlap on one GPU race (they share the array)."""
    ctx = ctx or default_context()
    succ = _dev(succ, torch.int32, "succ")
    heads = _dev(heads, torch.int32, "heads")
    rank = _dev(rank, torch.int32, "rank")
    L = _i32(succ.numel(), "list length", LIST_MAX)
    H = _i32(heads.numel(), "number of list heads")
    if rank.numel() < L:
        raise ValueError("rank is shorter than succ")
    _check(_lib.et_list_rank_noalloc(ctx.handle, _ptr(succ), L, _ptr(heads), H,
                                     _ptr(rank), _stream()), "et_list_rank_noalloc")
    return rank


# ------------------------------------------------------------------ trees and LCA

class Tree:
    """A built tree or batch of trees (``et_tree``): Euler tour, node
    statistics, Inlabel tables."""

    def __init__(self, handle, n, ctx, batch=0):
        self._h = handle
        self.n = n
        self.ctx = ctx
        self.batch = batch

    def export(self, fields=None):
        """Device tensors of the tree's tables; ``fields`` limits which are
        copied out (default: all that the tree kind provides)."""
        n = self.n
        dev = torch.device("cuda", self.ctx.device)
        if fields is not None:
            sizes = {"succ": 2 * n, "rank": 2 * n, "depth": n, "pre": n, "size": n, "inlabel": n, "asc": n}
            out = {k: torch.empty(sizes[k], dtype=torch.int32, device=dev) for k in fields}
            _check(_lib.et_tree_export(self._h, *[_ptr(out[k]) if k in out else None for k in
                                                  ("succ", "rank", "depth", "pre", "size", "inlabel", "asc")],
                                       _stream()), "et_tree_export")
            return out
        if self.batch:
            out = {k: torch.empty(n, dtype=torch.int32, device=dev) for k in ("depth", "pre", "size")}
            _check(_lib.et_tree_export(self._h, None, None, _ptr(out["depth"]), _ptr(out["pre"]),
                                       _ptr(out["size"]), None, None, _stream()), "et_tree_export")
            return out
        out = {
            "succ": torch.empty(2 * n, dtype=torch.int32, device=dev),
            "rank": torch.empty(2 * n, dtype=torch.int32, device=dev),
            "depth": torch.empty(n, dtype=torch.int32, device=dev),
            "pre": torch.empty(n, dtype=torch.int32, device=dev),
            "size": torch.empty(n, dtype=torch.int32, device=dev),
            "inlabel": torch.empty(n, dtype=torch.int32, device=dev),
            "asc": torch.empty(n, dtype=torch.int32, device=dev),
        }
        _check(_lib.et_tree_export(self._h, *[_ptr(out[k]) for k in
                                              ("succ", "rank", "depth", "pre", "size", "inlabel", "asc")],
                                   _stream()), "et_tree_export")
        return out

    def tour(self, out=None):
        """The half-edge at every tour position (2(n-1) entries)."""
        if out is None:
            out = torch.empty(max(2 * (self.n - 1), 0), dtype=torch.int32,
                              device=torch.device("cuda", self.ctx.device))
        _check(_lib.et_tree_export_tour(self._h, _ptr(out), _stream()), "et_tree_export_tour")
        return out

    def lca_batch(self, qtree, qx, qy, out=None):
        """LCA of local nodes qx[i], qy[i] of tree qtree[i] (local ids out)."""
        qt = _dev(qtree, torch.int32, "qtree")
        qx = _dev(qx, torch.int32, "qx")
        qy = _dev(qy, torch.int32, "qy")
        if not (qx.numel() == qy.numel() == qt.numel()):
            raise ValueError("query arrays differ in length")
        if out is None:
            out = torch.empty_like(qx)
        _check(_lib.et_lca_batch(self._h, _ptr(qt), _ptr(qx), _ptr(qy), qx.numel(), _ptr(out), _stream()),
               "et_lca_batch")
        return out

    def lca(self, qx, qy, out=None):
        qx = _dev(qx, torch.int32, "qx")
        qy = _dev(qy, torch.int32, "qy")
        if qx.numel() != qy.numel():
            raise ValueError("qx and qy differ in length")
        if out is None:
            out = torch.empty_like(qx)
        _check(_lib.et_lca(self._h, _ptr(qx), _ptr(qy), qx.numel(), _ptr(out), _stream()), "et_lca")
        return out

    def rmq_build(self, parent):
        """Add the RMQ query engine's tables (``parent``: the array the tree was built from)."""
        parent = _dev(parent, torch.int32, "parent")
        _check(_lib.et_tree_rmq_build(self._h, _ptr(parent), _stream()), "et_tree_rmq_build")
        return self

    def lca_rmq(self, qx, qy, out=None):
        """LCA queries answered by range minima over the Euler tour."""
        qx = _dev(qx, torch.int32, "qx")
        qy = _dev(qy, torch.int32, "qy")
        if qx.numel() != qy.numel():
            raise ValueError("qx and qy differ in length")
        if out is None:
            out = torch.empty_like(qx)
        _check(_lib.et_lca_rmq(self._h, _ptr(qx), _ptr(qy), qx.numel(), _ptr(out), _stream()), "et_lca_rmq")
        return out

    def nbytes(self):
        """Device bytes of this tree's tables (exact: the pool blocks it holds)."""
        b = _i64(0)
        _check(_lib.et_tree_bytes(self._h, ctypes.byref(b)), "et_tree_bytes")
        return b.value

    def free(self):
        """Return the tables to the context's pool, ordered on the current
        stream: later work on another stream that reuses them waits for it."""
        if self._h:
            _lib.et_tree_free(self._h, _stream())
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def et_list_scan(succ, weight, heads, rank=False, ctx=None):
    """Prefix sums of ``weight`` along the lists starting at ``heads``: the
    sum from each element's head through the element (int32, wrapping);
    with ``rank`` also the ranks (returns (sum, rank) then)."""
    ctx = ctx or default_context()
    succ = _dev(succ, torch.int32, "succ")
    weight = _dev(weight, torch.int32, "weight")
    heads = _dev(heads, torch.int32, "heads")
    if weight.numel() != succ.numel():
        raise ValueError("succ and weight differ in length")
    L = _i32(succ.numel(), "list length", LIST_MAX)
    H = _i32(heads.numel(), "number of list heads")
    out = torch.empty_like(succ)
    r = torch.empty_like(succ) if rank else None
    _check(_lib.et_list_scan(ctx.handle, _ptr(succ), _ptr(weight), L, _ptr(heads), H,
                             _ptr(r), _ptr(out), _stream()), "et_list_scan")
    return (out, r) if rank else out


def et_tree_build(parent, ctx=None):
    ctx = ctx or default_context()
    parent = _dev(parent, torch.int32, "parent")
    n = _i32(parent.numel(), "tree size", NODE_MAX)
    h = _P()
    _check(_lib.et_tree_build(ctx.handle, _ptr(parent), n, _stream(), ctypes.byref(h)),
           "et_tree_build")
    return Tree(h, n, ctx)


def et_tree_build_edges(u, v, n, root, ctx=None, parent_out=None):
    """Build from the unordered edge list (u[i], v[i]) of a tree on n nodes,
    rooted at ``root`` (the DCEL construction). With ``parent_out`` (an int32
    device tensor of n entries) the rooted parent array is written there."""
    ctx = ctx or default_context()
    u = _dev(u, torch.int32, "u")
    v = _dev(v, torch.int32, "v")
    n = _i32(n, "tree size", NODE_MAX)
    if u.numel() != n - 1 or v.numel() != n - 1:
        raise ValueError("a tree on n nodes has n - 1 edges")
    if parent_out is not None:
        parent_out = _dev(parent_out, torch.int32, "parent_out")
        if parent_out.numel() != n:
            raise ValueError("parent_out needs n entries")
    h = _P()
    _check(_lib.et_tree_build_edges(ctx.handle, _ptr(u) if n > 1 else None, _ptr(v) if n > 1 else None, int(n),
                                    int(root), _ptr(parent_out), _stream(), ctypes.byref(h)),
           "et_tree_build_edges")
    return Tree(h, int(n), ctx)


def et_lca(tree, qx, qy, out=None):
    return tree.lca(qx, qy, out)


def et_tree_build_batch(parent, offsets, ctx=None):
    """Build a batch of trees: ``parent`` holds each tree's local parent
    array back to back, ``offsets`` (int64, T+1) the tree boundaries."""
    ctx = ctx or default_context()
    parent = _dev(parent, torch.int32, "parent")
    offsets = _dev(offsets, torch.int64, "offsets")
    T = _i32(offsets.numel() - 1, "number of trees")
    _i32(parent.numel(), "batch size", NODE_MAX - 1)
    h = _P()
    _check(_lib.et_tree_build_batch(ctx.handle, _ptr(parent), _ptr(offsets), T, parent.numel(), _stream(),
                                    ctypes.byref(h)), "et_tree_build_batch")
    return Tree(h, parent.numel(), ctx, batch=T)


def et_lca_batch(tree, qtree, qx, qy, out=None):
    return tree.lca_batch(qtree, qx, qy, out)


def fused_order(offsets, qoffsets):
    """An order for :func:`et_lca_batch_fused` that hands out the costliest
    trees first (a tree's cost taken as its nodes plus a quarter of its
    queries), so that the launch does not end on a few large trees.
    ``offsets`` and ``qoffsets`` are host sequences of T + 1 offsets."""
    import numpy as np
    off = np.asarray(offsets, dtype=np.int64)
    qoff = np.asarray(qoffsets, dtype=np.int64)
    cost = np.diff(off) + np.diff(qoff) // 4
    return np.argsort(-cost, kind="stable").astype(np.int32)


def fused_graph_order(slots, vertices):
    """An order for :func:`et_bridges_batch_fused` that hands out the
    costliest graphs first (a graph's cost taken as its CSR slots plus twice
    its vertices); ``slots`` and ``vertices`` are host sequences, one entry
    per graph."""
    import numpy as np
    cost = np.asarray(slots, dtype=np.int64) + 2 * np.asarray(vertices, dtype=np.int64)
    return np.argsort(-cost, kind="stable").astype(np.int32)


def et_lca_batch_fused(parent, offsets, qoffsets, qx, qy, max_tree_nodes, out=None, stats=False, ctx=None,
                       order=None):
    """Build many small trees (at most ``FUSED_MAX_NODES`` nodes each, at most
    ``max_tree_nodes``) and answer their queries in one kernel launch.
    ``parent`` / ``offsets`` as for :func:`et_tree_build_batch`; the queries
    come grouped by tree: tree t's are ``[qoffsets[t], qoffsets[t+1])`` of
    ``qx`` / ``qy`` (local ids). ``order`` (optional, a permutation of the
    tree ids on the device, e.g. from :func:`fused_order`) is the order in
    which workgroups take the trees. Returns the answers (local ids), and
    with ``stats`` also per-node depth, preorder and subtree size within each
    tree."""
    ctx = ctx or default_context()
    parent = _dev(parent, torch.int32, "parent")
    offsets = _dev(offsets, torch.int64, "offsets")
    qoffsets = _dev(qoffsets, torch.int64, "qoffsets")
    qx = _dev(qx, torch.int32, "qx")
    qy = _dev(qy, torch.int32, "qy")
    T = _i32(offsets.numel() - 1, "number of trees")
    if qoffsets.numel() != offsets.numel():
        raise ValueError("qoffsets must have one entry per tree plus one")
    if qx.numel() != qy.numel():
        raise ValueError("qx and qy differ in length")
    q = qx.numel()
    if out is None:
        out = torch.empty(q, dtype=torch.int32, device=qx.device)
    else:
        out = _dev(out, torch.int32, "out")
        if out.numel() < q:
            raise ValueError("out is shorter than the queries")
    depth = pre = size = None
    if stats:
        depth, pre, size = (torch.empty(parent.numel(), dtype=torch.int32, device=parent.device) for _ in range(3))
    if order is not None:
        order = _dev(order, torch.int32, "order")
        if order.numel() != T:
            raise ValueError("order must name every tree once")
    _check(_lib.et_lca_batch_fused(ctx.handle, _ptr(parent), _ptr(offsets), T, parent.numel(),
                                   _i32(max_tree_nodes, "max_tree_nodes"), _ptr(qoffsets), _ptr(qx), _ptr(qy), q,
                                   _ptr(out), _ptr(depth), _ptr(pre), _ptr(size), _ptr(order), _stream()),
           "et_lca_batch_fused")
    if stats:
        return out, {"depth": depth, "pre": pre, "size": size}
    return out


# ------------------------------------------------------------------ bridges

def et_bridges(row_ptr, col, mask=None, ctx=None, count=True):
    """Per-slot bridge bitmask (int32 words, bit k of word k//32 = slot k)
    and, with ``count``, the number of bridges (waits for the stream)."""
    ctx = ctx or default_context()
    row_ptr = _dev(row_ptr, torch.int32, "row_ptr")
    col = _dev(col, torch.int32, "col")
    n = _i32(row_ptr.numel() - 1, "vertex count", NODE_MAX)
    nnz = _i32(col.numel(), "CSR slot count")
    if mask is None:
        mask = torch.empty(max((nnz + 31) // 32, 1), dtype=torch.int32, device=col.device)
    c = _i64(0)
    _check(_lib.et_bridges(ctx.handle, _ptr(row_ptr), _ptr(col), n, nnz, _ptr(mask),
                           ctypes.byref(c) if count else None, _stream()), "et_bridges")
    return mask, (int(c.value) if count else None)


def et_bridges_batch(graphs=None, *, row_ptr=None, col=None, voff=None, soff=None, slots=None, mask=None,
                     ctx=None, counts=True):
    """Bridges of a batch of graphs in one pass. Either ``graphs``, a list of
    (row_ptr, col) device pairs with local ids, or the concatenated arrays
    ``row_ptr`` (each graph's n_t + 1 entries back to back), ``col`` and
    int64 device offsets ``voff`` / ``soff`` (n_graphs + 1 each), with the
    host list ``slots`` of slot counts per graph (read back from ``soff``
    when absent) to size the output. Returns the per-graph word-aligned
    masks as one int32 tensor, the list of each graph's (start, words) in
    it, and with ``counts`` a device int64 tensor of bridges per graph."""
    ctx = ctx or default_context()
    if graphs is not None:
        if len(graphs) == 0:
            raise ValueError("a batch needs at least one graph")
        rps = [_dev(g[0], torch.int32, "row_ptr") for g in graphs]
        cols = [_dev(g[1], torch.int32, "col") for g in graphs]
        dev = rps[0].device
        vs = [r.numel() - 1 for r in rps]
        ss = [c.numel() for c in cols]
        row_ptr = torch.cat(rps)
        col = torch.cat(cols) if sum(ss) else torch.empty(0, dtype=torch.int32, device=dev)
        # offsets go up from pinned memory without waiting for the stream
        voff = torch.tensor([0] + vs, dtype=torch.int64).cumsum(0).pin_memory().to(dev, non_blocking=True)
        soff = torch.tensor([0] + ss, dtype=torch.int64).cumsum(0).pin_memory().to(dev, non_blocking=True)
    else:
        row_ptr = _dev(row_ptr, torch.int32, "row_ptr")
        col = _dev(col, torch.int32, "col")
        voff = _dev(voff, torch.int64, "voff")
        soff = _dev(soff, torch.int64, "soff")
        if soff.numel() != voff.numel():
            raise ValueError("voff and soff must have the same length")
        ss = list(slots) if slots is not None else torch.diff(soff).cpu().tolist()
    T = _i32(len(ss), "number of graphs")
    n_total = _i32(row_ptr.numel() - T, "total vertex count", NODE_MAX)
    nnz = _i32(col.numel(), "total CSR slot count")
    if T < 1 or n_total < 0 or sum(ss) != nnz:
        raise ValueError("offsets do not match the concatenated arrays")
    words = [(x + 31) // 32 for x in ss]
    starts = [0]
    for w in words[:-1]:
        starts.append(starts[-1] + w)
    total = sum(words)
    if mask is None:
        mask = torch.empty(max(total, 1), dtype=torch.int32, device=col.device)
    out = torch.empty(T, dtype=torch.int64, device=col.device) if counts else None
    _check(_lib.et_bridges_batch(ctx.handle, _ptr(row_ptr), _ptr(col), _ptr(voff), _ptr(soff), T, n_total, nnz,
                                 _ptr(mask), mask.numel(), _ptr(out) if counts else None, _stream()),
           "et_bridges_batch")
    return mask, list(zip(starts, words)), out


def et_bridges_batch_fused(graphs=None, *, row_ptr=None, col=None, voff=None, soff=None, slots=None,
                           vertices=None, moff=None, max_vertices=None, max_slots=None, mask=None, ctx=None,
                           counts=True, order=None):
    """Bridges of many small graphs (at most ``FUSED_MAX_VERTICES`` vertices
    and ``FUSED_MAX_SLOTS`` CSR slots each) in one kernel launch. Arguments
    and results as for :func:`et_bridges_batch` (``vertices``: the host list
    of vertex counts per graph, read back from ``voff`` when absent); the
    bounds default to the largest graph's. ``moff``, the device int64 word
    offsets of the graphs' masks, is uploaded from the slot counts when not
    given (give it to capture the call in a graph: the upload's pinned
    buffer would not outlive the capture). ``order`` (optional, a device
    permutation of the graph ids, e.g. from :func:`fused_graph_order`) is the
    order in which workgroups take the graphs."""
    ctx = ctx or default_context()
    if graphs is not None:
        if len(graphs) == 0:
            raise ValueError("a batch needs at least one graph")
        rps = [_dev(g[0], torch.int32, "row_ptr") for g in graphs]
        cols = [_dev(g[1], torch.int32, "col") for g in graphs]
        dev = rps[0].device
        vs = [r.numel() - 1 for r in rps]
        ss = [c.numel() for c in cols]
        row_ptr = torch.cat(rps)
        col = torch.cat(cols) if sum(ss) else torch.empty(0, dtype=torch.int32, device=dev)
        voff = torch.tensor([0] + vs, dtype=torch.int64).cumsum(0).pin_memory().to(dev, non_blocking=True)
        soff = torch.tensor([0] + ss, dtype=torch.int64).cumsum(0).pin_memory().to(dev, non_blocking=True)
    else:
        row_ptr = _dev(row_ptr, torch.int32, "row_ptr")
        col = _dev(col, torch.int32, "col")
        voff = _dev(voff, torch.int64, "voff")
        soff = _dev(soff, torch.int64, "soff")
        if soff.numel() != voff.numel():
            raise ValueError("voff and soff must have the same length")
        ss = list(slots) if slots is not None else torch.diff(soff).cpu().tolist()
        vs = list(vertices) if vertices is not None else torch.diff(voff).cpu().tolist()
    T = _i32(len(ss), "number of graphs")
    n_total = _i32(row_ptr.numel() - T, "total vertex count", NODE_MAX)
    nnz = _i32(col.numel(), "total CSR slot count")
    if T < 1 or sum(ss) != nnz or sum(vs) != n_total:
        raise ValueError("offsets do not match the concatenated arrays")
    words = [(x + 31) // 32 for x in ss]
    starts = [0]
    for w in words:
        starts.append(starts[-1] + w)
    if moff is None:
        moff = torch.tensor(starts, dtype=torch.int64).pin_memory().to(col.device, non_blocking=True)
    else:
        moff = _dev(moff, torch.int64, "moff")
    total = starts[-1]
    if mask is None:
        mask = torch.empty(max(total, 1), dtype=torch.int32, device=col.device)
    out = torch.empty(T, dtype=torch.int64, device=col.device) if counts else None
    mv = _i32(max(vs) if max_vertices is None else max_vertices, "max_vertices")
    ms = _i32(max(ss) if max_slots is None else max_slots, "max_slots")
    if order is not None:
        order = _dev(order, torch.int32, "order")
        if order.numel() != T:
            raise ValueError("order must name every graph once")
    _check(_lib.et_bridges_batch_fused(ctx.handle, _ptr(row_ptr), _ptr(col), _ptr(voff), _ptr(soff), _ptr(moff), T,
                                       n_total, nnz, mv, ms, _ptr(mask), mask.numel(), _ptr(out) if counts else None,
                                       _ptr(order), _stream()), "et_bridges_batch_fused")
    return mask, list(zip(starts[:-1], words)), out


def et_bridges_ck(row_ptr, col, spanning="bfs", mask=None, ctx=None, count=True):
    """Bridges by Chaitanya-Kothapalli marking on a BFS forest
    (``spanning="bfs"``) or on the connectivity forest rooted by the Euler
    tour (``spanning="forest"``, the hybrid); same output as et_bridges."""
    ctx = ctx or default_context()
    row_ptr = _dev(row_ptr, torch.int32, "row_ptr")
    col = _dev(col, torch.int32, "col")
    n = _i32(row_ptr.numel() - 1, "vertex count", NODE_MAX)
    nnz = _i32(col.numel(), "CSR slot count")
    if mask is None:
        mask = torch.empty(max((nnz + 31) // 32, 1), dtype=torch.int32, device=col.device)
    c = _i64(0)
    sp = {"bfs": 0, "forest": 1}[spanning]
    _check(_lib.et_bridges_ck(ctx.handle, _ptr(row_ptr), _ptr(col), n, nnz, sp, _ptr(mask),
                              ctypes.byref(c) if count else None, _stream()), "et_bridges_ck")
    return mask, (int(c.value) if count else None)


def et_levels(parent, out=None, ctx=None):
    """Node levels by pointer jumping (the naive algorithm's preprocessing)."""
    ctx = ctx or default_context()
    parent = _dev(parent, torch.int32, "parent")
    n = _i32(parent.numel(), "tree size", NODE_MAX)
    if out is None:
        out = torch.empty_like(parent)
    _check(_lib.et_levels(ctx.handle, _ptr(parent), n, _ptr(out), _stream()), "et_levels")
    return out


def et_lca_naive(parent, level, qx, qy, out=None, ctx=None):
    """LCA queries by climbing parent pointers with the levels of et_levels."""
    ctx = ctx or default_context()
    parent = _dev(parent, torch.int32, "parent")
    level = _dev(level, torch.int32, "level")
    qx = _dev(qx, torch.int32, "qx")
    qy = _dev(qy, torch.int32, "qy")
    if qx.numel() != qy.numel() or level.numel() != parent.numel():
        raise ValueError("array lengths differ")
    n = _i32(parent.numel(), "tree size", NODE_MAX)
    if out is None:
        out = torch.empty_like(qx)
    _check(_lib.et_lca_naive(ctx.handle, _ptr(parent), _ptr(level), n, _ptr(qx), _ptr(qy),
                             qx.numel(), _ptr(out), _stream()), "et_lca_naive")
    return out


class BatchGraph:
    """A batched build plus batched LCA queries captured once in a HIP graph
    and replayed as one launch.

    A warm-up call fills the context's scratch pool first, so the captured
    calls allocate nothing; the captured tree stays alive with the graph
    (its tables are what the replays write). Every library fill is a kernel,
    so the graph holds no memset nodes. Inputs are read from the same
    device buffers at every replay; results land in ``out``. The scratch
    blocks the graph writes go back to the context's pool after capture, so
    the context (a new one unless ``ctx`` is given) must run no other work
    while the graph lives.
    """

    def __init__(self, parent, offsets, qtree, qx, qy, ctx=None):
        self.ctx = ctx or Context()
        self.inputs = (parent, offsets, qtree, qx, qy)
        warm = et_tree_build_batch(parent, offsets, ctx=self.ctx)
        warm.lca_batch(qtree, qx, qy)
        torch.cuda.synchronize()
        warm.free()
        self.out = torch.empty_like(qx)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.tree = et_tree_build_batch(parent, offsets, ctx=self.ctx)
            self.tree.lca_batch(qtree, qx, qy, out=self.out)

    def replay(self):
        self.graph.replay()
        return self.out

    def close(self):
        torch.cuda.synchronize()
        self.graph = None
        if self.tree is not None:
            self.tree.free()
            self.tree = None


class FusedBatchGraph:
    """The one-launch small-tree batch (et_lca_batch_fused) captured in a HIP
    graph: each replay is one kernel node. It allocates nothing and writes
    only ``out``; its work counter resets itself at the end of every launch,
    so replays need no set-up node. The context must not run another
    et_lca_batch_fused call while a replay is in flight.

    ``order`` is the order in which the launch hands out the trees: "auto"
    (the default) takes the costliest trees first when some tree has more
    than 1024 nodes (1024-lane workgroups, where a launch ending on a few
    large trees leaves most compute units idle) and the stored order
    otherwise; None keeps the stored order; or a device permutation."""

    def __init__(self, parent, offsets, qoffsets, qx, qy, max_tree_nodes, ctx=None, order="auto"):
        self.ctx = ctx or Context()
        if isinstance(order, str):
            if order != "auto":
                raise ValueError("order must be 'auto', None or a device permutation")
            order = None
            if max_tree_nodes > 1024:
                order = torch.from_numpy(fused_order(offsets.cpu().numpy(), qoffsets.cpu().numpy())).to(qx.device)
        self.order = order
        self.inputs = (parent, offsets, qoffsets, qx, qy)
        self.out = torch.empty_like(qx)
        et_lca_batch_fused(parent, offsets, qoffsets, qx, qy, max_tree_nodes, out=self.out, ctx=self.ctx,
                           order=order)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            et_lca_batch_fused(parent, offsets, qoffsets, qx, qy, max_tree_nodes, out=self.out, ctx=self.ctx,
                               order=order)

    def replay(self):
        self.graph.replay()
        return self.out

    def close(self):
        torch.cuda.synchronize()
        self.graph = None


class SplitBatchGraph:
    """A batch of trees split by size and captured in one HIP graph: the
    leading trees of at most ``FUSED_MAX_NODES`` nodes go through the
    one-launch kernel (et_lca_batch_fused), the others through the
    multi-kernel batched build and queries (et_tree_build_batch +
    et_lca_batch), one after the other on the capturing stream.

    ``offsets`` and ``qoffsets`` are host sequences of T + 1 int64 offsets
    (trees concatenated in ``parent``, their queries grouped by tree in
    ``qx``/``qy``); the caller orders the small trees first, as a batching
    host does when it sorts work by size class (the split is the longest
    such prefix). Answers land in ``out`` in query order. The tree-id and
    offset arrays of the two parts are made once here; replays read the
    same device buffers. The context (a new one unless ``ctx`` is given)
    must run no other work while the graph lives."""

    def __init__(self, parent, offsets, qoffsets, qx, qy, ctx=None):
        import numpy as np
        off = np.asarray(offsets, dtype=np.int64)
        qoff = np.asarray(qoffsets, dtype=np.int64)
        T = len(off) - 1
        if T < 1 or len(qoff) != T + 1 or off[0] != 0 or qoff[0] != 0:
            raise ValueError("offsets and qoffsets need T + 1 >= 2 entries starting at 0")
        if off[-1] != parent.numel() or qoff[-1] != qx.numel() or qx.numel() != qy.numel():
            raise ValueError("offsets or qoffsets do not match the arrays")
        sizes = np.diff(off)
        if (sizes < 1).any() or (np.diff(qoff) < 0).any():
            raise ValueError("every tree needs a node; query offsets must not decrease")
        big = np.nonzero(sizes > FUSED_MAX_NODES)[0]
        k = int(big[0]) if len(big) else T  # trees [0, k) fit one workgroup
        self.split = k
        self.ctx = ctx or Context()
        dev = parent.device
        n_s, q_s = int(off[k]), int(qoff[k])
        self.out = torch.empty_like(qx)
        self._small = None
        if k > 0:
            mx = int(sizes[:k].max())
            # costliest first when the trees run 1024-lane workgroups (see FusedBatchGraph)
            order = torch.from_numpy(fused_order(off[:k + 1], qoff[:k + 1])).to(dev) if mx > 1024 else None
            self._small = (parent[:n_s], torch.from_numpy(off[:k + 1].copy()).to(dev),
                           torch.from_numpy(qoff[:k + 1].copy()).to(dev), qx[:q_s], qy[:q_s], mx, self.out[:q_s],
                           order)
        self._large = None
        if k < T:
            qt = np.repeat(np.arange(T - k, dtype=np.int32), np.diff(qoff[k:]))
            self._large = (parent[n_s:], torch.from_numpy(off[k:] - off[k]).to(dev),
                           torch.from_numpy(qt).to(dev), qx[q_s:], qy[q_s:], self.out[q_s:])
        self.tree = None
        self._run(keep=False)  # warm-up: fills the scratch pool, so the captured calls allocate nothing
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run(keep=True)

    def _run(self, keep):
        if self._small is not None:
            p, o, qo, x, y, mx, out, order = self._small
            et_lca_batch_fused(p, o, qo, x, y, mx, out=out, ctx=self.ctx, order=order)
        if self._large is not None:
            p, o, qt, x, y, out = self._large
            tree = et_tree_build_batch(p, o, ctx=self.ctx)
            tree.lca_batch(qt, x, y, out=out)
            if keep:
                self.tree = tree  # the captured tables stay alive with the graph
            else:
                tree.free()

    def replay(self):
        self.graph.replay()
        return self.out

    def close(self):
        torch.cuda.synchronize()
        self.graph = None
        if self.tree is not None:
            self.tree.free()
            self.tree = None


class BridgesFusedGraph:
    """The one-launch graph batch (et_bridges_batch_fused) captured in a HIP
    graph: each replay is one kernel node writing ``mask`` and ``counts``.
    The context must not run another one-launch call while a replay is in
    flight. ``order`` is the order in which the launch hands out the graphs:
    "auto" (the default) the costliest first (:func:`fused_graph_order`),
    None the stored order, or a device permutation."""

    def __init__(self, row_ptr, col, voff, soff, slots, vertices, ctx=None, order="auto"):
        self.ctx = ctx or Context()
        slots, vertices = list(slots), list(vertices)
        if isinstance(order, str):
            if order != "auto":
                raise ValueError("order must be 'auto', None or a device permutation")
            order = torch.from_numpy(fused_graph_order(slots, vertices)).to(col.device)
        self.order = order
        words = [(x + 31) // 32 for x in slots]
        starts = [0]
        for w in words:
            starts.append(starts[-1] + w)
        self.moff = torch.tensor(starts, dtype=torch.int64, device=col.device)
        self.inputs = (row_ptr, col, voff, soff, self.moff)
        kw = dict(row_ptr=row_ptr, col=col, voff=voff, soff=soff, slots=slots, vertices=vertices, moff=self.moff,
                  ctx=self.ctx, order=order)
        et_bridges_batch_fused(**kw)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.mask, self.spans, self.counts = et_bridges_batch_fused(**kw)

    def replay(self):
        self.graph.replay()
        return self.mask, self.counts

    def close(self):
        torch.cuda.synchronize()
        self.graph = None


class BridgesBatchGraph:
    """A batched bridge call (et_bridges_batch on concatenated arrays)
    captured once in a HIP graph and replayed as one launch; ``mask`` holds
    the per-graph word-aligned masks (``spans`` gives each graph's words)
    and ``counts`` the bridges per graph after every replay. Capture rules
    as for BatchGraph: a warm-up call fills the pool first, and the context
    (a new one unless ``ctx`` is given) runs no other work while the graph
    lives."""

    def __init__(self, row_ptr, col, voff, soff, slots, ctx=None):
        self.ctx = ctx or Context()
        self.inputs = (row_ptr, col, voff, soff)
        slots = list(slots)
        et_bridges_batch(row_ptr=row_ptr, col=col, voff=voff, soff=soff, slots=slots, ctx=self.ctx)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.mask, self.spans, self.counts = et_bridges_batch(row_ptr=row_ptr, col=col, voff=voff, soff=soff,
                                                                  slots=slots, ctx=self.ctx)

    def replay(self):
        self.graph.replay()
        return self.mask, self.counts

    def close(self):
        torch.cuda.synchronize()
        self.graph = None
