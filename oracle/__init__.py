"""CPU oracle for the Euler-tour hot path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. It wraps ``et_oracle.c`` (plain
sequential C, built by :func:`build` with gcc) through ctypes and shares no
code with the GPU library. Arrays go in and come out as numpy arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "et_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(path=None, flags=None):
    """Compile the oracle with gcc into ``oracle/liboracle.so`` (or ``path``);
    ``flags`` replaces the optimisation flags (a test builds it with
    sanitizers this way)."""
    out = path or _LIB
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *(flags or ["-O2"]), "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                           _SRC, "-o", tmp])
    os.replace(tmp, out)
    return out


def _bind(path):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "oracle_euler_tour": [P, i32, P, P, P, P, P, P],
        "oracle_list_rank": [P, i32, P, i32, P],
        "oracle_list_scan": [P, P, i32, P, i32, P, P],
        "oracle_lca_climb": [P, P, i32, P, P, i64, P],
        "oracle_lca_offline": [P, i32, P, P, i64, P],
        "oracle_sv_tables": [P, P, P, P, i32, P, P, P, P],
        "oracle_bridges": [P, P, i32, i64, P, P],
        "oracle_euler_tour_edges": [i32, i64, P, P, i32, P, P, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    other = os.environ.get("ET_ORACLE_LIB")   # another build of the same source (the sanitized one)
    if other:
        _lib = _bind(other)
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(_LIB)
    return _lib


def use_library(path):
    """Point this module at another build of the oracle source (used by the
    tests that plant mistakes in a copy of it); returns the previous one."""
    global _lib
    prev = _lib
    _lib = _bind(path) if isinstance(path, str) else path
    return prev


class OracleInputError(ValueError):
    """The oracle found the input malformed (code -4)."""


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc == -4:
        raise OracleInputError(f"{what}: malformed input")
    if rc != 0:
        raise RuntimeError(f"{what}: oracle error {rc}")


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def euler_tour(parent):
    """Euler tour of the tree (children in ascending id order).

    Returns a dict with ``tour`` [2(n-1)], ``rank`` [2n] (-1 on the root's
    two unused half-edge ids), ``depth``, ``pre``, ``size`` [n] and ``root``.
    Half-edge 2c goes down into c, 2c+1 goes up out of c.
    """
    parent = _i32(parent)
    n = parent.shape[0]
    tour = np.empty(max(2 * (n - 1), 0), dtype=np.int32)
    rank = np.empty(2 * n, dtype=np.int32)
    depth = np.empty(n, dtype=np.int32)
    pre = np.empty(n, dtype=np.int32)
    size = np.empty(n, dtype=np.int32)
    root = ctypes.c_int32(-1)
    rc = _load().oracle_euler_tour(_ptr(parent), n, _ptr(tour), _ptr(rank), _ptr(depth),
                                   _ptr(pre), _ptr(size), ctypes.cast(ctypes.pointer(root), ctypes.c_void_p))
    _check(rc, "euler_tour")
    return {"tour": tour, "rank": rank, "depth": depth, "pre": pre, "size": size,
            "root": int(root.value)}


def tree_succ(parent):
    """Successor array of the Euler tour built from the oracle's tour order
    (succ[tour[i]] = tour[i+1], -1 at the tail, -2 on the root's ids)."""
    t = euler_tour(parent)
    n = len(parent)
    succ = np.full(2 * n, -2, dtype=np.int32)
    tour = t["tour"]
    if tour.shape[0]:
        succ[tour[:-1]] = tour[1:]
        succ[tour[-1]] = -1
    head = int(tour[0]) if tour.shape[0] else -1
    return succ, head


def euler_tour_edges(n, eu, ev, root):
    """Euler tour of the tree given by the unordered edges (eu[i], ev[i]),
    rooted at ``root``, by the DCEL construction of Section 2.1.

    Half-edge 2i is (eu[i] -> ev[i]) and 2i+1 its twin. Returns ``succ`` and
    ``rank`` [2m] (succ -1 at the tail), ``tour`` (half-edge ids in order),
    and per node ``parent`` (-1 at the root), ``depth``, ``pre``, ``size``.
    """
    eu, ev = _i32(eu), _i32(ev)
    m = eu.shape[0]
    succ = np.empty(2 * m, dtype=np.int32)
    rank = np.empty(2 * m, dtype=np.int32)
    parent, depth, pre, size = (np.empty(n, dtype=np.int32) for _ in range(4))
    rc = _load().oracle_euler_tour_edges(int(n), m, _ptr(eu), _ptr(ev), int(root), _ptr(succ), _ptr(rank),
                                         _ptr(parent), _ptr(depth), _ptr(pre), _ptr(size))
    _check(rc, "euler_tour_edges")
    tour = np.empty(2 * m, dtype=np.int32)
    tour[rank] = np.arange(2 * m, dtype=np.int32)
    return {"succ": succ, "rank": rank, "tour": tour, "parent": parent, "depth": depth, "pre": pre,
            "size": size}


def list_rank(succ, heads):
    succ = _i32(succ)
    heads = _i32(heads)
    rank = np.empty(succ.shape[0], dtype=np.int32)
    rc = _load().oracle_list_rank(_ptr(succ), succ.shape[0], _ptr(heads), heads.shape[0], _ptr(rank))
    _check(rc, "list_rank")
    return rank


def list_scan(succ, weight, heads):
    """Weighted list ranking: per element the 32-bit wrapping sum of the
    weights from its list head through it, and its rank."""
    succ, weight, heads = _i32(succ), _i32(weight), _i32(heads)
    n = succ.shape[0]
    rank = np.empty(n, dtype=np.int32)
    out = np.empty(n, dtype=np.int32)
    rc = _load().oracle_list_scan(_ptr(succ), _ptr(weight), n, _ptr(heads), heads.shape[0], _ptr(rank), _ptr(out))
    _check(rc, "list_scan")
    return out, rank


def lca_climb(parent, depth, qx, qy):
    parent, depth, qx, qy = _i32(parent), _i32(depth), _i32(qx), _i32(qy)
    out = np.empty(qx.shape[0], dtype=np.int32)
    rc = _load().oracle_lca_climb(_ptr(parent), _ptr(depth), parent.shape[0], _ptr(qx), _ptr(qy),
                                  qx.shape[0], _ptr(out))
    _check(rc, "lca_climb")
    return out


def lca_offline(parent, qx, qy):
    parent, qx, qy = _i32(parent), _i32(qx), _i32(qy)
    out = np.empty(qx.shape[0], dtype=np.int32)
    rc = _load().oracle_lca_offline(_ptr(parent), parent.shape[0], _ptr(qx), _ptr(qy),
                                    qx.shape[0], _ptr(out))
    _check(rc, "lca_offline")
    return out


def sv_tables(parent, depth, pre, size):
    """Inlabel, ascendant and head tables from their definitions.

    ``head_parent``/``head_depth`` are indexed by inlabel value (n+1
    entries); labels that no path uses hold -3.
    """
    parent, depth, pre, size = _i32(parent), _i32(depth), _i32(pre), _i32(size)
    n = parent.shape[0]
    inl = np.empty(n, dtype=np.uint32)
    asc = np.empty(n, dtype=np.uint32)
    hp = np.empty(n + 1, dtype=np.int32)
    hd = np.empty(n + 1, dtype=np.int32)
    rc = _load().oracle_sv_tables(_ptr(parent), _ptr(depth), _ptr(pre), _ptr(size), n,
                                  _ptr(inl), _ptr(asc), _ptr(hp), _ptr(hd))
    _check(rc, "sv_tables")
    return {"inlabel": inl, "asc": asc, "head_parent": hp, "head_depth": hd}


def bridges(row_ptr, col):
    """Per-slot bridge bitmask (uint32 words) and bridge count."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = _i32(col)
    n = row_ptr.shape[0] - 1
    nnz = col.shape[0]
    mask = np.zeros(max((nnz + 31) // 32, 1), dtype=np.uint32)
    cnt = ctypes.c_int64(0)
    rc = _load().oracle_bridges(_ptr(row_ptr), _ptr(col), n, nnz, _ptr(mask),
                                ctypes.cast(ctypes.pointer(cnt), ctypes.c_void_p))
    _check(rc, "bridges")
    return mask[: (nnz + 31) // 32], int(cnt.value)


def mask_to_bool(mask, nnz):
    """Expand a per-slot bitmask into a bool array of length ``nnz``."""
    bits = np.unpackbits(np.asarray(mask, dtype=np.uint32).view(np.uint8), bitorder="little")
    return bits[:nnz].astype(bool)
