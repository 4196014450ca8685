"""CPU oracle for BFS levels and SSSP distances.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package.  It shares no code with the
HIP library and never calls it.

* ``bfs`` / ``dijkstra``: serial C implementations (``oracle.c``) of the plain
  definitions the paper's worklist BFS (Section 4.1) converges to, and of
  textbook single-source shortest paths (the paper states only BFS).
* ``kruskal``: the minimum spanning forest (serial Kruskal, ``oracle.c``) for
  the Boruvka workload of the Atomic construct (Section 3).
* ``floyd_warshall``: all-pairs min-plus closure in numpy, for tiny graphs.
* ``validate``: the invariants that characterize exact distances plus a
  valid parent tree, vectorized over the CSR.
* ``certify``: the same distance invariants as one serial C pass
  (``oracle_certify``), fast enough to check every full-size output.
* ``edges_scanned``: the TEPS numerator, the out-degree sum of the reached
  vertices (pinned by closed forms).
* ``mesh.check_mesh``: the complete validity check of a refined mesh for the
  Delaunay mesh refinement workload of the Exclusive construct (Section 3):
  conformity, Delaunay, quality bound, no encroached boundary edge, input
  points kept (``oracle/mesh.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .fw import floyd_warshall  # noqa: F401
from .validate import validate, validate_forest, ValidationError  # noqa: F401

INF = 0xFFFFFFFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_bfs.restype = ctypes.c_int64
        lib.oracle_bfs.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, u32p, i32p]
        lib.oracle_dijkstra.restype = ctypes.c_int64
        lib.oracle_dijkstra.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int32, u32p, i32p]
        lib.oracle_edges_scanned.restype = ctypes.c_int64
        lib.oracle_edges_scanned.argtypes = [ctypes.c_int32, i32p, u32p]
        lib.oracle_certify.restype = ctypes.c_int64
        lib.oracle_certify.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int32, u32p,
                                       ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_kruskal.restype = ctypes.c_int64
        lib.oracle_kruskal.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.POINTER(ctypes.c_uint8), i32p,
                                       ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    return rp, c


def bfs(row_ptr, col, src: int, with_parent: bool = True):
    """Queue BFS.  Returns (level uint32[n], parent int32[n] | None)."""
    rp, c = _csr(row_ptr, col)
    n = rp.size - 1
    level = np.empty(n, dtype=np.uint32)
    parent = np.empty(n, dtype=np.int32) if with_parent else None
    r = _load().oracle_bfs(n, _ptr(rp, ctypes.c_int32), _ptr(c, ctypes.c_int32), int(src),
                           _ptr(level, ctypes.c_uint32),
                           _ptr(parent, ctypes.c_int32) if with_parent else None)
    if r < 0:
        raise ValueError("oracle_bfs: invalid arguments")
    return level, parent


def dijkstra(row_ptr, col, w, src: int, with_parent: bool = True):
    """Binary-heap Dijkstra.  Returns (dist uint32[n], parent int32[n] | None)."""
    rp, c = _csr(row_ptr, col)
    ww = np.ascontiguousarray(w).view(np.uint32) if np.asarray(w).dtype.itemsize == 4 else \
        np.ascontiguousarray(w, dtype=np.uint32)
    n = rp.size - 1
    dist = np.empty(n, dtype=np.uint32)
    parent = np.empty(n, dtype=np.int32) if with_parent else None
    r = _load().oracle_dijkstra(n, _ptr(rp, ctypes.c_int32), _ptr(c, ctypes.c_int32),
                                _ptr(ww, ctypes.c_uint32), int(src), _ptr(dist, ctypes.c_uint32),
                                _ptr(parent, ctypes.c_int32) if with_parent else None)
    if r == -2:
        raise OverflowError("oracle_dijkstra: a distance does not fit in uint32")
    if r < 0:
        raise ValueError("oracle_dijkstra: invalid arguments")
    return dist, parent


def edges_scanned(row_ptr, level) -> int:
    """Sum of out-degrees over reached vertices (the TEPS numerator)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    lv = np.ascontiguousarray(level, dtype=np.uint32)
    return int(_load().oracle_edges_scanned(rp.size - 1, _ptr(rp, ctypes.c_int32),
                                            _ptr(lv, ctypes.c_uint32)))


_CERT_WHAT = {1: "d[src] != 0", 2: "an edge u -> v with d[v] > d[u] + w (or v unreached)",
              3: "a reached vertex without a tight in-edge", 4: "a zero weight"}


def certify(row_ptr, col, src: int, d, w=None) -> None:
    """Raise ValidationError unless ``d`` is exactly the shortest-path (BFS
    when ``w`` is None) distance vector from ``src``: the same three
    conditions as ``validate`` without parents, as one serial C pass
    (``oracle_certify``) that is fast enough for every full-size output."""
    rp, c = _csr(row_ptr, col)
    dd = np.ascontiguousarray(d).view(np.uint32) if np.asarray(d).dtype.itemsize == 4 else \
        np.ascontiguousarray(d, dtype=np.uint32)
    n = rp.size - 1
    if dd.size != n:
        raise ValidationError(f"distance array has {dd.size} entries, expected {n}")
    ww = None
    if w is not None:
        ww = np.ascontiguousarray(w).view(np.uint32) if np.asarray(w).dtype.itemsize == 4 else \
            np.ascontiguousarray(w, dtype=np.uint32)
    where = ctypes.c_int64()
    r = _load().oracle_certify(n, _ptr(rp, ctypes.c_int32), _ptr(c, ctypes.c_int32),
                               _ptr(ww, ctypes.c_uint32) if ww is not None else None, int(src),
                               _ptr(dd, ctypes.c_uint32), ctypes.byref(where))
    if r < 0:
        raise ValueError("oracle_certify: invalid arguments")
    if r:
        raise ValidationError(f"certificate fails: {_CERT_WHAT[int(r)]} at vertex {where.value}")


def kruskal(row_ptr, col, w):
    """Minimum spanning forest of a symmetric CSR under the total edge order
    (w, u, v).  Returns (weight, in_forest uint8[m] with both directions of
    every forest edge set, component int32[n] = smallest vertex id of the
    vertex's tree, number of forest edges)."""
    rp, c = _csr(row_ptr, col)
    ww = np.ascontiguousarray(w).view(np.uint32) if np.asarray(w).dtype.itemsize == 4 else \
        np.ascontiguousarray(w, dtype=np.uint32)
    n = rp.size - 1
    in_forest = np.empty(max(int(rp[-1]), 1), dtype=np.uint8)
    comp = np.empty(n, dtype=np.int32)
    edges = ctypes.c_int64()
    r = _load().oracle_kruskal(n, _ptr(rp, ctypes.c_int32), _ptr(c, ctypes.c_int32), _ptr(ww, ctypes.c_uint32),
                               _ptr(in_forest, ctypes.c_uint8), _ptr(comp, ctypes.c_int32), ctypes.byref(edges))
    if r == -3:
        raise ValueError("oracle_kruskal: the CSR is not symmetric (an edge lacks its equal-weight reverse)")
    if r < 0:
        raise ValueError("oracle_kruskal: invalid arguments")
    return int(r), in_forest[:int(rp[-1])], comp, int(edges.value)


def level_histogram(level) -> np.ndarray:
    """hist[k] = number of vertices at level k (reached vertices only)."""
    lv = np.asarray(level, dtype=np.uint32)
    reached = lv[lv != INF].astype(np.int64)
    if reached.size == 0:
        return np.zeros(0, dtype=np.int64)
    return np.bincount(reached)
