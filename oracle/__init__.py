"""Reference (oracle) implementations used to check the GPU library.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library under
``paper_2305_03317_amd`` never does, and this package never imports it.

Contents
--------
* ``bc`` / ``source_detail``: plain single-threaded Brandes betweenness
  centrality in C (``bc_oracle.c``), following the paper's BC specification
  (Appendix, Fig. "BC computation in StarPlat") and the BFS-DAG semantics of
  ``iterateInBFS`` / ``iterateInReverse`` (Section 2.3.2).
* ``sssp``: single-source shortest paths on a weighted CSR (``sssp_oracle.c``,
  Dijkstra): the distances the paper's SSSP (Section 2.2, Fig. "SSSP
  computation in StarPlat"; pull form in the Appendix) converges to.
* ``pagerank``: the paper's pull PageRank (Appendix, Fig. "PR computation
  in StarPlat"), double buffered, in numpy float64 (``pagerank.py``).
* ``triangles`` / ``triangles_at``: the paper's node-iterator triangle count
  (Appendix, Fig. "TC computation in StarPlat"), and the count through one
  vertex, in C (``tc_oracle.c``).
* ``csr_from_edges``: the CSR the paper's graph library stores (Section 2.3.1
  "Data Types": offsets plus concatenated neighbour lists), built from an edge
  list with plain numpy set operations.
* ``sigma_flag``: the overflow rule applied to path counts (any sigma above
  1e300 or not finite).

Every function here is pinned by ``tests/test_oracle_*.py`` against brute
force, closed forms and invariants rather than against itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .pagerank import pagerank  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "bc_oracle.c"), os.path.join(_HERE, "sssp_oracle.c"),
         os.path.join(_HERE, "tc_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SIGMA_LIMIT = 1e300


def build(force: bool = False) -> str:
    """Compile the oracle C sources with gcc: -O2, no FP contraction, no fast-math."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_bc.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, f64p, f64p]
        lib.oracle_bc.restype = ctypes.c_int
        lib.oracle_source_detail.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32,
                                             i32p, f64p, f64p, i32p]
        lib.oracle_source_detail.restype = ctypes.c_int
        lib.oracle_sssp.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, i32p]
        lib.oracle_sssp.restype = ctypes.c_int
        lib.oracle_tc.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_tc.restype = ctypes.c_int
        lib.oracle_tc_vertex.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_tc_vertex.restype = ctypes.c_int
        lib.oracle_tc_each.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_tc_each.restype = ctypes.c_int
        _lib = lib
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def bc(row_ptr, col_idx, sources, return_sigma_max: bool = False):
    """Betweenness centrality of every vertex over the source list.

    Returns a float64 array of n = len(row_ptr) - 1 values (and, optionally,
    the largest path count seen, for the overflow rule)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    src, srcp = _i32(sources if len(sources) else np.zeros(1, np.int32))
    n = len(rp) - 1
    out = np.zeros(max(n, 1), dtype=np.float64)
    smax = ctypes.c_double(0.0)
    rc = lib.oracle_bc(n, rpp, cip, srcp, len(sources), _f64(out), ctypes.byref(smax))
    if rc != 0:
        raise ValueError("oracle_bc rejected its input (code %d)" % rc)
    out = out[:n]
    return (out, smax.value) if return_sigma_max else out


def source_detail(row_ptr, col_idx, source: int):
    """(dist int32[n], sigma f64[n], delta f64[n]) of one source."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    n = len(rp) - 1
    dist = np.empty(n, np.int32)
    sigma = np.empty(n, np.float64)
    delta = np.empty(n, np.float64)
    reached = ctypes.c_int32(0)
    rc = lib.oracle_source_detail(n, rpp, cip, int(source),
                                  dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _f64(sigma), _f64(delta), ctypes.byref(reached))
    if rc != 0:
        raise ValueError("oracle_source_detail rejected its input (code %d)" % rc)
    return dist, sigma, delta


INF = np.iinfo(np.int32).max  # distance of a vertex no path reaches


def sssp(row_ptr, col_idx, weights, source: int):
    """Shortest-path distances (int32[n]) from `source`; INF where unreached.
    weights: int32 per CSR entry (aligned with col_idx), non-negative."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    w, wp = _i32(weights if len(weights) else np.zeros(1, np.int32))
    n = len(rp) - 1
    dist = np.empty(max(n, 1), np.int32)
    rc = lib.oracle_sssp(n, rpp, cip, wp, int(source),
                         dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("oracle_sssp rejected its input (code %d)" % rc)
    return dist[:n]


def triangles(row_ptr, col_idx) -> int:
    """Number of triangles (each once) of a simple undirected CSR with sorted rows."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    out = ctypes.c_int64(0)
    rc = lib.oracle_tc(len(rp) - 1, rpp, cip, ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_tc rejected its input (code %d)" % rc)
    return int(out.value)


def triangles_at(row_ptr, col_idx, v: int) -> int:
    """Triangles through vertex v (adjacent pairs of its neighbours)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    out = ctypes.c_int64(0)
    rc = lib.oracle_tc_vertex(len(rp) - 1, rpp, cip, int(v), ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_tc_vertex rejected its input (code %d)" % rc)
    return int(out.value)


def triangles_each(row_ptr, col_idx):
    """int64[V]: triangles through every vertex (one call)."""
    lib = _load()
    rp, rpp = _i32(row_ptr)
    ci, cip = _i32(col_idx if len(col_idx) else np.zeros(1, np.int32))
    n = len(rp) - 1
    out = np.zeros(max(n, 1), np.int64)
    rc = lib.oracle_tc_each(n, rpp, cip, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("oracle_tc_each rejected its input (code %d)" % rc)
    return out[:n]


def sigma_flag(sigma_max: float) -> bool:
    """True when the overflow rule fires: a path count above 1e300 or not finite."""
    return not (np.isfinite(sigma_max) and sigma_max <= SIGMA_LIMIT)


def csr_from_edges(n: int, src, dst):
    """Simple undirected CSR from an edge list: self-loops dropped, each edge
    stored in both directions, duplicates removed, rows sorted ascending.

    Returns (row_ptr int32[n+1], col_idx int32[nnz])."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    a = np.concatenate([src[keep], dst[keep]])
    b = np.concatenate([dst[keep], src[keep]])
    key = np.unique(a * np.int64(n) + b)
    rows = key // n
    cols = key % n
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32)
