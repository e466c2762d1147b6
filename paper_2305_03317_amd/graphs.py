"""Seeded synthetic graphs (stand-ins for the paper's inputs) as int32 CSR.

Thin ctypes wrapper over ``libspgraph.so`` (``csrc/graphgen.cpp``): the
uniform-random, RMAT and road-like recipes, the CSR builder (self-loops
dropped, both directions stored, rows sorted, duplicates removed) and the
seeded source draw.  The paper's own graphs (Section 5, Table "Input graphs")
are not available; these recipes mirror the uniform-random (UR), RMAT (RM)
and road (US, GR) rows.

``workload(k)`` returns the five benchmark workloads with fixed seeds
(graph seed 1000 + k, source seed 2000 + k).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libspgraph.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import _build
            _build.build_graphgen()
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.spg_uniform.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(vp)]
        lib.spg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(vp)]
        lib.spg_road.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(vp)]
        lib.spg_from_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.POINTER(vp)]
        lib.spg_size.argtypes = [vp, i32p, ctypes.POINTER(ctypes.c_int64)]
        lib.spg_copy.argtypes = [vp, i32p, i32p]
        lib.spg_release.argtypes = [vp]
        lib.spg_release.restype = None
        lib.spg_sources.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_uint64, i32p]
        lib.spg_weights.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_uint64, i32p]
        _lib = lib
    return _lib


def _take(rc, handle):
    lib = _load()
    if rc != 0:
        raise ValueError("graph generator rejected its arguments (code %d)" % rc)
    n = ctypes.c_int32()
    nnz = ctypes.c_int64()
    lib.spg_size(handle, ctypes.byref(n), ctypes.byref(nnz))
    rp = np.empty(n.value + 1, np.int32)
    ci = np.empty(max(nnz.value, 1), np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.spg_copy(handle, rp.ctypes.data_as(i32p), ci.ctypes.data_as(i32p))
    lib.spg_release(handle)
    return rp, ci[:nnz.value]


def uniform(n: int, m: int, seed: int):
    """n vertices, exactly m distinct undirected non-loop edges with uniform endpoints."""
    h = ctypes.c_void_p()
    return _take(_load().spg_uniform(n, m, seed, ctypes.byref(h)), h)


def rmat(scale: int, edge_factor: int = 16, abc=RMAT_ABC, seed: int = 0, permute: bool = True):
    """RMAT: 2^scale vertices, edge_factor * 2^scale quadrant-recursive draws."""
    h = ctypes.c_void_p()
    a, b, c = abc
    return _take(_load().spg_rmat(scale, edge_factor, a, b, c, seed, int(permute), ctypes.byref(h)), h)


def road(width: int, extra_fraction: float = 0.02, seed: int = 0):
    """Road-like: MST of a width x width grid with random weights + extra grid edges."""
    h = ctypes.c_void_p()
    return _take(_load().spg_road(width, extra_fraction, seed, ctypes.byref(h)), h)


def from_edges(n: int, src, dst):
    """Simple symmetric CSR of an undirected edge list."""
    s = np.ascontiguousarray(src, np.int32)
    d = np.ascontiguousarray(dst, np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    h = ctypes.c_void_p()
    rc = _load().spg_from_edges(n, len(s), s.ctypes.data_as(i32p), d.ctypes.data_as(i32p), ctypes.byref(h))
    return _take(rc, h)


def sources(row_ptr, count: int, seed: int, min_degree: int = 0):
    """count distinct vertices of degree >= min_degree, seeded, in draw order."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    out = np.empty(max(count, 1), np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = _load().spg_sources(len(rp) - 1, rp.ctypes.data_as(i32p), count, min_degree, seed,
                             out.ctypes.data_as(i32p))
    if rc != 0:
        raise ValueError("not enough candidate sources")
    return out[:count]


def weights(row_ptr, col_idx, seed: int, lo: int = 1, hi: int = 100):
    """int32 weight per CSR entry, uniform on [lo, hi], equal in both directions
    of an edge (the paper's recipe for graphs without weights, Section 5)."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    out = np.empty(max(len(ci), 1), np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = _load().spg_weights(len(rp) - 1, rp.ctypes.data_as(i32p), ci.ctypes.data_as(i32p), lo, hi, seed,
                             out.ctypes.data_as(i32p))
    if rc != 0:
        raise ValueError("weight generator rejected its arguments (code %d)" % rc)
    return out[:len(ci)]


def directed_from(row_ptr, col_idx, seed: int):
    """Directed CSR (rows = out-edges, sorted) that keeps each undirected edge
    {u, w} of a symmetric CSR as one arc, u -> w or w -> u by a seeded coin."""
    rp = np.asarray(row_ptr, np.int64)
    ci = np.asarray(col_idx, np.int64)
    n = len(rp) - 1
    u = np.repeat(np.arange(n), np.diff(rp))
    keep = u < ci
    a, b = u[keep], ci[keep]
    flip = np.random.default_rng(seed).random(len(a)) < 0.5
    src, dst = np.where(flip, b, a), np.where(flip, a, b)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    out_rp = np.zeros(n + 1, np.int64)
    np.add.at(out_rp, src + 1, 1)
    return np.cumsum(out_rp).astype(np.int32), dst.astype(np.int32)


WORKLOADS = {
    1: dict(name="uniform-4096", kind="uniform", n=4096, m=32768, n_sources=16, min_degree=0),
    2: dict(name="rmat-20", kind="rmat", scale=20, n_sources=256, min_degree=1),
    3: dict(name="rmat-22", kind="rmat", scale=22, n_sources=1024, min_degree=1),
    4: dict(name="road-4096", kind="road", width=4096, n_sources=64, min_degree=0),
}

# Serving mix: RMAT scales 16, 18, 20, 22 and road-like grids 512..4096.
SERVING_GRAPHS = [("rmat", 16), ("rmat", 18), ("rmat", 20), ("rmat", 22),
                  ("road", 512), ("road", 1024), ("road", 2048), ("road", 4096)]


def serving_requests(graph_sizes, count: int, seed: int = 2005):
    """Seeded request list of the serving workload: (graph index, sources).

    The graph is chosen uniformly; the source count is log-uniform on
    [1, 512]; sources are distinct vertices of degree >= 1 of that graph.
    graph_sizes: list of (row_ptr) arrays, one per resident graph.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        gi = int(rng.integers(0, len(graph_sizes)))
        k = int(min(512, max(1, np.floor(np.exp(rng.uniform(0.0, np.log(513.0)))))))
        out.append((gi, sources(graph_sizes[gi], k, int(rng.integers(0, 2**31 - 1)), min_degree=1)))
    return out


def serving_graphs(seed: int = 1005):
    """The eight resident graphs of the serving workload: [(name, row_ptr, col_idx)]."""
    res = []
    for i, (kind, size) in enumerate(SERVING_GRAPHS):
        rp, ci = make_graph(kind, size, seed + 100 * i)
        res.append(("%s-%d" % (kind, size), rp, ci))
    return res


def make_graph(kind: str, size: int, seed: int):
    if kind == "rmat":
        return rmat(size, 16, RMAT_ABC, seed)
    if kind == "road":
        return road(size, 0.02, seed)
    raise ValueError(kind)


def workload(k: int, n_sources: int | None = None):
    """(row_ptr, col_idx, sources, spec) of benchmark workload k in 1..4."""
    spec = dict(WORKLOADS[k])
    gseed, sseed = 1000 + k, 2000 + k
    if spec["kind"] == "uniform":
        rp, ci = uniform(spec["n"], spec["m"], gseed)
    elif spec["kind"] == "rmat":
        rp, ci = rmat(spec["scale"], 16, RMAT_ABC, gseed)
    else:
        rp, ci = road(spec["width"], 0.02, gseed)
    ns = spec["n_sources"] if n_sources is None else n_sources
    src = sources(rp, ns, sseed, spec["min_degree"])
    spec.update(graph_seed=gseed, source_seed=sseed)
    return rp, ci, src, spec
