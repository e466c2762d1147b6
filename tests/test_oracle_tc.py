"""Pins of the triangle-count oracle (``oracle/tc_oracle.c``) against things
other than itself, and proof that plausible slips in it fail them.

The oracle follows the paper's node iterator (Appendix, Fig. "TC computation
in StarPlat"): a triangle a < b < c is counted once, at b, with adjacency
tested by binary search in a sorted row.  Checked against: closed forms
(complete graphs C(n,3); trees, cycles longer than 3, grids and complete
bipartite graphs 0; wheels n - 1), brute force over all vertex triples,
trace(A^3) / 6 of the dense adjacency matrix, and networkx's per-vertex
triangles (also for the per-vertex count).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess

import networkx as nx
import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "tc_oracle.c")


def csr_of(G, oracle):
    G = nx.convert_node_labels_to_integers(G)
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return oracle.csr_from_edges(n, e[:, 0], e[:, 1])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 30])
def test_complete(oracle_mod, n):
    assert oracle_mod.triangles(*csr_of(nx.complete_graph(n), oracle_mod)) == math.comb(n, 3)


@pytest.mark.parametrize("G", [nx.random_labeled_tree(200, seed=1), nx.cycle_graph(9), nx.grid_2d_graph(9, 11),
                               nx.complete_bipartite_graph(7, 9), nx.path_graph(40)],
                         ids=["tree", "cycle9", "grid", "bipartite", "path"])
def test_triangle_free(oracle_mod, G):
    rp, ci = csr_of(G, oracle_mod)
    assert oracle_mod.triangles(rp, ci) == 0
    assert all(oracle_mod.triangles_at(rp, ci, v) == 0 for v in range(len(rp) - 1))


@pytest.mark.parametrize("n", [4, 5, 12, 100])
def test_wheel(oracle_mod, n):
    rp, ci = csr_of(nx.wheel_graph(n), oracle_mod)        # hub 0 + cycle of n - 1
    assert oracle_mod.triangles(rp, ci) == (n - 1 if n > 4 else 4)
    assert oracle_mod.triangles_at(rp, ci, 0) == (n - 1 if n > 4 else 3)


def test_brute_force_triples(oracle_mod):
    for seed in range(8):
        G = nx.gnp_random_graph(14, 0.45, seed=seed)
        rp, ci = csr_of(G, oracle_mod)
        adj = set(G.edges()) | {(b, a) for a, b in G.edges()}
        want = sum(1 for a, b, c in itertools.combinations(range(14), 3)
                   if (a, b) in adj and (b, c) in adj and (a, c) in adj)
        assert oracle_mod.triangles(rp, ci) == want


def test_trace_of_cube(oracle_mod):
    from paper_2305_03317_amd import graphs
    rp, ci = graphs.rmat(9, 16, seed=2)
    n = len(rp) - 1
    A = np.zeros((n, n), dtype=np.int64)
    for u in range(n):
        A[u, ci[rp[u]:rp[u + 1]]] = 1
    assert oracle_mod.triangles(rp, ci) == int(np.trace(A @ A @ A)) // 6


def test_networkx_per_vertex(oracle_mod):
    from paper_2305_03317_amd import graphs
    rp, ci = graphs.rmat(11, 16, seed=3)
    G = nx.Graph()
    G.add_nodes_from(range(len(rp) - 1))
    for u in range(len(rp) - 1):
        G.add_edges_from((u, int(w)) for w in ci[rp[u]:rp[u + 1]])
    t = nx.triangles(G)
    assert oracle_mod.triangles(rp, ci) == sum(t.values()) // 3
    for v in range(0, len(rp) - 1, 7):
        assert oracle_mod.triangles_at(rp, ci, v) == t[v]
    each = oracle_mod.triangles_each(rp, ci)
    assert list(each) == [t[v] for v in range(len(rp) - 1)]


def test_rejects_bad_input(oracle_mod):
    rp, ci = csr_of(nx.complete_graph(4), oracle_mod)
    with pytest.raises(ValueError):
        oracle_mod.triangles_at(rp, ci, 4)
    assert oracle_mod.triangles(np.array([0]), np.zeros(0)) == 0


MUTANTS = {
    "wrong_compare": ("if (col_idx[mid] < w) lo = mid + 1; else hi = mid - 1;",
                      "if (col_idx[mid] > w) lo = mid + 1; else hi = mid - 1;"),
    "search_misses_last": ("int64_t lo = row_ptr[u], hi = row_ptr[u + 1] - 1;",
                           "int64_t lo = row_ptr[u], hi = row_ptr[u + 1] - 2;"),
    "both_above": ("if (u >= v) continue;", "if (u <= v) continue;"),
    "w_above_u_not_v": ("if (w <= v) continue;", "if (w <= u) continue;"),
    "count_twice": ("count += is_an_edge(row_ptr, col_idx, u, w);", "count += 2 * is_an_edge(row_ptr, col_idx, u, w);"),
    "vertex_pairs_ordered": ("for (int64_t j = i + 1; j < row_ptr[v + 1]; ++j)",
                             "for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j)"),
}


def compile_variant(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(c)])
    lib = ctypes.CDLL(str(so))
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_tc.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_tc_vertex.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    return lib


class _Variant:
    def __init__(self, lib, oracle_mod):
        self.lib = lib
        self.csr_from_edges = oracle_mod.csr_from_edges

    def _call(self, f, rp, ci, *extra):
        rp = np.ascontiguousarray(rp, np.int32)
        ci = np.ascontiguousarray(ci if len(ci) else np.zeros(1), np.int32)
        out = ctypes.c_int64()
        q = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if f(len(rp) - 1, q(rp), q(ci), *extra, ctypes.byref(out)) != 0:
            raise ValueError
        return out.value

    def triangles(self, rp, ci):
        return self._call(self.lib.oracle_tc, rp, ci)

    def triangles_at(self, rp, ci, v):
        return self._call(self.lib.oracle_tc_vertex, rp, ci, int(v))

    def triangles_each(self, rp, ci):
        return [self.triangles_at(rp, ci, v) for v in range(len(rp) - 1)]


def battery_passes(m) -> bool:
    checks = [lambda: test_complete(m, 7), lambda: test_wheel(m, 12), lambda: test_brute_force_triples(m),
              lambda: test_networkx_per_vertex(m)]
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError):
            return False
    return True


def test_unmodified_tc_passes_battery(tmp_path, oracle_mod):
    assert battery_passes(_Variant(compile_variant(tmp_path, "orig", open(SRC).read()), oracle_mod))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_tc_mutant_is_caught(tmp_path, oracle_mod, name):
    text = open(SRC).read()
    cut = text.index("#include")
    head, code = text[:cut], text[cut:]
    old, new = MUTANTS[name]
    assert code.count(old) >= 1, "mutation site vanished: " + name
    lib = compile_variant(tmp_path, name, head + code.replace(old, new, 1))
    assert not battery_passes(_Variant(lib, oracle_mod))
