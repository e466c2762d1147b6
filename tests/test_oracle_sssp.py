"""Pins of the SSSP oracle (``oracle/sssp_oracle.c``) against things other
than itself, and proof that plausible slips in it fail them.

The paper's SSSP (Section 2.2, Fig. "SSSP computation in StarPlat"; pull form
in the Appendix) relaxes edges with an atomic Min until no distance changes;
what it converges to is the shortest-path distance.  The oracle computes that
with Dijkstra's algorithm.  Checked here against:

* the definition itself: the least weight over every simple path, by
  enumeration, on every graph of at most 6 vertices of the networkx atlas
  with random weights (zero weights included);
* the paper's own procedure, written as a plain synchronous Bellman-Ford
  fixed point in Python, on small random graphs;
* closed forms: unit weights give BFS hop counts (the paper's unweighted
  case); a weighted path gives prefix sums; a unit grid gives Manhattan
  distance; a cycle gives the shorter way round;
* networkx's Dijkstra on larger random graphs;
* invariants at any size: dist[src] = 0, no edge can be relaxed further, every
  reached vertex other than the source has a tight predecessor, unreached
  vertices have no reached neighbour;
* the error contract: negative weights and distances beyond int32 rejected.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import networkx as nx
import numpy as np
import pytest

from tests import brute

INF = np.iinfo(np.int32).max
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "sssp_oracle.c")


def csr_of(G, oracle):
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return oracle.csr_from_edges(n, e[:, 0], e[:, 1])


def sym_weights(rp, ci, rng, lo=1, hi=100):
    """Random weight per undirected edge, stored in both directions."""
    n = len(rp) - 1
    w = np.empty(len(ci), np.int32)
    table = {}
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            key = (min(u, int(ci[e])), max(u, int(ci[e])))
            if key not in table:
                table[key] = int(rng.integers(lo, hi + 1))
            w[e] = table[key]
    return w


def enumerate_min(rp, ci, w, s):
    """min over all simple s-t paths of the summed weights (INF if none)."""
    adj = brute.adjacency(rp, ci)
    wt = {}
    for u in range(len(rp) - 1):
        for e in range(rp[u], rp[u + 1]):
            wt[(u, int(ci[e]))] = int(w[e])
    best = [INF] * (len(rp) - 1)
    for p in brute.simple_paths_from(adj, s):
        c = sum(wt[(p[i], p[i + 1])] for i in range(len(p) - 1))
        best[p[-1]] = min(best[p[-1]], c)
    return best


def bellman_ford_fixed_point(rp, ci, w, s):
    """The paper's procedure: every vertex modified in the last round relaxes
    its edges with Min; repeat until no distance changed."""
    n = len(rp) - 1
    dist = [INF] * n
    dist[s] = 0
    modified = [False] * n
    modified[s] = True
    while any(modified):
        nxt = [False] * n
        for v in range(n):
            if not modified[v]:
                continue
            for e in range(rp[v], rp[v + 1]):
                u = int(ci[e])
                cand = dist[v] + int(w[e])
                if cand < dist[u]:
                    dist[u] = cand
                    nxt[u] = True
        modified = nxt
    return dist


def check_invariants(rp, ci, w, s, d):
    brute.sssp_invariants(rp, ci, w, s, d, INF)


# --------------------------------------------------------------------------
# Definition by enumeration and the paper's fixed point
# --------------------------------------------------------------------------

ATLAS = [G for G in nx.graph_atlas_g() if 0 < G.number_of_nodes() <= 6]


@pytest.mark.parametrize("lo", [0, 1])
def test_atlas_enumeration(oracle_mod, lo):
    rng = np.random.default_rng(11 + lo)
    for G in ATLAS:
        rp, ci = csr_of(G, oracle_mod)
        w = sym_weights(rp, ci, rng, lo, 9)
        for s in range(len(rp) - 1):
            assert list(oracle_mod.sssp(rp, ci, w, s)) == enumerate_min(rp, ci, w, s)


@pytest.mark.parametrize("seed", range(6))
def test_bellman_ford_fixed_point(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 60))
    G = nx.gnm_random_graph(n, int(rng.integers(n, 4 * n)), seed=seed)
    rp, ci = csr_of(G, oracle_mod)
    w = sym_weights(rp, ci, rng)
    for s in rng.choice(n, 4, replace=False):
        assert list(oracle_mod.sssp(rp, ci, w, int(s))) == bellman_ford_fixed_point(rp, ci, w, int(s))


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def test_unit_weights_are_bfs_hops(oracle_mod):
    from paper_2305_03317_amd import graphs
    rp, ci = graphs.uniform(3000, 9000, 21)
    adj = brute.adjacency(rp, ci)
    w = np.ones(len(ci), np.int32)
    for s in (0, 17, 2999):
        hops = [x if x >= 0 else INF for x in brute.bfs_dist(adj, s)]
        assert list(oracle_mod.sssp(rp, ci, w, s)) == hops


def test_weighted_path_prefix_sums(oracle_mod):
    n = 40
    rp, ci = oracle_mod.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))
    step = np.arange(1, n) * 3 % 17 + 1            # weight of edge (i, i+1)
    w = np.empty(len(ci), np.int32)
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            w[e] = step[min(u, ci[e])]
    pref = np.concatenate([[0], np.cumsum(step)])
    for s in (0, 13, n - 1):
        assert np.array_equal(oracle_mod.sssp(rp, ci, w, s), np.abs(pref - pref[s]))


def test_unit_grid_manhattan(oracle_mod):
    a, b = 23, 17
    G = nx.convert_node_labels_to_integers(nx.grid_2d_graph(a, b), ordering="sorted")
    rp, ci = csr_of(G, oracle_mod)
    w = np.ones(len(ci), np.int32)
    for s in (0, 5 * b + 7, a * b - 1):
        r0, c0 = divmod(s, b)
        want = [abs(r - r0) + abs(c - c0) for r in range(a) for c in range(b)]
        assert list(oracle_mod.sssp(rp, ci, w, s)) == want


def test_cycle_shorter_way_round(oracle_mod):
    n = 31
    G = nx.cycle_graph(n)
    rp, ci = csr_of(G, oracle_mod)
    w = np.full(len(ci), 7, np.int32)
    d = oracle_mod.sssp(rp, ci, w, 4)
    assert list(d) == [7 * min((v - 4) % n, (4 - v) % n) for v in range(n)]


# --------------------------------------------------------------------------
# Library cross-check and invariants
# --------------------------------------------------------------------------

def test_networkx_dijkstra(oracle_mod):
    from paper_2305_03317_amd import graphs
    rp, ci = graphs.rmat(11, 8, seed=5)
    w = graphs.weights(rp, ci, 9)
    G = nx.Graph()
    G.add_nodes_from(range(len(rp) - 1))
    for u in range(len(rp) - 1):
        for e in range(rp[u], rp[u + 1]):
            G.add_edge(u, int(ci[e]), weight=int(w[e]))
    for s in graphs.sources(rp, 5, 3, min_degree=1):
        ref = nx.single_source_dijkstra_path_length(G, int(s))
        got = oracle_mod.sssp(rp, ci, w, int(s))
        assert all(got[v] == ref.get(v, INF) for v in range(len(rp) - 1))


@pytest.mark.parametrize("kind", ["rmat", "road", "uniform"])
def test_invariants(oracle_mod, kind):
    from paper_2305_03317_amd import graphs
    if kind == "rmat":
        rp, ci = graphs.rmat(14, 16, seed=3)
    elif kind == "road":
        rp, ci = graphs.road(96, 0.02, seed=3)
    else:
        rp, ci = graphs.uniform(20000, 30000, 3)      # sparse: several components
    w = graphs.weights(rp, ci, 4)
    for s in graphs.sources(rp, 3, 8, min_degree=1):
        check_invariants(rp, ci, w, int(s), oracle_mod.sssp(rp, ci, w, int(s)))


def test_generator_weights_symmetric_and_in_range():
    from paper_2305_03317_amd import graphs
    rp, ci = graphs.rmat(10, 16, seed=1)
    w = graphs.weights(rp, ci, 2)
    assert w.min() >= 1 and w.max() <= 100
    u = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    pair = {}
    for a, b, x in zip(u, ci, w):
        pair[(int(a), int(b))] = int(x)
    assert all(pair[(b, a)] == x for (a, b), x in pair.items())
    counts = np.bincount(w, minlength=101)[1:]
    assert counts.min() > 0.5 * counts.mean()        # roughly uniform


def test_isolated_source_and_single_vertex(oracle_mod):
    rp = np.array([0], np.int32)
    rp1 = np.array([0, 0], np.int32)
    assert list(oracle_mod.sssp(rp1, np.zeros(0, np.int32), np.zeros(0, np.int32), 0)) == [0]
    rp, ci = oracle_mod.csr_from_edges(4, [1, 2], [2, 3])
    w = np.full(len(ci), 5, np.int32)
    assert list(oracle_mod.sssp(rp, ci, w, 0)) == [0, INF, INF, INF]
    assert list(oracle_mod.sssp(rp, ci, w, 1)) == [INF, 0, 5, 10]


def test_rejects_bad_input(oracle_mod):
    rp, ci = oracle_mod.csr_from_edges(3, [0, 1], [1, 2])
    w = np.array([1, -1, -1, 1], np.int32)
    with pytest.raises(ValueError):
        oracle_mod.sssp(rp, ci, w, 0)                 # negative weight
    with pytest.raises(ValueError):
        oracle_mod.sssp(rp, ci, np.ones(len(ci), np.int32), 3)
    big = np.full(len(ci), 2**30 + 7, np.int32)      # 2 hops exceed int32
    with pytest.raises(ValueError):
        oracle_mod.sssp(rp, ci, big, 0)


# --------------------------------------------------------------------------
# Mutants: one-place slips in a copy of the oracle must fail the pins above
# --------------------------------------------------------------------------

MUTANTS = {
    "max_heap_push": ("if (h[p].d <= x.d) break;", "if (h[p].d >= x.d) break;"),
    "pop_larger_child": ("if (c + 1 < *n && h[c + 1].d < h[c].d) ++c;",
                         "if (c + 1 < *n && h[c + 1].d > h[c].d) ++c;"),
    "weight_of_row_head": ("(int64_t)weight[e];", "(int64_t)weight[row_ptr[u]];"),
    "unit_weight": ("(int64_t)weight[e];", "(int64_t)1;"),
    "source_not_zero": ("dist[src] = 0;", "dist[src] = 1;"),
    "skip_first_edge": ("for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {",
                        "for (int64_t e = row_ptr[u] + 1; e < row_ptr[u + 1]; ++e) {"),
    "unreached_zero": ("if (dist[v] == INT64_MAX) {\n            dist_out[v] = INT32_MAX;",
                       "if (dist[v] == INT64_MAX) {\n            dist_out[v] = 0;"),
    "overflow_not_flagged": ("rc = 3;", "rc = 0;"),
    "relax_with_popped_weight": ("const int64_t nd = dist[u] + (int64_t)weight[e];",
                                 "const int64_t nd = (int64_t)weight[e];"),
}


def compile_variant(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(c)])
    lib = ctypes.CDLL(str(so))
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_sssp.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, i32p]
    return lib


class _Variant:
    """Duck-typed stand-in for the oracle module, calling a compiled variant."""

    def __init__(self, lib, oracle_mod):
        self.lib = lib
        self.csr_from_edges = oracle_mod.csr_from_edges

    def sssp(self, rp, ci, w, s):
        p = lambda a: np.ascontiguousarray(a if len(a) else np.zeros(1), np.int32)
        rp, ci, w = p(rp), p(ci), p(w)
        out = np.empty(len(rp) - 1, np.int32)
        q = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        rc = self.lib.oracle_sssp(len(rp) - 1, q(rp), q(ci), q(w), int(s), q(out))
        if rc != 0:
            raise ValueError(rc)
        return out


def battery_passes(mod) -> bool:
    checks = [lambda: test_atlas_enumeration(mod, 1), lambda: test_bellman_ford_fixed_point(mod, 0),
              lambda: test_weighted_path_prefix_sums(mod), lambda: test_cycle_shorter_way_round(mod),
              lambda: test_isolated_source_and_single_vertex(mod), lambda: test_rejects_bad_input(mod)]
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError):
            return False
        except pytest.fail.Exception:
            return False
    return True


def test_unmodified_sssp_passes_battery(tmp_path, oracle_mod):
    assert battery_passes(_Variant(compile_variant(tmp_path, "orig", open(SRC).read()), oracle_mod))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_sssp_mutant_is_caught(tmp_path, oracle_mod, name):
    text = open(SRC).read()
    cut = text.index("#include")
    head, code = text[:cut], text[cut:]
    old, new = MUTANTS[name]
    assert code.count(old) >= 1, "mutation site vanished: " + name
    lib = compile_variant(tmp_path, name, head + code.replace(old, new, 1))
    assert not battery_passes(_Variant(lib, oracle_mod))
