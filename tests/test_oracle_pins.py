"""Pins of the CPU oracle against things other than itself.

The oracle follows the paper's BC specification (Appendix, Fig. "BC
computation in StarPlat"; DAG-neighbour semantics of Section 2.3.2).  Here it
is checked against: exhaustive shortest-path enumeration on every graph with
at most 7 vertices, closed forms, invariants, and networkx's betweenness
routine.  ``test_oracle_mutants.py`` shows that plausible slips in the oracle
fail these pins.
"""
from __future__ import annotations

import math

import networkx as nx
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from tests import brute


def csr_of(G: nx.Graph, oracle):
    n = G.number_of_nodes()
    nodes = sorted(G.nodes())
    assert nodes == list(range(n))
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return oracle.csr_from_edges(n, e[:, 0], e[:, 1])


def close(a, b, rel=1e-12):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), 1.0))


# --------------------------------------------------------------------------
# CSR builder
# --------------------------------------------------------------------------

def test_csr_from_edges_matches_networkx_adjacency(oracle_mod):
    rng = np.random.default_rng(7)
    n = 50
    src = rng.integers(0, n, 400)
    dst = rng.integers(0, n, 400)
    rp, ci = oracle_mod.csr_from_edges(n, src, dst)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(src, dst) if a != b)
    assert rp[0] == 0 and rp[-1] == len(ci) == 2 * G.number_of_edges()
    for v in range(n):
        assert list(ci[rp[v]:rp[v + 1]]) == sorted(G.neighbors(v))


# --------------------------------------------------------------------------
# Exhaustive brute force: every graph of the networkx atlas (<= 7 vertices)
# --------------------------------------------------------------------------

ATLAS = nx.graph_atlas_g()


def test_atlas_is_complete():
    assert len(ATLAS) == 1253


@pytest.mark.parametrize("chunk", range(8))
def test_atlas_all_sources_bruteforce(oracle_mod, chunk):
    """dist, sigma exact and BC within 1e-12 on every atlas graph, all sources."""
    for G in ATLAS[chunk::8]:
        n = G.number_of_nodes()
        if n == 0:
            continue
        rp, ci = csr_of(G, oracle_mod)
        adj = brute.adjacency(rp, ci)
        for s in range(n):
            d_ref, sig_ref, del_ref = brute.brute_source(adj, s)
            d, sig, dl = oracle_mod.source_detail(rp, ci, s)
            assert list(d) == d_ref
            assert [int(x) for x in sig] == sig_ref
            for v in range(n):
                if v != s:
                    assert math.isclose(dl[v], float(del_ref[v]), rel_tol=1e-12, abs_tol=0)
        bc_ref = brute.brute_bc(adj, list(range(n)))
        assert close(oracle_mod.bc(rp, ci, np.arange(n)), [float(x) for x in bc_ref])


def test_atlas_random_source_lists(oracle_mod):
    """Arbitrary source lists, duplicates allowed (a listed vertex counts once per entry)."""
    rng = np.random.default_rng(11)
    for G in ATLAS[200::37]:
        n = G.number_of_nodes()
        rp, ci = csr_of(G, oracle_mod)
        adj = brute.adjacency(rp, ci)
        srcs = list(rng.integers(0, n, rng.integers(1, 2 * n + 1)))
        bc_ref = brute.brute_bc(adj, srcs)
        assert close(oracle_mod.bc(rp, ci, srcs), [float(x) for x in bc_ref])


@settings(max_examples=60, deadline=None)
@given(st.integers(2, 12), st.floats(0.05, 0.9), st.integers(0, 2**31 - 1))
def test_random_graphs_bruteforce(n, p, seed):
    import oracle
    G = nx.gnp_random_graph(n, p, seed=seed)
    rp, ci = csr_of(G, oracle)
    adj = brute.adjacency(rp, ci)
    rng = np.random.default_rng(seed)
    srcs = list(rng.integers(0, n, rng.integers(1, n + 1)))
    bc_ref = brute.brute_bc(adj, srcs, layered=True)
    assert close(oracle.bc(rp, ci, srcs), [float(x) for x in bc_ref])


# --------------------------------------------------------------------------
# Closed forms (all sources, no halving: ordered pairs)
# --------------------------------------------------------------------------

def all_src_bc(G, oracle):
    rp, ci = csr_of(G, oracle)
    return oracle.bc(rp, ci, np.arange(G.number_of_nodes()))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 301])
def test_path(oracle_mod, n):
    bc = all_src_bc(nx.path_graph(n), oracle_mod)
    assert list(bc) == [2.0 * i * (n - 1 - i) for i in range(n)]


@pytest.mark.parametrize("n", [2, 3, 10, 500])
def test_star(oracle_mod, n):
    bc = all_src_bc(nx.star_graph(n - 1), oracle_mod)
    assert bc[0] == (n - 1) * (n - 2) and np.all(bc[1:] == 0)


@pytest.mark.parametrize("n", [1, 2, 5, 40])
def test_complete(oracle_mod, n):
    assert np.all(all_src_bc(nx.complete_graph(n), oracle_mod) == 0)


@pytest.mark.parametrize("n", [3, 5, 9, 101])
def test_odd_cycle(oracle_mod, n):
    assert np.all(all_src_bc(nx.cycle_graph(n), oracle_mod) == (n - 1) * (n - 3) / 4)


@pytest.mark.parametrize("n", [4, 6, 10, 100])
def test_even_cycle(oracle_mod, n):
    # antipodal pairs have two shortest paths: exercises the division
    assert close(all_src_bc(nx.cycle_graph(n), oracle_mod), ((n - 2) / 2) ** 2)


@pytest.mark.parametrize("a,b", [(1, 5), (2, 3), (3, 7), (5, 5)])
def test_complete_bipartite(oracle_mod, a, b):
    bc = all_src_bc(nx.complete_bipartite_graph(a, b), oracle_mod)
    assert close(bc[:a], b * (b - 1) / a) and close(bc[a:], a * (a - 1) / b)


def tree_bc_closed_form(G):
    """BC(v) = (n-1)^2 - sum over components C of T - v of |C|^2."""
    n = G.number_of_nodes()
    out = np.zeros(n)
    for v in range(n):
        H = G.copy()
        H.remove_node(v)
        out[v] = (n - 1) ** 2 - sum(len(c) ** 2 for c in nx.connected_components(H))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_tree(oracle_mod, seed):
    G = nx.random_labeled_tree(60, seed=seed)
    assert np.array_equal(all_src_bc(G, oracle_mod), tree_bc_closed_form(G))


def test_tree_source_subset(oracle_mod):
    """On a tree, delta_s(v) = n - 1 - |component of T - v containing s|."""
    G = nx.random_labeled_tree(40, seed=5)
    n = 40
    rp, ci = csr_of(G, oracle_mod)
    srcs = [3, 17, 17, 29]
    expect = np.zeros(n)
    for v in range(n):
        H = G.copy()
        H.remove_node(v)
        comp = {u: len(c) for c in nx.connected_components(H) for u in c}
        for s in srcs:
            if s != v:
                expect[v] += n - 1 - comp[s]
    assert np.array_equal(oracle_mod.bc(rp, ci, srcs), expect)


def test_grid_sigma_binomial(oracle_mod):
    W = 28  # largest W whose corner-to-corner count stays below 2^53
    G = nx.convert_node_labels_to_integers(nx.grid_2d_graph(W, W), ordering="sorted")
    rp, ci = csr_of(G, oracle_mod)
    d, sig, _ = oracle_mod.source_detail(rp, ci, 0)
    for i in range(W):
        for j in range(W):
            assert d[i * W + j] == i + j
            assert sig[i * W + j] == math.comb(i + j, i)


def diamond_chain(k):
    """k 4-cycles glued end to end: sigma doubles at every joint."""
    edges = []
    for i in range(k):
        a, b, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        edges += [(a, b), (a, c), (b, d), (c, d)]
    return 3 * k + 1, np.array(edges)


@pytest.mark.parametrize("k,flag", [(10, False), (996, False), (997, True), (1024, True)])
def test_diamond_chain_sigma_and_overflow_rule(oracle_mod, k, flag):
    n, e = diamond_chain(k)
    rp, ci = oracle_mod.csr_from_edges(n, e[:, 0], e[:, 1])
    _, sig, _ = oracle_mod.source_detail(rp, ci, 0)
    assert sig[n - 1] == 2.0 ** k if k < 1024 else math.isinf(sig[n - 1])
    _, smax = oracle_mod.bc(rp, ci, [0], return_sigma_max=True)
    assert oracle_mod.sigma_flag(smax) == flag


# --------------------------------------------------------------------------
# Invariants and special cases
# --------------------------------------------------------------------------

def test_global_sum_invariant(oracle_mod):
    """sum_v BC(v) = sum_s sum_{t reached, t != s} (dist_s(t) - 1)."""
    G = nx.gnm_random_graph(300, 900, seed=3)
    rp, ci = csr_of(G, oracle_mod)
    srcs = list(range(0, 300, 7)) + [5, 5]
    total = 0
    for s in srcs:
        d, _, _ = oracle_mod.source_detail(rp, ci, s)
        total += int(np.sum(d[d > 0] - 1))
    assert math.isclose(oracle_mod.bc(rp, ci, srcs).sum(), total, rel_tol=1e-12)


def test_structural_invariants(oracle_mod):
    G = nx.gnm_random_graph(400, 1500, seed=9)
    rp, ci = csr_of(G, oracle_mod)
    for s in [0, 17, 399]:
        d, sig, dl = oracle_mod.source_detail(rp, ci, s)
        assert np.all((sig >= 1) == (d >= 0))
        assert np.all(dl[d == d.max()] == 0)                 # deepest level: no children
        for w in range(400):                                 # sigma = sum over DAG parents
            if d[w] > 0:
                par = [u for u in ci[rp[w]:rp[w + 1]] if d[u] == d[w] - 1]
                assert sig[w] == sum(sig[u] for u in par)
        ref = nx.single_source_shortest_path_length(G, s)
        assert all(d[v] == ref.get(v, -1) for v in range(400))


def test_duplicate_source_counts_twice(oracle_mod):
    G = nx.gnm_random_graph(80, 200, seed=2)
    rp, ci = csr_of(G, oracle_mod)
    one = oracle_mod.bc(rp, ci, [13])
    assert np.array_equal(oracle_mod.bc(rp, ci, [13, 13]), 2 * one)


def test_empty_and_isolated(oracle_mod):
    G = nx.path_graph(5)
    G.add_node(5)
    rp, ci = csr_of(G, oracle_mod)
    assert np.all(oracle_mod.bc(rp, ci, []) == 0)
    assert np.all(oracle_mod.bc(rp, ci, [5]) == 0)
    d, sig, dl = oracle_mod.source_detail(rp, ci, 5)
    assert list(d) == [-1] * 5 + [0] and list(sig) == [0] * 5 + [1]
    assert oracle_mod.bc(np.zeros(1, np.int32), np.zeros(0, np.int32), []).shape == (0,)


def test_disconnected_components(oracle_mod):
    G = nx.disjoint_union(nx.path_graph(6), nx.star_graph(4))
    bc = all_src_bc(G, oracle_mod)
    assert list(bc[:6]) == [2.0 * i * 5 - 2.0 * i * i for i in range(6)]
    assert bc[6] == 4 * 3 and np.all(bc[7:] == 0)


def test_rejects_bad_input(oracle_mod):
    rp, ci = oracle_mod.csr_from_edges(3, [0, 1], [1, 2])
    with pytest.raises(ValueError):
        oracle_mod.bc(rp, ci, [3])
    with pytest.raises(ValueError):
        oracle_mod.bc(rp, np.array([0, 5, 1, 2], np.int32), [0])


def test_networkx_cross_check(oracle_mod):
    """networkx's subset betweenness halves on undirected graphs: x2 gives ours."""
    G = nx.gnm_random_graph(1500, 6000, seed=4)
    rp, ci = csr_of(G, oracle_mod)
    srcs = list(range(0, 1500, 50))
    ref = nx.betweenness_centrality_subset(G, srcs, list(G.nodes()), normalized=False)
    assert close(oracle_mod.bc(rp, ci, srcs), [2 * ref[v] for v in range(1500)], rel=1e-10)
