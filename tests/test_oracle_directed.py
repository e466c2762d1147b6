"""Pins of the BC oracle on directed graphs (paper Section 2.3.1: the graph
type offers out-neighbours and nodes_to, so the BC program runs on directed
graphs too; Brandes then counts shortest directed paths).

The oracle's BFS and reverse sweep both walk a vertex's own CSR row, which
for a directed graph is its out-edges: parents of w are the v with an edge
v -> w one level up, children of v the w it points to one level down.
Checked against: exhaustive path enumeration on random digraphs; closed
forms (a directed path, a directed cycle, an out-star); networkx's
betweenness on DiGraphs (unnormalised, ordered pairs).
"""
from __future__ import annotations


import networkx as nx
import numpy as np
import pytest

from tests import brute


def close(a, b, rel=1e-12):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), 1.0))


@pytest.mark.parametrize("seed", range(10))
def test_random_digraphs_bruteforce(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 10))
    m = int(rng.integers(n, 3 * n))
    rp, ci = brute.directed_csr(n, rng.integers(0, n, m), rng.integers(0, n, m))
    adj = brute.adjacency(rp, ci)
    for s in range(n):
        d_ref, sig_ref, del_ref = brute.brute_source(adj, s)
        d, sig, dl = oracle_mod.source_detail(rp, ci, s)
        assert list(d) == d_ref and list(sig) == [float(x) for x in sig_ref]
        assert close(dl, [float(x) for x in del_ref])
    srcs = list(range(n))
    assert close(oracle_mod.bc(rp, ci, srcs), [float(x) for x in brute.brute_bc(adj, srcs)])


def test_directed_path(oracle_mod):
    n = 12
    rp, ci = brute.directed_csr(n, np.arange(n - 1), np.arange(1, n))
    bc = oracle_mod.bc(rp, ci, np.arange(n))
    assert list(bc) == [float(i * (n - 1 - i)) for i in range(n)]      # pairs s < i < t only


def test_directed_cycle(oracle_mod):
    n = 9
    rp, ci = brute.directed_csr(n, np.arange(n), (np.arange(n) + 1) % n)
    bc = oracle_mod.bc(rp, ci, np.arange(n))
    assert np.all(bc == (n - 1) * (n - 2) / 2)


def test_out_star_and_in_star(oracle_mod):
    n = 8
    rp, ci = brute.directed_csr(n, np.zeros(n - 1), np.arange(1, n))      # centre -> leaves
    assert np.all(oracle_mod.bc(rp, ci, np.arange(n)) == 0)
    src = np.concatenate([np.arange(1, 4), np.zeros(4)])                 # 1..3 -> 0 -> 4..7
    dst = np.concatenate([np.zeros(3), np.arange(4, 8)])
    rp, ci = brute.directed_csr(n, src, dst)
    bc = oracle_mod.bc(rp, ci, np.arange(n))
    assert bc[0] == 3 * 4 and np.all(bc[1:] == 0)


def test_networkx_digraph(oracle_mod):
    G = nx.gnp_random_graph(120, 0.04, seed=3, directed=True)
    e = np.array(list(G.edges()), dtype=np.int64)
    rp, ci = brute.directed_csr(120, e[:, 0], e[:, 1])
    ref = nx.betweenness_centrality(G, normalized=False)
    bc = oracle_mod.bc(rp, ci, np.arange(120))
    assert close(bc, [ref[v] for v in range(120)], 1e-12)
    srcs = [3, 17, 40, 41, 99]
    sub = nx.betweenness_centrality_subset(G, srcs, list(G.nodes()), normalized=False)
    assert close(oracle_mod.bc(rp, ci, srcs), [sub[v] for v in range(120)], 1e-12)
