"""Pins of the PageRank oracle (``oracle/pagerank.py``) against things other
than itself, and proof that plausible slips in it fail them.

The oracle follows the paper's pull PageRank (Appendix, Fig. "PR computation
in StarPlat"), double buffered, with the absolute-difference convergence
test (a reading: the printed signed sum would stop after one iteration).
Checked against: regular graphs (PageRank stays 1/N), the star's closed-form
fixed point, the linear system the fixed point solves, a dense-matrix power
iteration, mass conservation, directed examples worked by hand, networkx's
pagerank, and the stopping rule.
"""
from __future__ import annotations

import os
import types

import networkx as nx
import numpy as np
import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "pagerank.py")
D = 0.85


def csr_undirected(G, oracle):
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return oracle.csr_from_edges(n, e[:, 0], e[:, 1])


def csr_directed(n, edges):
    rows = [[] for _ in range(n)]
    for u, v in edges:
        rows[u].append(v)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([v for r in rows for v in sorted(r)], np.int64)
    return rp, ci


def dense_step_matrix(rp, ci):
    """M[v, u] = 1/outdeg(u) for every edge u -> v."""
    n = len(rp) - 1
    M = np.zeros((n, n))
    for u in range(n):
        deg = rp[u + 1] - rp[u]
        for e in range(rp[u], rp[u + 1]):
            M[ci[e], u] += 1.0 / deg
    return M


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("G", [nx.cycle_graph(17), nx.complete_graph(9), nx.hypercube_graph(5),
                               nx.grid_2d_graph(6, 7, periodic=True)], ids=["cycle", "complete", "cube", "torus"])
def test_regular_graphs_stay_uniform(oracle_mod, G):
    G = nx.convert_node_labels_to_integers(G)
    rp, ci = csr_undirected(G, oracle_mod)
    n = len(rp) - 1
    pr, it, diff = oracle_mod.pagerank(rp, ci, 1e-12, D, 50)
    assert np.allclose(pr, 1.0 / n, rtol=1e-14, atol=0) and it == 1 and diff < 1e-15


@pytest.mark.parametrize("n", [3, 5, 40])
def test_star_fixed_point(oracle_mod, n):
    rp, ci = oracle_mod.csr_from_edges(n, np.zeros(n - 1), np.arange(1, n))
    pr, it, _ = oracle_mod.pagerank(rp, ci, 1e-15, D, 10000)
    # c = (1-d)/n + d (n-1) l,  l = (1-d)/n + d c / (n-1)
    a = (1 - D) / n
    c = (a + D * (n - 1) * a) / (1 - D * D)
    leaf = a + D * c / (n - 1)
    assert abs(pr[0] - c) <= 1e-13 and np.all(np.abs(pr[1:] - leaf) <= 1e-13)
    assert it > 2                      # a signed difference would have stopped after one


def test_linear_system_fixed_point(oracle_mod):
    rng = np.random.default_rng(3)
    for seed in range(4):
        G = nx.connected_watts_strogatz_graph(60, 4, 0.3, seed=seed)
        rp, ci = csr_undirected(G, oracle_mod)
        n = len(rp) - 1
        M = dense_step_matrix(rp, ci)
        x = np.linalg.solve(np.eye(n) - D * M, np.full(n, (1 - D) / n))
        pr, _, _ = oracle_mod.pagerank(rp, ci, 1e-15, D, 100000)
        assert np.max(np.abs(pr - x) / x) < 1e-11
    del rng


def test_dense_power_iteration_step_by_step(oracle_mod):
    G = nx.gnm_random_graph(50, 160, seed=4)
    rp, ci = csr_undirected(G, oracle_mod)
    n = len(rp) - 1
    M = dense_step_matrix(rp, ci)          # isolated vertices: zero columns
    x = np.full(n, 1.0 / n)
    for k in range(1, 7):
        x = (1 - D) / n + D * (M @ x)
        pr, it, _ = oracle_mod.pagerank(rp, ci, 0.0, D, 100, iterations=k)
        assert it == k and np.max(np.abs(pr - x) / x) < 1e-14


def test_mass_and_dangling(oracle_mod):
    # 10 vertices: a 6-cycle plus 4 isolated ones
    rp, ci = oracle_mod.csr_from_edges(10, np.arange(6), (np.arange(6) + 1) % 6)
    for k in (1, 2, 5):
        pr, _, _ = oracle_mod.pagerank(rp, ci, 0.0, D, 100, iterations=k)
        assert np.allclose(pr[6:], (1 - D) / 10, rtol=1e-15)      # no in-neighbours
        # the cycle keeps its own mass: x_k = (1-d)/10 + d x_{k-1}, x_0 = 1/10
        x = 0.1
        for _ in range(k):
            x = (1 - D) / 10 + D * x
        assert np.allclose(pr[:6], x, rtol=1e-14)


def test_directed_examples_by_hand(oracle_mod):
    # 0 -> 1 only (N = 2): one iteration gives (1-d)/2 and (1-d)/2 + d/2
    rp, ci = csr_directed(2, [(0, 1)])
    pr, _, _ = oracle_mod.pagerank(rp, ci, 0.0, D, 10, iterations=1)
    assert np.allclose(pr, [(1 - D) / 2, (1 - D) / 2 + D * 0.5], rtol=1e-15)
    # directed 3-cycle stays uniform; reversing an edge set changes in-neighbours
    rp, ci = csr_directed(3, [(0, 1), (1, 2), (2, 0)])
    assert np.allclose(oracle_mod.pagerank(rp, ci, 0.0, D, 10, iterations=3)[0], 1 / 3, rtol=1e-15)
    # 0 -> 1, 0 -> 2, 1 -> 2: vertex 2 gathers from both, 0 from nobody
    rp, ci = csr_directed(3, [(0, 1), (0, 2), (1, 2)])
    pr, _, _ = oracle_mod.pagerank(rp, ci, 0.0, D, 10, iterations=1)
    a = (1 - D) / 3
    assert np.allclose(pr, [a, a + D * (1 / 3) / 2, a + D * ((1 / 3) / 2 + 1 / 3)], rtol=1e-15)


def test_networkx_pagerank(oracle_mod):
    G = nx.barabasi_albert_graph(300, 3, seed=5)        # connected, no dangling vertex
    rp, ci = csr_undirected(G, oracle_mod)
    pr, _, _ = oracle_mod.pagerank(rp, ci, 1e-15, D, 100000)
    ref = nx.pagerank(G, alpha=D, tol=1e-15, max_iter=100000)
    ref = np.array([ref[v] for v in range(300)])
    assert np.max(np.abs(pr - ref) / ref) < 1e-9


def test_stopping_rule(oracle_mod):
    G = nx.barabasi_albert_graph(200, 2, seed=6)
    rp, ci = csr_undirected(G, oracle_mod)
    _, it, diff = oracle_mod.pagerank(rp, ci, 1e-6, D, 1000)
    _, it_prev, diff_prev = oracle_mod.pagerank(rp, ci, 0.0, D, 1000, iterations=it - 1)
    assert diff <= 1e-6 < diff_prev and it_prev == it - 1
    _, it, diff = oracle_mod.pagerank(rp, ci, 1e-12, D, 7)
    assert it == 7 and diff > 1e-12
    assert oracle_mod.pagerank(np.array([0]), np.zeros(0), 1e-6, D, 10)[1] == 0


# --------------------------------------------------------------------------
# Mutants: one-place slips in a copy of the oracle must fail the pins above
# --------------------------------------------------------------------------

MUTANTS = {
    "teleport_not_divided": ("(1.0 - delta) / n + delta * s", "(1.0 - delta) + delta * s"),
    "share_not_divided": ("share[has] = pr[has] / outdeg[has]", "share[has] = pr[has]"),
    "signed_difference": ("np.sum(np.abs(val - pr))", "np.sum(val - pr)"),
    "gather_out_neighbours": ("np.bincount(ci, weights=share[src_of_entry]", "np.bincount(src_of_entry, weights=share[ci]"),
    "no_damping_on_sum": ("(1.0 - delta) / n + delta * s", "(1.0 - delta) / n + s"),
    "in_place_start": ("pr = np.full(n, 1.0 / n)", "pr = np.full(n, 1.0)"),
    "one_extra_iteration": ("elif not (diff > beta and it < max_iter):", "elif not (diff > beta and it <= max_iter):"),
}


def load_variant(text):
    mod = types.ModuleType("pagerank_variant")
    exec(compile(text, "pagerank_variant", "exec"), mod.__dict__)
    return mod


class _Variant:
    def __init__(self, mod, oracle_mod):
        self.pagerank = mod.pagerank
        self.csr_from_edges = oracle_mod.csr_from_edges


BATTERY = [lambda m: test_regular_graphs_stay_uniform(m, nx.cycle_graph(17)),
           lambda m: test_star_fixed_point(m, 5), test_linear_system_fixed_point,
           test_dense_power_iteration_step_by_step, test_mass_and_dangling,
           test_directed_examples_by_hand, test_stopping_rule]


def battery_passes(m) -> bool:
    for chk in BATTERY:
        try:
            chk(m)
        except (AssertionError, ValueError, IndexError, ZeroDivisionError, FloatingPointError):
            return False
    return True


def test_unmodified_pagerank_passes_battery(oracle_mod):
    assert battery_passes(_Variant(load_variant(open(SRC).read()), oracle_mod))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pagerank_mutant_is_caught(oracle_mod, name):
    text = open(SRC).read()
    old, new = MUTANTS[name]
    assert text.count(old) == 1, "mutation site vanished: " + name
    assert not battery_passes(_Variant(load_variant(text.replace(old, new)), oracle_mod))
