"""Graph generators and CSR builder (host code, CPU only)."""
from __future__ import annotations

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sps
import scipy.sparse.csgraph as csg

from paper_2305_03317_amd import graphs


def check_simple_symmetric(rp, ci):
    n = len(rp) - 1
    assert rp[0] == 0 and rp[-1] == len(ci)
    assert np.all(np.diff(rp) >= 0)
    assert np.all((ci >= 0) & (ci < n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(rows == ci), "self-loop"
    # strictly ascending within rows: sorted and duplicate-free
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    A = sps.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    assert (A != A.T).nnz == 0, "not symmetric"


def test_from_edges_matches_oracle_builder(oracle_mod):
    rng = np.random.default_rng(3)
    n = 300
    src = rng.integers(0, n, 5000)
    dst = rng.integers(0, n, 5000)
    rp, ci = graphs.from_edges(n, src, dst)
    orp, oci = oracle_mod.csr_from_edges(n, src, dst)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)


def test_uniform_exact_edge_count_and_determinism():
    rp, ci = graphs.uniform(4096, 32768, 1001)
    check_simple_symmetric(rp, ci)
    assert len(ci) == 65536
    rp2, ci2 = graphs.uniform(4096, 32768, 1001)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    rp3, ci3 = graphs.uniform(4096, 32768, 1002)
    assert not np.array_equal(ci, ci3)


def test_rmat_shape_and_determinism(monkeypatch):
    rp, ci = graphs.rmat(14, 16, graphs.RMAT_ABC, 7)
    check_simple_symmetric(rp, ci)
    n = 1 << 14
    assert len(rp) == n + 1
    deg = np.diff(rp)
    # skew: a heavy tail and many isolated vertices, as the recipe produces
    assert deg.max() > 50 * deg.mean()
    assert 0.2 < np.mean(deg == 0) < 0.5
    # chunked random streams: the thread count does not change the graph
    monkeypatch.setenv("SPG_THREADS", "1")
    rp1, ci1 = graphs.rmat(14, 16, graphs.RMAT_ABC, 7)
    assert np.array_equal(rp, rp1) and np.array_equal(ci, ci1)


def test_rmat_quadrant_probabilities_unpermuted():
    """Without relabelling, the top bit of (row, col) follows (a, b, c, d)."""
    # edge_factor 1 at scale 12: ~4K draws; check the fraction of draws whose
    # endpoints both lie in the low half (quadrant a), on the deduplicated graph
    rp, ci = graphs.rmat(12, 16, graphs.RMAT_ABC, 9, permute=False)
    n = 1 << 12
    rows = np.repeat(np.arange(n), np.diff(rp))
    low_low = np.mean((rows < n // 2) & (ci < n // 2))
    assert low_low > 0.45  # a = 0.57 before symmetrisation/dedupe


def test_road_tree_plus_extras():
    W = 64
    rp, ci = graphs.road(W, 0.02, 11)
    check_simple_symmetric(rp, ci)
    n = W * W
    grid_edges = 2 * W * (W - 1)
    extras = int(round(0.02 * grid_edges))
    assert len(ci) // 2 == (n - 1) + extras
    assert np.diff(rp).max() <= 4
    # every edge is a grid edge
    rows = np.repeat(np.arange(n), np.diff(rp))
    d = np.abs(rows - ci)
    assert np.all((d == 1) | (d == W))
    assert np.all((d != 1) | (np.minimum(rows, ci) % W != W - 1))
    A = sps.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    ncomp, _ = csg.connected_components(A, directed=False)
    assert ncomp == 1


def test_road_spanning_tree_is_minimal_shape():
    """With no extra edges the road graph is a spanning tree: BC has the tree closed form."""
    W = 12
    rp, ci = graphs.road(W, 0.0, 5)
    assert len(ci) // 2 == W * W - 1
    G = nx.Graph()
    rows = np.repeat(np.arange(W * W), np.diff(rp))
    G.add_edges_from(zip(rows.tolist(), ci.tolist()))
    assert nx.is_tree(G)


def test_sources_distinct_and_degree_rule():
    rp, ci = graphs.rmat(12, 16, graphs.RMAT_ABC, 3)
    s = graphs.sources(rp, 200, 44, min_degree=1)
    assert len(set(s.tolist())) == 200
    assert np.all(np.diff(rp)[s] >= 1)
    assert np.array_equal(s, graphs.sources(rp, 200, 44, min_degree=1))
    with pytest.raises(ValueError):
        graphs.sources(rp, len(rp), 1, min_degree=1)


def test_workload_one():
    rp, ci, src, spec = graphs.workload(1)
    assert spec["graph_seed"] == 1001 and spec["source_seed"] == 2001
    assert len(rp) == 4097 and len(ci) == 65536 and len(src) == 16
    assert len(set(src.tolist())) == 16
