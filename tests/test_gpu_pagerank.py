"""GPU parity of PageRank against the CPU oracle, through the C ABI (paper
Appendix, Fig. "PR computation in StarPlat"; absolute-difference stopping
test).

Bar: the GPU reports how many iterations it ran; the oracle runs exactly as
many, and every value agrees within 1e-9 relative (both are binary64; only
the order of each vertex's sum differs, so agreement is near 1e-15).  The
stopping decision is a floating-point comparison taken on both sides: the
GPU's count must be one the oracle's own differences allow (its last
difference at most beta, the one before above it, up to a 1e-12 absolute
slack for rounding), or max_iter.  Repeated runs must be bit-identical.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs

pytestmark = pytest.mark.gpu

D = 0.85
TOL = 1e-9


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


def check(sp, g, rp, ci, beta, max_iter, cfg=None, what=""):
    got = sp.sp_pagerank(g, beta, D, max_iter, config=cfg).cpu().numpy()
    st = sp.sp_pagerank_get_last_stats()
    k = st["iterations"]
    assert 1 <= k <= max_iter, what
    ref, it, diff = oracle.pagerank(rp, ci, beta, D, max_iter, iterations=k)
    assert it == k
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= TOL, "%s: max rel err %g" % (what, rel)
    # The stopping decision is consistent with the oracle's differences.  Near
    # convergence a difference is a small quantity taken from values of order
    # 1/N..1 whose sums were rounded in different orders (the oracle adds a
    # hub's row sequentially, with error up to about degree x 1e-16 of the
    # value), so it is compared with an absolute slack of 1e-12.
    slack = 1e-9 * diff + 1e-12
    assert abs(st["diff"] - diff) <= slack, (what, st["diff"], diff)
    if k < max_iter:
        assert diff <= beta + slack, what
    if k > 1:
        prev = oracle.pagerank(rp, ci, beta, D, max_iter, iterations=k - 1)[2]
        assert prev > beta - (1e-9 * prev + 1e-12), what
    return got, st


def small_graphs():
    yield "uniform-4096", graphs.uniform(4096, 32768, 7)
    yield "rmat-13", graphs.rmat(13, 16, seed=8)         # hubs and isolated vertices
    yield "road-80", graphs.road(80, 0.02, seed=9)
    yield "sparse-forest", graphs.uniform(5000, 3000, 10)


@pytest.mark.parametrize("beta", [1e-6, 1e-10, 0.0])
def test_small_graphs(sp, beta):
    for name, (rp, ci) in small_graphs():
        print(name, "beta", beta, flush=True)
        g = sp.sp_graph_upload(rp, ci)
        check(sp, g, rp, ci, beta, 60, what=name)
        g.release()


@pytest.mark.parametrize("cfg", [{"block_size": 128}, {"block_size": 512}, {"chunk_iters": -3},
                                 {"chunk_iters": 3}, {"chunk_iters": 1}])
def test_launch_configurations(sp, cfg):
    rp, ci = graphs.rmat(12, 16, seed=13)
    g = sp.sp_graph_upload(rp, ci)
    print(cfg, flush=True)
    check(sp, g, rp, ci, 1e-8, 100, cfg, what=str(cfg))


def test_reproducible_and_exact_counts(sp):
    rp, ci = graphs.rmat(13, 16, seed=14)
    g = sp.sp_graph_upload(rp, ci)
    a = sp.sp_pagerank(g, 1e-9, D, 100).cpu().numpy()
    k = sp.sp_pagerank_get_last_stats()["iterations"]
    b = sp.sp_pagerank(g, 1e-9, D, 100, config={"chunk_iters": -5}).cpu().numpy()
    assert np.array_equal(a, b) and sp.sp_pagerank_get_last_stats()["iterations"] == k
    sp.sp_pagerank(g, 0.0, D, 17)
    assert sp.sp_pagerank_get_last_stats()["iterations"] == 17
    sp.sp_pagerank(g, 4.0, D, 50)          # the summed change never exceeds 2
    assert sp.sp_pagerank_get_last_stats()["iterations"] == 1     # do-while: one always runs


def test_closed_forms(sp):
    # a cycle stays at 1/N; a star with a 3000-leaf hub reaches its fixed point
    n = 1000
    rp, ci = graphs.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    g = sp.sp_graph_upload(rp, ci)
    got = sp.sp_pagerank(g, 1e-12, D, 10).cpu().numpy()
    assert np.allclose(got, 1.0 / n, rtol=1e-14, atol=0)
    n = 3001
    rp, ci = graphs.from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    g = sp.sp_graph_upload(rp, ci)
    got = sp.sp_pagerank(g, 1e-15, D, 100000).cpu().numpy()
    a = (1 - D) / n
    c = (a + D * (n - 1) * a) / (1 - D * D)
    assert abs(got[0] - c) <= 1e-13 * c and np.allclose(got[1:], a + D * c / (n - 1), rtol=1e-12)
    check(sp, g, rp, ci, 1e-9, 500, what="star")


def test_edge_cases(sp):
    g = sp.sp_graph_upload(np.array([0, 0], np.int32), np.zeros(0, np.int32))
    assert list(sp.sp_pagerank(g, 1e-6, D, 10).cpu().numpy()) == [pytest.approx(1 - D, rel=1e-15)]
    g = sp.sp_graph_upload(np.array([0], np.int32), np.zeros(0, np.int32))
    assert sp.sp_pagerank(g, 1e-6, D, 10).numel() == 0
    rp, ci = graphs.from_edges(3, [0], [1])
    g = sp.sp_graph_upload(rp, ci)
    for bad in [dict(beta=-1.0), dict(delta=1.5), dict(max_iter=0)]:
        args = dict(beta=1e-6, delta=D, max_iter=10)
        args.update(bad)
        with pytest.raises(sp.SpError):
            sp.sp_pagerank(g, **args)
    with pytest.raises(sp.SpError):
        sp.sp_pagerank(g, config={"block_size": 64})
    got = sp.sp_pagerank(g, 0.0, 0.0, 3).cpu().numpy()          # delta 0: teleport only
    assert np.allclose(got, 1 / 3, rtol=1e-15)


@pytest.mark.parametrize("k", [3, 4])
def test_full_size(sp, k):
    rp, ci, _, spec = graphs.workload(k)
    print("workload", spec["name"], flush=True)
    g = sp.sp_graph_upload(rp, ci)
    got = sp.sp_pagerank(g, 0.0, D, 3).cpu().numpy()
    assert sp.sp_pagerank_get_last_stats()["iterations"] == 3
    ref, _, _ = oracle.pagerank(rp, ci, 0.0, D, 3, iterations=3)
    assert np.max(np.abs(got - ref) / ref) <= TOL


def directed_cases():
    """Directed graphs: RMAT arcs with seeded directions (hubs with long
    incoming rows, vertices without outgoing arcs), an in-star whose centre
    has 3000 incoming arcs and none outgoing, an out-star, and a directed
    cycle."""
    from tests import brute
    rp, ci = graphs.rmat(13, 16, seed=15)
    yield "rmat-13-directed", graphs.directed_from(rp, ci, 16)
    n = 3001
    yield "in-star", brute.directed_csr(n, np.arange(1, n), np.zeros(n - 1, np.int64))
    yield "out-star", brute.directed_csr(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    yield "cycle", brute.directed_csr(500, np.arange(500), (np.arange(500) + 1) % 500)


@pytest.mark.parametrize("name", ["rmat-13-directed", "in-star", "out-star", "cycle"])
@pytest.mark.parametrize("cfg", [None, {"block_size": 128}, {"chunk_iters": -3}])
def test_directed(sp, name, cfg):
    """PageRank over incoming arcs (the paper's nodes_to), shares divided by
    the outgoing row's length; a vertex with no outgoing arcs passes nothing
    on."""
    rp, ci = dict(directed_cases())[name]
    g = sp.sp_graph_upload(rp, ci, validate=True, directed=True)
    print(name, cfg, flush=True)
    got, _ = check(sp, g, rp, ci, 1e-10, 200, cfg, what=name)
    if name == "cycle":
        assert np.allclose(got, 1 / 500, rtol=1e-14, atol=0)
    if name == "in-star":  # leaves: teleport only; the centre gathers every leaf
        n = len(rp) - 1
        a = (1 - D) / n
        assert np.allclose(got[1:], a, rtol=1e-14)
        assert abs(got[0] - (a + D * (n - 1) * a)) <= 1e-13 * got[0]
    g.release()


def test_directed_full_size(sp):
    rp, ci, _, spec = graphs.workload(3)
    drp, dci = graphs.directed_from(rp, ci, 4003)
    g = sp.sp_graph_upload(drp, dci, directed=True)
    got = sp.sp_pagerank(g, 0.0, D, 3).cpu().numpy()
    ref, _, _ = oracle.pagerank(drp, dci, 0.0, D, 3, iterations=3)
    assert np.max(np.abs(got - ref) / ref) <= TOL
    g.release()
