"""GPU parity of betweenness centrality on directed graphs (paper Section
2.3.1 graph type with nodes_to; BC program of the Appendix), through the C
ABI: sp_graph_upload_directed, sp_bc / sp_bc_batch (per-source path), and
sp_bfs_levels.  Same bar as the undirected parity tests: distances and path
counts exact (below 2^53), delta and BC within 1e-9 relative, zeros exact.
"""
from __future__ import annotations

import networkx as nx
import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs
from tests import brute
from tests.test_gpu_parity import assert_bc, assert_sigma

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


def directed_rmat(scale, seed):
    """Directed RMAT: the undirected recipe's draws, each kept as one arc in a
    seeded random direction."""
    rp, ci = graphs.rmat(scale, 16, seed=seed)
    u = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    keep = u < ci
    a, b = u[keep], ci[keep]
    flip = np.random.default_rng(seed).random(len(a)) < 0.5
    return brute.directed_csr(len(rp) - 1, np.where(flip, b, a), np.where(flip, a, b))


def cases():
    yield "gnp-300", brute.directed_csr(300, *np.array(list(nx.gnp_random_graph(300, 0.02, seed=1, directed=True).edges())).T)
    yield "rmat-12-directed", directed_rmat(12, 2)
    yield "rmat-14-directed", directed_rmat(14, 3)
    yield "path-200", brute.directed_csr(200, np.arange(199), np.arange(1, 200))


@pytest.mark.parametrize("name", ["gnp-300", "rmat-12-directed", "rmat-14-directed", "path-200"])
def test_bc_and_levels(sp, name):
    rp, ci = dict(cases())[name]
    n = len(rp) - 1
    g = sp.sp_graph_upload(rp, ci, validate=True, directed=True)
    srcs = graphs.sources(rp, min(24, n), 5, min_degree=1)
    print(name, "sources", len(srcs), flush=True)
    ref = oracle.bc(rp, ci, srcs)
    for fn in (sp.sp_bc, sp.sp_bc_batch):
        got, st = fn(g, srcs)
        assert st == sp.SP_OK
        assert_bc(got.cpu().numpy(), ref, "%s %s" % (name, fn.__name__))
    for s in srcs[:4]:
        d, sig, dl, _ = sp.sp_bfs_levels(g, int(s), with_sigma=True, with_delta=True)
        d_ref, sig_ref, dl_ref = oracle.source_detail(rp, ci, int(s))
        assert np.array_equal(d.cpu().numpy(), d_ref)
        assert_sigma(sig.cpu().numpy(), sig_ref, name)
        assert_bc(dl.cpu().numpy(), dl_ref, name + " delta")


def test_split_hubs_directed(sp):
    # the split-hub graph with every edge given a seeded direction: hubs keep
    # about half their neighbours as out-arcs and half as in-arcs, so both
    # hub lists of the per-source path meet rows either side of 2048
    from tests.test_gpu_parity import HUB_DEGREES, split_hub_graph
    rp, ci = split_hub_graph()
    n = len(rp) - 1
    u = np.repeat(np.arange(n), np.diff(rp))
    keep = u < ci
    a, b = u[keep], ci[keep]
    flip = np.random.default_rng(41).random(len(a)) < 0.5
    drp, dci = brute.directed_csr(n, np.where(flip, b, a), np.where(flip, a, b))
    dout = np.diff(drp)
    print("hub out-degrees", dout[60000:], flush=True)
    g = sp.sp_graph_upload(drp, dci, validate=True, directed=True)
    hubs = np.arange(60000, 60000 + len(HUB_DEGREES), dtype=np.int32)
    srcs = np.concatenate([hubs, graphs.sources(drp, 17, 42, min_degree=1)]).astype(np.int32)
    srcs = np.unique(srcs)
    ref = oracle.bc(drp, dci, srcs)
    got, st = sp.sp_bc(g, srcs)
    assert st == sp.SP_OK
    assert_bc(got.cpu().numpy(), ref, "directed split hubs")
    for s in list(hubs[-2:]) + list(srcs[:2]):
        d_ref, sig_ref, del_ref = oracle.source_detail(drp, dci, int(s))
        d, sig, dl, _ = sp.sp_bfs_levels(g, int(s), with_sigma=True, with_delta=True)
        assert np.array_equal(d.cpu().numpy(), d_ref)
        assert_sigma(sig.cpu().numpy(), sig_ref, "sigma, source %d" % s)
        assert_bc(dl.cpu().numpy(), np.where(d_ref > 0, del_ref, 0.0), "delta, source %d" % s)
    g.release()


def test_directed_differs_from_symmetrised(sp):
    # the same arcs read as undirected edges give another BC: direction is used
    rp, ci = brute.directed_csr(6, [0, 1, 2, 3, 4], [1, 2, 3, 4, 5])
    g = sp.sp_graph_upload(rp, ci, directed=True)
    got, _ = sp.sp_bc(g, np.arange(6))
    assert list(got.cpu().numpy()) == [float(i * (5 - i)) for i in range(6)]


def test_undirected_only_calls_are_refused(sp):
    rp, ci = brute.directed_csr(4, [0, 1, 2], [1, 2, 3])
    g = sp.sp_graph_upload(rp, ci, directed=True)
    for call in (lambda: sp.sp_batch_levels(g, [0]), lambda: sp.sp_pagerank(g),
                 lambda: sp.sp_triangle_count(g), lambda: sp.sp_graph_set_weights(g, np.ones(3, np.int32)),
                 lambda: sp.sp_autotune(g, [0])):
        with pytest.raises(sp.SpError) as e:
            call()
        assert e.value.status == sp.SP_ERR_NOT_SUPPORTED
    with pytest.raises(sp.SpError):          # malformed: an id out of range
        sp.sp_graph_upload(np.array([0, 1, 1], np.int32), np.array([5], np.int32), directed=True)
    with pytest.raises(sp.SpError):          # unsorted row, with validation
        sp.sp_graph_upload(np.array([0, 2, 2, 2], np.int32), np.array([2, 1], np.int32), validate=True,
                           directed=True)
