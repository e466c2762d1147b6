"""GPU parity of triangle counting against the CPU oracle, through the C ABI
(paper Appendix, Fig. "TC computation in StarPlat").

Bar: integers, so bit-exact: the total and every vertex's count against the
oracle's node iterator on graphs it finishes in seconds; at the benchmark
graphs' full size, where the node iterator is quadratic in hub degree,
sampled vertices' counts (the oracle counts one vertex at a time) and the
identity sum of per-vertex counts = 3 x total.
"""
from __future__ import annotations

import math

import networkx as nx
import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


def csr_of(G):
    G = nx.convert_node_labels_to_integers(G)
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return graphs.from_edges(G.number_of_nodes(), e[:, 0], e[:, 1])


def valid_csr(rp, ci):
    """The oracle indexes rows by the ids it reads: check them before calling it."""
    n = len(rp) - 1
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    assert len(ci) == 0 or (ci.min() >= 0 and ci.max() < n)


def per_vertex_ref(rp, ci):
    valid_csr(rp, ci)
    return oracle.triangles_each(rp, ci).astype(np.uint64)


@pytest.mark.parametrize("name", ["uniform-4096", "rmat-13", "rmat-14", "road-80", "complete-60",
                                  "wheel-5000", "star-3000"])
def test_small_graphs(sp, name):
    if name == "uniform-4096":
        rp, ci = graphs.uniform(4096, 65536, 7)
    elif name.startswith("rmat"):
        rp, ci = graphs.rmat(int(name[5:]), 16, seed=8)
    elif name == "road-80":
        rp, ci = graphs.road(80, 0.02, seed=9)
    elif name == "complete-60":
        rp, ci = csr_of(nx.complete_graph(60))
    elif name == "wheel-5000":
        rp, ci = csr_of(nx.wheel_graph(5000))       # a hub of degree 4999
    else:
        rp, ci = csr_of(nx.star_graph(3000))
    print(name, flush=True)
    want_each = per_vertex_ref(rp, ci)
    want = oracle.triangles(rp, ci)
    g = sp.sp_graph_upload(rp, ci)
    total, per = sp.sp_triangle_count(g, per_vertex=True)
    assert total == want
    assert np.array_equal(per.cpu().numpy(), want_each)
    again, _ = sp.sp_triangle_count(g)
    assert again == total and sp.sp_tc_get_last_stats()["build_ms"] == 0.0   # rows kept


def test_closed_forms_and_edges(sp):
    for n in (1, 2, 3, 30):
        g = sp.sp_graph_upload(*csr_of(nx.complete_graph(n)))
        assert sp.sp_triangle_count(g)[0] == math.comb(n, 3)
    g = sp.sp_graph_upload(np.array([0], np.int32), np.zeros(0, np.int32))
    assert sp.sp_triangle_count(g)[0] == 0
    g = sp.sp_graph_upload(*csr_of(nx.random_labeled_tree(500, seed=2)))
    assert sp.sp_triangle_count(g)[0] == 0
    # a CSR that is not simple and symmetric is rejected
    g = sp.sp_graph_upload(np.array([0, 1, 1], np.int32), np.array([1], np.int32))
    with pytest.raises(sp.SpError):
        sp.sp_triangle_count(g)


@pytest.mark.parametrize("k", [3, 4])
def test_full_size(sp, k):
    rp, ci, src, spec = graphs.workload(k)
    print("workload", spec["name"], flush=True)
    valid_csr(rp, ci)
    deg = np.diff(rp)
    pick = [int(v) for v in src[:40] if deg[v] <= 3000]
    pick += [int(np.argmax(np.where(deg <= 3000, deg, 0)))]
    want = {v: oracle.triangles_at(rp, ci, v) for v in pick}
    g = sp.sp_graph_upload(rp, ci)
    total, per = sp.sp_triangle_count(g, per_vertex=True)
    per = per.cpu().numpy()
    assert int(per.sum()) == 3 * total
    for v in pick:
        assert int(per[v]) == want[v], v
    if k == 4:
        assert total == 0          # grid edges only: bipartite
