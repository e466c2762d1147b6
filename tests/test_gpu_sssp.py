"""GPU parity of single-source shortest paths against the CPU oracle, through
the C ABI (paper Section 2.2, Fig. "SSSP computation in StarPlat"; pull form
in the Appendix).

Bar: distances are integers, so bit-exact against the oracle (Dijkstra), in
every direction mode (automatic, push only, pull only), launch mode (captured
round chunks, direct launches) and block size.  At the benchmark graphs' full
sizes the oracle's Dijkstra still runs in seconds, so one source is compared
in full, and the other sources through the invariants that pin shortest-path
distances at any size (tests/brute.py).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs
from tests import brute

pytestmark = pytest.mark.gpu

INF = np.iinfo(np.int32).max
MODES = {"auto": None, "push": {"direction": 1}, "pull": {"direction": 2}}


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


def weighted(sp, rp, ci, w):
    g = sp.sp_graph_upload(rp, ci)
    sp.sp_graph_set_weights(g, w)
    return g


def run(sp, g, s, cfg=None):
    return sp.sp_sssp(g, int(s), config=cfg).cpu().numpy()


def small_graphs():
    yield "uniform-4096", graphs.uniform(4096, 32768, 7)
    yield "rmat-13", graphs.rmat(13, 16, seed=8)        # hubs: rows past 256 entries
    yield "road-80", graphs.road(80, 0.02, seed=9)       # deep: hundreds of rounds
    yield "sparse-forest", graphs.uniform(5000, 3000, 10)  # many components


@pytest.mark.parametrize("mode", sorted(MODES))
def test_small_graphs_all_modes(sp, mode):
    for name, (rp, ci) in small_graphs():
        w = graphs.weights(rp, ci, 11)
        g = weighted(sp, rp, ci, w)
        for s in graphs.sources(rp, 3, 12, min_degree=1):
            print(name, mode, "source", int(s), flush=True)
            got = run(sp, g, s, MODES[mode])
            assert np.array_equal(got, oracle.sssp(rp, ci, w, int(s))), (name, mode, int(s))
        g.release()


@pytest.mark.parametrize("cfg", [{"chunk_rounds": -3}, {"chunk_rounds": 3}, {"chunk_rounds": 1},
                                 {"block_size": 128}, {"block_size": 512},
                                 {"alpha": 1e6}, {"alpha": 1e-3, "chunk_rounds": -2},
                                 {"max_blocks": 3}, {"max_blocks": 1, "block_size": 512},
                                 {"local_hops": 1}, {"local_hops": 8, "chunk_rounds": -3},
                                 {"local_hops": 2, "block_size": 128}])
def test_launch_configurations(sp, cfg):
    rp, ci = graphs.rmat(12, 16, seed=13)
    w = graphs.weights(rp, ci, 14)
    g = weighted(sp, rp, ci, w)
    for s in graphs.sources(rp, 2, 15, min_degree=1):
        print(cfg, "source", int(s), flush=True)
        assert np.array_equal(run(sp, g, s, cfg), oracle.sssp(rp, ci, w, int(s)))
    st = sp.sp_sssp_get_last_stats()
    assert st["rounds"] == st["push_rounds"] + st["pull_rounds"] and st["rounds"] >= 2


@pytest.mark.parametrize("hops", [-1, 1, 2, 8, 32, 128])
def test_local_hops_on_meshes(sp, hops):
    # road-like graphs (rows of at most 8 entries) use local hops by default
    rp, ci = graphs.road(120, 0.02, seed=22)
    w = graphs.weights(rp, ci, 23)
    g = weighted(sp, rp, ci, w)
    for s in graphs.sources(rp, 3, 24, min_degree=1):
        got = run(sp, g, s, {"local_hops": hops})
        assert np.array_equal(got, oracle.sssp(rp, ci, w, int(s))), (hops, int(s))
    st = sp.sp_sssp_get_last_stats()
    assert st["local_hops"] == (0 if hops < 0 else hops)
    run(sp, g, 0)
    assert sp.sp_sssp_get_last_stats()["local_hops"] == 32


def test_unit_weights_match_bfs_levels(sp):
    rp, ci = graphs.rmat(12, 16, seed=16)
    g = weighted(sp, rp, ci, np.ones(len(ci), np.int32))
    for s in graphs.sources(rp, 3, 17, min_degree=1):
        d_bfs, _, _, _ = sp.sp_bfs_levels(g, int(s), with_sigma=False)
        d_bfs = d_bfs.cpu().numpy()
        want = np.where(d_bfs < 0, INF, d_bfs)
        for mode in MODES.values():
            assert np.array_equal(run(sp, g, s, mode), want)


def test_hub_source_and_zero_weights(sp):
    # a star whose centre has 3000 leaves (a hub from round 0), plus a path
    # of zero-weight edges hanging off one leaf
    n = 3010
    src = np.concatenate([np.zeros(3000, np.int64), np.arange(3000, 3009)])
    dst = np.concatenate([np.arange(1, 3001), np.arange(3001, 3010)])
    rp, ci = graphs.from_edges(n, src, dst)
    rng = np.random.default_rng(18)
    w = np.empty(len(ci), np.int32)
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            a, b = min(u, ci[e]), max(u, ci[e])
            w[e] = 0 if a >= 3000 else (a * 7919 + b) % 50 + 1
    g = weighted(sp, rp, ci, w)
    for s in (0, 1, 3000, 3009):
        for mode in MODES.values():
            assert np.array_equal(run(sp, g, s, mode), oracle.sssp(rp, ci, w, s)), (s, mode)
    del rng


def test_edge_cases(sp):
    # single vertex, no edges
    g = weighted(sp, np.array([0, 0], np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert list(run(sp, g, 0)) == [0]
    st = sp.sp_sssp_get_last_stats()
    assert st["reached"] == 1 and st["rounds"] == 1
    # isolated source inside a larger graph
    rp, ci = graphs.from_edges(6, [1, 2, 3], [2, 3, 4])
    w = np.full(len(ci), 9, np.int32)
    g = weighted(sp, rp, ci, w)
    for mode in MODES.values():
        assert list(run(sp, g, 0, mode)) == [0, INF, INF, INF, INF, INF]
        assert list(run(sp, g, 2, mode)) == [INF, 9, 0, 9, 18, INF]
    # a source at the last vertex id, and the largest weights that still fit
    rp, ci = graphs.from_edges(3, [0, 1], [1, 2])
    big = np.full(len(ci), (2**31 - 2) // 2, np.int32)
    g = weighted(sp, rp, ci, big)
    assert list(run(sp, g, 2)) == [2 * int(big[0]), int(big[0]), 0]


def test_errors(sp):
    rp, ci = graphs.from_edges(3, [0, 1], [1, 2])
    g = sp.sp_graph_upload(rp, ci)
    with pytest.raises(sp.SpError):                       # no weights yet
        sp.sp_sssp(g, 0)
    with pytest.raises(sp.SpError):                       # negative weight
        sp.sp_graph_set_weights(g, np.array([1, -1, -1, 1], np.int32))
    with pytest.raises(sp.SpError):                       # asymmetric, validated
        sp.sp_graph_set_weights(g, np.array([1, 2, 3, 4], np.int32), validate=True)
    sp.sp_graph_set_weights(g, np.array([2**30, 2**30, 2**30, 2**30], np.int32), validate=True)
    with pytest.raises(sp.SpError) as e:                  # 2 * 2^30 does not fit
        sp.sp_sssp(g, 0)
    assert e.value.status == sp.SP_ERR_NOT_SUPPORTED
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 3)
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 0, config={"block_size": 64})
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 0, config={"direction": 3})
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 0, config={"max_blocks": -1})
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 0, config={"local_hops": 3})
    with pytest.raises(sp.SpError):
        sp.sp_sssp(g, 0, config={"local_hops": 256})
    # still usable after errors
    sp.sp_graph_set_weights(g, np.array([5, 5, 6, 6], np.int32))
    assert list(run(sp, g, 0)) == [0, 5, 11]


def test_device_weights_and_reweighting(sp):
    import torch
    rp, ci = graphs.rmat(11, 16, seed=19)
    g = sp.sp_graph_upload(rp, ci)
    for seed in (20, 21):
        w = graphs.weights(rp, ci, seed)
        sp.sp_graph_set_weights(g, torch.from_numpy(w).cuda(), validate=True)
        s = int(graphs.sources(rp, 1, seed, min_degree=1)[0])
        assert np.array_equal(run(sp, g, s), oracle.sssp(rp, ci, w, s))


@pytest.mark.parametrize("k", [3, 4])
def test_full_size(sp, k):
    rp, ci, src, spec = graphs.workload(k)
    w = graphs.weights(rp, ci, 3000 + k)
    print("workload", spec["name"], "vertices", len(rp) - 1, flush=True)
    g = weighted(sp, rp, ci, w)
    s0 = int(src[0])
    got = run(sp, g, s0)
    assert np.array_equal(got, oracle.sssp(rp, ci, w, s0))
    for s in src[1:3]:
        print("invariants, source", int(s), flush=True)
        d = {m: run(sp, g, s, cfg) for m, cfg in MODES.items()}
        brute.sssp_invariants(rp, ci, w, int(s), d["auto"])
        assert np.array_equal(d["auto"], d["push"]) and np.array_equal(d["auto"], d["pull"])
