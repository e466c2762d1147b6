"""GPU parity: both HIP paths against the CPU oracle, through the C ABI.

Bar (Appendix Fig. "BC computation in StarPlat", DAG semantics of Section
2.3.2): distances and level membership bit-exact; path counts bit-exact while
below 2^53 (they are integers), else within 1e-12 relative; delta and BC
within 1e-9 relative, and exactly zero where the oracle is zero.
"""
from __future__ import annotations

import networkx as nx
import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs

pytestmark = pytest.mark.gpu

TOL = 1e-9
EXACT = 2.0 ** 53


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


def assert_bc(got, ref, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    zero = ref == 0
    assert np.all(got[zero] == 0), "%s: nonzero where oracle is zero" % what
    if np.any(~zero):
        rel = np.abs(got[~zero] - ref[~zero]) / np.abs(ref[~zero])
        assert rel.max() <= TOL, "%s: max rel err %g" % (what, rel.max())


def assert_sigma(got, ref, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    small = ref < EXACT
    assert np.array_equal(got[small], ref[small]), what
    if np.any(~small):
        rel = np.abs(got[~small] - ref[~small]) / ref[~small]
        assert rel.max() <= 1e-12, what


def csr_of(G):
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return graphs.from_edges(n, e[:, 0], e[:, 1])


def check_sources_detail(sp, g, rp, ci, srcs, config=None):
    """Per-source dist/sigma/delta: per-source path and one batched pass."""
    bd, bs, bdl, st = sp.sp_batch_levels(g, srcs, config=config)
    bd, bs, bdl = bd.cpu().numpy(), bs.cpu().numpy(), bdl.cpu().numpy()
    for i, s in enumerate(srcs):
        d_ref, sig_ref, del_ref = oracle.source_detail(rp, ci, int(s))
        d, sig, dl, _ = sp.sp_bfs_levels(g, int(s), with_sigma=True, with_delta=True)
        assert np.array_equal(d.cpu().numpy(), d_ref), "per-source dist, source %d" % s
        assert_sigma(sig.cpu().numpy(), sig_ref, "per-source sigma, source %d" % s)
        dref = np.where(d_ref > 0, del_ref, 0.0)
        assert_bc(dl.cpu().numpy(), dref, "per-source delta, source %d" % s)
        assert np.array_equal(bd[i], d_ref), "batched dist, source %d (slot %d)" % (s, i)
        assert_sigma(bs[i], sig_ref, "batched sigma, source %d" % s)
        assert_bc(bdl[i], dref, "batched delta, source %d" % s)


def both_paths(sp, g, srcs, config=None):
    a, sa = sp.sp_bc(g, srcs)
    b, sb = sp.sp_bc_batch(g, srcs, config=config)
    return a.cpu().numpy(), b.cpu().numpy(), sa, sb


# Launch configurations the parity tests run: every block size both paths
# are instantiated for, with the top-down -> bottom-up threshold at the
# built-in value (15) and at the one the autotuner picks on RMAT graphs (4).
# Set as the graph's tuned configuration, so sp_bc (block size) and
# sp_bc_batch (block size, alpha) both run it.
LAUNCH_CONFIGS = [(b, a) for b in (128, 256, 512) for a in (4.0, 15.0)]
LAUNCH_IDS = ["block%d-alpha%g" % c for c in LAUNCH_CONFIGS]


def use_launch_config(sp, g, block, alpha):
    sp.sp_graph_set_tuned(g, {"block_size": block, "alpha": alpha})


_REF = {}


def cached(key, make):
    """Oracle results shared by the parametrized cases of one input."""
    if key not in _REF:
        _REF[key] = make()
    return _REF[key]


# --------------------------------------------------------------------------

def test_workload_uniform_4096_full(sp):
    """Uniform random, 4,096 vertices, 32,768 edges, 16 sources: everything compared."""
    rp, ci, src, _ = graphs.workload(1)
    g = sp.sp_graph_upload(rp, ci, validate=True)
    check_sources_detail(sp, g, rp, ci, src)
    ref = oracle.bc(rp, ci, src)
    a, b, sa, sb = both_paths(sp, g, src)
    assert sa == sp.SP_OK and sb == sp.SP_OK
    assert_bc(a, ref, "sp_bc")
    assert_bc(b, ref, "sp_bc_batch")
    g.release()


@pytest.mark.parametrize("chunk", range(4))
def test_small_graph_atlas(sp, chunk):
    """Every 7th graph of the <= 7-vertex atlas, all sources, both paths."""
    for G in nx.graph_atlas_g()[1 + chunk::28]:
        rp, ci = csr_of(G)
        n = len(rp) - 1
        g = sp.sp_graph_upload(rp, ci, validate=True)
        srcs = np.arange(n, dtype=np.int32)
        ref = oracle.bc(rp, ci, srcs)
        a, b, _, _ = both_paths(sp, g, srcs)
        assert_bc(a, ref, "sp_bc atlas")
        assert_bc(b, ref, "sp_bc_batch atlas")
        check_sources_detail(sp, g, rp, ci, srcs)
        g.release()


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_random_disconnected_with_duplicates(sp, seed):
    rng = np.random.default_rng(seed)
    G = nx.disjoint_union(nx.gnm_random_graph(120, 300, seed=seed),
                          nx.gnm_random_graph(60, 90, seed=seed + 100))
    G.add_nodes_from(range(180, 185))  # isolated vertices
    rp, ci = csr_of(G)
    srcs = rng.integers(0, 185, 70).astype(np.int32)
    srcs[5] = srcs[6] = 182               # isolated source, listed twice
    srcs[10] = srcs[11] = srcs[12] = 7    # repeated source
    g = sp.sp_graph_upload(rp, ci, validate=True)
    ref = oracle.bc(rp, ci, srcs)
    a, b, _, _ = both_paths(sp, g, srcs)
    assert_bc(a, ref, "sp_bc")
    assert_bc(b, ref, "sp_bc_batch")
    check_sources_detail(sp, g, rp, ci, srcs[:64])
    g.release()


def test_single_vertex_and_empty_source_list(sp):
    g = sp.sp_graph_upload(np.array([0, 0], np.int32), np.zeros(0, np.int32))
    a, b, _, _ = both_paths(sp, g, [0, 0])
    assert a.tolist() == [0.0] and b.tolist() == [0.0]
    rp, ci = csr_of(nx.path_graph(9))
    g2 = sp.sp_graph_upload(rp, ci)
    a, b, _, _ = both_paths(sp, g2, [])
    assert np.all(a == 0) and np.all(b == 0)
    g.release()
    g2.release()


@pytest.mark.parametrize("width", [1, 7, 32, 64])
def test_batch_widths_and_partial_batches(sp, width):
    rp, ci = graphs.rmat(12, 16, graphs.RMAT_ABC, 77)
    srcs = graphs.sources(rp, 100, 78, min_degree=1)
    g = sp.sp_graph_upload(rp, ci)
    ref = oracle.bc(rp, ci, srcs)
    b, sb = sp.sp_bc_batch(g, srcs, config={"batch_width": width})
    assert sb == sp.SP_OK
    assert_bc(b.cpu().numpy(), ref, "width %d" % width)
    g.release()


@pytest.mark.parametrize("block,alpha", LAUNCH_CONFIGS, ids=LAUNCH_IDS)
def test_rmat_14_both_paths(sp, block, alpha):
    def make():
        rp, ci = graphs.rmat(14, 16, graphs.RMAT_ABC, 5)
        srcs = graphs.sources(rp, 130, 6, min_degree=1)
        return rp, ci, srcs, oracle.bc(rp, ci, srcs)
    rp, ci, srcs, ref = cached("rmat14", make)
    g = sp.sp_graph_upload(rp, ci)
    use_launch_config(sp, g, block, alpha)
    a, b, _, _ = both_paths(sp, g, srcs)
    st = sp.sp_get_last_stats()
    assert st["block_size"] == block and st["alpha"] == alpha
    assert_bc(a, ref, "sp_bc rmat14")
    assert_bc(b, ref, "sp_bc_batch rmat14")
    check_sources_detail(sp, g, rp, ci, srcs[:64])
    g.release()


HUB_DEGREES = (2048, 2049, 3000, 4096, 4097, 8193, 40000)


def split_hub_graph(seed=31):
    """Sparse random graph on 60000 vertices plus hubs (vertices 60000 on)
    of exactly the degrees in HUB_DEGREES: either side of the batched path's
    split threshold (2048) and of its piece-count steps (every 4096)."""
    n0 = 60000
    n = n0 + len(HUB_DEGREES)
    rng = np.random.default_rng(seed)
    base = graphs.uniform(n0, 120000, seed)
    src = [np.repeat(np.arange(n0, dtype=np.int64), np.diff(base[0]))]
    dst = [base[1].astype(np.int64)]
    for i, d in enumerate(HUB_DEGREES):
        src.append(np.full(d, n0 + i, np.int64))
        dst.append(rng.choice(n0, size=d, replace=False).astype(np.int64))
    rp, ci = graphs.from_edges(n, np.concatenate(src), np.concatenate(dst))
    assert list(np.diff(rp)[n0:]) == list(HUB_DEGREES)
    return rp, ci


@pytest.mark.parametrize("block,alpha", LAUNCH_CONFIGS, ids=LAUNCH_IDS)
@pytest.mark.parametrize("case", ["rmat-16", "synthetic"])
def test_split_hubs(sp, case, block, alpha):
    # hubs above 2048 neighbours are cut into 8m pieces numbered by row eighth
    # (both paths); sources include the hubs themselves (level-0 hubs)
    def make():
        if case == "rmat-16":
            rp, ci = graphs.rmat(16, 16, graphs.RMAT_ABC, 8)
            deg = np.diff(rp)
            assert (deg > 2048).sum() >= 10
            top = np.argsort(-deg, kind="stable")[:6].astype(np.int32)
        else:
            rp, ci = split_hub_graph()
            top = np.arange(60000, 60000 + len(HUB_DEGREES), dtype=np.int32)[::-1].copy()
        rest = [s for s in graphs.sources(rp, 80, 32, min_degree=1) if s not in set(top.tolist())]
        srcs = np.concatenate([top, np.array(rest[:64 - len(top)], np.int32)])
        return rp, ci, srcs, oracle.bc(rp, ci, srcs)
    rp, ci, srcs, ref = cached("split-" + case, make)
    print(case, "vertices", len(rp) - 1, "max degree", int(np.diff(rp).max()), flush=True)
    g = sp.sp_graph_upload(rp, ci)
    use_launch_config(sp, g, block, alpha)
    a, b, sa, sb = both_paths(sp, g, srcs)
    assert sa == sp.SP_OK and sb == sp.SP_OK
    assert_bc(a, ref, "sp_bc " + case)
    assert_bc(b, ref, "sp_bc_batch " + case)
    b2, _ = sp.sp_bc_batch(g, srcs[::-1].copy())
    assert_bc(b2.cpu().numpy(), ref, "sp_bc_batch reversed " + case)
    check_sources_detail(sp, g, rp, ci, srcs[:12])
    g.release()


@pytest.mark.parametrize("block", [128, 256, 512])
def test_road_grid_128(sp, block):
    """High diameter (hundreds of levels) and path counts beyond 2^53.  (Road
    graphs never switch to bottom-up levels, so alpha plays no part.)"""
    def make():
        rp, ci = graphs.road(128, 0.02, 9)
        srcs = graphs.sources(rp, 20, 10)
        return rp, ci, srcs, oracle.bc(rp, ci, srcs)
    rp, ci, srcs, ref = cached("road128", make)
    g = sp.sp_graph_upload(rp, ci)
    use_launch_config(sp, g, block, 15.0)
    a, b, _, _ = both_paths(sp, g, srcs)
    assert_bc(a, ref, "sp_bc road")
    assert_bc(b, ref, "sp_bc_batch road")
    assert sp.sp_get_last_stats()["engine"] == sp.SP_ENGINE_BLOCKS  # the automatic choice on roads
    check_sources_detail(sp, g, rp, ci, srcs)
    # the bitmap engine on the same road graph
    c, st = sp.sp_bc_batch(g, srcs, config={"engine": sp.SP_ENGINE_BITMAP})
    assert st == sp.SP_OK and sp.sp_get_last_stats()["engine"] == sp.SP_ENGINE_BITMAP
    assert_bc(c.cpu().numpy(), ref, "sp_bc_batch road, bitmap engine")
    check_sources_detail(sp, g, rp, ci, srcs, config={"engine": sp.SP_ENGINE_BITMAP})
    g.release()


def test_full_grid_sigma_is_binomial(sp):
    import math
    W = 40
    G = nx.convert_node_labels_to_integers(nx.grid_2d_graph(W, W), ordering="sorted")
    rp, ci = csr_of(G)
    g = sp.sp_graph_upload(rp, ci)
    d, sig, _, _ = sp.sp_bfs_levels(g, 0)
    _, bs, _, _ = sp.sp_batch_levels(g, [0, W * W - 1])
    exp = np.array([float(math.comb(i + j, i)) for i in range(W) for j in range(W)])
    assert np.array_equal(d.cpu().numpy(), np.add.outer(np.arange(W), np.arange(W)).ravel())
    assert_sigma(sig.cpu().numpy(), exp, "per-source grid sigma")
    assert_sigma(bs[0].cpu().numpy(), exp, "batched grid sigma")
    g.release()


@pytest.mark.parametrize("k,flag", [(996, False), (997, True), (1030, True)])
def test_sigma_overflow_flag(sp, k, flag):
    edges = []
    for i in range(k):
        a, b, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        edges += [(a, b), (a, c), (b, d), (c, d)]
    e = np.array(edges)
    n = 3 * k + 1
    rp, ci = graphs.from_edges(n, e[:, 0], e[:, 1])
    g = sp.sp_graph_upload(rp, ci)
    want = sp.SP_WARN_SIGMA_LARGE if flag else sp.SP_OK
    _, sa = sp.sp_bc(g, [0])
    for engine in (sp.SP_ENGINE_BLOCKS, sp.SP_ENGINE_BITMAP):
        _, sb = sp.sp_bc_batch(g, [0, n - 1], config={"engine": engine})
        assert sb == want, engine
        assert (sp.sp_get_last_stats()["sigma_flagged"] > 0) == flag
    assert sa == want
    if not flag:
        ref = oracle.bc(rp, ci, [0, n - 1])
        assert_bc(sp.sp_bc(g, [0, n - 1])[0].cpu().numpy(), ref)
        assert_bc(sp.sp_bc_batch(g, [0, n - 1])[0].cpu().numpy(), ref)
    g.release()


def test_runs_are_bit_identical(sp):
    rp, ci = graphs.rmat(13, 16, graphs.RMAT_ABC, 12)
    srcs = graphs.sources(rp, 70, 13, min_degree=1)
    g = sp.sp_graph_upload(rp, ci)
    a1, b1, _, _ = both_paths(sp, g, srcs)
    a2, b2, _, _ = both_paths(sp, g, srcs)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    g.release()


def test_results_do_not_depend_on_block_size(sp):
    """Sums run in CSR order and hub chunks are fixed by the degree, so each
    path gives the same bits at every block size."""
    rp, ci = graphs.rmat(13, 16, graphs.RMAT_ABC, 12)
    srcs = graphs.sources(rp, 70, 13, min_degree=1)
    g = sp.sp_graph_upload(rp, ci)
    got = {}
    for block in (128, 256, 512):
        use_launch_config(sp, g, block, 4.0)
        got[block] = both_paths(sp, g, srcs)[:2]
    for block in (128, 256):
        assert np.array_equal(got[block][0], got[512][0]), "sp_bc, block %d" % block
        assert np.array_equal(got[block][1], got[512][1]), "sp_bc_batch, block %d" % block
    g.release()


def test_invalid_source_leaves_output_untouched(sp):
    import torch
    rp, ci = csr_of(nx.path_graph(10))
    g = sp.sp_graph_upload(rp, ci)
    out = torch.full((10,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SpError) as ei:
        sp.sp_bc(g, [0, 10], out_bc=out)
    assert ei.value.status == sp.SP_ERR_INVALID_ARGUMENT
    with pytest.raises(sp.SpError):
        sp.sp_bc_batch(g, [-1], out_bc=out)
    for bad in ({"batch_width": 65}, {"block_size": 64}, {"alpha": -1.0},
                {"chunk_levels": 70000}, {"chunk_levels": -70000}):
        with pytest.raises(sp.SpError) as ei:
            sp.sp_bc_batch(g, [0, 1], out_bc=out, config=bad)
        assert ei.value.status == sp.SP_ERR_INVALID_ARGUMENT, bad
    assert torch.all(out == 7.0)
    g.release()


def test_upload_validation(sp):
    rp = np.array([0, 1, 1], np.int32)
    ci = np.array([1], np.int32)          # 0->1 without 1->0
    with pytest.raises(sp.SpError):
        sp.sp_graph_upload(rp, ci, validate=True)
    with pytest.raises(sp.SpError):       # id out of range: caught on the device
        sp.sp_graph_upload(np.array([0, 1, 2], np.int32), np.array([1, 5], np.int32))


@pytest.mark.parametrize("alpha,beta", [(1e-9, 24.0), (1e9, 1e-9), (1e9, 1e9)])
def test_direction_extremes(sp, alpha, beta):
    """Top-down only, bottom-up as early as possible, and bottom-up to the end."""
    rp, ci = graphs.rmat(13, 16, graphs.RMAT_ABC, 21)
    srcs = graphs.sources(rp, 40, 22, min_degree=1)
    g = sp.sp_graph_upload(rp, ci)
    ref = oracle.bc(rp, ci, srcs)
    b, _ = sp.sp_bc_batch(g, srcs, config={"alpha": alpha, "beta": beta})
    assert_bc(b.cpu().numpy(), ref, "alpha %g beta %g" % (alpha, beta))
    st = sp.sp_get_last_stats()
    if alpha > 1:
        assert st["bottomup_levels"] > 0
    else:
        assert st["bottomup_levels"] == 0
    g.release()


def test_star_and_meshes_never_switch_direction(sp):
    """Low-degree graphs run top-down only; the switch must not strand a level."""
    for G in (nx.star_graph(6), nx.grid_2d_graph(9, 9), nx.path_graph(50)):
        rp, ci = csr_of(nx.convert_node_labels_to_integers(G))
        n = len(rp) - 1
        g = sp.sp_graph_upload(rp, ci)
        srcs = np.arange(n)
        ref = oracle.bc(rp, ci, srcs)
        a, b, _, _ = both_paths(sp, g, srcs)
        assert_bc(a, ref, "sp_bc")
        assert_bc(b, ref, "sp_bc_batch")
        g.release()


@pytest.mark.parametrize("block", [128, 256, 512])
@pytest.mark.parametrize("case", ["rmat", "road"])
def test_hipgraph_capture_matches_direct_launches(sp, case, block):
    """The forward level chunk replayed from a captured hipGraph gives the same
    bits as direct launches, on every replay, with other device work between
    calls; an odd chunk length and a narrower batch (new slot set, so a new
    capture) still match the oracle."""
    def make():
        if case == "rmat":
            rp, ci = graphs.rmat(13, 16, graphs.RMAT_ABC, 21)
            srcs = graphs.sources(rp, 100, 22, min_degree=1)
        else:
            rp, ci = graphs.road(96, 0.02, 23)  # hundreds of levels: many replays per pass
            srcs = graphs.sources(rp, 70, 24)
        return rp, ci, srcs, oracle.bc(rp, ci, srcs)
    rp, ci, srcs, ref = cached("capture-" + case, make)
    g = sp.sp_graph_upload(rp, ci)
    use_launch_config(sp, g, block, 4.0)
    bitmap = sp.SP_ENGINE_BITMAP  # the engine whose levels are captured
    direct, st = sp.sp_bc_batch(g, srcs, config={"chunk_levels": -8, "engine": bitmap})
    assert st == sp.SP_OK and sp.sp_get_last_stats()["graph_launches"] == 0
    direct = direct.cpu().numpy()
    assert_bc(direct, ref, "%s direct launches" % case)
    for rep in range(3):
        got, st = sp.sp_bc_batch(g, srcs, config={"chunk_levels": 8, "engine": bitmap})
        assert st == sp.SP_OK
        assert sp.sp_get_last_stats()["graph_launches"] > 0
        assert np.array_equal(got.cpu().numpy(), direct), "%s replay %d differs" % (case, rep)
        sp.sp_bc(g, srcs[:2])  # eager work on the same stream between calls
    got, st = sp.sp_bc_batch(g, srcs, config={"chunk_levels": 3, "batch_width": 7, "engine": bitmap})
    assert st == sp.SP_OK
    assert_bc(got.cpu().numpy(), ref, "%s odd chunk, width 7" % case)
    g.release()


def blocks_engine_cases():
    """Graphs for the one-workgroup-per-source engine: its automatic target
    (road-like grids, rows of at most 4: fixed-width rows of 4), a grid with
    diagonal moves (rows of up to 8: fixed-width rows of 8), a directed road
    grid (fixed-width incoming rows too) and, forced, every other shape: a
    long path (a level per vertex), a uniform graph and RMAT with hubs and
    isolated vertices (rows through the CSR offsets), a directed RMAT, and a
    graph of two components."""
    yield "road-96", graphs.road(96, 0.02, 23), False
    k = 40
    x, y = np.meshgrid(np.arange(k), np.arange(k))
    x, y = x.ravel(), y.ravel()
    src, dst = [], []
    for dx, dy in ((1, 0), (0, 1), (1, 1), (-1, 1)):  # king moves, each edge once
        ok = (x + dx >= 0) & (x + dx < k) & (y + dy < k)
        src.append((y * k + x)[ok])
        dst.append(((y + dy) * k + x + dx)[ok])
    yield "king-40", graphs.from_edges(k * k, np.concatenate(src), np.concatenate(dst)), False
    rp, ci = graphs.road(60, 0.02, 25)
    yield "road-60-directed", graphs.directed_from(rp, ci, 26), True
    yield "path-3000", graphs.from_edges(3000, np.arange(2999), np.arange(1, 3000)), False
    yield "uniform-4096", graphs.uniform(4096, 32768, 5), False
    yield "rmat-13", graphs.rmat(13, 16, graphs.RMAT_ABC, 21), False
    rp, ci = graphs.rmat(12, 16, graphs.RMAT_ABC, 31)
    yield "rmat-12-directed", graphs.directed_from(rp, ci, 32), True
    a = graphs.road(20, 0.02, 3)
    yield "two-components", graphs.from_edges(
        800, np.concatenate([np.repeat(np.arange(400), np.diff(a[0])), np.arange(400, 799)]),
        np.concatenate([a[1], np.arange(401, 800)])), False


@pytest.mark.parametrize("block", [128, 256, 512, 1024])
@pytest.mark.parametrize("name", ["road-96", "king-40", "road-60-directed", "path-3000", "uniform-4096",
                                  "rmat-13", "rmat-12-directed", "two-components"])
def test_blocks_engine(sp, name, block):
    """SP_ENGINE_BLOCKS: BC over several batches (width 64 and 7, duplicate
    and isolated sources included) and every slot's dist / sigma / delta of
    one pass against the oracle."""
    (rp, ci), directed = {k: (v, d) for k, v, d in blocks_engine_cases()}[name]
    n = len(rp) - 1
    g = sp.sp_graph_upload(rp, ci, validate=True, directed=directed)
    srcs = graphs.sources(rp, min(90, n), 40)
    srcs = np.concatenate([srcs, srcs[:3]]).astype(np.int32)  # duplicates count twice
    iso = np.nonzero(np.diff(rp) == 0)[0]
    if len(iso):
        srcs = np.concatenate([srcs, iso[:2]]).astype(np.int32)
    print(name, "block", block, "sources", len(srcs), flush=True)
    ref = oracle.bc(rp, ci, srcs)
    for width in (64, 7):
        cfg = {"engine": sp.SP_ENGINE_BLOCKS, "block_size": block, "batch_width": width}
        got, st = sp.sp_bc_batch(g, srcs, config=cfg)
        assert st == sp.SP_OK
        assert sp.sp_get_last_stats()["engine"] == sp.SP_ENGINE_BLOCKS
        assert_bc(got.cpu().numpy(), ref, "%s block %d width %d" % (name, block, width))
    check_sources_detail(sp, g, rp, ci, srcs[:64], config={"engine": sp.SP_ENGINE_BLOCKS, "block_size": block})
    g.release()

