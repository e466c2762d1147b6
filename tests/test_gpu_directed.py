"""GPU parity of betweenness centrality on directed graphs (paper Section
2.3.1 graph type with nodes_to; BC program of the Appendix), through the C
ABI: sp_graph_upload_directed, sp_bc (per-source path), sp_bc_batch and
sp_batch_levels (batched path: discovery top-down over outgoing rows and
bottom-up over incoming rows, path counts over incoming rows with their own
per-level hub chunks, dependencies over outgoing rows), sp_bfs_levels, the
autotuner and the server.  Same bar as the undirected parity tests:
distances and path counts exact (below 2^53), delta and BC within 1e-9
relative, zeros exact.
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
    check_batch_detail(sp, g, rp, ci, srcs[:20], name)
    g.release()


def check_batch_detail(sp, g, rp, ci, srcs, what, config=None):
    """One batched pass over srcs: every slot's dist, sigma and delta against
    the oracle's single-source run."""
    bd, bs, bdl, st = sp.sp_batch_levels(g, srcs, config=config)
    assert st == sp.SP_OK
    bd, bs, bdl = bd.cpu().numpy(), bs.cpu().numpy(), bdl.cpu().numpy()
    for i, s in enumerate(srcs):
        d_ref, sig_ref, dl_ref = oracle.source_detail(rp, ci, int(s))
        assert np.array_equal(bd[i], d_ref), "%s: batched dist, source %d" % (what, s)
        assert_sigma(bs[i], sig_ref, "%s: batched sigma, source %d" % (what, s))
        assert_bc(bdl[i], np.where(d_ref > 0, dl_ref, 0.0), "%s: batched delta, source %d" % (what, s))


@pytest.mark.parametrize("block", [128, 256, 512])
@pytest.mark.parametrize("alpha", [4.0, 15.0, 1e9])
def test_batched_directed_configs(sp, block, alpha):
    """Batched BC on a directed RMAT graph at every block size, with the
    bottom-up switch (over incoming rows) at the tuned thresholds and as
    early as possible; widths 64 and 7 (several batches)."""
    rp, ci = directed_rmat(13, 6)
    g = sp.sp_graph_upload(rp, ci, validate=True, directed=True)
    srcs = graphs.sources(rp, 70, 7, min_degree=1)
    print("block", block, "alpha", alpha, flush=True)
    ref = oracle.bc(rp, ci, srcs)
    for width in (64, 7):
        cfg = {"block_size": block, "alpha": alpha, "batch_width": width}
        got, st = sp.sp_bc_batch(g, srcs, config=cfg)
        assert st == sp.SP_OK
        assert_bc(got.cpu().numpy(), ref, "block %d alpha %g width %d" % (block, alpha, width))
    stats = sp.sp_get_last_stats()
    assert stats["batch_width"] == 7 and stats["n_passes"] == 10
    if alpha > 1e6:
        assert stats["bottomup_levels"] > 0
    check_batch_detail(sp, g, rp, ci, srcs[:64], "block %d alpha %g" % (block, alpha),
                       config={"block_size": block, "alpha": alpha})
    g.release()


def test_directed_hub_rows_one_side(sp):
    """Hubs with only incoming arcs (path counts chunked over the reversed
    rows), only outgoing arcs (discovery and dependencies chunked), and both,
    on either side of the 2048-entry split."""
    rng = np.random.default_rng(9)
    n0 = 20000
    src = [np.arange(n0 - 1)]
    dst = [np.arange(1, n0)]
    extra = rng.integers(0, n0, size=(2, 40000))
    src.append(extra[0])
    dst.append(extra[1])
    hubs = {n0: ("in", 3000), n0 + 1: ("out", 3000), n0 + 2: ("in", 1500), n0 + 3: ("out", 5000),
            n0 + 4: ("both", 2600)}
    for h, (kind, d) in hubs.items():
        nb = rng.choice(n0, size=d, replace=False)
        if kind in ("in", "both"):
            src.append(nb)
            dst.append(np.full(d, h))
        if kind in ("out", "both"):
            nb2 = rng.choice(n0, size=d, replace=False)
            src.append(np.full(d, h))
            dst.append(nb2)
    a = np.concatenate(src)
    b = np.concatenate(dst)
    keep = a != b
    pairs = np.unique(np.stack([a[keep], b[keep]], 1), axis=0)
    rp, ci = brute.directed_csr(n0 + len(hubs), pairs[:, 0], pairs[:, 1])
    g = sp.sp_graph_upload(rp, ci, validate=True, directed=True)
    srcs = np.unique(np.concatenate([np.array(list(hubs), np.int32),
                                     graphs.sources(rp, 40, 10, min_degree=1)])).astype(np.int32)
    ref = oracle.bc(rp, ci, srcs)
    for block in (256, 512):
        got, st = sp.sp_bc_batch(g, srcs, config={"block_size": block})
        assert st == sp.SP_OK
        assert_bc(got.cpu().numpy(), ref, "one-sided hubs, block %d" % block)
    check_batch_detail(sp, g, rp, ci, srcs[:64], "one-sided hubs")
    g.release()


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
    for fn in (sp.sp_bc, sp.sp_bc_batch):
        got, st = fn(g, srcs)
        assert st == sp.SP_OK
        assert_bc(got.cpu().numpy(), ref, "directed split hubs, %s" % fn.__name__)
    check_batch_detail(sp, g, drp, dci, srcs[:64], "directed split hubs")
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
    for call in (lambda: sp.sp_triangle_count(g), lambda: sp.sp_graph_set_weights(g, np.ones(3, np.int32))):
        with pytest.raises(sp.SpError) as e:
            call()
        assert e.value.status == sp.SP_ERR_NOT_SUPPORTED
    with pytest.raises(sp.SpError):          # malformed: an id out of range
        sp.sp_graph_upload(np.array([0, 1, 1], np.int32), np.array([5], np.int32), directed=True)
    with pytest.raises(sp.SpError):          # unsorted row, with validation
        sp.sp_graph_upload(np.array([0, 2, 2, 2], np.int32), np.array([2, 1], np.int32), validate=True,
                           directed=True)


def test_autotune_and_server_on_directed(sp):
    """The autotuner's choice and the server's continuous batching on a
    directed graph, against the oracle."""
    import torch
    rp, ci = directed_rmat(12, 8)
    g = sp.sp_graph_upload(rp, ci, directed=True)
    srcs = graphs.sources(rp, 100, 11, min_degree=1)
    ref = oracle.bc(rp, ci, srcs)
    sp.sp_autotune(g, srcs)
    got, st = sp.sp_bc_batch(g, srcs)
    assert st == sp.SP_OK
    assert_bc(got.cpu().numpy(), ref, "autotuned")
    srv = sp.Server(memory_budget=2 << 30)
    gid = srv.add_graph(g)
    outs = [torch.empty(len(rp) - 1, dtype=torch.float64, device="cuda") for _ in range(3)]
    parts = [srcs[:30], srcs[30:33], srcs[33:]]
    reqs = [srv.submit(gid, p, out_bc=o) for p, o in zip(parts, outs)]
    for r, p, o in zip(reqs, parts, outs):
        assert r.wait() == sp.SP_OK
        r.release()
        assert_bc(o.cpu().numpy(), oracle.bc(rp, ci, p), "served request")
    srv.destroy()
    g.release()
