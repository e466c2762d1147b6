"""Serving loop on the GPU: continuous batching over several resident graphs.

Each request's BC must match the oracle, and be bit-identical whether the
request runs alone or mixed with others (its chunks may share passes with
other requests' chunks, and several of its chunks may run at once)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


@pytest.fixture(scope="module")
def resident(sp):
    specs = [graphs.uniform(4096, 32768, 1001), graphs.rmat(12, 16, graphs.RMAT_ABC, 31),
             graphs.road(48, 0.02, 32)]
    gs = [sp.sp_graph_upload(rp, ci) for rp, ci in specs]
    yield specs, gs
    for g in gs:
        g.release()


def requests_for(specs, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(9):
        gi = k % 3
        rp, _ = specs[gi]
        n = len(rp) - 1
        size = int(rng.integers(1, 100))
        reqs.append((gi, rng.integers(0, n, size).astype(np.int32)))
    return reqs


def test_alone_equals_mixed_and_oracle(sp, resident):
    specs, gs = resident
    reqs = requests_for(specs, 5)
    srv = sp.Server(n_streams=2)
    ids = [srv.add_graph(g) for g in gs]
    alone = []
    for gi, src in reqs:
        r = srv.submit(ids[gi], src)
        assert r.wait() == sp.SP_OK
        alone.append(r.out_bc[:gs[gi].n].cpu().numpy().copy())
        r.release()
    live = [srv.submit(ids[gi], src) for gi, src in reqs]
    for (gi, src), r, a in zip(reqs, live, alone):
        assert r.wait() == sp.SP_OK
        got = r.out_bc[:gs[gi].n].cpu().numpy()
        assert np.array_equal(got, a), "mixed result differs from the same request alone"
        rp, ci = specs[gi]
        ref = oracle.bc(rp, ci, src)
        nz = ref != 0
        assert np.all(got[~nz] == 0)
        assert np.max(np.abs(got[nz] - ref[nz]) / ref[nz]) <= 1e-9
        assert r.latency_us() > 0
        r.release()
    st = srv.stats()
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    assert st["slots_used"] == 2 * sum(len(s) for _, s in reqs)
    srv.destroy()


def test_memory_budget_admission_and_rejection(sp, resident):
    specs, gs = resident
    need = max(sp.sp_bc_workspace_bytes(g, 64) for g in gs)
    srv = sp.Server(memory_budget=need + 1024, n_streams=2)
    ids = [srv.add_graph(g) for g in gs]
    reqs = requests_for(specs, 6)
    live = [(gi, src, srv.submit(ids[gi], src)) for gi, src in reqs]
    for gi, src, r in live:
        assert r.wait() == sp.SP_OK
        rp, ci = specs[gi]
        ref = oracle.bc(rp, ci, src)
        got = r.out_bc[:gs[gi].n].cpu().numpy()
        nz = ref != 0
        assert np.max(np.abs(got[nz] - ref[nz]) / ref[nz]) <= 1e-9
        r.release()
    st = srv.stats()
    # workspaces stay within the budget; a chunk buffer (V doubles) may go
    # over it only when its pass has nothing else to run
    assert st["peak_admitted_bytes"] <= need + 1024 + max(8 * g.n for g in gs)
    srv.destroy()
    tiny = sp.Server(memory_budget=4096, n_streams=1)
    gid = tiny.add_graph(gs[0])
    with pytest.raises(sp.SpError) as ei:
        tiny.submit(gid, [1, 2, 3])
    assert ei.value.status == sp.SP_ERR_REJECTED
    assert tiny.stats()["rejected"] == 1
    tiny.destroy()


def test_cancel_invalid_and_empty(sp, resident):
    specs, gs = resident
    srv = sp.Server(n_streams=1, max_batch=8)
    gid = srv.add_graph(gs[1])
    first = srv.submit(gid, np.arange(1, 400, dtype=np.int32) % gs[1].n)
    last = srv.submit(gid, [5, 6, 7])
    rc = last.cancel()
    if rc == sp.SP_OK:
        assert last.wait() == sp.SP_ERR_CANCELLED
        assert srv.stats()["cancelled"] == 1
    else:  # already started: it completes normally
        assert last.wait() == sp.SP_OK
    assert first.wait() == sp.SP_OK
    with pytest.raises(sp.SpError):
        srv.submit(gid, [gs[1].n])          # source out of range
    with pytest.raises(sp.SpError):
        srv.submit(gid + 7, [0])            # unknown graph
    empty = srv.submit(gid, [])
    assert empty.wait() == sp.SP_OK
    assert np.all(empty.out_bc[:gs[1].n].cpu().numpy() == 0)
    for r in (first, last, empty):
        r.release()
    srv.destroy()


def test_sigma_warning_goes_only_to_the_request_that_overflowed(sp):
    """A diamond chain of 1030 diamonds (2^1030 shortest paths from its first
    vertex, above the 1e300 flag) plus a separate path: two requests that
    share one pass; only the chain request carries the warning, and the path
    request's BC matches the oracle."""
    k = 1030
    edges = []
    for i in range(k):
        a, b, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        edges += [(a, b), (a, c), (b, d), (c, d)]
    base = 3 * k + 1
    edges += [(base + i, base + i + 1) for i in range(9)]
    e = np.array(edges)
    n = base + 10
    rp, ci = graphs.from_edges(n, e[:, 0], e[:, 1])
    g = sp.sp_graph_upload(rp, ci)
    frp, fci = graphs.road(256, 0.02, 3)  # a long first pass keeps the one worker busy
    fg = sp.sp_graph_upload(frp, fci)
    srv = sp.Server(n_streams=1)
    gid = srv.add_graph(g)
    fid = srv.add_graph(fg)
    filler = srv.submit(fid, graphs.sources(frp, 64, 4))
    ra = srv.submit(gid, [0])                  # both wait for the filler,
    rb = srv.submit(gid, [base + 2, base + 7])  # then share one pass
    assert ra.wait() == sp.SP_WARN_SIGMA_LARGE
    assert rb.wait() == sp.SP_OK
    ref = oracle.bc(rp, ci, np.array([base + 2, base + 7], np.int32))
    got = rb.out_bc[:n].cpu().numpy()
    assert np.array_equal(got == 0, ref == 0)
    nz = ref != 0
    assert np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-9
    assert filler.wait() == sp.SP_OK
    for r in (ra, rb, filler):
        r.release()
    srv.destroy()
    g.release()
    fg.release()


@pytest.mark.parametrize("graph", ["rmat-12", "road-48"])
def test_large_request_chunks_run_together(sp, resident, graph):
    """A 330-source request (six chunks of 64, the last of 10) on four streams:
    several of its chunks are on the device at once, alone and in a mix with
    smaller requests, and the result is the same bits either way and matches
    the oracle."""
    specs, gs = resident
    gi = {"rmat-12": 1, "road-48": 2}[graph]
    rp, ci = specs[gi]
    big = graphs.sources(rp, 330, 77, min_degree=1)
    srv = sp.Server(n_streams=4)
    ids = [srv.add_graph(g) for g in gs]
    r = srv.submit(ids[gi], big)
    st = r.wait()
    assert st == sp.SP_OK, (st, sp.sp_last_error())
    alone = r.out_bc[:gs[gi].n].cpu().numpy().copy()
    r.release()
    others = requests_for(specs, 9)
    live = [srv.submit(ids[g2], s2) for g2, s2 in others[:4]]
    rb = srv.submit(ids[gi], big)
    live += [srv.submit(ids[g2], s2) for g2, s2 in others[4:]]
    st = rb.wait()
    assert st == sp.SP_OK, (st, sp.sp_last_error())
    got = rb.out_bc[:gs[gi].n].cpu().numpy()
    assert np.array_equal(got, alone), "large request: mixed differs from alone"
    ref = oracle.bc(rp, ci, big)
    nz = ref != 0
    assert np.all(got[~nz] == 0) and np.max(np.abs(got[nz] - ref[nz]) / ref[nz]) <= 1e-9
    for x in live:
        assert x.wait() == sp.SP_OK
        x.release()
    rb.release()
    st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == 2 + len(others)
    srv.destroy()
