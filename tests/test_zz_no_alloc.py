"""sp_bc_noalloc (per-source BC on the library's fixed device workspace)
against sp_bc, through the C ABI: the same kernels on the same inputs, so the
outputs must agree bit for bit (and hence within the 1e-9 relative bar of the
oracle parity tests).  Two calls in a row, the second on a smaller graph, so
anything the first call leaves in the shared workspace would show; plus the
size limit and the oracle on the second graph."""
from __future__ import annotations

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


def assert_same(sp, g, srcs, what):
    ref, st_ref = sp.sp_bc(g, srcs)
    ref = ref.cpu().numpy()
    got, st = sp.sp_bc_noalloc(g, srcs)
    got = got.cpu().numpy()
    assert st == st_ref, what
    assert np.array_equal(got, ref), "%s: max abs diff %g" % (what, np.max(np.abs(got - ref)))
    return got


def test_two_calls_second_smaller(sp):
    # first: RMAT scale 14 (hubs above the 256-entry threshold, so the hub
    # chunk lists and partial sums of the workspace are used), 24 sources
    rp1, ci1 = graphs.rmat(14, seed=71)
    s1 = graphs.sources(rp1, 24, seed=72, min_degree=1)
    g1 = sp.sp_graph_upload(rp1, ci1)
    print("noalloc: rmat-14, 24 sources", flush=True)
    assert_same(sp, g1, s1, "rmat-14")
    # second: a smaller road-like grid (many levels, short rows) right after
    rp2, ci2 = graphs.road(40, seed=73)
    s2 = graphs.sources(rp2, 5, seed=74)
    g2 = sp.sp_graph_upload(rp2, ci2)
    print("noalloc: road-40, 5 sources", flush=True)
    got = assert_same(sp, g2, s2, "road-40 after rmat-14")
    ref = oracle.bc(rp2, ci2, s2)
    zero = ref == 0
    assert np.all(got[zero] == 0)
    assert np.max(np.abs(got[~zero] - ref[~zero]) / np.abs(ref[~zero])) <= 1e-9
    # and the larger graph again, after the smaller one
    print("noalloc: rmat-14 again", flush=True)
    assert_same(sp, g1, s1[:7], "rmat-14 after road-40")
    g1.release()
    g2.release()


def test_edge_cases(sp):
    import torch
    rp, ci = graphs.uniform(300, 1200, seed=75)
    g = sp.sp_graph_upload(rp, ci)
    out = torch.full((300,), 7.0, dtype=torch.float64, device="cuda")
    _, st = sp.sp_bc_noalloc(g, [], out_bc=out)  # no sources: zeroed output
    assert st == sp.SP_OK and torch.count_nonzero(out).item() == 0
    assert_same(sp, g, [5, 5, 17], "duplicate source")
    with pytest.raises(sp.SpError) as e:
        sp.sp_bc_noalloc(g, [300])
    assert e.value.status == sp.SP_ERR_INVALID_ARGUMENT
    g.release()


def test_graph_above_the_limit_is_rejected(sp):
    import torch
    n = 2_000_000  # 40 bytes per vertex: above the 64 MiB workspace
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[2:] = 2  # one edge 0 - 1
    ci = np.array([1, 0], dtype=np.int32)
    g = sp.sp_graph_upload(rp, ci)
    out = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SpError) as e:
        sp.sp_bc_noalloc(g, [0], out_bc=out)
    assert e.value.status == sp.SP_ERR_INVALID_ARGUMENT
    assert "64" in sp.sp_last_error() or "bytes" in sp.sp_last_error()
    assert torch.all(out == 3.0).item(), "output written on error"
    g.release()
