"""Parity at the benchmark workloads' full sizes, in the benchmark's launch
configuration (batches of 64 sources through the multi-source path).

At these sizes the oracle takes about a second per source, so whole batches
run on the GPU and a few of their slots are compared in full (distance
bit-exact; path counts and dependencies as in the small-graph parity tests),
and BC over a short source list is compared vertex by vertex.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_03317_amd import graphs
from tests.test_gpu_parity import assert_bc, assert_sigma

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_03317_amd import sp as spmod
    spmod.lib()
    return spmod


@pytest.mark.parametrize("k,slots,alpha", [(2, (0, 37), 15.0), (3, (0, 63), 4.0), (4, (5, 50), 15.0)])
def test_full_size_batch_slots(sp, k, slots, alpha):
    """Block 512 (the built-in default); on RMAT-22 with the threshold the
    autotuner picks there (alpha 4)."""
    rp, ci, src, spec = graphs.workload(k)
    print("workload", spec["name"], "vertices", len(rp) - 1, flush=True)
    g = sp.sp_graph_upload(rp, ci)
    batch = src[:64]
    bd, bs, bdl, st = sp.sp_batch_levels(g, batch, config={"block_size": 512, "alpha": alpha})
    assert st == sp.SP_OK
    for i in slots:
        s = int(batch[i])
        d_ref, sig_ref, del_ref = oracle.source_detail(rp, ci, s)
        assert np.array_equal(bd[i].cpu().numpy(), d_ref), "dist, slot %d" % i
        assert_sigma(bs[i].cpu().numpy(), sig_ref, "sigma, slot %d" % i)
        assert_bc(bdl[i].cpu().numpy(), np.where(d_ref > 0, del_ref, 0.0), "delta, slot %d" % i)
    del bd, bs, bdl
    few = src[:2]
    ref = oracle.bc(rp, ci, few)
    got, st = sp.sp_bc_batch(g, few)
    assert st == sp.SP_OK
    assert_bc(got.cpu().numpy(), ref, "%s BC over 2 sources" % spec["name"])
    g.release()


@pytest.mark.parametrize("k", [3, 4])
def test_full_size_global_sum_invariant(sp, k):
    """Sum over v of BC(v) equals the sum over sources s and reached targets t
    of (dist_s(t) - 1): every shortest s-t path has dist_s(t) - 1 interior
    vertices and each is counted with weight sigma_st(v)/sigma_st, which sums
    to one per interior position.  Checked over every source of the workload
    (RMAT-22: 1,024; road-4096: 64), with the distances from the batched
    pass (their values are pinned against the oracle by the slot test above)."""
    import torch
    rp, ci, src, spec = graphs.workload(k)
    g = sp.sp_graph_upload(rp, ci)
    bc, st = sp.sp_bc_batch(g, src)
    assert st == sp.SP_OK
    total_bc = float(bc.double().sum().item())
    want = 0
    for b in range(0, len(src), 64):
        d, _, _, st = sp.sp_batch_levels(g, src[b:b + 64], with_sigma=False, with_delta=False)
        assert st == sp.SP_OK
        d = d.long()
        want += int(torch.where(d > 0, d - 1, torch.zeros_like(d)).sum().item())
        del d
    print(spec["name"], total_bc, want, flush=True)
    assert abs(total_bc - want) <= 1e-9 * want
    g.release()
