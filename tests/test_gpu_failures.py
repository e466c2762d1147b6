"""Failure paths forced from the host: an allocation hook makes the library's
device allocations fail after the graph upload; both BC paths must return
SP_ERR_OUT_OF_MEMORY and leave the output untouched.  Runs in a child process
because the hook is read once per process."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, %r)
from paper_2305_03317_amd import graphs, sp
rp, ci = graphs.uniform(512, 2048, 5)
g = sp.sp_graph_upload(rp, ci)          # allocations 0, 1, 2 succeed
out = torch.full((512,), 7.0, dtype=torch.float64, device="cuda")
codes = []
for fn in (sp.sp_bc_batch, sp.sp_bc):
    try:
        fn(g, [1, 2, 3], out_bc=out)
        codes.append(0)
    except sp.SpError as e:
        codes.append(e.status)
assert codes == [sp.SP_ERR_OUT_OF_MEMORY] * 2, codes
assert torch.all(out == 7.0).item()
print("ok")
""" % ROOT


def test_allocation_failure_leaves_output_untouched():
    env = dict(os.environ, SP_TEST_FAIL_ALLOC_AFTER="3")
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
