"""Host-side measurement tooling, without a GPU: the rocprofv3 summariser
(name parsing, counter calibration, per-family bytes, source digest) and the
bench's roofline arithmetic, traffic lookup, parity rule and one-GPU guard."""
from __future__ import annotations

import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
from paper_2305_03317_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HUB = "void sp::k_ms_delta_hub<%d>(sp::LevelCtl*, int const*, int const*, double*, int)"
NEG = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)>(int)"


def test_short_names_keep_template_arguments():
    assert rs.short_name(HUB % 512) == "k_ms_delta_hub<512>"
    assert rs.base_name(rs.short_name(HUB % 512)) == "k_ms_delta_hub"
    assert rs.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
    assert rs.short_name("void sp::k_wg_bc_ell<1024, 4>(int const*)") == "k_wg_bc_ell<1024, 4>"


def write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def counter_run(d, counter, rows):
    """rows: (kernel name, value in KiB) per dispatch."""
    write_csv(os.path.join(d, "x", "run_counter_collection.csv"),
              ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
              [[i + 1, k, counter, v] for i, (k, v) in enumerate(rows)])


def test_summary_calibrates_counters_and_keeps_the_most_launched_instance(tmp_path, monkeypatch):
    gib = 1 << 30
    stats = tmp_path / "stats"
    write_csv(str(stats / "run_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
              [[HUB % 512, 4, 4.0e6, 1.0e6, 90.0], [NEG, 1, 4.0e5, 4.0e5, 10.0]])
    # the calibration kernel reads and writes 1 GiB; the counters see 2 GiB
    # fetched and 0.5 GiB written, so the factors are 0.5 and 2
    fetch_rows = [(NEG, 2.0 * gib / 1024)] + [(HUB % 512, 3000.0)] * 4 + [(HUB % 256, 9000.0)]
    write_rows = [(NEG, 0.5 * gib / 1024)] + [(HUB % 512, 100.0)] * 4 + [(HUB % 256, 50.0)]
    counter_run(str(tmp_path / "fetch"), "FETCH_SIZE", fetch_rows)
    counter_run(str(tmp_path / "write"), "WRITE_SIZE", write_rows)
    md, js = tmp_path / "s.md", tmp_path / "s.json"
    monkeypatch.setattr(sys, "argv", ["rocprof_summary", "--stats", str(stats), "--fetch", str(tmp_path / "fetch"),
                                      "--write", str(tmp_path / "write"), "--copy-gib", "1", "--workload", "w",
                                      "--command", "cmd", "--md", str(md), "--json", str(js)])
    rs.main()
    doc = json.loads(js.read_text())
    assert doc["fetch_scale"] == pytest.approx(0.5)
    assert doc["write_scale"] == pytest.approx(2.0)
    assert doc["source_digest"] == rs.source_digest()
    fam = doc["families"]["ms_delta_hub"]
    assert fam["kernel"] == "k_ms_delta_hub<512>" and fam["dispatches"] == 4
    assert fam["fetch_bytes_per_launch"] == pytest.approx(3000.0 * 1024 * 0.5)
    assert fam["write_bytes_per_launch"] == pytest.approx(100.0 * 1024 * 2.0)
    assert fam["traffic_bytes_per_launch"] == pytest.approx(3000.0 * 512 + 100.0 * 2048)
    text = md.read_text()
    assert "cmd" in text and "k_ms_delta_hub<512>" in text


def test_summary_refuses_counter_runs_without_the_calibration_kernel(tmp_path):
    counter_run(str(tmp_path), "FETCH_SIZE", [(HUB % 512, 3000.0)])
    per = rs.read_pmc(str(tmp_path), "FETCH_SIZE")
    with pytest.raises(SystemExit):
        rs.calibration(per, float(1 << 30))


def test_digest_follows_the_kernel_sources(tmp_path, monkeypatch):
    for name, body in (("a.hip", "x"), ("b.h", "y")):
        (tmp_path / name).write_text(body)
    monkeypatch.setattr(rs, "CSRC", str(tmp_path))
    d0 = rs.source_digest()
    (tmp_path / "b.h").write_text("y ")
    d1 = rs.source_digest()
    (tmp_path / "notes.txt").write_text("z")
    assert d0 != d1 and rs.source_digest() == d1


class FakeProfiler:
    """Stands in for the binding's profiling calls: a timed run, then a
    counted run (with half as many launches, as when the counted run is a
    shorter sample)."""
    SP_PROFILE_TIMES, SP_PROFILE_COUNTS = 1, 2

    def __init__(self, timed, counted):
        self.reads = [{}, timed, counted]
        self.modes = []

    def sp_profile_enable(self, mode):
        self.modes.append(mode)

    def sp_profile_read(self):
        return self.reads.pop(0)


def test_roofline_is_algorithmic_bytes_of_the_dominant_kernel_over_its_time():
    timed = {"ms_delta_hub": {"launches": 10, "total_ms": 5.0}, "ms_sigma": {"launches": 10, "total_ms": 2.0}}
    counted = {"ms_delta_hub": {"launches": 5, "edges": 1e8, "pairs": 5e7},
               "ms_sigma": {"launches": 5, "items": 1e6, "edges": 1e7, "pairs": 1e6, "item_slots": 1e6}}
    fake = FakeProfiler(timed, counted)
    calls = []
    kernels, roof = bench.profile_kernels(fake, lambda: calls.append(1), per=2)
    assert len(calls) == 2 and fake.modes == [1, 2, False]
    # 20 B per edge + 8 B per pair, counted over half the launches
    alg = (20 * 1e8 + 8 * 5e7) * 2
    assert kernels["ms_delta_hub"]["algorithmic_bytes_per_launch"] == int(alg / 10)
    assert kernels["ms_delta_hub"]["ms_per_unit"] == 2.5
    assert roof["kernel"] == "ms_delta_hub" and roof["bound"] == "hbm"
    assert roof["achieved"] == pytest.approx(alg / 5.0e-3 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0, abs=1e-4)
    assert roof["avg_launch_ms"] == 0.5 and roof["traffic"] is None


def test_byte_model_covers_every_profiled_family():
    import re
    names = open(os.path.join(ROOT, "paper_2305_03317_amd", "csrc", "profile.hip")).read()
    table = re.search(r"kProfNames\[\w*\]\s*=\s*\{(.*?)\};", names, re.S).group(1)
    fams = re.findall(r'"(\w+)"', table)
    assert fams, "profile family names not found"
    # the PageRank hub finish (a thread per hub adding its chunk sums) counts
    # no units of its own: its rows are counted by the pull kernel's chunks
    missing = [f for f in fams if f not in bench.BYTE_MODEL and f != "pr_hub"]
    assert not missing, missing
    for f in bench.FORWARD:
        assert f in bench.BYTE_MODEL


def test_traffic_is_used_only_while_the_sources_match(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic_rmat-22.json")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    doc = json.load(open(path))
    monkeypatch.setattr(rs, "source_digest", lambda: doc["source_digest"])
    roof = bench.attach_traffic({"kernel": "ms_delta_hub", "traffic": None}, "rmat-22")
    assert roof["traffic"] == round(doc["families"]["ms_delta_hub"]["traffic_bytes_per_launch"])
    monkeypatch.setattr(rs, "source_digest", lambda: "0" * 16)
    roof = bench.attach_traffic({"kernel": "ms_delta_hub", "traffic": None}, "rmat-22")
    assert roof["traffic"] is None


def test_parity_rule():
    ref = np.array([0.0, 1.0, 3.0])
    assert bench.bc_parity(ref.copy(), ref)["pass"]
    assert bench.bc_parity(ref * (1 + 5e-10), ref)["pass"]
    assert not bench.bc_parity(ref * (1 + 2e-9), ref)["pass"]
    assert not bench.bc_parity(ref + np.array([1e-300, 0, 0]), ref)["pass"]


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
