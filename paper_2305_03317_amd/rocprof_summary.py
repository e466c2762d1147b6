"""Summarise rocprofv3 output of a bench.py run into text for profiles/.

Inputs are the CSV directories of three runs of the same bench.py command:

* ``--stats DIR``: ``rocprofv3 --kernel-trace --stats --output-format csv``
  (per-kernel calls, total and average duration);
* ``--fetch DIR`` / ``--write DIR``: ``rocprofv3 --pmc FETCH_SIZE`` and
  ``--pmc WRITE_SIZE`` (KiB per dispatch), each run with ``bench.py
  --copy-gib G`` so that one elementwise kernel that reads G GiB and writes
  G GiB (int32 negation) calibrates the counters: factor = known bytes /
  counted bytes.  Optional: without them only the kernel trace is summarised.

Writes a Markdown summary (the commands, the kernel table, calibrated HBM bytes
per dispatch) and a JSON file of per-family bytes per launch that bench.py
reads for ``roofline.traffic``, stamped with a digest of the kernel sources so
that it is ignored once a kernel changes.

    python -m paper_2305_03317_amd.rocprof_summary --stats D1 --fetch D2 \\
        --write D3 --copy-gib 1 --workload rmat-22 --command "..." \\
        --md profiles/x.md --json profiles/x.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# kernel function name -> profile family reported by sp_profile_read
FAMILY = {
    "k_ms_topdown": "ms_topdown", "k_ms_bottomup": "ms_bottomup", "k_ms_sigma": "ms_sigma",
    "k_ms_sigma_hub": "ms_sigma_hub", "k_ms_delta": "ms_delta", "k_ms_delta_hub": "ms_delta_hub",
    "k_ms_expand": "ms_expand", "k_ms_bc": "ms_bc", "k_src_topdown": "src_topdown", "k_src_bottomup": "src_bottomup",
    "k_src_sigma": "src_sigma", "k_src_sigma_hub": "src_sigma_hub", "k_src_delta": "src_delta",
    "k_src_delta_hub": "src_delta_hub", "k_sssp_push": "sssp_push", "k_sssp_pull": "sssp_pull",
    "k_pr_pull": "pr_pull", "k_pr_hub_fin": "pr_hub", "k_tc_count": "tc_count",
    "k_wg_bc": "wg_bc", "k_wg_bc_ell": "wg_bc", "k_wg_bc_sum": "wg_bc_sum", "k_ms_sigma_push": "ms_sigma_push",
}


def source_digest() -> str:
    """sha256 over the HIP sources and headers of the library (sorted by name)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    m = re.search(r"(?:sp::)?(\w+)(<[^>(]*>)?\s*\(", full)
    if m:
        return m.group(1) + (m.group(2) or "")
    return full.split("(")[0][:60]


def base_name(short: str) -> str:
    return short.split("<")[0]


def _one(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise SystemExit("no %s under %s" % (pattern, d))
    return hits[0]


def read_stats(d):
    rows = []
    with open(_one(d, "*kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append(dict(name=short_name(r["Name"]), calls=int(r["Calls"]),
                             total_ms=float(r["TotalDurationNs"]) / 1e6,
                             avg_us=float(r["AverageNs"]) / 1e3, pct=float(r["Percentage"])))
    return rows


def read_pmc(d, counter):
    """{short kernel name: [values per dispatch]} plus the copy kernel's values."""
    per = defaultdict(list)
    with open(_one(d, "*counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            per[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> B
    return per


def calibration(per, copy_bytes):
    """Factor = known bytes of the calibration kernel / bytes the counter saw.
    The calibration kernel is the one elementwise negation bench.py runs with
    --copy-gib; its dispatches are summed in case the runtime splits it."""
    hits = [v for k, vals in per.items() if "neg" in k.lower() for v in vals if v >= copy_bytes / 16]
    if not hits:
        raise SystemExit("no calibration kernel in the counter run (run bench.py with --copy-gib)")
    seen = sum(hits)
    return copy_bytes / seen, seen


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-gib", type=float, default=1.0)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", action="append", default=[], help="command line(s) that made the runs")
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    a = ap.parse_args()

    copy_bytes = a.copy_gib * (1 << 30)
    stats = read_stats(a.stats)
    counters = bool(a.fetch and a.write)
    fetch = read_pmc(a.fetch, "FETCH_SIZE") if counters else {}
    write = read_pmc(a.write, "WRITE_SIZE") if counters else {}
    cf, fb = calibration(fetch, copy_bytes) if counters else (0.0, 0.0)
    cw, wb = calibration(write, copy_bytes) if counters else (0.0, 0.0)
    digest = source_digest()

    fam = {}
    lines = ["# rocprofv3 summary: %s" % a.workload, ""]
    lines += ["Commands (run from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", ""]
    lines += ["    " + c for c in a.command] + [""]
    lines += ["Kernel sources digest: `%s` (sha256 prefix over csrc/*.hip, csrc/*.h)." % digest, ""]
    lines += ["## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -r["total_ms"])[:20]:
        lines.append("| %s | %d | %.3f | %.2f | %.2f |" % (r["name"], r["calls"], r["total_ms"], r["avg_us"], r["pct"]))
    if not counters:
        lines += ["", "(No counter runs for this workload.)"]
    lines += [] if not counters else ["", "## HBM traffic (--pmc FETCH_SIZE, --pmc WRITE_SIZE, separate runs)", "",
              "Calibration: one elementwise kernel (int32 negation) that reads and writes %.0f MiB "
              "counted FETCH_SIZE %.1f MiB and WRITE_SIZE %.1f MiB, so FETCH_SIZE is scaled by %.4f "
              "and WRITE_SIZE by %.4f." % (copy_bytes / 2**20, fb / 2**20, wb / 2**20, cf, cw), "",
              "| kernel | dispatches | FETCH MiB/dispatch (raw) | WRITE MiB/dispatch (raw) | "
              "calibrated MB/dispatch | calibrated GB total |", "|---|---:|---:|---:|---:|---:|"]
    names = sorted(set(fetch) | set(write), key=lambda k: -sum(fetch.get(k, [])))
    for k in names:
        fv, wv = fetch.get(k, []), write.get(k, [])
        if not fv or base_name(k) not in FAMILY:
            continue
        nd = len(fv)
        f_avg = sum(fv) / nd
        w_avg = sum(wv) / max(len(wv), 1)
        per = f_avg * cf + w_avg * cw
        tot = sum(fv) * cf + sum(wv) * cw
        lines.append("| %s | %d | %.2f | %.2f | %.2f | %.2f |" % (k, nd, f_avg / 2**20, w_avg / 2**20, per / 1e6, tot / 1e9))
        # several instances of a family (block sizes tried by the autotuner):
        # keep the one launched most, the configuration the timed steps use
        f = FAMILY[base_name(k)]
        if f not in fam or nd > fam[f]["dispatches"]:
            fam[f] = dict(kernel=k, dispatches=nd, fetch_bytes_per_launch=f_avg * cf,
                          write_bytes_per_launch=w_avg * cw, traffic_bytes_per_launch=per)
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    with open(a.md, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(a.json, "w") as f:
        json.dump(dict(workload=a.workload, source_digest=digest, fetch_scale=cf, write_scale=cw,
                       copy_bytes=copy_bytes, families=fam, commands=a.command), f, indent=1)
    print("wrote", a.md, a.json)


if __name__ == "__main__":
    main()
