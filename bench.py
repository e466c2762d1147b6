#!/usr/bin/env python3
"""Benchmark: batched betweenness centrality on one MI355X.

One step = the whole hot path over one batch of synthetic input: sp_bc_batch
on the workload's full source list (per-batch init, level-synchronous
multi-source forward pass, reverse pass, BC accumulation, sigma overflow
check), with the graph already resident in HBM.  The graph is built and
uploaded once before timing; upload time is reported separately.

Default workload: RMAT scale 22 (4,194,304 vertices, edge factor 16,
a/b/c = 0.57/0.19/0.19, deduplicated, vertex ids permuted), 1,024 seeded
sources among vertices of degree >= 1, batches of 64.  TEPS = sources x
undirected edges / step time.

Regions: (1) the timed steps, in the production configuration (forward level
chunks replayed from captured hipGraphs) -> value, ms_per_step; (2) the same
steps with a HIP event pair around every kernel launch and device work
counters -> kernels, roofline (dominant kernel: algorithmic bytes per launch /
average launch time against 8 TB/s; traffic from the committed rocprofv3
counter summary while the kernel sources are unchanged), forward_pass.
Also: the per-source GPU path on the same sources (the batched vs per-source
ratio, and its own kernel roofline on a sample), the CPU oracle on a bounded
sample (cpu_baseline, which doubles as a parity check of this run), the
per-source path on RMAT scale 20 (256 sources), batched BC on the 4096 x 4096
road-like grid (64 sources in one batch, captured level loop, sigma overflow
check, oracle parity on two sources), the serving workload (eight
resident graphs, seeded Poisson request stream; p50/p99 latency and TEPS),
single-source shortest paths on the RMAT and road graphs with the paper's
uniform [1, 100] weights (per-source time, kernel roofline, Dijkstra oracle),
PageRank on the same graphs (time per iteration, kernel roofline, numpy
oracle), the triangle count of the RMAT graph, and BC on a directed version
of it (both paths).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BC TEPS (sources×edges/s) batched vs per-source at 1e-9 rel err; p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {"uniform-4096": 1, "rmat-20": 2, "rmat-22": 3, "road-4096": 4}

# Algorithmic bytes per unit of work, per kernel family (units counted on the
# device while timing): items = vertices (per-source) or (vertex, level)
# entries (batched); edges = adjacency entries scanned; pairs = DAG edges
# (per-source) or (slot, DAG edge) pairs (batched); item_slots = slots over
# entries (batched).
BYTE_MODEL = {
    "ms_sigma": dict(items=72, edges=20, pairs=8, item_slots=8),
    "ms_sigma_hub": dict(edges=20, pairs=8),
    # pushed path counts: items = parent entries (queue, qmask, qvb, row
    # offsets), edges = their outgoing entries (column id, child's front
    # record), pairs = (slot, DAG edge) atomic adds (read and write of the
    # child's value)
    "ms_sigma_push": dict(items=24, edges=20, pairs=16),
    "ms_delta": dict(items=40, edges=20, pairs=8, item_slots=24),
    "ms_delta_hub": dict(edges=20, pairs=8),
    "ms_topdown": dict(items=20, edges=20),
    # fused road-like level: items = frontier entries (queue, front record,
    # qmask/qvb writes, row offsets), edges = their adjacency (column id, seen,
    # claim), pairs = (slot, parent) pairs summed, item_slots = entries of the
    # new vertices' rows read while gathering parent slots (column id, front)
    "ms_expand": dict(items=40, edges=16, pairs=8, item_slots=20),
    "ms_bottomup": dict(items=16, edges=20),
    "ms_bc": dict(items=24, item_slots=8),
    # blocks engine, one workgroup per source, forward and reverse levels in
    # one kernel: items = vertices reached, edges = outgoing entries expanded,
    # pairs = DAG edges summed (path counts and dependencies); per source the
    # forward and reverse byte models added up (28 + 44 per vertex, 8 + 8 per
    # adjacency entry, 16 per DAG edge and pass)
    "wg_bc": dict(items=72, edges=16, pairs=16),
    "src_topdown": dict(items=12, edges=8),
    "src_bottomup": dict(items=12, edges=8),
    "src_sigma": dict(items=20, edges=8, pairs=8),
    "src_sigma_hub": dict(edges=8, pairs=8),
    "src_delta_hub": dict(edges=8, pairs=16),
    "src_delta": dict(items=44, edges=8, pairs=16),
    # SSSP rounds: items = frontier vertices (push: queue entry, row offsets,
    # own distance) or all vertices (pull: row offsets), edges = adjacency
    # entries (packed {neighbour, weight} plus the neighbour's {dist, stamp})
    "sssp_push": dict(items=20, edges=16),
    "sssp_pull": dict(items=8, edges=16),
    # PageRank iteration: items = non-hub vertices (row offsets, own value
    # read, value and share written), edges = adjacency entries (column id,
    # neighbour's share); hub chunks count their entries the same way
    "pr_pull": dict(items=28, edges=12),
    # triangle count: edges = list elements walked (one 4-byte id each); the
    # per-entry reads (row id, neighbour id, four offsets) are added
    # separately from the oriented-entry count
    "tc_count": dict(edges=4),
}
FORWARD = ("ms_topdown", "ms_bottomup", "ms_sigma", "ms_sigma_hub", "ms_sigma_push", "ms_expand")


_WORKLOAD_CACHE = {}


def workload_graph(k):
    """graphs.workload(k), generated once per run (several legs share it)."""
    if k not in _WORKLOAD_CACHE:
        from paper_2305_03317_amd import graphs
        _WORKLOAD_CACHE[k] = graphs.workload(k)
    return _WORKLOAD_CACHE[k]


def algorithmic_bytes(name, prof):
    model = BYTE_MODEL.get(name, {})
    return sum(coef * prof.get(unit, 0) for unit, coef in model.items())


def load_traffic(workload):
    """Per-family HBM bytes per launch from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel
    sources changed since it was taken."""
    from paper_2305_03317_amd import rocprof_summary
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("source_digest") != rocprof_summary.source_digest():
        return None
    doc["path"] = os.path.relpath(path, ROOT)
    return doc


def sssp_benchmark(sp, torch, workload, n_sources):
    """Single-source shortest paths on a benchmark graph with the paper's
    synthetic weights (uniform on [1, 100], Section 5), one source at a time:
    wall time per source (distances in HBM when the call returns), then the
    same sources with kernel events, then once with work counters; the
    oracle's Dijkstra on the first source is the CPU baseline and a parity
    check."""
    import numpy as np
    import oracle
    from paper_2305_03317_amd import graphs
    k = WORKLOADS[workload]
    rp, ci, src, spec = workload_graph(k)
    w = graphs.weights(rp, ci, 3000 + k)
    m = len(ci) // 2
    g = sp.sp_graph_upload(rp, ci)
    sp.sp_graph_set_weights(g, w)
    out = torch.empty(len(rp) - 1, dtype=torch.int32, device="cuda")
    srcs = [int(x) for x in src[:n_sources]]
    sp.sp_sssp(g, srcs[0], out)  # warm: workspace and captured round chunks
    times, rounds = [], []
    for s in srcs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp.sp_sssp(g, s, out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rounds.append(sp.sp_sssp_get_last_stats()["rounds"])
        print("sssp %s source %d: %.2f ms, %d rounds" % (workload, s, times[-1] * 1e3, rounds[-1]),
              file=sys.stderr, flush=True)
    per_s = float(np.mean(times))
    sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_TIMES)
    for s in srcs:
        sp.sp_sssp(g, s, out)
    prof = sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_COUNTS)
    for s in srcs:
        sp.sp_sssp(g, s, out)
    counted = sp.sp_profile_read()
    sp.sp_profile_enable(False)
    kernels = {}
    for kname, p in prof.items():
        c = counted.get(kname, {})
        launches = max(p["launches"], 1)
        alg = algorithmic_bytes(kname, c) * (p["launches"] / max(c.get("launches", 1), 1))
        kernels[kname] = {"launches": p["launches"], "ms_per_source": round(p["total_ms"] / len(srcs), 3),
                          "avg_launch_ms": round(p["total_ms"] / launches, 4),
                          "edges_per_source": int(c.get("edges", 0) / len(srcs)),
                          "GBps_algorithmic": round(alg / max(p["total_ms"], 1e-9) / 1e6, 1)}
    dom = max(kernels.items(), key=lambda kv: kv[1]["ms_per_source"]) if kernels else None
    roofline = None
    if dom:
        achieved = dom[1]["GBps_algorithmic"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom[0],
                    "avg_launch_ms": dom[1]["avg_launch_ms"]}
        attach_traffic(roofline, "sssp_" + workload)
    t0 = time.perf_counter()
    ref = oracle.sssp(rp, ci, w, srcs[0])
    cpu_s = time.perf_counter() - t0
    got = sp.sp_sssp(g, srcs[0], out).cpu().numpy()
    g.release()
    edges_scanned = sum(v["edges_per_source"] for v in kernels.values())
    return {"workload": "%s, weights uniform [1,100] (seed %d)" % (spec["name"], 3000 + k),
            "sources": len(srcs), "ms_per_source": round(per_s * 1e3, 3), "teps": m / per_s,
            "unit": "TEPS (undirected edges / time per source)",
            "rounds_mean": float(np.mean(rounds)), "entries_scanned_over_nnz": round(edges_scanned / len(ci), 2),
            "kernels": kernels, "roofline": roofline,
            "cpu_baseline": {"value": m / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
                             "sample": "Dijkstra from the first source, single-threaded C oracle, %.2f s" % cpu_s},
            "parity": {"sources": 1, "bit_exact": bool(np.array_equal(got, ref))}}


def pagerank_benchmark(sp, torch, workload, iterations):
    """PageRank (the paper's pull form, damping 0.85) on a benchmark graph:
    a fixed number of iterations (beta = 0, so every run does exactly that
    many), wall time with the graph resident; then the same run with kernel
    events and once with work counters; the numpy oracle on the same
    iterations is the CPU baseline and a parity check."""
    import numpy as np
    import oracle
    from paper_2305_03317_amd import graphs
    directed = workload.endswith("-directed")
    k = WORKLOADS[workload[:-len("-directed")] if directed else workload]
    rp, ci, _, spec = workload_graph(k)
    if directed:  # each undirected edge kept as one arc, seeded direction (as the directed BC leg)
        rp, ci = graphs.directed_from(rp, ci, 4000 + k)
    g = sp.sp_graph_upload(rp, ci, directed=directed)
    out = torch.empty(len(rp) - 1, dtype=torch.float64, device="cuda")
    sp.sp_pagerank(g, 0.0, 0.85, iterations, out)  # warm: workspace, hub list, captured chunk
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp.sp_pagerank(g, 0.0, 0.85, iterations, out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    per_iter = float(np.min(times)) / iterations
    sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_TIMES)
    sp.sp_pagerank(g, 0.0, 0.85, iterations, out)
    prof = sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_COUNTS)
    sp.sp_pagerank(g, 0.0, 0.85, iterations, out)
    counted = sp.sp_profile_read()
    sp.sp_profile_enable(False)
    kernels = {}
    for kname, p in prof.items():
        c = counted.get(kname, {})
        launches = max(p["launches"], 1)
        alg = algorithmic_bytes(kname, c)
        kernels[kname] = {"launches": p["launches"], "ms_per_iteration": round(p["total_ms"] / iterations, 4),
                          "avg_launch_ms": round(p["total_ms"] / launches, 4),
                          "GBps_algorithmic": round(alg / max(p["total_ms"], 1e-9) / 1e6, 1)}
    dom = max(kernels.items(), key=lambda kv: kv[1]["ms_per_iteration"]) if kernels else None
    roofline = None
    if dom:
        achieved = dom[1]["GBps_algorithmic"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom[0],
                    "avg_launch_ms": dom[1]["avg_launch_ms"]}
        attach_traffic(roofline, "pagerank_" + workload)
    t0 = time.perf_counter()
    ref, _, _ = oracle.pagerank(rp, ci, 0.0, 0.85, iterations, iterations=iterations)
    cpu_s = time.perf_counter() - t0
    got = out.cpu().numpy()
    g.release()
    m = len(ci) // 2
    return {"workload": "%s%s, damping 0.85, %d iterations"
                        % (spec["name"], ", each edge one arc (seed %d)" % (4000 + k) if directed else "",
                           iterations),
            "ms_per_iteration": round(per_iter * 1e3, 4), "teps": len(ci) / per_iter,
            "unit": "TEPS (adjacency entries gathered / time per iteration)", "undirected_edges": m,
            "kernels": kernels, "roofline": roofline,
            "cpu_baseline": {"value": len(ci) * iterations / cpu_s, "unit": "TEPS", "cores": 1,
                             "kind": "oracle", "sample": "the same %d iterations, numpy oracle, %.1f s"
                                                         % (iterations, cpu_s)},
            "parity": {"max_rel_err": float(np.max(np.abs(got - ref) / ref)),
                       "pass": bool(np.max(np.abs(got - ref) / ref) <= 1e-9)}}


def tc_benchmark(sp, torch, workload, small_scale=16):
    """Triangle count of a benchmark graph: the first call builds the
    oriented rows (kept with the graph), later calls only count.  The
    oracle's node iterator is quadratic in hub degree, so the CPU baseline
    runs it on the same recipe at RMAT scale 16 (and the GPU beside it)."""
    import numpy as np
    import oracle
    from paper_2305_03317_amd import graphs
    k = WORKLOADS[workload]
    rp, ci, _, spec = workload_graph(k)
    m = len(ci) // 2
    g = sp.sp_graph_upload(rp, ci)
    count, _ = sp.sp_triangle_count(g)
    build_ms = sp.sp_tc_get_last_stats()["build_ms"]
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        again, _ = sp.sp_triangle_count(g)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        assert again == count
    count_s = float(np.min(times))
    sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_TIMES)
    sp.sp_triangle_count(g)
    prof = sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_COUNTS)
    sp.sp_triangle_count(g)
    counted = sp.sp_profile_read()
    sp.sp_profile_enable(False)
    p, c = prof.get("tc_count"), counted.get("tc_count", {})
    roofline = None
    if p:
        alg = algorithmic_bytes("tc_count", c) + 24 * m
        achieved = alg / (p["total_ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "tc_count",
                    "avg_launch_ms": round(p["total_ms"] / max(p["launches"], 1), 4),
                    "list_elements_walked": int(c.get("edges", 0))}
        attach_traffic(roofline, "tc_" + workload)
    g.release()
    out = {"workload": spec["name"], "triangles": count, "count_ms": round(count_s * 1e3, 3),
           "build_ms": round(build_ms, 3), "teps": m / count_s,
           "unit": "TEPS (undirected edges / count time)", "roofline": roofline}
    if small_scale <= 0:
        return out
    srp, sci = graphs.rmat(small_scale, 16, graphs.RMAT_ABC, 1000 + k)
    sg = sp.sp_graph_upload(srp, sci)
    sp.sp_triangle_count(sg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    small, _ = sp.sp_triangle_count(sg)
    torch.cuda.synchronize()
    small_s = time.perf_counter() - t0
    sg.release()
    t0 = time.perf_counter()
    ref = oracle.triangles(srp, sci)
    cpu_s = time.perf_counter() - t0
    sm = len(sci) // 2
    out.update({"small_gpu_teps": sm / small_s,
                "cpu_baseline": {"value": sm / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
                                 "sample": "node iterator on RMAT scale %d of the same recipe (seed %d), "
                                           "single-threaded C oracle, %.1f s" % (small_scale, 1000 + k, cpu_s)},
                "parity": {"graph": "rmat-%d" % small_scale, "gpu": small, "oracle": ref, "pass": small == ref}})
    return out


def attach_traffic(roofline, profile_name):
    """roofline["traffic"]: calibrated HBM bytes per launch of its kernel from
    the committed counter summary `profile_name`, while the kernel sources
    are unchanged (else it stays null)."""
    if not roofline:
        return roofline
    doc = load_traffic(profile_name)
    fam = doc["families"].get(roofline["kernel"]) if doc else None
    if fam:
        roofline["traffic"] = round(fam["traffic_bytes_per_launch"])
        roofline["traffic_source"] = doc["path"]
    return roofline


def directed_benchmark(sp, torch, workload, n_sources):
    """Betweenness centrality on a directed graph: the workload graph with
    each undirected edge kept as one arc in a seeded direction.  Both paths
    on the first n_sources of its sources (per-source: one BFS pass per
    source; batched: one multi-source pass, parents from the reversed rows),
    the batched path also on the workload's whole source list; kernel
    roofline of the batched pass; the oracle on two sources is the CPU
    baseline and a parity check of both paths."""
    import numpy as np
    import oracle
    from paper_2305_03317_amd import graphs
    k = WORKLOADS[workload]
    urp, uci, src, spec = workload_graph(k)
    rp, ci = graphs.directed_from(urp, uci, 4000 + k)
    arcs = len(ci)
    g = sp.sp_graph_upload(rp, ci, directed=True)
    srcs = src[:n_sources]
    out = torch.empty(len(rp) - 1, dtype=torch.float64, device="cuda")

    def timed(fn, s, reps=1):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = fn(g, s, out)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        return best, st, sp.sp_get_last_stats()

    sp.sp_bc(g, srcs[:1], out)
    ps_wall, st, ps_stats = timed(sp.sp_bc, srcs)
    t0 = time.perf_counter()
    tuned = sp.sp_autotune(g, src)
    tuning_s = time.perf_counter() - t0
    sp.sp_bc_batch(g, srcs, out)  # warm: workspace, captured chunks
    b_wall, bst, b_stats = timed(sp.sp_bc_batch, srcs, reps=3)
    sp.sp_bc_batch(g, src, out)
    ball_wall, ballst, ball_stats = timed(sp.sp_bc_batch, src, reps=2)
    kernels, roofline = profile_kernels(sp, lambda: sp.sp_bc_batch(g, srcs, out), 1)
    attach_traffic(roofline, "directed_" + workload)
    t0 = time.perf_counter()
    ref = oracle.bc(rp, ci, srcs[:2])
    cpu_s = time.perf_counter() - t0
    par = {}
    for name, fn in (("per_source", sp.sp_bc), ("batched", sp.sp_bc_batch)):
        got, _ = fn(g, srcs[:2], out)
        par[name] = bc_parity(got.cpu().numpy(), ref)
    g.release()
    per_source = {"sources": len(srcs), "ms_per_source": round(ps_wall * 1e3 / len(srcs), 3),
                  "teps": len(srcs) * arcs / ps_wall, "status": st, "levels_max": ps_stats["max_levels"]}
    batched = {"sources": len(srcs), "ms": round(b_wall * 1e3, 2), "teps": len(srcs) * arcs / b_wall,
               "status": bst, "levels_max": b_stats["max_levels"],
               "topdown_levels": b_stats["topdown_levels"], "bottomup_levels": b_stats["bottomup_levels"],
               "config": {k2: tuned[k2] for k2 in ("batch_width", "block_size", "alpha", "beta", "chunk_levels")},
               "tuning_s": round(tuning_s, 2)}
    batched_all = {"sources": len(src), "ms": round(ball_wall * 1e3, 1), "teps": len(src) * arcs / ball_wall,
                   "status": ballst, "passes": ball_stats["n_passes"]}
    return {"workload": "%s, each edge one arc (seed %d)" % (spec["name"], 4000 + k), "arcs": arcs,
            "unit": "TEPS (sources x arcs / time)",
            "batched_over_per_source": batched["teps"] / per_source["teps"],
            "per_source": per_source, "batched": batched, "batched_all_sources": batched_all,
            "roofline": roofline, "kernels": kernels,
            "cpu_baseline": {"value": 2 * arcs / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
                             "sample": "first 2 sources, single-threaded C oracle, %.2f s" % cpu_s},
            "parity": dict(sources=2, **{k2: v for k2, v in par.items()},
                           all_pass=all(v["pass"] for v in par.values()))}


def profile_kernels(sp, run, per):
    """Run `run()` once with a HIP event pair around every kernel launch, then
    once with the device work counters on; per-kernel launches, time per
    `per` unit, average launch time and algorithmic GB/s, and the roofline of
    the kernel with the most time (algorithmic bytes per launch over its
    average launch time, against 8 TB/s)."""
    sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_TIMES)
    run()
    prof = sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_COUNTS)
    run()
    counted = sp.sp_profile_read()
    sp.sp_profile_enable(False)
    kernels = {}
    for kname, p in prof.items():
        c = counted.get(kname, {})
        scale = p["launches"] / c["launches"] if c.get("launches") else 0.0
        alg = algorithmic_bytes(kname, c) * scale
        launches = max(p["launches"], 1)
        kernels[kname] = {"launches": p["launches"], "ms_per_unit": round(p["total_ms"] / per, 4),
                          "avg_launch_ms": round(p["total_ms"] / launches, 4),
                          "algorithmic_bytes_per_launch": int(alg / launches),
                          "GBps_algorithmic": round(alg / max(p["total_ms"], 1e-9) / 1e6, 1)}
    dom = max(kernels.items(), key=lambda kv: kv[1]["ms_per_unit"]) if kernels else None
    roofline = None
    if dom:
        achieved = dom[1]["GBps_algorithmic"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom[0],
                    "launches": dom[1]["launches"], "avg_launch_ms": dom[1]["avg_launch_ms"],
                    "algorithmic_bytes_per_launch": dom[1]["algorithmic_bytes_per_launch"]}
    return kernels, roofline


def bc_parity(got, ref):
    import numpy as np
    nz = ref != 0
    rel = float(np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz]))) if nz.any() else 0.0
    return {"max_rel_err": rel, "zero_exact": bool(np.all(got[~nz] == 0)),
            "pass": bool(rel <= 1e-9 and np.all(got[~nz] == 0))}


def per_source_benchmark(sp, torch, workload, n_sources, profile_sample=32, oracle_sources=4):
    """Per-source BC path (sp_bc: one BFS pass per source) on a benchmark
    graph: wall time over n_sources with the graph resident, the kernel
    roofline over a sample of them, and the oracle on a few sources as CPU
    baseline and parity check."""
    import oracle
    k = WORKLOADS[workload]
    rp, ci, src, spec = workload_graph(k)
    m = len(ci) // 2
    srcs = src[:n_sources]
    g = sp.sp_graph_upload(rp, ci)
    out = torch.empty(len(rp) - 1, dtype=torch.float64, device="cuda")
    sp.sp_bc(g, srcs[:1], out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = sp.sp_bc(g, srcs, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = sp.sp_get_last_stats()
    sample = srcs[:profile_sample]
    kernels, roofline = profile_kernels(sp, lambda: sp.sp_bc(g, sample, out), len(sample))
    attach_traffic(roofline, "bc_per_source_" + workload)
    res = {"workload": "%s per-source BC" % spec["name"], "sources": len(srcs), "status": st,
           "ms_per_source": round(wall * 1e3 / len(srcs), 3), "teps": len(srcs) * m / wall,
           "unit": "TEPS (sources x undirected edges / time)", "block_size": stats["block_size"],
           "levels_max": stats["max_levels"], "roofline": roofline,
           "roofline_sample": "first %d sources" % len(sample), "kernels": kernels}
    if oracle_sources > 0:
        cs = srcs[:oracle_sources]
        t0 = time.perf_counter()
        ref = oracle.bc(rp, ci, cs)
        cpu_s = time.perf_counter() - t0
        got, _ = sp.sp_bc(g, cs, out)
        res["cpu_baseline"] = {"value": len(cs) * m / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
                               "sample": "first %d sources, single-threaded C oracle, %.1f s" % (len(cs), cpu_s)}
        res["parity"] = dict(sources=len(cs), **bc_parity(got.cpu().numpy(), ref))
    g.release()
    return res


def road_batched_benchmark(sp, torch, workload, n_sources, runs=3, oracle_sources=2, compare_bitmap=True):
    """Batched BC on the road-like grid: every source in one batch, in the
    library's automatic engine for road-like graphs (one workgroup per source,
    the whole pass in one launch); wall time per pass with the graph resident
    (best of `runs`), level count and sigma-overflow status, the kernel
    roofline, the other engine (one multi-source bitmap pass, levels replayed
    from captured hipGraphs) timed for comparison, and the oracle on a few of
    the sources (a separate batch of them) as parity check."""
    import numpy as np
    import oracle
    k = WORKLOADS[workload]
    rp, ci, src, spec = workload_graph(k)
    m = len(ci) // 2
    srcs = src[:n_sources]
    g = sp.sp_graph_upload(rp, ci)
    out = torch.empty(len(rp) - 1, dtype=torch.float64, device="cuda")
    sp.sp_bc_batch(g, srcs, out)  # warm: workspace and captured level chunks
    times = []
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = sp.sp_bc_batch(g, srcs, out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print("road batched pass: %.1f ms" % (times[-1] * 1e3), file=sys.stderr, flush=True)
    stats = sp.sp_get_last_stats()
    best = float(np.min(times))
    kernels, roofline = profile_kernels(sp, lambda: sp.sp_bc_batch(g, srcs, out), 1)
    attach_traffic(roofline, "bc_batch_" + workload)
    bitmap_ms = bitmap_levels = None
    if compare_bitmap:
        bitmap = {"engine": sp.SP_ENGINE_BITMAP}
        sp.sp_bc_batch(g, srcs, out, config=bitmap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp.sp_bc_batch(g, srcs, out, config=bitmap)
        torch.cuda.synchronize()
        bitmap_ms = round((time.perf_counter() - t0) * 1e3, 1)
        bitmap_levels = sp.sp_get_last_stats()["graph_launches"]
    cs = srcs[:oracle_sources]
    t0 = time.perf_counter()
    ref = oracle.bc(rp, ci, cs)
    cpu_s = time.perf_counter() - t0
    got, _ = sp.sp_bc_batch(g, cs, out)
    g.release()
    return {"workload": "%s batched BC" % spec["name"], "sources": len(srcs), "status": st,
            "sigma_flagged_sources": stats["sigma_flagged"], "sigma_max": stats["sigma_max"],
            "ms_per_pass": round(best * 1e3, 1), "ms_per_pass_runs": [round(t * 1e3, 1) for t in times],
            "teps": len(srcs) * m / best, "unit": "TEPS (sources x undirected edges / time)",
            "levels_max": stats["max_levels"], "batch_width": stats["batch_width"],
            "engine": {1: "bitmap", 2: "blocks"}.get(stats["engine"], stats["engine"]),
            "block_size": stats["block_size"],
            "chunk_levels": stats["chunk_levels"], "graph_launches": stats["graph_launches"],
            "roofline": roofline, "kernels": kernels,
            "bitmap_engine": {"ms_per_pass": bitmap_ms, "graph_launches": bitmap_levels},
            "cpu_baseline": {"value": len(cs) * m / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
                             "sample": "first %d sources, single-threaded C oracle, %.1f s" % (len(cs), cpu_s)},
            "parity": dict(sources=len(cs), **bc_parity(got.cpu().numpy(), ref))}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def serving_benchmark(sp, torch, n_requests, seed=2005, budget_gb=230):
    """Serving workload: eight resident graphs, seeded requests (graph uniform,
    1..512 sources log-uniform), continuous batching by the library's server.
    Phase "burst" submits every request at once (saturation throughput);
    phases at 50% and 80% of that rate submit them with seeded exponential
    gaps (Poisson arrivals).  Latency is the library's submit-to-completion
    time of each request."""
    import numpy as np
    from paper_2305_03317_amd import graphs
    t0 = time.perf_counter()
    gs = graphs.serving_graphs()
    reqs = graphs.serving_requests([rp for _, rp, _ in gs], n_requests, seed)
    build_s = time.perf_counter() - t0
    handles = [sp.sp_graph_upload(rp, ci) for _, rp, ci in gs]
    edges = [len(ci) // 2 for _, _, ci in gs]
    # an explicit workspace budget (the library's default is a quarter of the
    # free memory at creation, which depends on what ran before): room for a
    # workspace of every graph on each of the four workers (about 190 GB, most
    # of it road-4096's 30 GB per worker), so admission never has to evict
    srv = sp.Server(memory_budget=budget_gb << 30)
    ids = [srv.add_graph(h) for h in handles]
    outs = [torch.empty(max(h.n, 1), dtype=torch.float64, device="cuda") for h in handles]
    for gid, h in zip(ids, handles):  # warm: workspaces and captured graphs exist before timing
        r = srv.submit(gid, graphs.sources(gs[gid][1], 64, 7, min_degree=1), out_bc=outs[gid])
        assert r.wait() == sp.SP_OK
        r.release()
    work = sum(len(src) * edges[gi] for gi, src in reqs)

    def phase(rate):
        rng = np.random.default_rng(seed + 1)
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        live = []
        start = time.perf_counter()
        t_next = start
        for (gi, src), gap in zip(reqs, gaps):
            t_next += gap
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            out = torch.empty(max(handles[gi].n, 1), dtype=torch.float64, device="cuda")
            live.append(srv.submit(ids[gi], src, out_bc=out))
        bad, warned, errors = 0, 0, {}
        for k, r in enumerate(live):
            st = r.wait()
            if (k + 1) % 20 == 0:
                print("  %d/%d requests done, %.1f s" % (k + 1, len(live), time.perf_counter() - start),
                      file=sys.stderr, flush=True)
            if st < 0:
                bad += 1
                msg = sp.lib().sp_last_error()
                msg = msg.decode() if isinstance(msg, bytes) else str(msg)
                errors[msg] = errors.get(msg, 0) + 1
            elif st > 0:
                warned += 1
        wall = time.perf_counter() - start
        lat = np.array([r.latency_us() for r in live]) / 1e3
        for r in live:
            r.release()
        by_graph = {}
        for gi in sorted(set(g for g, _ in reqs)):
            sel = np.array([g == gi for g, _ in reqs])
            big = max(len(src) for g, src in reqs if g == gi)
            by_graph[gs[gi][0]] = {"requests": int(sel.sum()), "largest_sources": big,
                                   "p50_ms": round(float(np.percentile(lat[sel], 50)), 1),
                                   "p99_ms": round(float(np.percentile(lat[sel], 99)), 1)}
        print("serving phase rate=%s: %.1f s" % (rate, wall), file=sys.stderr, flush=True)
        return {"offered_qps": round(rate, 3) if rate else None, "achieved_qps": round(len(reqs) / wall, 3),
                "teps": work / wall, "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2), "max_ms": round(float(lat.max()), 2),
                "wall_s": round(wall, 2), "failed": int(bad), "sigma_warnings": int(warned),
                "errors": errors or None, "by_graph": by_graph}

    burst = phase(0)
    sat = burst["achieved_qps"]
    res = {"graphs": [n for n, _, _ in gs], "requests": len(reqs),
           "mean_sources": round(float(np.mean([len(s) for _, s in reqs])), 1),
           "graph_build_s": round(build_s, 1), "burst": burst,
           "load50": phase(0.5 * sat), "load80": phase(0.8 * sat), "load95": phase(0.95 * sat)}
    st = srv.stats()
    res["passes"] = st["passes"]
    res["mean_slots_per_pass"] = round(st["slots_used"] / max(st["passes"], 1), 1)
    res["peak_admitted_GB"] = round(st["peak_admitted_bytes"] / 1e9, 2)
    res["memory_budget_GB"] = round((budget_gb << 30) / 1e9, 1)
    res["workspaces_created"] = st["workspaces_created"]
    res["workspaces_evicted"] = st["workspaces_evicted"]
    srv.destroy()
    for h in handles:
        h.release()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-22", choices=sorted(WORKLOADS))
    ap.add_argument("--sources", type=int, default=None, help="override the workload's source count")
    ap.add_argument("--batch-width", type=int, default=0,
                    help="fixed batch width (skips the autotuner)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in defaults instead of sp_autotune's choice")
    ap.add_argument("--per-source-sample", type=int, default=-1,
                    help="sources timed through the per-source path (-1 = all, 0 = skip)")
    ap.add_argument("--cpu-sample", type=int, default=16,
                    help="sources timed through the single-threaded CPU oracle (0 = skip)")
    ap.add_argument("--cpu-parallel-sample", type=int, default=4,
                    help="sources per host thread of the parallel oracle baseline (0 = skip)")
    ap.add_argument("--per-source-profile", type=int, default=32,
                    help="sources of the per-source path run with kernel timing (its roofline)")
    ap.add_argument("--per-source-legs", default="rmat-20:256",
                    help="per-source BC legs as workload:sources, comma-separated ('' = skip)")
    ap.add_argument("--road-batched", default="road-4096:64",
                    help="batched BC legs on road-like grids as workload:sources ('' = skip)")
    ap.add_argument("--serving-requests", type=int, default=400,
                    help="requests per phase of the serving workload (0 = skip)")
    ap.add_argument("--sssp-sources", default="rmat-22:16,road-4096:2",
                    help="SSSP legs as workload:sources, comma-separated ('' = skip)")
    ap.add_argument("--pagerank", default="rmat-22:20,road-4096:20,rmat-22-directed:20",
                    help="PageRank legs as workload:iterations, comma-separated ('' = skip)")
    ap.add_argument("--tc", default="rmat-22",
                    help="triangle-count workloads, comma-separated ('' = skip)")
    ap.add_argument("--tc-small-scale", type=int, default=16,
                    help="RMAT scale of the triangle-count CPU baseline and parity graph (0 = skip)")
    ap.add_argument("--only-tc", action="store_true",
                    help="run only the triangle-count legs and print their JSON object")
    ap.add_argument("--directed", default="rmat-22:64",
                    help="directed BC legs as workload:sources, comma-separated ('' = skip)")
    ap.add_argument("--only-directed", action="store_true",
                    help="run only the directed BC legs and print their JSON object")
    ap.add_argument("--only-sssp", action="store_true",
                    help="run only the SSSP legs and print their JSON object")
    ap.add_argument("--only-pagerank", action="store_true",
                    help="run only the PageRank legs and print their JSON object")
    ap.add_argument("--road-no-bitmap", action="store_true",
                    help="skip the road leg's timing of the other (bitmap) engine (profiling runs)")
    ap.add_argument("--only-road", action="store_true",
                    help="run only the road-like batched BC legs and print their JSON object")
    ap.add_argument("--only-serving", action="store_true",
                    help="run only the serving workload and print its JSON object")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="first run one elementwise kernel that reads and writes this many GiB "
                         "(a known-size kernel that calibrates hardware byte counters in a "
                         "profiler run)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(BC over a source set would shard sources across GPUs and all-reduce BC; "
              "not implemented here).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2305_03317_amd import graphs, sp
    if not os.path.exists(sp.LIB_PATH):
        from paper_2305_03317_amd import _build
        _build.build_all()

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_gib > 0:
        # one full-grid elementwise kernel that reads and writes copy_gib GiB
        # (int32 negation), found by name in the counter output
        nbytes = int(args.copy_gib * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    # Device copy bandwidth on this machine (a 2 GiB device-to-device copy, best of
    # 3): the streaming reference that the kernels' rates are also quoted against.
    # Skipped in counter-calibration runs, whose only large copy must be the
    # calibration copy above.
    cbuf = torch.empty(1 << 29, dtype=torch.int32, device="cuda").fill_(1)
    cdst = torch.empty_like(cbuf)
    copy_gbps = float("nan")
    for _ in range(0 if args.copy_gib > 0 else 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cdst.copy_(cbuf)
        e1.record()
        torch.cuda.synchronize()
        rate = 2 * cbuf.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        copy_gbps = rate if copy_gbps != copy_gbps else max(copy_gbps, rate)
    del cbuf, cdst
    if args.only_sssp or args.only_pagerank or args.only_tc or args.only_directed or args.only_road or \
            args.only_serving:
        legs = {}
        if args.only_serving:
            legs["serving"] = serving_benchmark(sp, torch, args.serving_requests)
        if args.only_road:
            legs["road_batched"] = {wl: road_batched_benchmark(sp, torch, wl, int(ns),
                                                               compare_bitmap=not args.road_no_bitmap) for wl, ns in
                                    (leg.split(":") for leg in filter(None, args.road_batched.split(",")))}
        if args.only_directed:
            legs["directed_bc"] = {wl: directed_benchmark(sp, torch, wl, int(ns)) for wl, ns in
                                   (leg.split(":") for leg in filter(None, args.directed.split(",")))}
        if args.only_tc:
            legs["triangles"] = {wl: tc_benchmark(sp, torch, wl, args.tc_small_scale)
                                 for wl in filter(None, args.tc.split(","))}
        if args.only_sssp:
            legs["sssp"] = {wl: sssp_benchmark(sp, torch, wl, int(ns)) for wl, ns in
                            (leg.split(":") for leg in filter(None, args.sssp_sources.split(",")))}
        if args.only_pagerank:
            legs["pagerank"] = {wl: pagerank_benchmark(sp, torch, wl, int(it)) for wl, it in
                                (leg.split(":") for leg in filter(None, args.pagerank.split(",")))}
        print(json.dumps(legs))
        return
    k = WORKLOADS[args.workload]

    t0 = time.perf_counter()
    rp, ci, src, spec = workload_graph(k) if args.sources is None else graphs.workload(k, args.sources)
    gen_s = time.perf_counter() - t0
    n = len(rp) - 1
    m = len(ci) // 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sp.sp_graph_upload(rp, ci)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    cfg = {"batch_width": args.batch_width} if args.batch_width else None
    tuned = None
    if cfg is None and not args.no_autotune:
        # sp_autotune times candidate configurations on (up to) 128 of the
        # sources and caches its choice on the graph; sp_bc_batch with no
        # config then uses it.  Not part of the timed region.
        t0 = time.perf_counter()
        tuned = sp.sp_autotune(g, src)
        tuned = {k: tuned[k] for k in ("batch_width", "block_size", "alpha", "beta", "chunk_levels")}
        tuned["tuning_s"] = round(time.perf_counter() - t0, 2)
        report = sp.sp_autotune_get_last_report()
        tuned["group_ms"] = round(report["group_ms"], 1)
        tuned["sample_sources"] = report["sample_sources"]
        tuned["repetitions"] = report["repetitions"]
        tuned["candidates"] = [dict(c["cfg"], ms_per_source=round(c["ms_per_source"], 4), accepted=c["accepted"])
                               for c in report["candidates"]]
        for c in tuned["candidates"]:
            c.pop("reserved", None)
        print("autotuned:", tuned, file=sys.stderr, flush=True)

    out = torch.empty(n, dtype=torch.float64, device="cuda")
    group_ms = tuned["group_ms"] if tuned else 0.0
    for _ in range(args.warmup):
        sp.sp_bc_batch(g, src, out_bc=out, config=cfg)
        group_ms += sp.sp_get_last_stats()["group_ms"]  # nonzero only on the call that computes it
    torch.cuda.synchronize()

    def run_steps(tag):
        return run_steps_n(args.steps, tag)

    def run_steps_n(k, tag):
        times, dev_ms, statuses = [], [], []
        for _ in range(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = sp.sp_bc_batch(g, src, out_bc=out, config=cfg)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            dev_ms.append(sp.sp_get_last_stats()["device_ms"])
            statuses.append(st)
            print("%s step %d: %.1f ms" % (tag, len(times), times[-1] * 1e3), file=sys.stderr, flush=True)
        return times, dev_ms, statuses

    # Timed region: the production configuration (forward level chunks
    # replayed from captured hipGraphs, no per-kernel events).
    times, dev_ms, statuses = run_steps("timed")
    stats = sp.sp_get_last_stats()
    step_s = float(np.mean(times))
    value = len(src) * m / step_s

    # Kernel-timed region: the same steps again with a HIP event pair around
    # every launch (on the library's stream); the level chunks are launched
    # directly here, since events cannot be read per kernel inside a replayed
    # graph.  Then one more step with the device work counters on (they add
    # reductions to the kernels, so they are not on while timing): the work is
    # the same every step, so the counts per launch apply to the timed launches.
    sp.sp_profile_read()  # discard anything earlier
    sp.sp_profile_enable(sp.SP_PROFILE_TIMES)
    ptimes, _, pstat = run_steps("kernel-timed")
    prof = sp.sp_profile_read()
    sp.sp_profile_enable(sp.SP_PROFILE_COUNTS)
    _, _, cstat = run_steps_n(1, "counted")
    counted = sp.sp_profile_read()
    sp.sp_profile_enable(False)
    statuses += pstat + cstat
    for kname, p in prof.items():  # counts per launch x timed launches
        c = counted.get(kname)
        scale = p["launches"] / c["launches"] if c and c["launches"] else 0.0
        for unit in ("items", "edges", "pairs", "item_slots"):
            p[unit] = (c[unit] * scale) if c else 0

    traffic_doc = load_traffic(spec["name"])
    # dominant kernel: most time inside the kernel-timed region
    dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"]) if prof else None
    roofline = None
    if dom:
        name, p = dom
        launches = max(p["launches"], 1)
        achieved = algorithmic_bytes(name, p) / (p["total_ms"] * 1e-3) / 1e9
        tr = traffic_doc["families"].get(name) if traffic_doc else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(tr["traffic_bytes_per_launch"]) if tr else None,
                    "kernel": name, "launches": p["launches"],
                    "avg_launch_ms": round(p["total_ms"] / launches, 4),
                    "algorithmic_bytes_per_launch": int(algorithmic_bytes(name, p) / launches),
                    "traffic_source": traffic_doc["path"] if tr else None}
        roofline["frac_of_measured_copy"] = round(achieved / copy_gbps, 4) if copy_gbps == copy_gbps else None
        if tr:
            roofline["traffic_GBps"] = round(tr["traffic_bytes_per_launch"] / (p["total_ms"] / launches * 1e-3) / 1e9, 1)
    kernels = {}
    for kname, p in prof.items():
        launches = max(p["launches"], 1)
        e = {"launches": p["launches"], "ms_per_step": round(p["total_ms"] / args.steps, 3),
             "avg_launch_ms": round(p["total_ms"] / launches, 4),
             "GBps_algorithmic": round(algorithmic_bytes(kname, p) / max(p["total_ms"], 1e-9) / 1e6, 1),
             "per_launch": {u: int(p[u] / launches) for u in ("items", "edges", "pairs", "item_slots") if p[u]}}
        tr = traffic_doc["families"].get(kname) if traffic_doc else None
        if tr:
            e["GBps_hbm_counters"] = round(tr["traffic_bytes_per_launch"] * p["launches"] / max(p["total_ms"], 1e-9) / 1e6, 1)
        kernels[kname] = e
    fwd = [prof[k] for k in FORWARD if k in prof]
    forward = None
    if fwd:
        f_ms = sum(p["total_ms"] for p in fwd)
        f_alg = sum(algorithmic_bytes(k, prof[k]) for k in FORWARD if k in prof)
        forward = {"ms_per_step": round(f_ms / args.steps, 2),
                   "GBps_algorithmic": round(f_alg / (f_ms * 1e-3) / 1e9, 1)}
        if traffic_doc and all(k in traffic_doc["families"] for k in FORWARD if k in prof):
            hw = sum(traffic_doc["families"][k]["traffic_bytes_per_launch"] * prof[k]["launches"]
                     for k in FORWARD if k in prof)
            forward["GBps_hbm_counters"] = round(hw / (f_ms * 1e-3) / 1e9, 1)
            forward["frac_of_peak_hbm_counters"] = round(hw / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    # per-source GPU path on a sample of the same sources
    per_source = None
    if args.per_source_sample != 0:
        ps_src = src if args.per_source_sample < 0 else src[:args.per_source_sample]
        sp.sp_bc(g, ps_src[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp.sp_bc(g, ps_src)
        torch.cuda.synchronize()
        ps_s = time.perf_counter() - t0
        per_source = {"sources": len(ps_src), "teps": len(ps_src) * m / ps_s,
                      "ms_per_source": ps_s * 1e3 / len(ps_src),
                      "block_size": sp.sp_get_last_stats()["block_size"]}
        if args.per_source_profile > 0:
            sample = ps_src[:args.per_source_profile]
            pk, proof = profile_kernels(sp, lambda: sp.sp_bc(g, sample), len(sample))
            attach_traffic(proof, "bc_per_source_" + spec["name"])
            per_source["roofline"] = proof
            per_source["roofline_sample"] = "first %d sources" % len(sample)
            per_source["kernels"] = pk

    # CPU oracle on a bounded sample (also a parity check at full size)
    cpu = None
    cpu_par = None
    parity = None
    if args.cpu_sample > 0:
        import oracle
        oracle.build()
        cs = src[:args.cpu_sample]
        t0 = time.perf_counter()
        ref = oracle.bc(rp, ci, cs)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": len(cs) * m / cpu_s, "unit": "TEPS", "cores": 1, "kind": "oracle",
               "sample": "first %d of the %d sources, single-threaded C oracle, %.1f s"
                         % (len(cs), len(src), cpu_s), "cpu_model": cpu_model()}
        # The same oracle function on P host threads over disjoint chunks of a
        # larger sample (ctypes releases the GIL during each call); per-thread
        # BC summed in chunk order.
        if args.cpu_parallel_sample > 0:
            import concurrent.futures as cf
            P = max(1, min(16, os.cpu_count() or 1))
            ps_src = src[:P * args.cpu_parallel_sample]
            chunks = [ps_src[i::P] for i in range(P)]
            t0 = time.perf_counter()
            with cf.ThreadPoolExecutor(P) as ex:
                list(ex.map(lambda c: oracle.bc(rp, ci, c), chunks))
            par_s = time.perf_counter() - t0
            cpu_par = {"value": len(ps_src) * m / par_s, "unit": "TEPS", "cores": P, "kind": "oracle",
                       "sample": "first %d sources, %d threads x %d sources, %.1f s"
                                 % (len(ps_src), P, args.cpu_parallel_sample, par_s)}
        got, _ = sp.sp_bc_batch(g, cs, config=cfg)
        got = got.cpu().numpy()
        parity = dict(sources=len(cs), **bc_parity(got, ref))

    g.release()
    del out
    per_source_legs = {wl: per_source_benchmark(sp, torch, wl, int(ns)) for wl, ns in
                       (leg.split(":") for leg in filter(None, args.per_source_legs.split(",")))}
    road = {wl: road_batched_benchmark(sp, torch, wl, int(ns), compare_bitmap=not args.road_no_bitmap)
            for wl, ns in
            (leg.split(":") for leg in filter(None, args.road_batched.split(",")))}
    sssp = {}
    for leg in filter(None, args.sssp_sources.split(",")):
        wl, ns = leg.split(":")
        sssp[wl] = sssp_benchmark(sp, torch, wl, int(ns))
    pagerank = {}
    for leg in filter(None, args.pagerank.split(",")):
        wl, it = leg.split(":")
        pagerank[wl] = pagerank_benchmark(sp, torch, wl, int(it))
    triangles = {wl: tc_benchmark(sp, torch, wl, args.tc_small_scale) for wl in filter(None, args.tc.split(","))}
    directed = {wl: directed_benchmark(sp, torch, wl, int(ns)) for wl, ns in
                (leg.split(":") for leg in filter(None, args.directed.split(",")))}
    serving = None
    if args.serving_requests > 0:
        serving = serving_benchmark(sp, torch, args.serving_requests)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "batched_over_per_source": (value / per_source["teps"]) if per_source else None,
        "forward_GBps_algorithmic": forward["GBps_algorithmic"] if forward else None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s batched BC" % spec["name"], "vertices": n, "undirected_edges": m,
                   "nnz": len(ci), "sources": len(src), "batch_width": stats["batch_width"],
                   "graph_seed": spec["graph_seed"], "source_seed": spec["source_seed"],
                   "levels_max": stats["max_levels"], "topdown_levels": stats["topdown_levels"],
                   "bottomup_levels": stats["bottomup_levels"], "block_size": stats["block_size"],
                   "alpha": stats["alpha"], "beta": stats["beta"], "chunk_levels": stats["chunk_levels"],
                   "autotuned": tuned},
        "device_ms_per_step": float(np.mean(dev_ms)),
        "ms_per_step_kernel_timed": float(np.mean(ptimes)) * 1e3,
        "graph_launches_per_step": stats["graph_launches"],
        "status": max(statuses),
        "upload_ms": upload_ms,
        "source_grouping_ms": round(group_ms, 1),
        "hbm_copy_GBps_measured": round(copy_gbps, 1) if copy_gbps == copy_gbps else None,
        "graph_build_s": gen_s,
        "roofline": roofline,
        "per_source_path": per_source,
        "per_source_legs": per_source_legs or None,
        "road_batched": road or None,
        "forward_pass": forward,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "cpu_baseline_parallel": cpu_par,
        "parity": parity,
        "serving": serving,
        "sssp": sssp or None,
        "pagerank": pagerank or None,
        "triangles": triangles or None,
        "directed_bc": directed or None,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
