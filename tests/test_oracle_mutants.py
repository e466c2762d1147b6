"""Plausible slips planted in a copy of the oracle must fail the pins.

Each mutant is a one-place edit of ``oracle/bc_oracle.c`` (a dropped term, a
swapped operand, a wrong index or sign, a missing skip or reset), compiled
on the CPU into a temporary library and run through a small battery drawn
from the pins in ``test_oracle_pins.py``: exhaustive path enumeration on
small graphs (dist, sigma and BC), including the path and cycle closed-form
graphs.
The unmodified source must pass the same battery.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import networkx as nx
import numpy as np
import pytest

from tests import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bc_oracle.c")

MUTANTS = {
    "drop_one_plus_delta": ("(1.0 + delta[w])", "(delta[w])"),
    "swap_sigma_ratio": ("(sigma[v] / sigma[w])", "(sigma[w] / sigma[v])"),
    "delta_wrong_index": ("(1.0 + delta[w])", "(1.0 + delta[v])"),
    "delta_wrong_sign": ("delta[v] = delta[v] + (sigma", "delta[v] = delta[v] - (sigma"),
    "source_not_skipped": ("if (v == src) continue;", ""),
    "sigma_not_summed": ("sigma[w] = sigma[w] + sigma[v];", "sigma[w] = sigma[v];"),
    "sigma_source_zero": ("sigma[src] = 1.0;", "sigma[src] = 2.0;"),
    "reverse_all_neighbours": ("if (dist[w] == dist[v] + 1)\n                delta",
                               "if (dist[w] != dist[v] - 1)\n                delta"),
    "forward_same_level_edges": ("if (dist[w] == dist[v] + 1)          /*",
                                 "if (dist[w] >= dist[v])          /*"),
    "halved": ("bc[v] = bc[v] + delta[v];", "bc[v] = bc[v] + 0.5 * delta[v];"),
    "bc_not_zeroed": ("for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;", ""),
    "delta_not_reset": ("        delta[v] = 0.0;\n", "\n"),
    "dist_step_two": ("dist[w] = dist[v] + 1;", "dist[w] = dist[v] + 2;"),
    "reverse_forward_order": ("for (int32_t i = tail - 1; i >= 0; --i) {",
                              "for (int32_t i = 0; i < tail; ++i) {"),
}


def compile_variant(tmp_path, name, text):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_bc.argtypes = [ctypes.c_int32, i32p, i32p, i32p, ctypes.c_int32, f64p, f64p]
    lib.oracle_source_detail.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32,
                                         i32p, f64p, f64p, i32p]
    return lib


def run_detail(lib, rp, ci, s):
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci if len(ci) else np.zeros(1, np.int32), np.int32)
    n = len(rp) - 1
    d = np.empty(n, np.int32)
    sig = np.empty(n)
    dl = np.empty(n)
    r = ctypes.c_int32(0)
    p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    assert lib.oracle_source_detail(n, p(rp, ctypes.c_int32), p(ci, ctypes.c_int32), s,
                                    p(d, ctypes.c_int32), p(sig, ctypes.c_double),
                                    p(dl, ctypes.c_double), ctypes.byref(r)) == 0
    return d, sig


def run_bc(lib, rp, ci, srcs):
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci if len(ci) else np.zeros(1, np.int32), np.int32)
    s = np.ascontiguousarray(srcs, np.int32)
    n = len(rp) - 1
    out = np.full(n, 1.0)        # not zero: a missing reset must show
    p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    rc = lib.oracle_bc(n, p(rp, ctypes.c_int32), p(ci, ctypes.c_int32), p(s, ctypes.c_int32),
                       len(s), p(out, ctypes.c_double), None)
    assert rc == 0
    return out


def battery_passes(lib, oracle_mod) -> bool:
    """True when the variant passes every check of the battery."""
    graphs = [nx.path_graph(7), nx.cycle_graph(6), nx.complete_bipartite_graph(2, 3),
              nx.gnm_random_graph(9, 16, seed=1), nx.gnm_random_graph(10, 20, seed=2)]
    graphs += [g for g in nx.graph_atlas_g()[100::97]]
    for G in graphs:
        n = G.number_of_nodes()
        e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
        rp, ci = oracle_mod.csr_from_edges(n, e[:, 0], e[:, 1])
        adj = brute.adjacency(rp, ci)
        d_ref, sig_ref, _ = brute.brute_source(adj, 0, layered=True)
        d, sig = run_detail(lib, rp, ci, 0)
        if list(d) != d_ref or [float(x) for x in sig_ref] != list(sig):
            return False
        for srcs in (list(range(n)), [n // 2], [0, n - 1]):
            ref = np.array([float(x) for x in brute.brute_bc(adj, srcs, layered=True)])
            got = run_bc(lib, rp, ci, srcs)
            if not np.all(np.abs(got - ref) <= 1e-12 * np.maximum(np.abs(ref), 1.0)):
                return False
    return True


def test_unmodified_passes(tmp_path, oracle_mod):
    assert battery_passes(compile_variant(tmp_path, "orig", open(SRC).read()), oracle_mod)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, oracle_mod, name):
    text = open(SRC).read()
    cut = text.index("#include")          # mutate code, not the header comment
    head, code = text[:cut], text[cut:]
    old, new = MUTANTS[name]
    assert code.count(old) >= 1, "mutation site vanished: " + name
    lib = compile_variant(tmp_path, name, head + code.replace(old, new, 1))
    assert not battery_passes(lib, oracle_mod)
