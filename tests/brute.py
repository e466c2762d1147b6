"""Brute-force betweenness centrality straight from its definition.

BC(v) = sum over sources s in S, over targets t != s, t != v, of
sigma_st(v) / sigma_st, where sigma_st counts shortest s-t paths and
sigma_st(v) those of them that pass through v.  Computed here by listing
paths explicitly and summing exact rationals, with no recursion over
predecessors, so it shares no step with the Brandes recursion the oracle and
the GPU library use.
"""
from __future__ import annotations

from collections import deque
from fractions import Fraction


def adjacency(row_ptr, col_idx):
    n = len(row_ptr) - 1
    return [list(int(x) for x in col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]


def simple_paths_from(adj, s):
    """Every simple path that starts at s (as tuples), by plain DFS."""
    out = []
    stack = [(s,)]
    while stack:
        p = stack.pop()
        out.append(p)
        last = p[-1]
        for w in adj[last]:
            if w not in p:
                stack.append(p + (w,))
    return out


def shortest_paths_by_enumeration(adj, s):
    """{t: list of shortest s-t paths}: all simple paths from s, keep the
    shortest per endpoint.  Exponential; for graphs of <= 8 vertices."""
    best = {}
    for p in simple_paths_from(adj, s):
        t = p[-1]
        if t not in best or len(p) < len(best[t][0]):
            best[t] = [p]
        elif len(p) == len(best[t][0]):
            best[t].append(p)
    return best


def bfs_dist(adj, s):
    n = len(adj)
    d = [-1] * n
    d[s] = 0
    q = deque([s])
    while q:
        u = q.popleft()
        for w in adj[u]:
            if d[w] < 0:
                d[w] = d[u] + 1
                q.append(w)
    return d


def shortest_paths_layered(adj, s):
    """{t: list of shortest s-t paths} by extending paths one hop at a time
    along edges that raise the BFS distance by one.  For graphs of <= ~14
    vertices (counts stay small)."""
    d = bfs_dist(adj, s)
    out = {s: [(s,)]}
    frontier = [(s,)]
    while frontier:
        nxt = []
        for p in frontier:
            u = p[-1]
            for w in adj[u]:
                if d[w] == d[u] + 1:
                    q = p + (w,)
                    out.setdefault(w, []).append(q)
                    nxt.append(q)
        frontier = nxt
    return out


def brute_source(adj, s, layered=False):
    """(dist list, sigma list of ints, delta list of Fractions) of source s."""
    n = len(adj)
    paths = shortest_paths_layered(adj, s) if layered else shortest_paths_by_enumeration(adj, s)
    dist = [-1] * n
    sigma = [0] * n
    delta = [Fraction(0)] * n
    for t, plist in paths.items():
        dist[t] = len(plist[0]) - 1
        sigma[t] = len(plist)
        if t == s:
            continue
        for p in plist:
            for v in p[1:-1]:
                delta[v] += Fraction(1, len(plist))
    return dist, sigma, delta


def brute_bc(adj, sources, layered=False):
    n = len(adj)
    bc = [Fraction(0)] * n
    for s in sources:
        _, _, delta = brute_source(adj, s, layered)
        for v in range(n):
            if v != s:
                bc[v] += delta[v]
    return bc


def sssp_invariants(rp, ci, w, s, d, inf=2**31 - 1):
    """Properties that make d the shortest-path distances from s, at any size
    (vectorised): d[s] = 0; no edge out of a reached vertex can lower its
    target; every reached vertex but s has a neighbour with d[u] + w = d[v]
    (so d[v] is the length of a real path, by induction on d); a reached
    vertex has only reached neighbours.  With positive weights these force d
    to equal the true distances: the first two bound d from above by
    induction along a shortest path, the third from below by induction on d
    (with zero weights a zero cycle could hold a too-small value up)."""
    import numpy as np
    n = len(rp) - 1
    d = np.asarray(d, np.int64)
    assert d[s] == 0, "source distance %d" % d[s]
    u = np.repeat(np.arange(n), np.diff(np.asarray(rp)))
    v = np.asarray(ci, np.int64)
    ww = np.asarray(w, np.int64)
    ru = d[u] != inf
    assert np.all(d[v][ru] != inf), "a reached vertex has an unreached neighbour"
    assert np.all(d[v][ru] <= d[u][ru] + ww[ru]), "an edge can still be relaxed"
    tight = ru & (d[u] + ww == d[v])
    has = np.zeros(n, bool)
    has[v[tight]] = True
    reached = d != inf
    reached[s] = False
    assert np.all(has[reached]), "a reached vertex has no tight predecessor"


def directed_csr(n, src, dst):
    """CSR of a simple directed graph (rows = out-edges, sorted, duplicates
    and self-loops dropped) from an edge list."""
    import numpy as np
    s = np.asarray(src, np.int64)
    d = np.asarray(dst, np.int64)
    keep = s != d
    key = np.unique(s[keep] * n + d[keep])
    s, d = key // n, key % n
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, s + 1, 1)
    return np.cumsum(rp).astype(np.int32), d.astype(np.int32)
