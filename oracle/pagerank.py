"""Reference (oracle) PageRank.  TEST INFRASTRUCTURE ONLY (see the package
docstring): plain numpy in float64, no blocking or reordering beyond the
paper's steps.

Paper: Appendix, Fig. "PR computation in StarPlat" (pull form, double
buffered).  Every vertex starts at 1/N.  One iteration computes, for every
vertex v,

    sum  = sum over in-neighbours u of v of  pr[u] / outdeg(u)
    val  = (1 - delta) / N + delta * sum
    diff = diff + |val - pr[v]|
    pr_next[v] = val

then replaces pr by pr_next and counts the iteration; it repeats while
diff > beta and fewer than max_iter iterations have run.

Reading: the paper accumulates the signed difference val - pr[v]; over a
graph without dangling vertices that sum is zero after the first iteration
(the iteration keeps total mass), so the loop would stop at once.  The
convergence test here uses the absolute difference (the L1 norm of the
change).  A vertex without out-edges passes nothing on: its term pr[u] /
outdeg(u) appears in no sum, so its mass leaves the system each iteration
(it is not redistributed; the formula sums over in-neighbours only).
"""
from __future__ import annotations

import numpy as np


def pagerank(row_ptr, col_idx, beta: float, delta: float, max_iter: int, iterations: int | None = None):
    """(pr float64[N], iterations run, diff of the last iteration).

    row_ptr/col_idx: CSR of out-edges (u -> col_idx[e] for e in row u).
    iterations: when given, run exactly that many iterations (no test).
    """
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    n = len(rp) - 1
    if n <= 0:
        return np.zeros(0), 0, 0.0
    outdeg = np.diff(rp)
    src_of_entry = np.repeat(np.arange(n), outdeg)
    pr = np.full(n, 1.0 / n)
    it = 0
    diff = 0.0
    while True:
        # pr[u] / outdeg(u) for every edge u -> v, added into v
        share = np.zeros(n)
        has = outdeg > 0
        share[has] = pr[has] / outdeg[has]
        s = np.bincount(ci, weights=share[src_of_entry], minlength=n)
        val = (1.0 - delta) / n + delta * s
        diff = float(np.sum(np.abs(val - pr)))
        pr = val
        it += 1
        if iterations is not None:
            if it >= iterations:
                break
        elif not (diff > beta and it < max_iter):
            break
    return pr, it, diff
