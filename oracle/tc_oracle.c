/*
 * Reference (oracle) triangle count of a simple undirected CSR graph.
 * TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg have a plain, slow, obviously correct answer
 * to compare the GPU library against.  No product code links or calls it, and
 * it shares no code, header or helper with the GPU library.
 *
 * What it computes (paper: Appendix, Fig. "TC computation in StarPlat"): the
 * number of triangles, each counted once.  The paper's node iterator visits
 * every vertex v, every neighbour u < v and every neighbour w > v, and counts
 * the pair when u and w are adjacent, so a triangle a < b < c is counted once,
 * at b.  That is the plain definition written here: for every vertex v, count
 * the pairs (u, w) of its neighbours with u < v < w that are adjacent, with
 * adjacency tested by binary search in u's sorted row (the paper's
 * is_an_edge on a sorted CSR).
 *
 * Rows must be sorted ascending and duplicate-free.
 */
#include <stdint.h>

static int is_an_edge(const int32_t *row_ptr, const int32_t *col_idx, int32_t u, int32_t w) {
    int64_t lo = row_ptr[u], hi = row_ptr[u + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == w) return 1;
        if (col_idx[mid] < w) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

/* Returns 0 and the count in *out, or 1 for a bad argument. */
int oracle_tc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int64_t *out) {
    if (n < 0 || !row_ptr || !out) return 1;
    int64_t count = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i) {
            const int32_t u = col_idx[i];
            if (u >= v) continue;
            for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
                const int32_t w = col_idx[j];
                if (w <= v) continue;
                count += is_an_edge(row_ptr, col_idx, u, w);
            }
        }
    *out = count;
    return 0;
}

/* Triangles through vertex v (each once): adjacent pairs among v's
 * neighbours.  The per-vertex counts sum to three times the total.
 * Returns 0 and the count in *out, or 1 for a bad argument. */
int oracle_tc_vertex(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t v, int64_t *out) {
    if (n < 0 || v < 0 || v >= n || !row_ptr || !out) return 1;
    int64_t count = 0;
    for (int64_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i)
        for (int64_t j = i + 1; j < row_ptr[v + 1]; ++j)
            count += is_an_edge(row_ptr, col_idx, col_idx[i], col_idx[j]);
    *out = count;
    return 0;
}

/* oracle_tc_vertex for every vertex: out[v] for v in [0, n). */
int oracle_tc_each(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int64_t *out) {
    if (n < 0 || !row_ptr || (n > 0 && !out)) return 1;
    for (int32_t v = 0; v < n; ++v)
        if (oracle_tc_vertex(n, row_ptr, col_idx, v, out + v) != 0) return 1;
    return 0;
}
