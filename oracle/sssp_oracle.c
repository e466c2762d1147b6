/*
 * Reference (oracle) single-source shortest paths on a weighted CSR graph.
 * TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg have a plain, slow, obviously correct answer
 * to compare the GPU library against.  No product code links or calls it, and
 * it shares no code, header or helper with the GPU library.
 *
 * What it computes (paper: Section 2.2, Fig. "SSSP computation in StarPlat",
 * and the pull form in the Appendix): dist[v] = the least total edge weight
 * of a path from src to v, with dist[src] = 0 and INT32_MAX for vertices no
 * path reaches (the paper initialises every distance to INT_MAX).  The paper
 * reaches it by repeated relaxation until no distance changes (a Bellman-Ford
 * variant); the result is the plain shortest-path distance, so this oracle
 * writes that definition out with Dijkstra's algorithm (weights must be
 * non-negative): a binary heap of (distance, vertex) pairs, stale pairs
 * skipped when popped, every edge of a settled vertex relaxed once.
 *
 * Distances are accumulated in 64 bits; a finite distance that does not fit
 * below INT32_MAX is reported as an error (code 3) rather than wrapped.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t d;
    int32_t v;
} item;

static void heap_push(item *h, int64_t *n, item x) {
    int64_t i = (*n)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= x.d) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = x;
}

static item heap_pop(item *h, int64_t *n) {
    item top = h[0];
    item last = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= *n) break;
        if (c + 1 < *n && h[c + 1].d < h[c].d) ++c;
        if (h[c].d >= last.d) break;
        h[i] = h[c];
        i = c;
    }
    h[i] = last;
    return top;
}

/* Returns 0, or 1 for a bad argument, 2 for a negative weight, 3 for a
 * distance that does not fit in int32, 4 for an allocation failure. */
int oracle_sssp(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *weight,
                int32_t src, int32_t *dist_out) {
    if (n <= 0 || src < 0 || src >= n || !row_ptr || !dist_out) return 1;
    const int64_t nnz = row_ptr[n];
    for (int64_t e = 0; e < nnz; ++e)
        if (weight[e] < 0) return 2;
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    char *done = (char *)calloc((size_t)n, 1);
    item *heap = (item *)malloc(sizeof(item) * (size_t)(nnz + 1));
    if (!dist || !done || !heap) {
        free(dist);
        free(done);
        free(heap);
        return 4;
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = INT64_MAX;
    int64_t hn = 0;
    dist[src] = 0;
    heap_push(heap, &hn, (item){0, src});
    while (hn > 0) {
        const item it = heap_pop(heap, &hn);
        const int32_t u = it.v;
        if (done[u] || it.d != dist[u]) continue; /* stale pair */
        done[u] = 1;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t w = col_idx[e];
            const int64_t nd = dist[u] + (int64_t)weight[e];
            if (nd < dist[w]) {
                dist[w] = nd;
                heap_push(heap, &hn, (item){nd, w});
            }
        }
    }
    int rc = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (dist[v] == INT64_MAX) {
            dist_out[v] = INT32_MAX;
        } else if (dist[v] >= INT32_MAX) {
            rc = 3;
            dist_out[v] = INT32_MAX;
        } else {
            dist_out[v] = (int32_t)dist[v];
        }
    }
    free(dist);
    free(done);
    free(heap);
    return rc;
}
