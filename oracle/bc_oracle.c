/*
 * Reference (oracle) implementation of betweenness centrality over a source
 * set.  TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke check and
 * the benchmark's CPU-baseline leg have a plain, slow, obviously correct answer
 * to compare the GPU library against.  No product code links or calls it, and
 * it shares no code, header or helper with the GPU library.
 *
 * What it computes (paper: Appendix, Fig. "BC computation in StarPlat", with
 * the traversal semantics of Section 2.3.2 "Parallelization and Iteration
 * Schemes"):
 *
 *   BC is zeroed once (attachNodeProperty(BC = 0)).  Then, for every source
 *   src of the source list, in list order:
 *     sigma := 0, delta := 0, sigma[src] := 1;
 *     a breadth-first traversal from src visits vertices level by level; for
 *       every visited v and every BFS-DAG child w of v (a neighbour one level
 *       further from src), sigma[w] := sigma[w] + sigma[v];
 *     a reverse traversal visits the same vertices in reverse level order,
 *       skipping src itself; for every visited v and every BFS-DAG child w of
 *       v, delta[v] := delta[v] + (sigma[v] / sigma[w]) * (1 + delta[w]);
 *       then BC[v] := BC[v] + delta[v].
 *
 * Section 2.3.2 states that inside the BFS/reverse constructs "neighbours"
 * means neighbours in the BFS DAG, not in the whole graph: for vertex v at
 * distance d, its DAG children are the adjacent w at distance d + 1.  Vertices
 * the traversal never reaches keep distance -1 (the unvisited sentinel the
 * generated BFS code of Section 3.5 uses), sigma 0 and delta 0.
 *
 * Readings taken where the paper is silent:
 *   - sigma, delta and BC are all binary64 (the paper declares BC and delta
 *     float, sigma double); every operation is a single IEEE-754 operation
 *     with round-to-nearest-even: this file must be compiled without
 *     floating-point contraction (-ffp-contract=off) and without fast-math.
 *   - The source list is a list: a vertex listed twice contributes twice.
 *   - Order: sigma[w] accumulates in the order its parents leave the FIFO
 *     queue; delta[v] accumulates over v's adjacency in CSR order; BC[v]
 *     accumulates in source-list order.
 *   - No halving for undirected graphs and no normalisation: every ordered
 *     (source, target) pair contributes, as the specification accumulates
 *     delta over every source.
 *
 * The graph is CSR: row_ptr[n + 1] offsets into col_idx[nnz], vertex ids in
 * [0, n).  An undirected graph is expected stored in both directions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Return codes. */
#define ORACLE_OK 0
#define ORACLE_BAD_ARG (-1)
#define ORACLE_NO_MEMORY (-2)

static int check_graph(int32_t n, const int32_t *row_ptr, const int32_t *col_idx)
{
    if (n < 0 || (n > 0 && (row_ptr == NULL))) return ORACLE_BAD_ARG;
    if (n == 0) return ORACLE_OK;
    if (row_ptr[0] != 0) return ORACLE_BAD_ARG;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORACLE_BAD_ARG;
    if (row_ptr[n] > 0 && col_idx == NULL) return ORACLE_BAD_ARG;
    for (int32_t e = 0; e < row_ptr[n]; ++e)
        if (col_idx[e] < 0 || col_idx[e] >= n) return ORACLE_BAD_ARG;
    return ORACLE_OK;
}

/*
 * One source: forward BFS with path counting, then the reverse sweep.
 * dist, sigma, delta: caller arrays of n entries, fully overwritten.
 * order: caller array of n entries; receives the vertices in the order the
 *   FIFO queue popped them (non-decreasing distance); *n_reached their count.
 * bc: nullable; when given, bc[v] += delta[v] for every reached v != src.
 */
int oracle_brandes_source(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          int32_t src, int32_t *dist, double *sigma, double *delta,
                          int32_t *order, int32_t *n_reached, double *bc)
{
    if (src < 0 || src >= n || !dist || !sigma || !delta || !order || !n_reached)
        return ORACLE_BAD_ARG;

    for (int32_t v = 0; v < n; ++v) {
        dist[v] = -1;
        sigma[v] = 0.0;
        delta[v] = 0.0;
    }
    dist[src] = 0;
    sigma[src] = 1.0;

    /* Forward: FIFO breadth-first traversal.  'order' doubles as the queue:
     * entries [head, tail) are discovered but not yet expanded. */
    int32_t head = 0, tail = 0;
    order[tail++] = src;
    while (head < tail) {
        int32_t v = order[head++];
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] < 0) {
                dist[w] = dist[v] + 1;
                order[tail++] = w;
            }
            if (dist[w] == dist[v] + 1)          /* w is a DAG child of v */
                sigma[w] = sigma[w] + sigma[v];
        }
    }
    *n_reached = tail;

    /* Reverse: vertices in reverse discovery order, which is non-increasing
     * distance, so every DAG child's delta is final before its parents read
     * it.  The source itself is skipped. */
    for (int32_t i = tail - 1; i >= 0; --i) {
        int32_t v = order[i];
        if (v == src) continue;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t w = col_idx[e];
            if (dist[w] == dist[v] + 1)
                delta[v] = delta[v] + (sigma[v] / sigma[w]) * (1.0 + delta[w]);
        }
        if (bc) bc[v] = bc[v] + delta[v];
    }
    return ORACLE_OK;
}

/*
 * BC over a source list: bc[n] is zeroed, then every source contributes in
 * list order.  Returns ORACLE_OK, or an error with bc untouched.
 * If sigma_max is non-null it receives the largest sigma seen in any source
 * (NaN/inf propagate), so callers can apply the overflow rule
 * "sigma > 1e300 or not finite".
 */
int oracle_bc(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              const int32_t *sources, int32_t n_sources, double *bc, double *sigma_max)
{
    int rc = check_graph(n, row_ptr, col_idx);
    if (rc != ORACLE_OK) return rc;
    if (n_sources < 0 || (n_sources > 0 && !sources) || (n > 0 && !bc)) return ORACLE_BAD_ARG;
    for (int32_t i = 0; i < n_sources; ++i)
        if (sources[i] < 0 || sources[i] >= n) return ORACLE_BAD_ARG;

    double smax = 0.0;
    if (n == 0) {
        if (sigma_max) *sigma_max = smax;
        return ORACLE_OK;
    }
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *sigma = (double *)malloc(sizeof(double) * (size_t)n);
    double *delta = (double *)malloc(sizeof(double) * (size_t)n);
    if (!dist || !order || !sigma || !delta) {
        free(dist); free(order); free(sigma); free(delta);
        return ORACLE_NO_MEMORY;
    }
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;

    for (int32_t i = 0; i < n_sources; ++i) {
        int32_t reached = 0;
        oracle_brandes_source(n, row_ptr, col_idx, sources[i], dist, sigma, delta,
                              order, &reached, bc);
        for (int32_t j = 0; j < reached; ++j) {
            double s = sigma[order[j]];
            if (!(s <= smax)) smax = s;      /* also captures NaN */
        }
    }
    if (sigma_max) *sigma_max = smax;
    free(dist); free(order); free(sigma); free(delta);
    return ORACLE_OK;
}

/* Per-source detail for parity tests: dist/sigma/delta of one source, plus
 * the number of reached vertices.  Arrays of n entries, overwritten. */
int oracle_source_detail(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t src, int32_t *dist, double *sigma, double *delta,
                         int32_t *n_reached)
{
    int rc = check_graph(n, row_ptr, col_idx);
    if (rc != ORACLE_OK) return rc;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!order) return ORACLE_NO_MEMORY;
    rc = oracle_brandes_source(n, row_ptr, col_idx, src, dist, sigma, delta, order,
                               n_reached, NULL);
    free(order);
    return rc;
}
