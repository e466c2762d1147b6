/*
 * sp.h — C ABI of the MI355X (gfx950) betweenness-centrality library
 * (libsp.so).
 *
 * The library computes Brandes betweenness centrality over a source list on
 * a simple, undirected, unweighted graph held as int32 CSR, on one AMD GPU,
 * single-source shortest paths once the graph is given edge weights,
 * PageRank and triangle counts.
 * The operation is the paper's computeBC (Appendix, Fig. "BC computation in
 * StarPlat"): BC is zeroed, then for every source a level-synchronous
 * breadth-first pass counts shortest paths (sigma[w] += sigma[v] over BFS-DAG
 * children, Section 2.3.2 "iterateInBFS") and a reverse level-order pass
 * accumulates delta[v] += (sigma[v] / sigma[w]) * (1 + delta[w]) over the same
 * DAG children and adds delta[v] to BC[v] for every v other than the source
 * ("iterateInReverse").  All arithmetic is IEEE binary64 (the paper declares
 * BC and delta float; this library keeps every quantity in double).  No
 * halving for undirected graphs and no normalisation: every ordered
 * (source, target) pair contributes.
 *
 * Conventions shared by every entry point
 *   - Return value: SP_OK (0); a negative SP_ERR_* code, in which case no
 *     output buffer has been written; or a positive SP_WARN_* bit mask, in
 *     which case outputs were written and carry the stated caveat.
 *   - Streams: `sp_stream` is a hipStream_t (NULL = the default stream).
 *     Work is ordered on that stream.  Entry points that return a warning
 *     synchronise the stream before returning, so the status is final.
 *   - Host pointers are read before the call returns and never retained.
 *   - Device output buffers are caller-owned and must be valid device
 *     memory (e.g. a torch CUDA tensor on the current device).
 *   - The source list is a list, not a set: a vertex listed twice
 *     contributes twice.
 *   - Thread safety: distinct sp_graph handles are independent; one handle
 *     may be used by several threads when each passes its own stream (each
 *     call takes its own workspace).  A server (sp_server) is thread-safe.
 *   - Every entry point is exception-free and never aborts the process;
 *     sp_last_error() returns a thread-local human-readable detail of the
 *     last failure on the calling thread.
 */
#ifndef SP_H
#define SP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sp_status;

#define SP_OK 0
/* Warning bit: some path count sigma exceeded 1e300 or was not finite; BC
 * may hold inf or NaN (the paper's sigma is double and overflows the same
 * way).  Outputs are written. */
#define SP_WARN_SIGMA_LARGE 1
#define SP_ERR_INVALID_ARGUMENT (-1) /* null pointer, bad size, source out of range, malformed CSR */
#define SP_ERR_OUT_OF_MEMORY (-2)    /* device or host allocation failed, or memory budget exceeded */
#define SP_ERR_DEVICE (-3)           /* HIP runtime error; detail in sp_last_error() */
#define SP_ERR_NOT_SUPPORTED (-4)    /* no usable gfx950 device, or a request outside documented limits */
#define SP_ERR_REJECTED (-5)         /* serving: request can never fit, or the server is shutting down */
#define SP_ERR_TIMEOUT (-6)          /* serving: wait timed out (request still in flight) */
#define SP_ERR_CANCELLED (-7)        /* serving: request was cancelled before it ran */

/* Upload flags. */
#define SP_PTR_DEVICE 1u /* row_ptr/col_idx are device pointers (else host) */
#define SP_VALIDATE 2u   /* check: offsets monotone, ids in range, rows sorted and
                            duplicate-free, no self-loops, symmetric */

typedef struct sp_graph_s *sp_graph;
typedef struct sp_server_s *sp_server;
typedef struct sp_request_s *sp_request;
typedef void *sp_stream;

/* ------------------------------------------------------------------------
 * Status and diagnostics
 * ------------------------------------------------------------------------ */

/* Static text of a status code. Never NULL. */
const char *sp_status_string(sp_status s);

/* Thread-local detail of the last failure on this thread ("" if none).
 * Valid until the next library call on this thread. */
const char *sp_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t sp_version(void);

/* First 8 bytes (little-endian) of the SHA-256 of this header file as the
 * library was built from it.  A binding compares it with the header it was
 * written against before exchanging any struct. */
uint64_t sp_header_hash(void);

/* ------------------------------------------------------------------------
 * Graphs (paper Section 2.3.1 "Data Types" and Section 3.1 "Graph
 * Representation and Storage": CSR offsets + neighbour lists, copied to the
 * device once; the graph is static)
 * ------------------------------------------------------------------------ */

/* Copy a CSR graph into library-owned device memory on the current device.
 *   n_vertices  V >= 0; vertex ids are [0, V).  V < 2^31 - 1.
 *   nnz         number of CSR entries (2x the undirected edges), 0 <= nnz < 2^31.
 *   row_ptr     V + 1 int32 offsets, row_ptr[0] = 0, row_ptr[V] = nnz.
 *   col_idx     nnz int32 neighbour ids.  An undirected edge {u, w} must
 *               appear as w in row u and as u in row w.
 *   flags       SP_PTR_DEVICE if the two arrays are device pointers (else
 *               host); SP_VALIDATE to check the CSR (on the host, copying
 *               device arrays back first) before uploading.
 *   s           stream used for the copies; the call synchronises it.
 *   out         receives the handle (unchanged on error).
 * Every upload checks on the device that offsets are monotone within
 * [0, nnz] and ids lie in [0, V) (SP_ERR_INVALID_ARGUMENT otherwise), so no
 * kernel can index outside the arrays.  Without SP_VALIDATE the remaining
 * properties (sorted, duplicate-free, loop-free, symmetric rows) are trusted;
 * a CSR that breaks them gives BC of the directed multigraph it encodes. */
sp_status sp_graph_upload(int32_t n_vertices, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, uint32_t flags, sp_stream s, sp_graph *out);

/* Copy a directed graph: row u of the CSR lists the heads of u's out-edges.
 * Same arguments as sp_graph_upload; the offsets and ids are always checked
 * on the host (the reversed rows of incoming edges are built there and
 * uploaded too), SP_VALIDATE adds sorted, duplicate-free rows without
 * self-loops.  Betweenness centrality then follows edge directions (paper
 * Section 2.3.1: the graph type offers neighbors and nodes_to; Brandes on a
 * directed graph counts shortest directed paths).  Both BC paths read
 * parents from the incoming rows and children from the outgoing ones:
 * discovery walks outgoing rows top-down and incoming rows bottom-up, path
 * counts pull over incoming rows (long ones chunked, listed per level),
 * dependencies over outgoing rows.  sp_bc, sp_bc_batch, sp_bfs_levels,
 * sp_batch_levels, sp_autotune and the server accept directed graphs, and
 * so does sp_pagerank (gathering over the reversed rows); edge weights /
 * SSSP and triangle counting need an undirected graph and return
 * SP_ERR_NOT_SUPPORTED. */
sp_status sp_graph_upload_directed(int32_t n_vertices, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, uint32_t flags, sp_stream s, sp_graph *out);

/* Free the graph's device memory.  The caller must ensure no call using the
 * graph is still running.  NULL is accepted (no-op). */
sp_status sp_graph_release(sp_graph g);

/* Sizes of an uploaded graph.  Any output pointer may be NULL. */
sp_status sp_graph_info(sp_graph g, int32_t *n_vertices, int64_t *nnz, size_t *device_bytes);

/* ------------------------------------------------------------------------
 * Betweenness centrality
 * ------------------------------------------------------------------------ */

/* Tuning of the batched path.  Zero in a field means "choose automatically"
 * (autotuned value cached per graph, else the built-in default). */
typedef struct sp_batch_config {
    int32_t batch_width;  /* sources per multi-source pass, 1..64 */
    int32_t block_size;   /* threads per workgroup: 128, 256 or 512 */
    double alpha;         /* bottom-up when frontier edges * alpha > unsettled edges */
    double beta;          /* back to top-down when frontier vertices * beta < V */
    int32_t chunk_levels; /* k > 0: the batched path captures k levels (rounded up
                             to even) in one hipGraph and replays it, checking the
                             device "done" flag on the host after each replay;
                             k < 0: |k| levels per check, launched directly (no
                             capture).  |k| <= 65536.  (Bitmap engine only.) */
    int32_t engine;       /* SP_ENGINE_* below; 0 = SP_ENGINE_AUTO */
    int32_t reserved[2];  /* must be zero */
} sp_batch_config;

/* How a batch runs:
 *   SP_ENGINE_BITMAP  one multi-source pass: a 64-bit source bitmap per vertex,
 *                     all slots advancing level by level together, each level
 *                     a few grid-wide kernels (levels captured in hipGraphs).
 *   SP_ENGINE_BLOCKS  one workgroup per source, the whole pass (forward and
 *                     reverse levels) inside one launch with the workgroup
 *                     barrier between levels; per-slot level/value records
 *                     and delta source-major (32 bytes per vertex and slot),
 *                     rows copied once to a fixed width of 4 or 8 when every
 *                     row fits.  For graphs of many small levels.
 *   SP_ENGINE_AUTO    SP_ENGINE_BLOCKS on road-like graphs (no vertex with
 *                     more than 8 neighbours in or out), else SP_ENGINE_BITMAP.
 * Both compute the same per-source quantities; the bitmap engine, and the
 * blocks engine over fixed-width rows, regroup the reverse sum (sigma(v)
 * times the sum of (1 + delta(w)) / sigma(w)); the blocks engine over longer
 * rows sums (sigma(v) / sigma(w)) (1 + delta(w)) as written, so their BC
 * differs by rounding only. */
#define SP_ENGINE_AUTO 0
#define SP_ENGINE_BITMAP 1
#define SP_ENGINE_BLOCKS 2

/* Counters of the last sp_bc / sp_bc_batch call on the calling thread. */
typedef struct sp_stats {
    int32_t n_sources;
    int32_t n_passes;        /* BFS passes: sources for sp_bc, batches for sp_bc_batch */
    int32_t max_levels;      /* deepest BFS (levels incl. level 0) over all passes */
    int32_t sigma_flagged;   /* passes in which some sigma > 1e300 or not finite */
    int64_t levels_total;    /* sum of levels over passes */
    int64_t topdown_levels;  /* levels expanded top-down (frontier push) */
    int64_t bottomup_levels; /* levels expanded bottom-up (unvisited pull) */
    int64_t reached_total;   /* sum over sources of reached vertices */
    double sigma_max;        /* largest path count seen */
    double device_ms;        /* time from the first init kernel to BC ready (HIP events) */
    int32_t batch_width;     /* configuration actually used */
    int32_t block_size;
    double alpha, beta;
    int32_t chunk_levels;
    int32_t graph_launches;  /* hipGraph launches used */
    double group_ms;         /* sp_bc_batch: host time spent in this call computing the
                                graph's source-grouping keys (0 once cached; not part
                                of device_ms) */
    int32_t engine;          /* sp_bc_batch: SP_ENGINE_BITMAP or SP_ENGINE_BLOCKS (0 for sp_bc) */
} sp_stats;

/* Per-source path: one BFS pass per source, sources in list order.
 *   sources    host array of n_sources vertex ids in [0, V).
 *   out_bc     device array of V doubles: zeroed, then receives BC.
 * Returns SP_OK or SP_WARN_SIGMA_LARGE (synchronises the stream). */
sp_status sp_bc(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc,
                sp_stream s);

/* Batched path: sources are cut into batches of cfg->batch_width; each batch
 * runs as one multi-source BFS with a 64-bit source bitmap per vertex (one bit
 * per batch slot), all slots advancing level by level together.  Same inputs,
 * outputs and status as sp_bc; cfg may be NULL.  When the sources need more
 * than one batch they are first grouped so that a batch holds sources with
 * similar BFS depth profiles (fewer distinct levels per vertex, so less work):
 * ordered by their summed distance to the four highest-degree vertices
 * (computed once per graph, on the first such call), then by descending
 * degree, then by list position.  BC is accumulated per vertex batch by batch
 * in that order, slot order within a batch; the order is a function of the
 * graph and the source list alone, so results are reproducible. */
sp_status sp_bc_batch(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc,
                      const sp_batch_config *cfg, sp_stream s);

/* sp_bc for callers that cannot allocate device memory while they run (tight
 * serving loops, harnesses that forbid hipMalloc).  The same per-source
 * computation and kernels, so bit-identical results, with the whole
 * workspace (distances, path counts, dependencies, queue, level offsets, hub
 * lists, control block: about 40 bytes per vertex plus a few dozen per vertex
 * of degree > 256) carved from one fixed 64 MiB device array that the
 * library holds on every GPU it runs on until the process ends.  Calls no
 * device or pinned allocation routine.  Not capturable in a HIP graph (it
 * reads level counts back to the host).  Same arguments, outputs and status
 * as sp_bc, plus:
 *   SP_ERR_INVALID_ARGUMENT  the graph's workspace exceeds 64 MiB (roughly
 *                            V > 1.6M vertices): use sp_bc; nothing written.
 *   SP_ERR_NOT_SUPPORTED     kernel profiling is on (it creates events).
 * Calls on one GPU share that GPU's array: they are serialised on the host
 * (each holds the GPU's lock until its stream has synchronised), so calls on
 * different streams of one GPU never overlap.  The array keeps the last
 * call's contents; every value a call reads is written by that call first. */
sp_status sp_bc_noalloc(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc,
                        sp_stream s);

/* Counters of the last sp_bc / sp_bc_batch call on this thread. */
sp_status sp_get_last_stats(sp_stats *out);

/* Forward pass of one source through the per-source path:
 *   out_dist   device int32[V]: BFS distance, -1 where unreached.
 *   out_sigma  device double[V] (nullable): shortest-path counts, 0 where unreached.
 *   out_delta  device double[V] (nullable): when given, the reverse pass runs too
 *              and delta is written (0 at the source and where unreached). */
sp_status sp_bfs_levels(sp_graph g, int32_t source, int32_t *out_dist, double *out_sigma,
                        double *out_delta, sp_stream s);

/* One multi-source pass (at most 64 sources) through the batched path,
 * exposing per-source results, source-major: entry [i * V + v] belongs to
 * sources[i].  Any output may be NULL except out_dist. Used to check that the
 * batched path reaches the same distances and counts as the per-source one. */
sp_status sp_batch_levels(sp_graph g, const int32_t *sources, int32_t n_sources,
                          int32_t *out_dist, double *out_sigma, double *out_delta,
                          const sp_batch_config *cfg, sp_stream s);

/* Device workspace the batched path allocates for one pass of `batch_width`
 * slots on this graph (bytes). */
sp_status sp_bc_workspace_bytes(sp_graph g, int32_t batch_width, size_t *bytes);

/* Autotuner: times candidate configurations of the batched path and writes
 * the fastest to *out.  The sample is up to 128 consecutive sources of
 * `sources` in the order sp_bc_batch would batch them (grouped, see above),
 * taken from the middle of that order, so candidates run the batches
 * production runs.  The engine is the graph's SP_ENGINE_AUTO choice (not
 * searched).  Search: coordinate descent from the built-in defaults (width
 * 64, block 512, alpha 15, beta 24, chunk_levels 8), one field at a time:
 * block {256, 128}, width {32, 48}, alpha {4, 60} and beta {8, 96} (graphs
 * with a vertex of degree > 8 only), chunk_levels {16, 32}; for the blocks
 * engine from block 1024, width 64: block {512, 256}, width {32, 48}.  Each
 * candidate runs the sample once untimed, then twice timed (HIP events); its
 * score is the faster of the two, per source, and it replaces the running
 * best only when 2% faster.  The choice is kept on the graph (used whenever
 * a later call passes a zero field, by sp_bc for the block size) and in a
 * process-wide cache keyed by the graph's fingerprint (sp_graph_fingerprint):
 * a graph whose fingerprint is cached is not timed again, and an upload of a
 * graph with a cached fingerprint starts with that configuration.  When the
 * environment variable SP_TUNE_CACHE names a file, the cache is read from it
 * on first use and every new choice is appended to it (one line per graph:
 * fingerprint in hex, width, block, alpha, beta, chunk_levels).  Output
 * buffers are not touched.  Synchronises the stream. */
sp_status sp_autotune(sp_graph g, const int32_t *sources, int32_t n_sources,
                      sp_batch_config *out, sp_stream s);

/* One configuration timed by the last sp_autotune call on this thread. */
typedef struct sp_tune_candidate {
    sp_batch_config cfg;
    double ms_per_source;   /* the faster of the two timed repetitions, per source */
    int32_t accepted;       /* 1: became the running best when timed */
    int32_t reserved;
} sp_tune_candidate;

#define SP_TUNE_MAX_CANDIDATES 16

/* Report of the last sp_autotune call on this thread. */
typedef struct sp_tune_report {
    uint64_t fingerprint;
    int32_t from_cache;      /* 1: the configuration came from the cache; nothing was timed */
    int32_t sample_sources;  /* sources in the timed sample */
    int32_t repetitions;     /* timed repetitions per candidate */
    int32_t n_candidates;    /* entries of cand[] filled, in the order timed */
    double tuning_ms;        /* host time of the whole call, grouping keys included */
    double group_ms;         /* of which computing the source-grouping keys */
    sp_batch_config chosen;
    sp_tune_candidate cand[SP_TUNE_MAX_CANDIDATES];
} sp_tune_report;
sp_status sp_autotune_get_last_report(sp_tune_report *out);

/* 64-bit fingerprint of an uploaded graph: a hash of V, nnz, whether it is
 * directed, the maximum degree, the sum of squared degrees and the
 * histogram of degrees by power of two (in-degrees too for a directed
 * graph).  Graphs with equal fingerprints share a cached tuning. */
sp_status sp_graph_fingerprint(sp_graph g, uint64_t *out);

/* Set the graph's tuned configuration (as if sp_autotune had chosen it; for
 * example one saved by an earlier process), or clear it with NULL.  Fields
 * are checked as for sp_bc_batch; zero fields keep their built-in defaults.
 * Does not touch the fingerprint cache. */
sp_status sp_graph_set_tuned(sp_graph g, const sp_batch_config *cfg);

/* Empty the process-wide tuning cache (the SP_TUNE_CACHE file is kept). */
sp_status sp_tune_cache_clear(void);

/* ------------------------------------------------------------------------
 * Single-source shortest paths on a weighted graph (paper Section 2.2,
 * Fig. "SSSP computation in StarPlat"; the pull form in the Appendix)
 *
 * dist[v] is the least total weight of a path from the source to v
 * (dist[source] = 0; INT32_MAX where no path reaches v).  The paper computes
 * it by rounds of relaxation: every vertex whose distance dropped in the last
 * round offers dist + weight to its neighbours through an atomic Min (push),
 * or every vertex takes the Min over such neighbours (pull), until a round
 * lowers nothing.  The library runs those rounds on the device, choosing the
 * direction per round; the result is the shortest-path distance, exact in
 * int32 whatever the direction or scheduling.
 * ------------------------------------------------------------------------ */

/* Attach edge weights to an uploaded graph (replacing earlier ones).
 *   weights  nnz int32 values aligned with the graph's col_idx: weights[e] is
 *            the weight of CSR entry e.  Each must lie in [0, 2^31 - 2].  The
 *            two entries of an undirected edge must carry the same weight
 *            (pull rounds read a vertex's own row as its incoming edges).
 *   flags    SP_PTR_DEVICE if `weights` is a device pointer (else host);
 *            SP_VALIDATE to check on the host that the weights are symmetric.
 *   s        stream used for the copies; the call synchronises it.
 * The range of every weight is always checked (SP_ERR_INVALID_ARGUMENT).
 * Without SP_VALIDATE symmetry is trusted; asymmetric weights give distances
 * that depend on the direction chosen per round.  No sp_sssp call on the
 * graph may be running.  Adds 8 bytes per CSR entry of device memory (the
 * adjacency packed with its weights) plus 16 bytes per vertex of degree
 * above 256. */
sp_status sp_graph_set_weights(sp_graph g, const int32_t *weights, uint32_t flags, sp_stream s);

/* Direction of the relaxation rounds. */
#define SP_SSSP_AUTO 0 /* per round: pull when the frontier's adjacency entries
                          times alpha exceed the graph's (never on graphs whose
                          rows all hold at most 8 entries, nor with alpha <= 1) */
#define SP_SSSP_PUSH 1 /* every round pushes */
#define SP_SSSP_PULL 2 /* every round pulls */

typedef struct sp_sssp_config {
    int32_t direction;    /* SP_SSSP_AUTO, SP_SSSP_PUSH or SP_SSSP_PULL */
    int32_t block_size;   /* threads per workgroup: 128, 256 or 512 (0 = 256) */
    double alpha;         /* automatic direction threshold, >= 0 (0 = 1.0: push only;
                             measured on RMAT graphs, a pull round costs about as
                             much as the push round it replaces, or more) */
    int32_t chunk_rounds; /* k > 0: rounds are captured k at a time (rounded up to
                             even) in a hipGraph and replayed, checking the device
                             "done" flag after each replay; k < 0: |k| rounds per
                             check launched directly; 0 = 8.  |k| <= 65536. */
    int32_t max_blocks;   /* workgroups per round kernel, >= 0 (0 = automatic) */
    int32_t local_hops;   /* push rounds: a workgroup also follows its own lowerings for
                             this many more hops inside the round (a power of two up
                             to 128; -1 = none; 0 = automatic: 32 on graphs whose rows
                             all hold at most 8 entries, else none).  The distances do
                             not change. */
    int32_t reserved[1];  /* must be zero */
} sp_sssp_config;

typedef struct sp_sssp_stats {
    int32_t rounds;         /* relaxation rounds run, the last one lowering nothing */
    int32_t push_rounds;
    int32_t pull_rounds;
    int32_t reached;        /* vertices with a finite distance */
    double device_ms;       /* HIP-event time from the first kernel to distances ready */
    int32_t graph_launches; /* hipGraph launches used */
    int32_t block_size;     /* configuration actually used */
    double alpha;
    int32_t direction;
    int32_t chunk_rounds;
    int32_t local_hops;
} sp_sssp_stats;

/* Distances from `source` to every vertex.
 *   out_dist  device int32[V]: receives the distances (INT32_MAX where
 *             unreached).  Written only when the call succeeds.
 *   cfg       may be NULL (all defaults).
 * Requires weights (sp_graph_set_weights), else SP_ERR_INVALID_ARGUMENT.
 * A reachable vertex whose distance is INT32_MAX or more makes the call fail
 * with SP_ERR_NOT_SUPPORTED (the distances do not fit in int32); longer
 * detours that are not shortest paths do not.  Synchronises the stream. */
sp_status sp_sssp(sp_graph g, int32_t source, int32_t *out_dist, const sp_sssp_config *cfg,
                  sp_stream s);

/* Counters of the last sp_sssp call on the calling thread. */
sp_status sp_sssp_get_last_stats(sp_sssp_stats *out);

/* ------------------------------------------------------------------------
 * PageRank (paper Appendix, Fig. "PR computation in StarPlat": pull form,
 * double buffered)
 *
 * Every vertex starts at 1/N.  Each iteration computes, from the previous
 * iteration's values,
 *     pr'[v] = (1 - delta) / N + delta * sum over in-neighbours u of pr[u] / outdeg(u)
 * and the run stops after the first iteration whose sum over vertices of
 * |pr'[v] - pr[v]| is at most beta, or after max_iter iterations (at least
 * one runs).  The paper writes the signed difference; its sum is zero on a
 * graph without isolated vertices (the iteration keeps total mass), which
 * would stop the loop at once, so the absolute difference is used.  On an
 * undirected graph a vertex's in-neighbours are its row and outdeg its
 * degree; on a directed one (sp_graph_upload_directed) the in-neighbours are
 * its row of the reversed graph (the paper's nodes_to) and outdeg the length
 * of its outgoing row.  A vertex without outgoing edges passes nothing on:
 * its mass leaves the system (not redistributed).  All arithmetic is
 * binary64; each vertex's sum is taken in an order fixed by its row, so
 * results are reproducible.
 * ------------------------------------------------------------------------ */

typedef struct sp_pagerank_config {
    int32_t block_size;  /* 128, 256 or 512 (0 = 256) */
    int32_t chunk_iters; /* k > 0: iterations captured k at a time (rounded up to
                            even) in a hipGraph, the device "done" flag checked
                            after each replay; k < 0: |k| per check, launched
                            directly; 0 = 8.  |k| <= 65536. */
    int32_t reserved[4]; /* must be zero */
} sp_pagerank_config;

typedef struct sp_pagerank_stats {
    int32_t iterations;     /* iterations run */
    int32_t graph_launches; /* hipGraph launches used */
    double diff;            /* sum of |change| in the last iteration (accurate to
                               about 1e-15: block sums are added in fixed point) */
    double device_ms;       /* HIP-event time of the call's device work */
} sp_pagerank_stats;

/* PageRank of every vertex.
 *   beta      stopping threshold on the summed |change|, >= 0
 *   delta     damping factor in [0, 1]
 *   max_iter  >= 1
 *   out_pr    device double[V]: receives the values of the last iteration.
 *   cfg       may be NULL.
 * Synchronises the stream. */
sp_status sp_pagerank(sp_graph g, double beta, double delta, int32_t max_iter, double *out_pr,
                      const sp_pagerank_config *cfg, sp_stream s);

/* Counters of the last sp_pagerank call on the calling thread. */
sp_status sp_pagerank_get_last_stats(sp_pagerank_stats *out);

/* ------------------------------------------------------------------------
 * Triangle counting (paper Appendix, Fig. "TC computation in StarPlat")
 *
 * The number of triangles of the graph, each counted once: the count the
 * paper's node iterator produces (for every vertex v, the adjacent pairs
 * (u, w) of neighbours with u < v < w).  The library counts every triangle
 * once at its lowest edge under the (degree, id) order, which bounds the
 * work by O(m^1.5); the number is the same.  The graph must be simple and
 * undirected (each edge stored in both rows once, no self-loops), else
 * SP_ERR_INVALID_ARGUMENT.  The oriented rows (8 bytes per undirected edge +
 * 4 per vertex) are built on the first call and kept with the graph.
 * ------------------------------------------------------------------------ */

typedef struct sp_tc_stats {
    int64_t triangles;
    int64_t oriented_edges; /* entries of the oriented rows (undirected edges) */
    double build_ms;        /* orienting the rows (0 when they were already built) */
    double count_ms;        /* the counting kernel (HIP events) */
} sp_tc_stats;

/*   out_count       host: receives the number of triangles.
 *   out_per_vertex  device uint64[V] (nullable): triangles through each vertex
 *                   (they sum to three times the count).
 * Synchronises the stream. */
sp_status sp_triangle_count(sp_graph g, int64_t *out_count, uint64_t *out_per_vertex, sp_stream s);

/* Counters of the last sp_triangle_count call on the calling thread. */
sp_status sp_tc_get_last_stats(sp_tc_stats *out);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support)
 * ------------------------------------------------------------------------ */

/* Per kernel family: launches, HIP-event time, and the work it did. */
typedef struct sp_kernel_profile {
    char name[32];      /* kernel family, e.g. "ms_delta" */
    int64_t launches;   /* launches while profiling was on (either bit) */
    double total_ms;    /* sum over launches of the time between HIP events recorded
                           on the launch stream immediately before and after it
                           (0 unless SP_PROFILE_TIMES) */
    int64_t items;      /* vertices (per-source path) or (vertex, level) entries (batched) */
    int64_t edges;      /* adjacency entries scanned */
    int64_t pairs;      /* DAG edges accumulated (per-source) or (slot, DAG edge) pairs (batched) */
    int64_t item_slots; /* batched: sum over entries of their slot count; per-source: = items */
} sp_kernel_profile;

/* What sp_profile_enable turns on for all later launches of this process
 * (0 = off, the default).  Either one makes the batched path launch its
 * level kernels directly instead of replaying captured graphs. */
#define SP_PROFILE_TIMES 1  /* a HIP event pair around every launch (total_ms) */
#define SP_PROFILE_COUNTS 2 /* device work counters (items, edges, pairs, item_slots); they
                               add reductions to the kernels, so time and count in
                               separate runs when the times matter */
sp_status sp_profile_enable(int32_t what); /* SP_ERR_INVALID_ARGUMENT on unknown bits */

/* Synchronise every stream used, write up to `cap` families with at least one
 * launch into out[], their count into *n_out, and reset the totals. */
sp_status sp_profile_read(sp_kernel_profile *out, int32_t cap, int32_t *n_out);

/* ------------------------------------------------------------------------
 * Serving: continuous batching over several resident graphs
 * ------------------------------------------------------------------------ */

typedef struct sp_server_config {
    size_t memory_budget;  /* device bytes the server may hold for workspaces (0 = 25% of free) */
    int32_t max_batch;     /* slots per multi-source pass, 1..64 (0 = 64) */
    int32_t n_streams;     /* concurrent passes on the device, 1..8 (0 = 4) */
    int32_t reserved[4];   /* must be zero */
} sp_server_config;

typedef struct sp_server_stats {
    int64_t submitted, completed, failed, cancelled, rejected;
    int64_t passes;          /* multi-source passes run */
    int64_t slots_used;      /* sum over passes of filled slots */
    int64_t edges_traversed; /* sum over completed sources of undirected edge count */
    size_t admitted_bytes;   /* workspace bytes currently held */
    size_t peak_admitted_bytes;
    int32_t queue_depth;     /* sources waiting */
    int32_t in_flight;       /* passes on the device */
    int64_t workspaces_created;  /* pass workspaces allocated */
    int64_t workspaces_evicted;  /* idle workspaces freed to admit another graph's */
} sp_server_stats;

/* Start a server: n_streams worker threads, each with its own HIP stream (on
 * the device current at creation), pack queued sources of each graph into
 * multi-source passes and run them.  Workspaces and chunk buffers are
 * admitted against memory_budget. */
sp_status sp_server_create(const sp_server_config *cfg, sp_server *out);

/* Make an uploaded graph servable.  The graph must outlive the server. */
sp_status sp_server_add_graph(sp_server srv, sp_graph g, int32_t *graph_id);

/* Queue BC over `sources` on graph `graph_id`.  out_bc: device double[V],
 * zeroed by the server before the first contribution and complete when the
 * request completes.  The sources are cut into chunks of max_batch
 * consecutive sources; a pass takes whole chunks, possibly of several
 * requests, and up to n_streams chunks of one request may run at once on
 * different streams.  Chunk 0 accumulates into out_bc, each later chunk into
 * a V-double buffer the server holds (counted with its workspaces) until it
 * is added into out_bc in chunk order.  A chunk's sources are added in list
 * order, so each request's BC is a function of its own source list: the
 * same bits alone or in a mix.  out_req receives a handle to wait on and
 * release. */
sp_status sp_stream_submit(sp_server srv, int32_t graph_id, const int32_t *sources,
                           int32_t n_sources, double *out_bc, sp_request *out_req);

/* Wait until the request finishes or timeout_us passes (< 0 waits forever).
 * Returns SP_OK when finished (its status in *result), SP_ERR_TIMEOUT
 * otherwise.  A request's status carries SP_WARN_SIGMA_LARGE only when one of
 * its own sources overflowed; when it failed (negative status),
 * sp_last_error() on the waiting thread then gives the detail. */
sp_status sp_request_wait(sp_request r, int64_t timeout_us, sp_status *result);

/* Non-blocking: 1 in *done if finished (status in *result), else 0. */
sp_status sp_request_poll(sp_request r, int32_t *done, sp_status *result);

/* Cancel a request whose sources have not started; returns SP_ERR_REJECTED
 * if it is already running or finished (it then completes normally). */
sp_status sp_request_cancel(sp_request r);

/* Submission-to-completion latency in microseconds (after completion). */
sp_status sp_request_latency_us(sp_request r, double *latency_us);

/* Release a request handle (after completion or cancellation). */
sp_status sp_request_release(sp_request r);

sp_status sp_server_get_stats(sp_server srv, sp_server_stats *out);

/* Stop accepting work, finish everything queued, free workspaces, join the
 * scheduler thread.  Requests not yet released stay valid handles. */
sp_status sp_server_destroy(sp_server srv);

#ifdef __cplusplus
}
#endif

#endif /* SP_H */
