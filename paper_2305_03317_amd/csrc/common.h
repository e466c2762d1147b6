// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sp.h"

namespace sp {

// ---------------------------------------------------------------------------
// Errors: a thread-local detail string plus status codes; no exceptions cross
// the C ABI.
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define SP_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::sp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                            __FILE__, __LINE__);                                      \
            return e_ == hipErrorOutOfMemory ? SP_ERR_OUT_OF_MEMORY : SP_ERR_DEVICE;  \
        }                                                                             \
    } while (0)

#define SP_TRY(expr)                        \
    do {                                    \
        sp_status st_ = (expr);             \
        if (st_ < 0) return st_;            \
    } while (0)

// Device allocation with an optional global test hook that makes the n-th
// allocation fail (environment SP_TEST_FAIL_ALLOC_AFTER=n), so the
// out-of-memory paths can be exercised without a full device.
sp_status dev_alloc(void **p, size_t bytes);
void dev_free(void *p);

// ---------------------------------------------------------------------------
// Graph
// ---------------------------------------------------------------------------
struct BatchWorkspace;
struct SourceWorkspace;
struct SsspWorkspace;
struct PrWorkspace;
struct HubEntry;

struct TuneEntry {
    bool valid = false;
    sp_batch_config cfg{};
};

}  // namespace sp

struct sp_graph_s {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *row_ptr = nullptr;  // device, n + 1
    int32_t *col_idx = nullptr;  // device, nnz (>= 1 element allocated)
    // Rows of incoming edges: the same arrays as row_ptr/col_idx for an
    // undirected graph, the reversed graph's for a directed one.
    int32_t *rp_in = nullptr;
    int32_t *ci_in = nullptr;
    bool directed = false;
    int32_t max_degree = 0;
    int32_t n_hubs = 0;          // vertices of degree > kHubDeg
    int64_t hub_chunks = 0;      // sum over hubs of ceil(degree / kHubChunk)
    int32_t n_hubs_in = 0;       // the same for incoming rows (= n_hubs when undirected)
    int64_t hub_chunks_in = 0;
    int64_t split_hub_chunks = 0;     // sum over hubs of split_hub_span(degree) (BC paths)
    int64_t split_hub_chunks_in = 0;  // the same for incoming rows (= split_hub_chunks when undirected)
    size_t bytes = 0;
    uint64_t fingerprint = 0;    // graph_fingerprint(): keys the tuning cache
    std::vector<int32_t> host_deg;   // host, n: vertex degrees (from the upload)
    std::vector<int32_t> host_deg_in;  // host, n: in-degrees (directed graphs only)
    std::vector<int32_t> group_key;  // host, n: summed distance to the highest-degree vertices
                                     // (unreached: n each); empty until first needed
    std::mutex mu;               // guards `tuned`, `group_key` and the workspace pools
    sp::TuneEntry tuned;
    std::vector<sp::SourceWorkspace *> src_pool;
    std::vector<sp::BatchWorkspace *> batch_pool;
    // Edge weights (sp_graph_set_weights), null until set: the adjacency
    // packed as {neighbour, weight} per CSR entry, so one 8-byte load gives
    // both.
    int2 *adjw = nullptr;            // device, nnz (>= 1 element allocated)
    // Every hub with its chunk range, in vertex order, and the hub of each
    // chunk; built on first use by the whole-graph kernels (ensure_static_hubs).
    sp::HubEntry *hub_static = nullptr;  // device, n_hubs (>= 1)
    int32_t *owner_static = nullptr;     // device, hub_chunks (>= 1)
    // PageRank's hub chunks, cut by row eighths (ensure_pr_hubs).
    sp::HubEntry *pr_hubs = nullptr;     // device, n_hubs (>= 1)
    int32_t *pr_owner = nullptr;         // device, pr_chunks (>= 1)
    int64_t pr_chunks = 0;
    int32_t pr_n_hubs = 0;               // entries of pr_hubs
    // Triangle counting: rows oriented toward higher (degree, id) rank, built
    // on first use (ensure_oriented): offsets, entries, and each entry's row.
    int32_t *tc_orp = nullptr;       // device, n + 1
    int32_t *tc_oci = nullptr;       // device, tc_m (>= 1)
    int32_t *tc_osrc = nullptr;      // device, tc_m (>= 1)
    int64_t tc_m = 0;
    int32_t max_weight = 0;
    size_t weight_bytes = 0;
    std::vector<sp::SsspWorkspace *> sssp_pool;
    std::vector<sp::PrWorkspace *> pr_pool;
};

namespace sp {

// Per-thread stats of the last BC call (what sp_get_last_stats returns).
sp_stats &tls_stats();

// Makes device d current for the guard's scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d) {
        if (hipGetDevice(&prev) == hipSuccess && prev != d) (void)hipSetDevice(d);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// ---------------------------------------------------------------------------
// Level-loop control block shared by the kernels of one BFS pass.  It lives in
// device memory; the kernels of a level read it, the `advance` kernel updates
// it, and the host reads it back once per chunk of levels.
// ---------------------------------------------------------------------------
enum : int32_t { MODE_TOPDOWN = 0, MODE_BOTTOMUP = 1 };

// Vertices with more than kHubDeg neighbours ("hubs") are not reduced inside
// the wave that holds their entry (which would walk a long row while its other
// entries wait): their adjacency is cut into chunks of kHubChunk entries, each
// chunk is reduced by its own wave into a partial, and a finishing kernel adds
// the partials in chunk order.  The result depends only on the degree, not on
// scheduling.  256/512 measured best on RMAT-22 among thresholds 128-1024 and
// chunks 256-1024.
constexpr int32_t kHubDeg = 256;
constexpr int32_t kHubChunk = 512;

// Both BC paths: a hub of more than kHubSplitDeg neighbours is cut into 8*m
// chunks of near-equal length (at most kHubChunk), m = ceil(deg/(8*kHubChunk)),
// numbered so that chunk id mod 8 names the eighth of the row the chunk lies
// in, with the hub's first id a multiple of 8.  Workgroups are dispatched to
// the device's 8 XCDs round-robin, so when the chunk kernels give the waves of
// block b the chunk ids congruent to b mod 8, each XCD (with its own L2)
// gathers from one eighth of every such hub row: one eighth of the vertex ids
// when they are randomly numbered.  A registration reserves 7 ids more than it
// uses, to align its first id.  Smaller hubs keep kHubChunk-entry chunks (at
// most 4), so a hub is split exactly when it has 8 or more chunks.
constexpr int32_t kXcds = 8;
constexpr int32_t kHubSplitDeg = 4 * kHubChunk;
__host__ __device__ constexpr int32_t split_hub_nchunks(int32_t deg) {
    return deg > kHubSplitDeg ? kXcds * ((deg + kXcds * kHubChunk - 1) / (kXcds * kHubChunk))
                              : (deg + kHubChunk - 1) / kHubChunk;
}
__host__ __device__ constexpr int32_t split_hub_span(int32_t deg) {
    return deg > kHubSplitDeg ? split_hub_nchunks(deg) + kXcds - 1 : split_hub_nchunks(deg);
}

// One hub occurrence on a level: vertex, its queue entry, and the range of
// level-local chunk ids [chunk_base, chunk_base + nchunks).
struct HubEntry {
    int32_t v;
    int32_t entry;
    int32_t chunk_base;
    int32_t nchunks;
};

// Counters that many workgroups update with atomics each sit on their own
// 128-byte line, so updates of one do not queue behind another's.
struct alignas(128) HotU64 {
    unsigned long long v;
    unsigned long long pad[15];
};
struct alignas(128) HotI32 {
    int32_t v;
    int32_t pad[31];
};

struct LevelCtl {
    // read-mostly part (written by init/advance)
    int32_t level;      // level of the current frontier
    int32_t lo, hi;     // current frontier = queue[lo, hi)
    int32_t done;       // 1 once a level produced no new vertex
    int32_t mode;       // MODE_* chosen for expanding the current frontier
    int32_t n_vertices;
    int32_t topdown_levels, bottomup_levels;
    unsigned long long front_deg;  // adjacency entries of the current frontier
    unsigned long long unset_deg;  // adjacency entries of vertices not yet reached
    unsigned long long reached_pairs;  // (slot, vertex) pairs reached (per-source: vertices)
    double alpha, beta;                // direction thresholds
    unsigned long long live;           // batched: slots with a nonempty current frontier
    unsigned long long active;         // batched: slots in use in this pass
    int32_t bwd_level, bwd_last;       // batched reverse pass: level being swept, deepest level
    int32_t chunk_next;                // batched: first owner-map slot of the level being built
    // Hubs: entries of the level being built are appended at hub_next, with
    // hub_pack = (count << 40) | chunks accumulating; `advance` turns them into
    // the current level's segment [hub_lo, hub_hi) with hub_nchunks chunks.
    int32_t hub_lo, hub_hi, hub_nchunks, hub_next;
    // contended counters
    HotI32 tail_;       // append position for the next frontier (starts at hi)
    HotI32 overflow_;   // capacity of the queue, hub list or value store exceeded
    HotU64 next_deg_;   // adjacency entries of the next frontier (accumulating)
    HotU64 settled_deg_;  // batched: adjacency entries of vertices every slot has reached
    HotU64 vtail_;      // batched: next free value (compact storage)
    HotU64 hub_pack_;
    HotU64 sigma_max_bits_;  // bit pattern of the largest sigma (>= 0, so integer order =
                             // value order; NaN sorts above inf)
    HotU64 flagged_slots_;   // slots with sigma > 1e300 / non-finite
    HotU64 nlive_;           // batched: slots of the next frontier (accumulating)
    HotI32 blocks_done_;     // batched: blocks of the current kernel that finished (last one
                             // ends the level); zero between kernels
    // Per-source path on a directed graph: the level's vertices whose
    // incoming row is longer than kHubDeg (their path counts are chunked),
    // listed afresh each level: [0, in_hub_n) with in_hub_nchunks chunks;
    // in_hub_pack_ accumulates the level being built as (count << 40) | chunks.
    int32_t in_hub_n, in_hub_nchunks;
    HotU64 in_hub_pack_;
    // Batched path, path counts of the level being built: pull_cost_
    // accumulates the incoming row lengths of its new vertices (the entries a
    // pull reads); sigma_push = 1 when the level's path counts are pushed from
    // the parents instead (set by `advance`, for the level it opens).
    HotU64 pull_cost_;
    int32_t sigma_push;
    unsigned long long val_lo;  // batched: first value of the current level
};


// Measurement: kernel families timed with HIP events when profiling is on,
// each with device counters of the work it did.
enum ProfKind : int {
    P_SRC_TOPDOWN, P_SRC_BOTTOMUP, P_SRC_SIGMA, P_SRC_SIGMA_HUB, P_SRC_DELTA, P_SRC_DELTA_HUB,
    P_MS_TOPDOWN, P_MS_BOTTOMUP, P_MS_SIGMA, P_MS_SIGMA_HUB, P_MS_EXPAND, P_MS_DELTA, P_MS_DELTA_HUB,
    P_MS_BC, P_SSSP_PUSH, P_SSSP_PULL, P_PR_PULL, P_PR_HUB, P_TC_COUNT, P_WG_BC,
    P_MS_SIGMA_PUSH, P_COUNT
};
constexpr int kProfCounters = 4;  // items, edges, pairs, item_slots
extern const char *const kProfNames[P_COUNT];
bool prof_enabled();
unsigned long long *prof_counters(int kind);  // device u64[kProfCounters], null when off
class ProfScope {
  public:
    ProfScope(int kind, hipStream_t s);
    ~ProfScope();
  private:
    int kind_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

// Launch shape helpers.
int device_cu_count();
int grid_for(int64_t items, int block, int max_blocks);

// Grids of the hub chunk kernels: a multiple of kXcds blocks (at least kXcds,
// at most max_blocks when that is a multiple), so that every XCD holds blocks.
inline int xcd_grid(int grid, int max_blocks) {
    const int g = (std::max(grid, kXcds) + kXcds - 1) / kXcds * kXcds;
    return g <= max_blocks ? g : std::max(kXcds, max_blocks / kXcds * kXcds);
}

// ---------------------------------------------------------------------------
// Per-source path (source_path.hip)
// ---------------------------------------------------------------------------
struct SourceWorkspace {
    int device = -1;
    int32_t n = 0;
    int32_t *dist = nullptr;
    double *sigma = nullptr;
    double *delta = nullptr;
    int32_t *queue = nullptr;
    int32_t *level_off = nullptr;  // device, levels + 2
    int32_t level_cap = 0;
    HubEntry *hub_list = nullptr;  // device, n_hubs + 1 (a hub occurs once per source)
    HubEntry *in_hub_list = nullptr;  // device, n_hubs_in + 1 (directed graphs)
    int32_t *hub_off = nullptr;    // device, levels + 2: hub segment of each level
    int32_t *hub_lvl_chunks = nullptr;  // device, levels + 1: chunk count of each level
    unsigned int *hub_cnt = nullptr;    // device, n_hubs + 1: finished chunks per hub
    double *partial = nullptr;     // device, max(hub_chunks, hub_chunks_in) + 1
    LevelCtl *ctl = nullptr;       // device
    LevelCtl *ctl_host = nullptr;  // pinned mirror
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
sp_status source_ws_create(sp_graph g, SourceWorkspace &ws);
void source_ws_destroy(SourceWorkspace &ws);

// Built-in configuration of both BC paths (used where neither the caller nor
// the autotuner set a field); the autotuner starts its search here.
constexpr int32_t kDefaultWidth = 64;
constexpr int kDefaultBlock = 512;
constexpr double kDefaultAlpha = 15.0;
constexpr double kDefaultBeta = 24.0;
constexpr int kDefaultChunkLevels = 8;
constexpr int kDefaultBlocksEngineBlock = 1024;  // workgroup size of the blocks engine

struct SourceRunOpts {
    double alpha = kDefaultAlpha, beta = kDefaultBeta;
    int block = kDefaultBlock;
    int chunk_levels = kDefaultChunkLevels;
};
struct SourceResult {
    int32_t levels = 0;   // levels including level 0
    int32_t reached = 0;
    double sigma_max = 0.0;
    bool flagged = false;  // some sigma > 1e300 or not finite
    int32_t td = 0, bu = 0;
};
// One source: forward (+ backward when with_backward); bc may be null.
sp_status source_run(sp_graph g, SourceWorkspace &ws, int32_t src, double *bc, bool with_backward,
                     const SourceRunOpts &o, hipStream_t s, SourceResult *res);
// sp_bc's work on a given workspace (api.hip): BC zeroed, then every source
// in list order; counters added to *stats.  Synchronises the stream.
sp_status bc_per_source(sp_graph g, SourceWorkspace &ws, const int32_t *sources, int32_t n_sources,
                        double *out_bc, hipStream_t st, sp_stats *stats);
// sp_bc's argument checks (null graph or output, sources in range).
sp_status check_bc_args(sp_graph g, const int32_t *sources, int32_t n_sources, const double *out_bc,
                        const char *what);

// ---------------------------------------------------------------------------
// Batched path (batch_path.hip)
// ---------------------------------------------------------------------------
constexpr int kSlots = 64;  // bits per source bitmap; also the slot stride of sigma/delta rows

// Output BC array of each slot of a pass (null: the slot adds to no output).
struct SlotTable {
    double *out[kSlots];
};

// Per-slot summary written by the workgroup engine.
// Blocks engine, per (slot, vertex): the BFS level (-1 unreached) and a
// value -- sigma after the forward pass; with fixed-width rows, rho =
// (1 + delta) / sigma once the reverse pass has finished the vertex.
struct alignas(16) WgRec {
    int32_t dist;
    int32_t pad;
    double val;
};

struct WgSlotResult {
    int32_t levels;   // levels including level 0
    int32_t reached;  // vertices reached
    double sigma_max;
    int32_t flagged;  // some sigma > 1e300 or not finite
    int32_t pad;
};

struct CapturedChunk {
    hipGraphExec_t exec = nullptr;
    std::array<long long, 12> key{};
};

struct BatchWorkspace {
    int device = -1;
    int32_t engine = SP_ENGINE_BITMAP;   // SP_ENGINE_BITMAP or SP_ENGINE_BLOCKS
    // Workgroup engine (wg_path.hip), source-major [slot][V] per slot:
    WgRec *wg_rec = nullptr;
    int32_t *wg_queue = nullptr, *wg_loff = nullptr;  // loff: [slot][V + 2]
    double *wg_delta = nullptr;  // [slot][V]
    WgSlotResult *wg_res = nullptr, *wg_res_host = nullptr;
    // Rows of width wg_ell_w (4 or 8; 0: rows read through the CSR offsets):
    // neighbour k of v at [v * w + k], -1 past the row's end; the incoming
    // rows' copy too on a directed graph.  Built on the first pass.
    int32_t *wg_ell = nullptr, *wg_ell_in = nullptr;
    int32_t wg_ell_w = 0;
    bool wg_ell_built = false;
    int32_t n = 0;
    unsigned long long *seen = nullptr;  // V: slots that reached v at any level so far
    unsigned long long *nxt = nullptr;   // V: slots discovering v at the level being built
    uint4 *front[2] = {nullptr, nullptr};  // V: {mask lo, mask hi, level tag, pad} by level parity
    // Values of an entry (v, level, mask m) are stored compactly: slot s of m
    // lives at val[vb + rank_m(s)], rank_m(s) = set bits of m below s, where vb
    // is the entry's value base.  val holds sigma after the forward pass and
    // rho = (1 + delta) / sigma once the reverse pass has visited the entry.
    double *val = nullptr;               // vcap values
    int64_t vcap = 0;
    double *dlt = nullptr;               // V x 64, vertex-major: delta[v * 64 + slot] (for BC)
    int32_t *queue = nullptr;            // entries: vertex ids, levels concatenated
    unsigned long long *qmask = nullptr; // entries: slot mask of the vertex at that level
    uint32_t *qvb = nullptr;             // entries: value base
    int64_t qcap = 0;
    int32_t *level_off = nullptr;        // device, level_cap + 2
    int32_t level_cap = 0;
    int32_t *slot_src = nullptr;         // device, 64: source vertex of each slot (-1 = empty)
    HubEntry *hub_list = nullptr;        // device, hub_cap entries
    int64_t hub_cap = 0;
    int32_t *owner = nullptr;            // device, owner_cap: hub list index of each hub chunk,
    int64_t owner_cap = 0;               //   levels concatenated
    int32_t *chunk_off = nullptr;        // device, level_cap: first owner slot of each level
    int32_t *hub_off = nullptr;          // device, level_cap: hub segment of each level
    int32_t *hub_lvl_chunks = nullptr;   // device, level_cap
    unsigned int *hub_cnt = nullptr;     // device, n_hubs + 1
    double *partial = nullptr;           // device, partial_rows x 64
    HubEntry *in_hub_list = nullptr;     // device, directed graphs: one level's incoming-row hubs
    int64_t in_hub_cap = 0;
    LevelCtl *ctl = nullptr;
    LevelCtl *ctl_host = nullptr;
    void *staging = nullptr;             // pinned: level-0 entries and slot sources
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    size_t bytes = 0;
    int32_t width = 0;                   // slots the value store is sized for
    // Chunks of levels captured once as HIP graphs (on a private stream) and
    // replayed on the caller's stream while their keys still hold: short and
    // long forward chunks, and the reverse chunk.
    hipStream_t cap_stream = nullptr;
    CapturedChunk fwd_short, fwd_long, bwd;
};
size_t batch_ws_bytes(sp_graph g, int64_t qcap, int32_t width, int32_t engine);
sp_status batch_ws_create(sp_graph g, int64_t qcap, int32_t width, int32_t engine, BatchWorkspace &ws);
// The engine SP_ENGINE_AUTO resolves to on this graph.
int32_t auto_engine(sp_graph g);
// Workgroup engine (wg_path.hip).
size_t wg_ws_bytes(sp_graph g, int32_t width);
sp_status wg_ws_alloc(sp_graph g, int32_t width, BatchWorkspace &ws);
void wg_ws_free(BatchWorkspace &ws);
void batch_ws_destroy(BatchWorkspace &ws);

struct BatchRunOpts {
    double alpha = kDefaultAlpha, beta = kDefaultBeta;
    int block = kDefaultBlock;
    int chunk_levels = kDefaultChunkLevels;
    int32_t engine = SP_ENGINE_BITMAP;  // resolved: SP_ENGINE_BITMAP or SP_ENGINE_BLOCKS
};

// Per-slot results of a pass, source-major ([slot * V + v]); any may be null.
struct BatchExtract {
    int32_t *dist = nullptr;
    double *sigma = nullptr;
    double *delta = nullptr;
};

// One multi-source pass over up to 64 sources (slot i <- srcs[i]).
//   bc_of_slot: per slot, the device BC array its delta is added to (may repeat);
//     slots are reduced in ascending slot order per vertex.
struct BatchResult {
    int32_t levels = 0;
    int64_t reached = 0;    // (slot, vertex) pairs reached
    int64_t entries = 0;    // (vertex, level) entries
    double sigma_max = 0.0;
    int32_t flagged = 0;    // slots with some sigma > 1e300 or not finite
    unsigned long long flagged_mask = 0;  // which slots
    int32_t td = 0, bu = 0;
    int32_t graph_launches = 0;
};
sp_status batch_run(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                    double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s,
                    BatchResult *res, const BatchExtract *ex = nullptr);
sp_status wg_run(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                 double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s, BatchResult *res,
                 const BatchExtract *ex);


// ---------------------------------------------------------------------------
// Single-source shortest paths (sssp_path.hip)
// ---------------------------------------------------------------------------
enum : int32_t { SSSP_PUSH = 0, SSSP_PULL = 1 };

// Round-loop control block of one SSSP run (device memory).  Round r expands
// the frontier: the vertices whose distance dropped in round r - 1 (the
// source in round 0).  They sit in queue[r & 1]; the hubs among them in
// hubs[r & 1], their chunks' owners in owner[r & 1].  The last working block
// of a round's kernel closes the round.
struct SsspCtl {
    // Everything a block needs to decide whether and how it takes part in a
    // round, written by the closing block in one 64-bit store and read by
    // every block in one 64-bit load, so no block sees half of a round's
    // state: bits 0-30 frontier size, 31-54 its hubs' chunk count, 55 round
    // parity, 56 pull round, 57 done.
    unsigned long long state;
    int32_t round;       // round being run (read by the round's working blocks)
    int32_t done;        // host mirror of the done bit
    int32_t n_vertices;
    int32_t forced;      // -1: choose per round; else the mode of every round
    int32_t push_rounds, pull_rounds;
    int32_t static_chunks;  // chunks of every hub of the graph (pull rounds)
    long long nnz;
    double alpha;        // a round pulls when its frontier's entries * alpha > nnz
    HotI32 tail_;        // entries of the next frontier
    HotI32 overflow_;    // a candidate distance reached INT32_MAX (checked after the rounds)
    HotI32 capacity_;    // 1: a queue, hub list or owner map would have overflowed (never
                         //   expected: a vertex joins a frontier at most once per round);
                         // 2 (after the rounds): a distance does not fit in int32
    HotU64 next_deg_;    // adjacency entries of the next frontier
    HotU64 hub_pack_;    // next frontier's hubs: (count << 40) | chunks
    HotI32 blocks_done_; // working blocks of the current kernel that finished
    HotU64 reached_;     // export: vertices with a finite distance
};

struct SsspWorkspace {
    int device = -1;
    int32_t n = 0;
    int2 *ds = nullptr;              // V: {distance, stamp}; stamp = last round whose
                                     //   frontier holds the vertex (-1: never)
    int32_t *queue[2] = {nullptr, nullptr};  // V each: frontier by round parity
    HubEntry *hubs[2] = {nullptr, nullptr};  // n_hubs + 1 each: frontier hubs by parity
    int32_t *owner[2] = {nullptr, nullptr};  // hub_chunks + 1 each: hub index of each chunk
    SsspCtl *ctl = nullptr;
    SsspCtl *ctl_host = nullptr;     // pinned mirror
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_stream = nullptr;
    CapturedChunk rounds_short, rounds_long;
};
sp_status sssp_ws_create(sp_graph g, SsspWorkspace &ws);
void sssp_ws_destroy(SsspWorkspace &ws);

struct SsspOpts {
    int forced = -1;       // -1 auto, else SSSP_PUSH / SSSP_PULL
    double alpha = 1.0;    // a frontier never holds more than every entry: no pull rounds
    int block = 256;
    int chunk_rounds = 8;
    int max_blocks = 0;    // 0: automatic
    int local_hops = 0;    // 0: automatic, < 0: none, else hops per round (a power of two <= 128)
};
// Local hops a run uses (sssp_path.hip).
int sssp_local_hops(sp_graph g, int requested);
struct SsspResult {
    int32_t rounds = 0, push_rounds = 0, pull_rounds = 0;
    int32_t reached = 0;
    int32_t graph_launches = 0;
    bool overflow = false;   // some distance does not fit in int32 (nothing exported)
};
// One source; writes the distance of every vertex (INT32_MAX where unreached)
// to out_dist unless the result overflows.
sp_status sssp_run(sp_graph g, SsspWorkspace &ws, int32_t src, int32_t *out_dist, const SsspOpts &o,
                   hipStream_t s, SsspResult *res);

// ---------------------------------------------------------------------------
// PageRank (pr_path.hip)
// ---------------------------------------------------------------------------
// Iteration control block.  `state` = iteration * 2 + done, written by the
// closing block in one store and read once per block (a block that starts
// after its iteration was closed sees another parity and returns).
struct PrCtl {
    int32_t state;
    int32_t max_iter;
    double beta;         // continue while diff > beta
    double last_diff;    // diff of the last iteration run
    HotU64 diff_;        // this iteration's sum of |change|, fixed point (2^-kPrDiffBits units)
    HotI32 blocks_done_; // working blocks of the closing kernel that finished
};
// Each block rounds its sum of |change| to a multiple of 2^-60 and adds it
// with an integer atomic: the total is the same whatever the order, so the
// stopping decision is reproducible.  Its error is at most blocks x 2^-61
// (under 2e-15 for 4096 blocks); the sum itself is at most 2 (the values
// start at 1/N and each iteration's total is at most 1), below the 16 that
// 64 bits hold at this scale.
constexpr int kPrDiffBits = 60;

struct PrWorkspace {
    int device = -1;
    double *pr[2] = {nullptr, nullptr};     // V each: PageRank by iteration parity
    double *share[2] = {nullptr, nullptr};  // V each: pr / out-degree (0 without out-edges)
    double *partial = nullptr;              // hub_chunks + 1: hub chunk sums
    PrCtl *ctl = nullptr;
    PrCtl *ctl_host = nullptr;              // pinned mirror
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_stream = nullptr;
    CapturedChunk iters;
};
sp_status pr_ws_create(sp_graph g, PrWorkspace &ws);
void pr_ws_destroy(PrWorkspace &ws);

struct PrOpts {
    int block = 256;
    int chunk_iters = 8;   // > 0: captured chunks; < 0: direct launches
};
struct PrResult {
    int32_t iterations = 0;
    double diff = 0.0;
    int32_t graph_launches = 0;
};
// PageRank of every vertex into out_pr (device, V doubles).
sp_status pr_run(sp_graph g, PrWorkspace &ws, double beta, double delta, int32_t max_iter,
                 double *out_pr, const PrOpts &o, hipStream_t s, PrResult *res);

// ---------------------------------------------------------------------------
// Triangle counting (tc_path.hip)
// ---------------------------------------------------------------------------
// Builds the oriented rows once per graph (thread-safe).
sp_status ensure_oriented(sp_graph g, hipStream_t s);
// Adds the graph's triangle count to *d_total (device, zeroed here) and, when
// per is not null, each vertex's triangle count to per[v] (zeroed here).
sp_status tc_run(sp_graph g, unsigned long long *d_total, unsigned long long *per, hipStream_t s);

// SP_ERR_NOT_SUPPORTED with a message, for entry points that need an
// undirected graph.
sp_status undirected_only(const char *what);

// SP_ERR_INVALID_ARGUMENT with a message unless every field of cfg (nullable)
// is within its documented range.
sp_status check_batch_cfg(const sp_batch_config *cfg);

// Builds g->hub_static / g->owner_static once (thread-safe).
sp_status ensure_static_hubs(sp_graph g, hipStream_t s);
// Builds g->pr_hubs / g->pr_owner once (thread-safe).
sp_status ensure_pr_hubs(sp_graph g, hipStream_t s);

// Workspace pools and configuration shared by the entry points and the server.
int64_t initial_qcap(int32_t n, int32_t width);
sp_status acquire_batch_ws(sp_graph g, int32_t width, int32_t engine, BatchWorkspace **out);
void release_batch_ws(sp_graph g, BatchWorkspace *ws);
BatchRunOpts resolve_batch(sp_graph g, const sp_batch_config *cfg, int32_t *width);

// Order in which sp_bc_batch cuts `sources` into batches of `width` (see
// sp_bc_batch); *key_ms receives the time spent computing the per-graph
// grouping keys in this call (0 when they were already cached).
sp_status source_groups(sp_graph g, const int32_t *sources, int32_t n_sources, int32_t width,
                        hipStream_t st, std::vector<int32_t> &order, double *key_ms);

// Tuning cache keyed by graph fingerprint (autotune.hip): a hash of the
// vertex and entry counts, direction and degree statistics, computed at
// upload.  Process-wide; also kept in the file named by the environment
// variable SP_TUNE_CACHE when it is set.
uint64_t graph_fingerprint(const sp_graph_s *g, const int32_t *in_deg);
bool tune_cache_lookup(uint64_t fp, sp_batch_config *out);
void tune_cache_store(uint64_t fp, const sp_batch_config &cfg);

// Kernels used by several files.
sp_status launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
sp_status launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

}  // namespace sp
