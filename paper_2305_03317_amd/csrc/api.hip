// C ABI of the library: argument checks, graph upload, workspace pools and
// the per-source / batched BC entry points.  Every entry point catches all
// C++ exceptions and returns a status; nothing here aborts the process.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <new>

#include "common.h"
#include "devutil.h"

namespace sp {

// ---------------------------------------------------------------------------
// Errors, stats, allocation
// ---------------------------------------------------------------------------
static thread_local char g_err[512];
static thread_local sp_stats g_stats;

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }
sp_stats &tls_stats() { return g_stats; }

static std::atomic<long long> g_alloc_count{0};
static long long alloc_fail_after() {
    static long long v = [] {
        const char *e = std::getenv("SP_TEST_FAIL_ALLOC_AFTER");
        return e ? std::atoll(e) : -1ll;
    }();
    return v;
}

sp_status dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    const long long lim = alloc_fail_after();
    if (lim >= 0 && g_alloc_count.fetch_add(1) >= lim) {
        set_error("device allocation of %zu bytes refused by SP_TEST_FAIL_ALLOC_AFTER", bytes);
        return SP_ERR_OUT_OF_MEMORY;
    }
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SP_ERR_OUT_OF_MEMORY : SP_ERR_DEVICE;
    }
    return SP_OK;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

int device_cu_count() {
    static int cus[64] = {0};
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return 256;
    if (!cus[d]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || c <= 0)
            c = 256;
        cus[d] = c;
    }
    return cus[d];
}

int grid_for(int64_t items, int block, int max_blocks) {
    int64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

// The library runs on gfx950 only; checked once per device.
static sp_status check_device(int *dev_out) {
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("no HIP device: %s", hipGetErrorString(e));
        return SP_ERR_NOT_SUPPORTED;
    }
    static std::atomic<int> ok[64];
    if (d < 0 || d >= 64) return SP_ERR_NOT_SUPPORTED;
    if (ok[d].load() == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) != hipSuccess) {
            set_error("hipGetDeviceProperties failed");
            return SP_ERR_DEVICE;
        }
        ok[d].store(std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2);
    }
    if (ok[d].load() != 1) {
        set_error("device %d is not gfx950", d);
        return SP_ERR_NOT_SUPPORTED;
    }
    if (dev_out) *dev_out = d;
    return SP_OK;
}


// ---------------------------------------------------------------------------
// CSR checks
// ---------------------------------------------------------------------------
// Device-side range check run on every upload: offsets monotone within
// [0, nnz], ids within [0, n).  bad[0] counts violations.
__global__ void k_check_csr(const int32_t *rp, const int32_t *ci, int32_t n, int64_t nnz,
                            unsigned int *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned int b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n + 1; i += stride) {
        const int32_t r = rp[i];
        if (r < 0 || (int64_t)r > nnz) ++b;
        if (i == 0 && r != 0) ++b;
        if (i == n && (int64_t)r != nnz) ++b;
        if (i < n && rp[i + 1] < r) ++b;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
        const int32_t c = ci[i];
        if (c < 0 || c >= n) ++b;
    }
    if (b) atomicAdd(bad, b);
}

// Host check of the full contract (SP_VALIDATE).
static bool host_validate(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci) {
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[V] must equal nnz");
        return false;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) {
            set_error("row_ptr decreases at vertex %d", v);
            return false;
        }
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t w = ci[e];
            if (w < 0 || w >= n) {
                set_error("col_idx[%d] = %d out of range", e, w);
                return false;
            }
            if (w == v) {
                set_error("self-loop at vertex %d", v);
                return false;
            }
            if (e > rp[v] && ci[e - 1] >= w) {
                set_error("row %d not strictly ascending (unsorted or duplicate)", v);
                return false;
            }
            // symmetric: v must appear in row w (binary search, rows sorted)
            const int32_t *b = ci + rp[w], *en = ci + rp[w + 1];
            const int32_t *f = std::lower_bound(b, en, v);
            if (f == en || *f != v) {
                set_error("edge %d->%d has no reverse entry", v, w);
                return false;
            }
        }
    }
    return true;
}

// Fingerprint of a freshly uploaded graph, and the tuned configuration the
// cache holds for it (if any) as its starting configuration.
static void adopt_cached_tuning(sp_graph g, const int32_t *in_deg) {
    g->fingerprint = graph_fingerprint(g, in_deg);
    sp_batch_config c{};
    const bool hit = tune_cache_lookup(g->fingerprint, &c);
    std::lock_guard<std::mutex> lk(g->mu);
    g->tuned = TuneEntry{};
    if (hit) {
        g->tuned.valid = true;
        g->tuned.cfg = c;
    }
}

// ---------------------------------------------------------------------------
// Workspace pools
// ---------------------------------------------------------------------------
static sp_status acquire_source_ws(sp_graph g, SourceWorkspace **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->src_pool.empty()) {
            *out = g->src_pool.back();
            g->src_pool.pop_back();
            return SP_OK;
        }
    }
    auto *ws = new (std::nothrow) SourceWorkspace;
    if (!ws) return SP_ERR_OUT_OF_MEMORY;
    sp_status st = source_ws_create(g, *ws);
    if (st < 0) {
        source_ws_destroy(*ws);
        delete ws;
        return st;
    }
    *out = ws;
    return SP_OK;
}

static void release_source_ws(sp_graph g, SourceWorkspace *ws) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->src_pool.push_back(ws);
}

int64_t initial_qcap(int32_t n, int32_t width) {
    const int64_t V = std::max(n, 1);
    return V * std::min(width, 16) + kSlots;
}

sp_status acquire_batch_ws(sp_graph g, int32_t width, int32_t engine, BatchWorkspace **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (size_t i = 0; i < g->batch_pool.size(); ++i)
            if (g->batch_pool[i]->width >= width && g->batch_pool[i]->engine == engine) {
                *out = g->batch_pool[i];
                g->batch_pool.erase(g->batch_pool.begin() + i);
                return SP_OK;
            }
    }
    auto *ws = new (std::nothrow) BatchWorkspace;
    if (!ws) return SP_ERR_OUT_OF_MEMORY;
    sp_status st = batch_ws_create(g, initial_qcap(g->n, width), width, engine, *ws);
    if (st < 0) {
        batch_ws_destroy(*ws);
        delete ws;
        return st;
    }
    *out = ws;
    return SP_OK;
}

void release_batch_ws(sp_graph g, BatchWorkspace *ws) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->batch_pool.push_back(ws);
}

static sp_status check_sources(sp_graph g, const int32_t *sources, int32_t n_sources) {
    if (n_sources < 0 || (n_sources > 0 && !sources)) {
        set_error("sources must be a host array of n_sources >= 0 ids");
        return SP_ERR_INVALID_ARGUMENT;
    }
    for (int32_t i = 0; i < n_sources; ++i)
        if (sources[i] < 0 || sources[i] >= g->n) {
            set_error("sources[%d] = %d outside [0, %d)", i, sources[i], g->n);
            return SP_ERR_INVALID_ARGUMENT;
        }
    return SP_OK;
}

sp_status check_bc_args(sp_graph g, const int32_t *sources, int32_t n_sources, const double *out_bc,
                        const char *what) {
    if (!g || (g->n > 0 && !out_bc)) {
        set_error("%s: null graph or output", what);
        return SP_ERR_INVALID_ARGUMENT;
    }
    return check_sources(g, sources, n_sources);
}

// Effective batched configuration: explicit fields, else tuned, else defaults.
BatchRunOpts resolve_batch(sp_graph g, const sp_batch_config *cfg, int32_t *width) {
    sp_batch_config t{};
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->tuned.valid) t = g->tuned.cfg;
    }
    auto pick_i = [](int32_t a, int32_t b, int32_t d) { return a ? a : (b ? b : d); };
    auto pick_d = [](double a, double b, double d) { return a > 0 ? a : (b > 0 ? b : d); };
    BatchRunOpts o;
    *width = pick_i(cfg ? cfg->batch_width : 0, t.batch_width, kDefaultWidth);
    o.block = pick_i(cfg ? cfg->block_size : 0, t.block_size, kDefaultBlock);
    o.alpha = pick_d(cfg ? cfg->alpha : 0, t.alpha, kDefaultAlpha);
    o.beta = pick_d(cfg ? cfg->beta : 0, t.beta, kDefaultBeta);
    o.chunk_levels = pick_i(cfg ? cfg->chunk_levels : 0, t.chunk_levels, kDefaultChunkLevels);
    o.engine = pick_i(cfg ? cfg->engine : 0, t.engine, auto_engine(g));
    if (o.engine == SP_ENGINE_BLOCKS)  // its own default workgroup size
        o.block = pick_i(cfg ? cfg->block_size : 0, t.engine == SP_ENGINE_BLOCKS ? t.block_size : 0,
                         kDefaultBlocksEngineBlock);
    return o;
}

sp_status check_batch_cfg(const sp_batch_config *cfg) {
    if (!cfg) return SP_OK;
    if (cfg->batch_width < 0 || cfg->batch_width > kSlots) {
        set_error("batch_width %d outside 0..64", cfg->batch_width);
        return SP_ERR_INVALID_ARGUMENT;
    }
    const int b = cfg->block_size;
    if (b != 0 && b != 128 && b != 256 && b != 512 && !(b == 1024 && cfg->engine == SP_ENGINE_BLOCKS)) {
        set_error("block_size %d not one of 128, 256, 512 (1024: with engine SP_ENGINE_BLOCKS only)", b);
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (cfg->alpha < 0 || cfg->beta < 0 || !std::isfinite(cfg->alpha) || !std::isfinite(cfg->beta)) {
        set_error("alpha/beta must be finite and >= 0");
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (cfg->chunk_levels < -65536 || cfg->chunk_levels > 65536) {
        set_error("chunk_levels %d outside -65536..65536", cfg->chunk_levels);
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (cfg->engine != SP_ENGINE_AUTO && cfg->engine != SP_ENGINE_BITMAP && cfg->engine != SP_ENGINE_BLOCKS) {
        set_error("engine %d not one of SP_ENGINE_AUTO, _BITMAP, _BLOCKS", cfg->engine);
        return SP_ERR_INVALID_ARGUMENT;
    }
    for (int r : cfg->reserved)
        if (r) {
            set_error("reserved fields must be zero");
            return SP_ERR_INVALID_ARGUMENT;
        }
    return SP_OK;
}

// Export helpers for sp_bfs_levels.
__global__ void k_src_export(int32_t n, const int32_t *dist, const double *sigma, const double *delta,
                             int32_t *out_dist, double *out_sigma, double *out_delta) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t d = dist[v];
        out_dist[v] = d;
        if (out_sigma) out_sigma[v] = d >= 0 ? sigma[v] : 0.0;
        if (out_delta) out_delta[v] = d > 0 ? delta[v] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Weighted graphs (SSSP)
// ---------------------------------------------------------------------------
static thread_local sp_sssp_stats g_sssp_stats;

// Pack each CSR entry with its weight; count weights outside [0, INT32_MAX - 1]
// and track the largest.
__global__ void k_pack_weights(const int32_t *__restrict__ ci, const int32_t *__restrict__ w,
                               int64_t nnz, int2 *adjw, unsigned int *bad, int *maxw) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned int b = 0;
    int m = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        const int32_t x = w[e];
        if (x < 0 || x == INT32_MAX) ++b;
        m = max(m, x);
        adjw[e] = make_int2(ci[e], x);
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
    if (b) atomicAdd(bad, b);
    if (lane_id() == 0 && m > 0) atomicMax(maxw, m);
}

// Host check (SP_VALIDATE): the entry of v in row u and of u in row v carry
// the same weight.  Rows must be sorted (binary search).
static bool weights_symmetric(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *w) {
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = ci[e];
            const int32_t *b = ci + rp[v], *z = ci + rp[v + 1];
            const int32_t *f = std::lower_bound(b, z, u);
            if (f == z || *f != u) {
                set_error("edge (%d, %d) has no reverse entry (or row %d is unsorted)", u, v, v);
                return false;
            }
            if (w[f - ci] != w[e]) {
                set_error("edge {%d, %d} has weights %d and %d in its two entries", u, v, w[e], w[f - ci]);
                return false;
            }
        }
    return true;
}

static sp_status acquire_sssp_ws(sp_graph g, SsspWorkspace **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->sssp_pool.empty()) {
            *out = g->sssp_pool.back();
            g->sssp_pool.pop_back();
            return SP_OK;
        }
    }
    auto *ws = new (std::nothrow) SsspWorkspace;
    if (!ws) return SP_ERR_OUT_OF_MEMORY;
    sp_status st = sssp_ws_create(g, *ws);
    if (st < 0) {
        sssp_ws_destroy(*ws);
        delete ws;
        return st;
    }
    *out = ws;
    return SP_OK;
}

static void release_sssp_ws(sp_graph g, SsspWorkspace *ws) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->sssp_pool.push_back(ws);
}

sp_status undirected_only(const char *what) {
    set_error("%s: not available for directed graphs", what);
    return SP_ERR_NOT_SUPPORTED;
}

static thread_local sp_pagerank_stats g_pr_stats;
static thread_local sp_tc_stats g_tc_stats;

static sp_status acquire_pr_ws(sp_graph g, PrWorkspace **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->pr_pool.empty()) {
            *out = g->pr_pool.back();
            g->pr_pool.pop_back();
            return SP_OK;
        }
    }
    auto *ws = new (std::nothrow) PrWorkspace;
    if (!ws) return SP_ERR_OUT_OF_MEMORY;
    sp_status st = pr_ws_create(g, *ws);
    if (st < 0) {
        delete ws;
        return st;
    }
    *out = ws;
    return SP_OK;
}

static void release_pr_ws(sp_graph g, PrWorkspace *ws) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->pr_pool.push_back(ws);
}

static void free_weights(sp_graph g) {
    dev_free(g->adjw);
    g->adjw = nullptr;
    g->max_weight = 0;
    g->bytes -= g->weight_bytes;
    g->weight_bytes = 0;
}

// Upload a hub list and its chunk owner map; on success the device copies go
// to *hub_out / *owner_out and their bytes are added to the graph's size.
static sp_status upload_hub_layout(sp_graph g, const std::vector<HubEntry> &hubs,
                                   const std::vector<int32_t> &owners, hipStream_t st,
                                   HubEntry **hub_out, int32_t **owner_out) {
    HubEntry *hub_dev = nullptr;
    int32_t *owner_dev = nullptr;
    const size_t hb = sizeof(HubEntry) * std::max<size_t>(hubs.size(), 1);
    const size_t ob = sizeof(int32_t) * std::max<size_t>(owners.size(), 1);
    sp_status rc = dev_alloc((void **)&hub_dev, hb);
    if (rc == SP_OK) rc = dev_alloc((void **)&owner_dev, ob);
    hipError_t e = hipSuccess;
    if (rc == SP_OK && !hubs.empty())
        e = hipMemcpyAsync(hub_dev, hubs.data(), hubs.size() * sizeof(HubEntry), hipMemcpyHostToDevice, st);
    if (rc == SP_OK && e == hipSuccess && !owners.empty())
        e = hipMemcpyAsync(owner_dev, owners.data(), owners.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st);
    if (rc == SP_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    if (rc != SP_OK || e != hipSuccess) {
        dev_free(hub_dev);
        dev_free(owner_dev);
        if (e != hipSuccess) set_error("hub list upload failed: %s", hipGetErrorString(e));
        return rc != SP_OK ? rc : SP_ERR_DEVICE;
    }
    *hub_out = hub_dev;
    *owner_out = owner_dev;
    g->bytes += hb + ob;
    return SP_OK;
}

// Every hub of the graph with its chunk range, in vertex order, and the hub
// of every chunk: built once per graph on first use (SSSP pull rounds,
// triangle counting), kept until the graph is released.
sp_status ensure_static_hubs(sp_graph g, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->hub_static) return SP_OK;
    std::vector<HubEntry> hubs;
    std::vector<int32_t> owners;
    for (int32_t v = 0; v < g->n; ++v)
        if (g->host_deg[v] > kHubDeg) {
            const int32_t nch = (g->host_deg[v] + kHubChunk - 1) / kHubChunk;
            hubs.push_back(HubEntry{v, 0, (int32_t)owners.size(), nch});
            owners.insert(owners.end(), (size_t)nch, (int32_t)hubs.size() - 1);
        }
    return upload_hub_layout(g, hubs, owners, st, &g->hub_static, &g->owner_static);
}

// PageRank's hub layout over the rows it gathers (a vertex's in-neighbours:
// its own row when undirected, its reversed row when directed): every hub cut
// by row eighths into 8m near-equal pieces of at most kHubChunk entries
// (split_piece), m = ceil(deg / (8 * kHubChunk)); every hub's first chunk id
// is a multiple of 8.
sp_status ensure_pr_hubs(sp_graph g, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->pr_hubs) return SP_OK;
    const std::vector<int32_t> &deg = g->directed ? g->host_deg_in : g->host_deg;
    std::vector<HubEntry> hubs;
    std::vector<int32_t> owners;
    for (int32_t v = 0; v < g->n; ++v)
        if (deg[v] > kHubDeg) {
            const int32_t nch = kXcds * ((deg[v] + kXcds * kHubChunk - 1) / (kXcds * kHubChunk));
            hubs.push_back(HubEntry{v, 0, (int32_t)owners.size(), nch});
            owners.insert(owners.end(), (size_t)nch, (int32_t)hubs.size() - 1);
        }
    SP_TRY(upload_hub_layout(g, hubs, owners, st, &g->pr_hubs, &g->pr_owner));
    g->pr_chunks = (int64_t)owners.size();
    g->pr_n_hubs = (int32_t)hubs.size();
    return SP_OK;
}

// The per-source loop shared by sp_bc and sp_bc_noalloc: out_bc zeroed,
// then one pass per source in list order (block size from the graph's tuned
// configuration).  Times the call with ws's events when it has them.
sp_status bc_per_source(sp_graph g, SourceWorkspace &ws, const int32_t *sources, int32_t n_sources,
                        double *out_bc, hipStream_t st, sp_stats *stats) {
    sp_batch_config tcfg{};
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->tuned.valid) tcfg = g->tuned.cfg;
    }
    SourceRunOpts o;
    if (tcfg.block_size && tcfg.block_size <= 512) o.block = tcfg.block_size;  // (1024: blocks engine only)
    const bool timed = ws.ev0 && ws.ev1;
    if (timed) SP_HIP(hipEventRecord(ws.ev0, st));
    SP_TRY(launch_fill_f64(out_bc, g->n, 0.0, st));
    bool flagged = false;
    for (int32_t i = 0; i < n_sources; ++i) {
        SourceResult r;
        SP_TRY(source_run(g, ws, sources[i], out_bc, true, o, st, &r));
        stats->n_passes++;
        stats->max_levels = std::max(stats->max_levels, r.levels);
        stats->levels_total += r.levels;
        stats->topdown_levels += r.td;
        stats->bottomup_levels += r.bu;
        stats->reached_total += r.reached;
        stats->sigma_max = std::max(stats->sigma_max, r.sigma_max);
        if (r.flagged) {
            stats->sigma_flagged++;
            flagged = true;
        }
    }
    if (timed) {
        SP_HIP(hipEventRecord(ws.ev1, st));
        SP_HIP(hipEventSynchronize(ws.ev1));
        float ms = 0;
        SP_HIP(hipEventElapsedTime(&ms, ws.ev0, ws.ev1));
        stats->device_ms = ms;
    } else {
        SP_HIP(hipStreamSynchronize(st));
    }
    stats->batch_width = 1;
    stats->block_size = o.block;
    stats->alpha = o.alpha;
    stats->beta = o.beta;
    stats->chunk_levels = o.chunk_levels;
    return flagged ? SP_WARN_SIGMA_LARGE : SP_OK;
}

}  // namespace sp

using namespace sp;

#define SP_GUARD_BEGIN try {
#define SP_GUARD_END                                       \
    }                                                      \
    catch (const std::bad_alloc &) {                       \
        set_error("host allocation failed");               \
        return SP_ERR_OUT_OF_MEMORY;                       \
    }                                                      \
    catch (...) {                                          \
        set_error("unexpected C++ exception");             \
        return SP_ERR_DEVICE;                              \
    }

extern "C" {

const char *sp_status_string(sp_status s) {
    switch (s) {
        case SP_OK: return "ok";
        case SP_WARN_SIGMA_LARGE: return "warning: some path count exceeded 1e300 or was not finite";
        case SP_ERR_INVALID_ARGUMENT: return "invalid argument";
        case SP_ERR_OUT_OF_MEMORY: return "out of memory";
        case SP_ERR_DEVICE: return "device error";
        case SP_ERR_NOT_SUPPORTED: return "not supported";
        case SP_ERR_REJECTED: return "rejected";
        case SP_ERR_TIMEOUT: return "timed out";
        case SP_ERR_CANCELLED: return "cancelled";
        default: return s > 0 ? "warning" : "unknown error";
    }
}

const char *sp_last_error(void) { return g_err; }

int32_t sp_version(void) { return 100; }

uint64_t sp_header_hash(void) { return SP_HEADER_HASH; }

sp_status sp_graph_upload(int32_t n_vertices, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, uint32_t flags, sp_stream s, sp_graph *out) {
    SP_GUARD_BEGIN
    clear_error();
    if (!out || n_vertices < 0 || n_vertices == INT32_MAX || nnz < 0 || nnz >= INT32_MAX ||
        !row_ptr || (nnz > 0 && !col_idx) ||
        (flags & ~(SP_PTR_DEVICE | SP_VALIDATE))) {
        set_error("sp_graph_upload: bad arguments");
        return SP_ERR_INVALID_ARGUMENT;
    }
    int dev = 0;
    SP_TRY(check_device(&dev));
    hipStream_t st = (hipStream_t)s;
    const bool on_dev = flags & SP_PTR_DEVICE;
    if (flags & SP_VALIDATE) {
        std::vector<int32_t> hr, hc;
        const int32_t *rp = row_ptr, *ci = col_idx;
        if (on_dev) {
            hr.resize((size_t)n_vertices + 1);
            hc.resize((size_t)nnz);
            SP_HIP(hipMemcpyAsync(hr.data(), row_ptr, hr.size() * 4, hipMemcpyDeviceToHost, st));
            if (nnz) SP_HIP(hipMemcpyAsync(hc.data(), col_idx, hc.size() * 4, hipMemcpyDeviceToHost, st));
            SP_HIP(hipStreamSynchronize(st));
            rp = hr.data();
            ci = hc.data();
        }
        if (!host_validate(n_vertices, nnz, rp, ci)) return SP_ERR_INVALID_ARGUMENT;
    }
    auto *g = new sp_graph_s;
    g->device = dev;
    g->n = n_vertices;
    g->nnz = nnz;
    sp_status rc = dev_alloc((void **)&g->row_ptr, ((size_t)n_vertices + 1) * 4);
    if (rc == SP_OK) rc = dev_alloc((void **)&g->col_idx, (size_t)std::max<int64_t>(nnz, 1) * 4);
    unsigned int *bad = nullptr;
    if (rc == SP_OK) rc = dev_alloc((void **)&bad, 4);
    if (rc != SP_OK) {
        dev_free(g->row_ptr);
        dev_free(g->col_idx);
        dev_free(bad);
        delete g;
        return rc;
    }
    auto fail = [&](sp_status code) {
        dev_free(g->row_ptr);
        dev_free(g->col_idx);
        dev_free(bad);
        delete g;
        return code;
    };
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    unsigned int h_bad = 0;
    std::vector<int32_t> deg_rp;
    hipError_t e = hipMemcpyAsync(g->row_ptr, row_ptr, ((size_t)n_vertices + 1) * 4, kind, st);
    if (e == hipSuccess && nnz) e = hipMemcpyAsync(g->col_idx, col_idx, (size_t)nnz * 4, kind, st);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, 4, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_check_csr, dim3(grid_for(std::max<int64_t>(nnz, n_vertices + 1), 256, 2048)),
                           dim3(256), 0, st, (const int32_t *)g->row_ptr, (const int32_t *)g->col_idx,
                           n_vertices, nnz, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) {
        deg_rp.resize((size_t)n_vertices + 1);
        e = hipMemcpyAsync(deg_rp.data(), g->row_ptr, deg_rp.size() * 4, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error("graph upload failed: %s", hipGetErrorString(e));
        return fail(SP_ERR_DEVICE);
    }
    if (h_bad) {
        set_error("CSR has %u out-of-range offsets or ids", h_bad);
        return fail(SP_ERR_INVALID_ARGUMENT);
    }
    dev_free(bad);
    bad = nullptr;
    int32_t md = 0;
    g->host_deg.resize(n_vertices);
    for (int32_t v = 0; v < n_vertices; ++v) {
        const int32_t d = deg_rp[v + 1] - deg_rp[v];
        g->host_deg[v] = d;
        md = std::max(md, d);
        if (d > kHubDeg) {
            g->n_hubs++;
            g->hub_chunks += (d + kHubChunk - 1) / kHubChunk;
            g->split_hub_chunks += split_hub_span(d);
        }
    }
    g->max_degree = md;
    g->rp_in = g->row_ptr;
    g->ci_in = g->col_idx;
    g->n_hubs_in = g->n_hubs;
    g->hub_chunks_in = g->hub_chunks;
    g->split_hub_chunks_in = g->split_hub_chunks;
    g->bytes = ((size_t)n_vertices + 1) * 4 + (size_t)std::max<int64_t>(nnz, 1) * 4;
    adopt_cached_tuning(g, nullptr);
    *out = g;
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_graph_upload_directed(int32_t n_vertices, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, uint32_t flags, sp_stream s, sp_graph *out) {
    SP_GUARD_BEGIN
    clear_error();
    if (!out || n_vertices < 0 || n_vertices == INT32_MAX || nnz < 0 || nnz >= INT32_MAX || !row_ptr ||
        (nnz > 0 && !col_idx) || (flags & ~(SP_PTR_DEVICE | SP_VALIDATE))) {
        set_error("sp_graph_upload_directed: bad arguments");
        return SP_ERR_INVALID_ARGUMENT;
    }
    int dev = 0;
    SP_TRY(check_device(&dev));
    hipStream_t st = (hipStream_t)s;
    // host copies: the reversed rows are built on the host
    std::vector<int32_t> hr((size_t)n_vertices + 1), hc((size_t)nnz);
    if (flags & SP_PTR_DEVICE) {
        SP_HIP(hipMemcpyAsync(hr.data(), row_ptr, hr.size() * 4, hipMemcpyDeviceToHost, st));
        if (nnz) SP_HIP(hipMemcpyAsync(hc.data(), col_idx, hc.size() * 4, hipMemcpyDeviceToHost, st));
        SP_HIP(hipStreamSynchronize(st));
    } else {
        std::memcpy(hr.data(), row_ptr, hr.size() * 4);
        if (nnz) std::memcpy(hc.data(), col_idx, hc.size() * 4);
    }
    // offsets and ids are always checked here (the reversal indexes by them)
    bool ok = hr[0] == 0 && (int64_t)hr[n_vertices] == nnz;
    for (int32_t v = 0; ok && v < n_vertices; ++v) ok = hr[v] <= hr[v + 1];
    for (int64_t e = 0; ok && e < nnz; ++e) ok = hc[e] >= 0 && hc[e] < n_vertices;
    if (ok && (flags & SP_VALIDATE))  // sorted, duplicate-free rows without self-loops
        for (int32_t v = 0; ok && v < n_vertices; ++v)
            for (int32_t e = hr[v]; ok && e < hr[v + 1]; ++e)
                ok = hc[e] != v && (e == hr[v] || hc[e - 1] < hc[e]);
    if (!ok) {
        set_error("directed CSR is malformed (offsets, ids%s)",
                  (flags & SP_VALIDATE) ? ", row order, duplicates or self-loops" : "");
        return SP_ERR_INVALID_ARGUMENT;
    }
    std::vector<int32_t> ir((size_t)n_vertices + 1, 0), ic((size_t)std::max<int64_t>(nnz, 1));
    for (int64_t e = 0; e < nnz; ++e) ir[hc[e] + 1]++;
    for (int32_t v = 0; v < n_vertices; ++v) ir[v + 1] += ir[v];
    {
        std::vector<int32_t> pos(ir.begin(), ir.end() - 1);
        for (int32_t u = 0; u < n_vertices; ++u)  // sources ascending: reversed rows come out sorted
            for (int32_t e = hr[u]; e < hr[u + 1]; ++e) ic[pos[hc[e]]++] = u;
    }
    sp_graph g = nullptr;
    SP_TRY(sp_graph_upload(n_vertices, nnz, hr.data(), hc.data(), 0, s, &g));
    int32_t *rp_in = nullptr, *ci_in = nullptr;
    sp_status rc = dev_alloc((void **)&rp_in, ir.size() * 4);
    if (rc == SP_OK) rc = dev_alloc((void **)&ci_in, ic.size() * 4);
    hipError_t e = hipSuccess;
    if (rc == SP_OK) e = hipMemcpyAsync(rp_in, ir.data(), ir.size() * 4, hipMemcpyHostToDevice, st);
    if (rc == SP_OK && e == hipSuccess) e = hipMemcpyAsync(ci_in, ic.data(), ic.size() * 4, hipMemcpyHostToDevice, st);
    if (rc == SP_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    if (rc != SP_OK || e != hipSuccess) {
        dev_free(rp_in);
        dev_free(ci_in);
        sp_graph_release(g);
        if (e != hipSuccess) set_error("directed graph upload failed: %s", hipGetErrorString(e));
        return rc != SP_OK ? rc : SP_ERR_DEVICE;
    }
    int32_t md = g->max_degree;
    int32_t nh_in = 0;
    int64_t nch_in = 0, split_in = 0;
    for (int32_t v = 0; v < n_vertices; ++v) {
        const int32_t d = ir[v + 1] - ir[v];
        md = std::max(md, d);
        if (d > kHubDeg) {
            ++nh_in;
            nch_in += (d + kHubChunk - 1) / kHubChunk;
            split_in += split_hub_span(d);
        }
    }
    g->rp_in = rp_in;
    g->ci_in = ci_in;
    g->directed = true;
    g->max_degree = md;
    g->n_hubs_in = nh_in;  // n_hubs / hub_chunks count the outgoing rows
    g->hub_chunks_in = nch_in;
    g->split_hub_chunks_in = split_in;
    g->bytes += ir.size() * 4 + ic.size() * 4;
    {
        std::vector<int32_t> in_deg(n_vertices);
        for (int32_t v = 0; v < n_vertices; ++v) in_deg[v] = ir[v + 1] - ir[v];
        adopt_cached_tuning(g, in_deg.data());
        g->host_deg_in = std::move(in_deg);
    }
    *out = g;
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_graph_release(sp_graph g) {
    SP_GUARD_BEGIN
    if (!g) return SP_OK;
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();
    for (auto *ws : g->src_pool) {
        source_ws_destroy(*ws);
        delete ws;
    }
    for (auto *ws : g->batch_pool) {
        batch_ws_destroy(*ws);
        delete ws;
    }
    for (auto *ws : g->sssp_pool) {
        sssp_ws_destroy(*ws);
        delete ws;
    }
    for (auto *ws : g->pr_pool) {
        pr_ws_destroy(*ws);
        delete ws;
    }
    free_weights(g);
    if (g->directed) {
        dev_free(g->rp_in);
        dev_free(g->ci_in);
    }
    dev_free(g->tc_orp);
    dev_free(g->tc_oci);
    dev_free(g->tc_osrc);
    dev_free(g->hub_static);
    dev_free(g->owner_static);
    dev_free(g->pr_hubs);
    dev_free(g->pr_owner);
    dev_free(g->row_ptr);
    dev_free(g->col_idx);
    delete g;
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_graph_info(sp_graph g, int32_t *n_vertices, int64_t *nnz, size_t *device_bytes) {
    if (!g) {
        set_error("null graph");
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (n_vertices) *n_vertices = g->n;
    if (nnz) *nnz = g->nnz;
    if (device_bytes) *device_bytes = g->bytes;
    return SP_OK;
}

sp_status sp_get_last_stats(sp_stats *out) {
    if (!out) return SP_ERR_INVALID_ARGUMENT;
    *out = g_stats;
    return SP_OK;
}

sp_status sp_bc(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    SP_TRY(check_bc_args(g, sources, n_sources, out_bc, "sp_bc"));
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    sp_stats stats{};
    stats.n_sources = n_sources;
    if (g->n == 0) {
        g_stats = stats;
        return SP_OK;
    }
    SourceWorkspace *ws = nullptr;
    SP_TRY(acquire_source_ws(g, &ws));
    struct Rel {
        sp_graph g;
        SourceWorkspace *ws;
        ~Rel() { release_source_ws(g, ws); }
    } rel{g, ws};
    const sp_status rc = bc_per_source(g, *ws, sources, n_sources, out_bc, st, &stats);
    if (rc >= 0) g_stats = stats;
    return rc;
    SP_GUARD_END
}

}  // extern "C"

namespace sp {

// Order in which sp_bc_batch cuts `sources` into batches: ascending summed
// BFS distance to the kGroupHubs highest-degree vertices, then descending
// degree, then list position.  Sources with similar depth profiles share a
// batch, so each vertex is reached at fewer distinct levels per batch.  The
// distances are computed once per graph with the per-source path.
constexpr int kGroupHubs = 4;

sp_status source_groups(sp_graph g, const int32_t *sources, int32_t n_sources, int32_t width,
                        hipStream_t st, std::vector<int32_t> &order, double *key_ms) {
    order.resize(n_sources);
    for (int32_t i = 0; i < n_sources; ++i) order[i] = i;
    if (key_ms) *key_ms = 0.0;
    if (n_sources <= width) return SP_OK;
    bool ready;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        ready = !g->group_key.empty();
    }
    if (!ready) {
        const auto t0 = std::chrono::steady_clock::now();
        const int32_t n = g->n;
        std::vector<int32_t> hubs(n);
        for (int32_t v = 0; v < n; ++v) hubs[v] = v;
        const int32_t k = std::min(kGroupHubs, n);
        std::partial_sort(hubs.begin(), hubs.begin() + k, hubs.end(), [&](int32_t a, int32_t b) {
            return g->host_deg[a] != g->host_deg[b] ? g->host_deg[a] > g->host_deg[b] : a < b;
        });
        std::vector<int32_t> key(n, 0), dist(n);
        SourceWorkspace *ws = nullptr;
        SP_TRY(acquire_source_ws(g, &ws));
        struct Rel {
            sp_graph g;
            SourceWorkspace *ws;
            ~Rel() { release_source_ws(g, ws); }
        } rel{g, ws};
        SourceRunOpts o;
        for (int32_t h = 0; h < k; ++h) {
            SourceResult r;
            SP_TRY(source_run(g, *ws, hubs[h], nullptr, false, o, st, &r));
            SP_HIP(hipMemcpyAsync(dist.data(), ws->dist, (size_t)n * 4, hipMemcpyDeviceToHost, st));
            SP_HIP(hipStreamSynchronize(st));
            for (int32_t v = 0; v < n; ++v) key[v] += dist[v] >= 0 ? dist[v] : n;
        }
        if (key_ms)
            *key_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->group_key.empty()) g->group_key = std::move(key);
    }
    const std::vector<int32_t> &key = g->group_key;  // immutable once set
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int32_t sa = sources[a], sb = sources[b];
        if (key[sa] != key[sb]) return key[sa] < key[sb];
        return g->host_deg[sa] > g->host_deg[sb];
    });
    return SP_OK;
}

}  // namespace sp

extern "C" {

sp_status sp_bc_batch(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc,
                      const sp_batch_config *cfg, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || (g->n > 0 && !out_bc)) {
        set_error("sp_bc_batch: null graph or output");
        return SP_ERR_INVALID_ARGUMENT;
    }
    SP_TRY(check_sources(g, sources, n_sources));
    SP_TRY(check_batch_cfg(cfg));
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    int32_t width = 64;
    const BatchRunOpts o = resolve_batch(g, cfg, &width);
    sp_stats stats{};
    stats.n_sources = n_sources;
    stats.batch_width = width;
    stats.block_size = o.block;
    stats.alpha = o.alpha;
    stats.beta = o.beta;
    stats.chunk_levels = o.chunk_levels;
    if (g->n == 0) {
        g_stats = stats;
        return SP_OK;
    }
    BatchWorkspace *ws = nullptr;
    stats.engine = o.engine;
    SP_TRY(acquire_batch_ws(g, width, o.engine, &ws));
    struct Rel {
        sp_graph g;
        BatchWorkspace *ws;
        ~Rel() { release_batch_ws(g, ws); }
    } rel{g, ws};
    hipEvent_t e0, e1;
    SP_HIP(hipEventCreate(&e0));
    SP_HIP(hipEventCreate(&e1));
    struct EvRel {
        hipEvent_t a, b;
        ~EvRel() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evrel{e0, e1};
    std::vector<int32_t> order;
    double key_ms = 0.0;
    SP_TRY(source_groups(g, sources, n_sources, width, st, order, &key_ms));
    stats.group_ms = key_ms;
    std::vector<int32_t> grouped(n_sources);
    for (int32_t i = 0; i < n_sources; ++i) grouped[i] = sources[order[i]];
    SP_HIP(hipEventRecord(e0, st));
    SP_TRY(launch_fill_f64(out_bc, g->n, 0.0, st));
    double *slots[kSlots];
    for (auto &p : slots) p = out_bc;
    bool flagged = false;
    for (int32_t b = 0; b < n_sources; b += width) {
        const int32_t nb = std::min(width, n_sources - b);
        BatchResult r;
        SP_TRY(batch_run(g, *ws, grouped.data() + b, nb, slots, o, st, &r));
        stats.n_passes++;
        stats.max_levels = std::max(stats.max_levels, r.levels);
        stats.levels_total += r.levels;
        stats.topdown_levels += r.td;
        stats.bottomup_levels += r.bu;
        stats.reached_total += r.reached;
        stats.sigma_max = std::max(stats.sigma_max, r.sigma_max);
        stats.graph_launches += r.graph_launches;
        if (r.flagged) {
            stats.sigma_flagged += r.flagged;
            flagged = true;
        }
    }
    SP_HIP(hipEventRecord(e1, st));
    SP_HIP(hipEventSynchronize(e1));
    float ms = 0;
    SP_HIP(hipEventElapsedTime(&ms, e0, e1));
    stats.device_ms = ms;
    g_stats = stats;
    return flagged ? SP_WARN_SIGMA_LARGE : SP_OK;
    SP_GUARD_END
}

sp_status sp_bfs_levels(sp_graph g, int32_t source, int32_t *out_dist, double *out_sigma,
                        double *out_delta, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || !out_dist || source < 0 || source >= g->n) {
        set_error("sp_bfs_levels: null graph/output or source out of range");
        return SP_ERR_INVALID_ARGUMENT;
    }
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    SourceWorkspace *ws = nullptr;
    SP_TRY(acquire_source_ws(g, &ws));
    struct Rel {
        sp_graph g;
        SourceWorkspace *ws;
        ~Rel() { release_source_ws(g, ws); }
    } rel{g, ws};
    SourceRunOpts o;
    SourceResult r;
    SP_TRY(source_run(g, *ws, source, nullptr, out_delta != nullptr, o, st, &r));
    hipLaunchKernelGGL(k_src_export, dim3(grid_for(g->n, 256, 4096)), dim3(256), 0, st, g->n,
                       (const int32_t *)ws->dist, (const double *)ws->sigma,
                       (const double *)ws->delta, out_dist, out_sigma, out_delta);
    SP_HIP(hipGetLastError());
    SP_HIP(hipStreamSynchronize(st));
    return r.flagged ? SP_WARN_SIGMA_LARGE : SP_OK;
    SP_GUARD_END
}

sp_status sp_batch_levels(sp_graph g, const int32_t *sources, int32_t n_sources, int32_t *out_dist,
                          double *out_sigma, double *out_delta, const sp_batch_config *cfg,
                          sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || !out_dist || n_sources < 1 || n_sources > kSlots) {
        set_error("sp_batch_levels: null graph/output or n_sources outside 1..64");
        return SP_ERR_INVALID_ARGUMENT;
    }
    SP_TRY(check_sources(g, sources, n_sources));
    SP_TRY(check_batch_cfg(cfg));
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    int32_t width = 64;
    const BatchRunOpts o = resolve_batch(g, cfg, &width);
    BatchWorkspace *ws = nullptr;
    SP_TRY(acquire_batch_ws(g, n_sources, o.engine, &ws));
    struct Rel {
        sp_graph g;
        BatchWorkspace *ws;
        ~Rel() { release_batch_ws(g, ws); }
    } rel{g, ws};
    BatchResult r;
    BatchExtract ex;
    ex.dist = out_dist;
    ex.sigma = out_sigma;
    ex.delta = out_delta;
    SP_TRY(batch_run(g, *ws, sources, n_sources, nullptr, o, st, &r, &ex));
    SP_HIP(hipStreamSynchronize(st));
    return r.flagged ? SP_WARN_SIGMA_LARGE : SP_OK;
    SP_GUARD_END
}

sp_status sp_bc_workspace_bytes(sp_graph g, int32_t batch_width, size_t *bytes) {
    if (!g || !bytes || batch_width < 1 || batch_width > kSlots) {
        set_error("sp_bc_workspace_bytes: bad arguments");
        return SP_ERR_INVALID_ARGUMENT;
    }
    int32_t width = 0;
    const BatchRunOpts o = resolve_batch(g, nullptr, &width);
    *bytes = batch_ws_bytes(g, initial_qcap(g->n, batch_width), batch_width, o.engine);
    return SP_OK;
}

sp_status sp_graph_set_weights(sp_graph g, const int32_t *weights, uint32_t flags, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || (g->nnz > 0 && !weights) || (flags & ~(SP_PTR_DEVICE | SP_VALIDATE))) {
        set_error("sp_graph_set_weights: bad arguments");
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (g->directed) return undirected_only("sp_graph_set_weights");
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    const bool on_dev = flags & SP_PTR_DEVICE;
    const int64_t nnz = g->nnz;
    if (flags & SP_VALIDATE) {
        std::vector<int32_t> hr((size_t)g->n + 1), hc((size_t)nnz), hw;
        const int32_t *w = weights;
        SP_HIP(hipMemcpyAsync(hr.data(), g->row_ptr, hr.size() * 4, hipMemcpyDeviceToHost, st));
        if (nnz) SP_HIP(hipMemcpyAsync(hc.data(), g->col_idx, hc.size() * 4, hipMemcpyDeviceToHost, st));
        if (on_dev && nnz) {
            hw.resize((size_t)nnz);
            SP_HIP(hipMemcpyAsync(hw.data(), weights, hw.size() * 4, hipMemcpyDeviceToHost, st));
            w = hw.data();
        }
        SP_HIP(hipStreamSynchronize(st));
        if (!weights_symmetric(g->n, hr.data(), hc.data(), w)) return SP_ERR_INVALID_ARGUMENT;
    }
    SP_TRY(ensure_static_hubs(g, st));
    int2 *adjw = nullptr;
    int32_t *wdev = nullptr;
    unsigned int *bad = nullptr;  // bad[0]: count, bad[1]: largest weight (as int)
    auto cleanup = [&](sp_status code) {
        dev_free(adjw);
        dev_free(wdev);
        dev_free(bad);
        return code;
    };
    const size_t adj_bytes = sizeof(int2) * (size_t)std::max<int64_t>(nnz, 1);
    sp_status rc = dev_alloc((void **)&adjw, adj_bytes);
    if (rc == SP_OK) rc = dev_alloc((void **)&bad, 8);
    if (rc == SP_OK && !on_dev && nnz) rc = dev_alloc((void **)&wdev, (size_t)nnz * 4);
    if (rc != SP_OK) return cleanup(rc);
    unsigned int h_bad[2] = {0, 0};
    hipError_t e = hipMemsetAsync(bad, 0, 8, st);
    if (e == hipSuccess && wdev) e = hipMemcpyAsync(wdev, weights, (size_t)nnz * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz) {
        hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, st,
                           (const int32_t *)g->col_idx, (const int32_t *)(wdev ? wdev : weights), nnz,
                           adjw, bad, (int *)(bad + 1));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h_bad, bad, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error("weight upload failed: %s", hipGetErrorString(e));
        return cleanup(SP_ERR_DEVICE);
    }
    if (h_bad[0]) {
        set_error("%u weights lie outside [0, 2^31 - 2]", h_bad[0]);
        return cleanup(SP_ERR_INVALID_ARGUMENT);
    }
    dev_free(wdev);
    dev_free(bad);
    wdev = nullptr;
    bad = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        free_weights(g);
        g->adjw = adjw;
        g->max_weight = (int32_t)h_bad[1];
        g->weight_bytes = adj_bytes;
        g->bytes += g->weight_bytes;
    }
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_sssp(sp_graph g, int32_t source, int32_t *out_dist, const sp_sssp_config *cfg,
                  sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || !out_dist || source < 0 || source >= g->n) {
        set_error("sp_sssp: null graph/output or source out of range");
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (!g->adjw) {
        set_error("sp_sssp: the graph has no weights (sp_graph_set_weights)");
        return SP_ERR_INVALID_ARGUMENT;
    }
    SsspOpts o;
    if (cfg) {
        const bool bad = cfg->direction < SP_SSSP_AUTO || cfg->direction > SP_SSSP_PULL ||
                         (cfg->block_size != 0 && cfg->block_size != 128 && cfg->block_size != 256 &&
                          cfg->block_size != 512) ||
                         !(cfg->alpha >= 0.0) || std::isinf(cfg->alpha) ||
                         std::abs((int64_t)cfg->chunk_rounds) > 65536 || cfg->max_blocks < 0 ||
                         (cfg->local_hops < -1 || cfg->local_hops > 128 ||
                          (cfg->local_hops > 0 && (cfg->local_hops & (cfg->local_hops - 1)))) ||
                         cfg->reserved[0];
        if (bad) {
            set_error("sp_sssp: invalid configuration");
            return SP_ERR_INVALID_ARGUMENT;
        }
        o.forced = cfg->direction == SP_SSSP_PUSH ? SSSP_PUSH : cfg->direction == SP_SSSP_PULL ? SSSP_PULL : -1;
        if (cfg->block_size) o.block = cfg->block_size;
        if (cfg->alpha > 0) o.alpha = cfg->alpha;
        if (cfg->chunk_rounds) o.chunk_rounds = cfg->chunk_rounds;
        o.max_blocks = cfg->max_blocks;
        o.local_hops = cfg->local_hops;
    }
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    SsspWorkspace *ws = nullptr;
    SP_TRY(acquire_sssp_ws(g, &ws));
    struct Rel {
        sp_graph g;
        SsspWorkspace *ws;
        ~Rel() { release_sssp_ws(g, ws); }
    } rel{g, ws};
    SsspResult r;
    SP_HIP(hipEventRecord(ws->ev0, st));
    SP_TRY(sssp_run(g, *ws, source, out_dist, o, st, &r));
    SP_HIP(hipEventRecord(ws->ev1, st));
    SP_HIP(hipEventSynchronize(ws->ev1));
    float ms = 0.f;
    SP_HIP(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
    sp_sssp_stats &t = g_sssp_stats;
    t = sp_sssp_stats{};
    t.rounds = r.rounds;
    t.push_rounds = r.push_rounds;
    t.pull_rounds = r.pull_rounds;
    t.reached = r.reached;
    t.device_ms = ms;
    t.graph_launches = r.graph_launches;
    t.block_size = o.block;
    t.alpha = o.alpha;
    t.direction = o.forced == SSSP_PUSH ? SP_SSSP_PUSH : o.forced == SSSP_PULL ? SP_SSSP_PULL : SP_SSSP_AUTO;
    t.chunk_rounds = o.chunk_rounds;
    t.local_hops = sssp_local_hops(g, o.local_hops);
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_sssp_get_last_stats(sp_sssp_stats *out) {
    if (!out) return SP_ERR_INVALID_ARGUMENT;
    *out = g_sssp_stats;
    return SP_OK;
}

sp_status sp_pagerank(sp_graph g, double beta, double delta, int32_t max_iter, double *out_pr,
                      const sp_pagerank_config *cfg, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || (g->n > 0 && !out_pr) || !(beta >= 0.0) || std::isinf(beta) || !(delta >= 0.0 && delta <= 1.0) ||
        max_iter < 1) {
        set_error("sp_pagerank: null graph/output, beta < 0, delta outside [0, 1] or max_iter < 1");
        return SP_ERR_INVALID_ARGUMENT;
    }
    PrOpts o;
    if (cfg) {
        if ((cfg->block_size != 0 && cfg->block_size != 128 && cfg->block_size != 256 &&
             cfg->block_size != 512) ||
            std::abs((int64_t)cfg->chunk_iters) > 65536 || cfg->reserved[0] || cfg->reserved[1] ||
            cfg->reserved[2] || cfg->reserved[3]) {
            set_error("sp_pagerank: invalid configuration");
            return SP_ERR_INVALID_ARGUMENT;
        }
        if (cfg->block_size) o.block = cfg->block_size;
        if (cfg->chunk_iters) o.chunk_iters = cfg->chunk_iters;
    }
    g_pr_stats = sp_pagerank_stats{};
    if (g->n == 0) return SP_OK;
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    SP_TRY(ensure_pr_hubs(g, st));
    PrWorkspace *ws = nullptr;
    SP_TRY(acquire_pr_ws(g, &ws));
    struct Rel {
        sp_graph g;
        PrWorkspace *ws;
        ~Rel() { release_pr_ws(g, ws); }
    } rel{g, ws};
    PrResult r;
    SP_HIP(hipEventRecord(ws->ev0, st));
    SP_TRY(pr_run(g, *ws, beta, delta, max_iter, out_pr, o, st, &r));
    SP_HIP(hipEventRecord(ws->ev1, st));
    SP_HIP(hipEventSynchronize(ws->ev1));
    float ms = 0.f;
    SP_HIP(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
    g_pr_stats.iterations = r.iterations;
    g_pr_stats.graph_launches = r.graph_launches;
    g_pr_stats.diff = r.diff;
    g_pr_stats.device_ms = ms;
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_pagerank_get_last_stats(sp_pagerank_stats *out) {
    if (!out) return SP_ERR_INVALID_ARGUMENT;
    *out = g_pr_stats;
    return SP_OK;
}

sp_status sp_triangle_count(sp_graph g, int64_t *out_count, uint64_t *out_per_vertex, sp_stream s) {
    SP_GUARD_BEGIN
    clear_error();
    if (!g || !out_count) {
        set_error("sp_triangle_count: null graph or output");
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (g->directed) return undirected_only("sp_triangle_count");
    g_tc_stats = sp_tc_stats{};
    DeviceGuard dg(g->device);
    hipStream_t st = (hipStream_t)s;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    unsigned long long *d_total = nullptr;
    struct Cleanup {
        hipEvent_t *ev[3];
        unsigned long long **p;
        ~Cleanup() {
            for (auto *e : ev)
                if (*e) (void)hipEventDestroy(*e);
            dev_free(*p);
        }
    } cleanup{{&e0, &e1, &e2}, &d_total};
    SP_HIP(hipEventCreate(&e0));
    SP_HIP(hipEventCreate(&e1));
    SP_HIP(hipEventCreate(&e2));
    SP_TRY(dev_alloc((void **)&d_total, sizeof(unsigned long long)));
    const bool built = g->tc_orp != nullptr;
    SP_HIP(hipEventRecord(e0, st));
    SP_TRY(ensure_oriented(g, st));
    SP_HIP(hipEventRecord(e1, st));
    SP_TRY(tc_run(g, d_total, (unsigned long long *)out_per_vertex, st));
    SP_HIP(hipEventRecord(e2, st));
    unsigned long long total = 0;
    SP_HIP(hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, st));
    SP_HIP(hipStreamSynchronize(st));
    float b_ms = 0.f, c_ms = 0.f;
    SP_HIP(hipEventElapsedTime(&b_ms, e0, e1));
    SP_HIP(hipEventElapsedTime(&c_ms, e1, e2));
    *out_count = (int64_t)total;
    g_tc_stats.triangles = (int64_t)total;
    g_tc_stats.oriented_edges = g->tc_m;
    g_tc_stats.build_ms = built ? 0.0 : b_ms;
    g_tc_stats.count_ms = c_ms;
    return SP_OK;
    SP_GUARD_END
}

sp_status sp_tc_get_last_stats(sp_tc_stats *out) {
    if (!out) return SP_ERR_INVALID_ARGUMENT;
    *out = g_tc_stats;
    return SP_OK;
}

}  // extern "C"
