// Autotuner for the batched path: times candidate configurations on a sample
// of the caller's sources, grouped and batched as sp_bc_batch would run them,
// and keeps the fastest per graph and per graph fingerprint.
//
// Search: coordinate descent from the built-in defaults, one field at a time:
// block size {256, 128}, batch width {32, 48}, the top-down -> bottom-up
// threshold alpha {4, 60} and the bottom-up -> top-down threshold beta
// {8, 96} (only where bottom-up levels can run), levels per captured chunk
// {16, 32}.  Each candidate runs the sample once untimed and twice timed
// (HIP events); the faster repetition, per source, is its score, and it
// replaces the running best only when 2% faster.
#include <chrono>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <unordered_map>
#include <vector>

#include "common.h"

using namespace sp;

namespace {

constexpr int kTimedReps = 2;
constexpr int32_t kSampleMax = 2 * kSlots;
constexpr double kMargin = 0.98;

thread_local sp_tune_report g_report;

// ---------------------------------------------------------------------------
// Fingerprint cache
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;
std::unordered_map<uint64_t, sp_batch_config> g_cache;
bool g_cache_file_read = false;

const char *cache_path() {
    const char *p = std::getenv("SP_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Lines "fingerprint width block alpha beta chunk_levels [engine]"; later
// lines win.
void read_cache_file_locked() {
    if (g_cache_file_read) return;
    g_cache_file_read = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long fp = 0;
        sp_batch_config c{};
        if (std::sscanf(line, "%llx %d %d %lf %lf %d %d", &fp, &c.batch_width, &c.block_size, &c.alpha,
                        &c.beta, &c.chunk_levels, &c.engine) >= 6 &&
            check_batch_cfg(&c) == SP_OK)
            g_cache[(uint64_t)fp] = c;
    }
    std::fclose(f);
    clear_error();
}

uint64_t mix(uint64_t h, uint64_t x) {
    // one splitmix64 finalisation per word folded in
    h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h ^= h >> 30;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 27;
    h *= 0x94d049bb133111ebull;
    h ^= h >> 31;
    return h;
}

uint64_t degree_stats(uint64_t h, const int32_t *deg, int32_t n) {
    uint64_t hist[33] = {};
    unsigned long long sq = 0;
    int32_t md = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = deg[v];
        md = std::max(md, d);
        sq += (unsigned long long)d * (unsigned long long)d;
        hist[d > 0 ? 32 - __builtin_clz((unsigned)d) : 0]++;
    }
    h = mix(h, (uint64_t)md);
    h = mix(h, (uint64_t)sq);
    for (uint64_t b : hist) h = mix(h, b);
    return h;
}

sp_status time_config(sp_graph g, BatchWorkspace &ws, const int32_t *src, int32_t n, int32_t width,
                      const BatchRunOpts &o, hipStream_t s, double *ms_per_source) {
    hipEvent_t e0, e1;
    SP_HIP(hipEventCreate(&e0));
    SP_HIP(hipEventCreate(&e1));
    struct Rel {
        hipEvent_t a, b;
        ~Rel() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } rel{e0, e1};
    double best = 0.0;
    for (int rep = 0; rep <= kTimedReps; ++rep) {  // rep 0 warms up (captures, workspace growth)
        SP_HIP(hipEventRecord(e0, s));
        for (int32_t b = 0; b < n; b += width) {
            BatchResult r;
            SP_TRY(batch_run(g, ws, src + b, std::min(width, n - b), nullptr, o, s, &r));
        }
        SP_HIP(hipEventRecord(e1, s));
        SP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0 && (rep == 1 || ms < best)) best = ms;
    }
    *ms_per_source = best / std::max(n, 1);
    return SP_OK;
}

BatchRunOpts opts_of(sp_graph g, const sp_batch_config &c) {
    BatchRunOpts o;
    o.block = c.block_size;
    o.alpha = c.alpha;
    o.beta = c.beta;
    o.chunk_levels = c.chunk_levels;
    o.engine = c.engine ? c.engine : sp::auto_engine(g);
    return o;
}

}  // namespace

namespace sp {

uint64_t graph_fingerprint(const sp_graph_s *g, const int32_t *in_deg) {
    uint64_t h = mix(0x5350u, (uint64_t)(uint32_t)g->n);
    h = mix(h, (uint64_t)g->nnz);
    h = mix(h, (uint64_t)(in_deg != nullptr));
    h = degree_stats(h, g->host_deg.data(), g->n);
    if (in_deg) h = degree_stats(h, in_deg, g->n);
    return h;
}

bool tune_cache_lookup(uint64_t fp, sp_batch_config *out) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    read_cache_file_locked();
    auto it = g_cache.find(fp);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

void tune_cache_store(uint64_t fp, const sp_batch_config &c) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    read_cache_file_locked();
    g_cache[fp] = c;
    if (const char *path = cache_path()) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%016" PRIx64 " %d %d %.17g %.17g %d %d\n", fp, c.batch_width, c.block_size,
                         c.alpha, c.beta, c.chunk_levels, c.engine);
            std::fclose(f);
        }
    }
}

}  // namespace sp

extern "C" sp_status sp_autotune(sp_graph g, const int32_t *sources, int32_t n_sources,
                                 sp_batch_config *out, sp_stream s) {
    try {
        clear_error();
        if (!g || !out || n_sources < 1 || !sources) {
            set_error("sp_autotune: need a graph, an output and at least one source");
            return SP_ERR_INVALID_ARGUMENT;
        }
        for (int32_t i = 0; i < n_sources; ++i)
            if (sources[i] < 0 || sources[i] >= g->n) {
                set_error("sources[%d] out of range", i);
                return SP_ERR_INVALID_ARGUMENT;
            }
        const auto t0 = std::chrono::steady_clock::now();
        auto elapsed_ms = [&] {
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        };
        sp_tune_report rep{};
        rep.fingerprint = g->fingerprint;
        rep.repetitions = kTimedReps;
        sp_batch_config cached{};
        if (tune_cache_lookup(g->fingerprint, &cached)) {
            {
                std::lock_guard<std::mutex> lk(g->mu);
                g->tuned.valid = true;
                g->tuned.cfg = cached;
            }
            rep.from_cache = 1;
            rep.chosen = cached;
            rep.tuning_ms = elapsed_ms();
            g_report = rep;
            *out = cached;
            return SP_OK;
        }
        hipStream_t st = (hipStream_t)s;
        // The sample: up to kSampleMax consecutive sources of the grouped
        // order, from its middle, starting at a batch boundary.
        std::vector<int32_t> order;
        SP_TRY(source_groups(g, sources, n_sources, kDefaultWidth, st, order, &rep.group_ms));
        const int32_t n = std::min(n_sources, kSampleMax);
        const int32_t first = (n_sources - n) / 2 / kDefaultWidth * kDefaultWidth;
        std::vector<int32_t> sample(n);
        for (int32_t i = 0; i < n; ++i) sample[i] = sources[order[first + i]];
        rep.sample_sources = n;

        BatchWorkspace *ws = nullptr;
        const int32_t engine = auto_engine(g);  // the engine is not searched
        SP_TRY(acquire_batch_ws(g, kSlots, engine, &ws));
        struct Rel {
            sp_graph g;
            BatchWorkspace *ws;
            ~Rel() { release_batch_ws(g, ws); }
        } rel{g, ws};

        sp_batch_config best{};
        best.engine = engine;
        best.batch_width = kDefaultWidth;
        best.block_size = engine == SP_ENGINE_BLOCKS ? kDefaultBlocksEngineBlock : kDefaultBlock;
        best.alpha = kDefaultAlpha;
        best.beta = kDefaultBeta;
        best.chunk_levels = kDefaultChunkLevels;
        auto record = [&](const sp_batch_config &c, double ms, bool accepted) {
            if (rep.n_candidates >= SP_TUNE_MAX_CANDIDATES) return;
            sp_tune_candidate &k = rep.cand[rep.n_candidates++];
            k.cfg = c;
            k.ms_per_source = ms;
            k.accepted = accepted ? 1 : 0;
        };
        double best_ms = 0;
        SP_TRY(time_config(g, *ws, sample.data(), n, best.batch_width, opts_of(g, best), st, &best_ms));
        record(best, best_ms, true);
        auto try_field = [&](auto setter, const std::vector<double> &values) -> sp_status {
            for (double v : values) {
                sp_batch_config c = best;
                setter(c, v);
                double ms = 0;
                SP_TRY(time_config(g, *ws, sample.data(), n, c.batch_width, opts_of(g, c), st, &ms));
                const bool win = ms < best_ms * kMargin;
                record(c, ms, win);
                if (win) {
                    best_ms = ms;
                    best = c;
                }
            }
            return SP_OK;
        };
        if (engine == SP_ENGINE_BLOCKS)
            SP_TRY(try_field([](sp_batch_config &c, double v) { c.block_size = (int32_t)v; }, {512, 256}));
        else
            SP_TRY(try_field([](sp_batch_config &c, double v) { c.block_size = (int32_t)v; }, {256, 128}));
        SP_TRY(try_field([](sp_batch_config &c, double v) { c.batch_width = (int32_t)v; }, {32, 48}));
        if (engine == SP_ENGINE_BITMAP) {  // the other fields do not apply to the blocks engine
            if (g->max_degree > 8) {  // bottom-up levels never run on sparser graphs
                SP_TRY(try_field([](sp_batch_config &c, double v) { c.alpha = v; }, {4, 60}));
                SP_TRY(try_field([](sp_batch_config &c, double v) { c.beta = v; }, {8, 96}));
            }
            SP_TRY(try_field([](sp_batch_config &c, double v) { c.chunk_levels = (int32_t)v; }, {16, 32}));
        }
        {
            std::lock_guard<std::mutex> lk(g->mu);
            g->tuned.valid = true;
            g->tuned.cfg = best;
        }
        tune_cache_store(g->fingerprint, best);
        rep.chosen = best;
        rep.tuning_ms = elapsed_ms();
        g_report = rep;
        *out = best;
        return SP_OK;
    } catch (...) {
        set_error("sp_autotune: unexpected failure");
        return SP_ERR_DEVICE;
    }
}

extern "C" sp_status sp_autotune_get_last_report(sp_tune_report *out) {
    if (!out) {
        set_error("sp_autotune_get_last_report: null output");
        return SP_ERR_INVALID_ARGUMENT;
    }
    *out = g_report;
    return SP_OK;
}

extern "C" sp_status sp_graph_fingerprint(sp_graph g, uint64_t *out) {
    if (!g || !out) {
        set_error("sp_graph_fingerprint: null argument");
        return SP_ERR_INVALID_ARGUMENT;
    }
    *out = g->fingerprint;
    return SP_OK;
}

extern "C" sp_status sp_graph_set_tuned(sp_graph g, const sp_batch_config *cfg) {
    clear_error();
    if (!g) {
        set_error("sp_graph_set_tuned: null graph");
        return SP_ERR_INVALID_ARGUMENT;
    }
    SP_TRY(check_batch_cfg(cfg));
    std::lock_guard<std::mutex> lk(g->mu);
    g->tuned = TuneEntry{};
    if (cfg) {
        g->tuned.valid = true;
        g->tuned.cfg = *cfg;
    }
    return SP_OK;
}

extern "C" sp_status sp_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.clear();
    g_cache_file_read = true;  // the file is not read again in this process
    return SP_OK;
}
