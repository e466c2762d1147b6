// Serving loop: continuous batching of BC requests over several resident
// graphs.
//
// A request is (graph, source list, output BC array).  Its sources queue per
// graph in arrival order.  Worker threads, one HIP stream each, repeatedly
// take the graph with the oldest waiting source, fill one multi-source pass
// (up to max_batch slots) with waiting sources of that graph -- possibly from
// several requests -- and run it; passes on different workers overlap on the
// device.  Requests that arrive while others run join the next pass that has
// room.  A pass needs a workspace for its graph; workspaces are admitted
// against the memory budget and kept for reuse (the idle ones of other graphs
// are freed first when the budget is tight).
//
// A request's sources are cut into chunks of max_batch consecutive sources
// (the last may be shorter), fixed at submission.  A pass takes whole chunks
// only, possibly of several requests, and several chunks of one request may
// be on the device at once, on different workers (up to n_streams chunks
// past the last one merged).  Chunk 0 accumulates into the request's output;
// chunk c >= 1 into a V-double buffer of the graph's pool, which is added
// into the output once chunks 0..c-1 have been (in chunk order, by whichever
// worker finishes the chunk that completes the prefix).
//
// Result independence: each slot's delta depends only on its own source, a
// chunk's slots are reduced in ascending order into a buffer that starts at
// zero, and chunk sums are added in chunk order, so every request's BC is
// ((chunk 0) + chunk 1) + ... over a cut of its own source list: bit-identical
// alone and in a mix, whatever else shares its passes.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <new>
#include <thread>

#include "common.h"

namespace {

using Clock = std::chrono::steady_clock;

}  // namespace

struct sp_request_s {
    sp_server_s *srv = nullptr;
    int32_t graph_id = -1;
    std::vector<int32_t> sources;
    double *out_bc = nullptr;
    int32_t chunk = 64;        // sources per chunk
    int32_t n_chunks = 0;
    int32_t next_chunk = 0;    // first chunk not yet given to a pass
    int32_t merged = 0;        // chunks added into out_bc (chunk order)
    int32_t in_flight = 0;     // chunks on the device
    bool merging = false;      // a worker is adding finished chunks into out_bc
    std::vector<double *> part;     // chunk c >= 1: its BC buffer while unmerged
    std::vector<char> chunk_done;   // chunk c's pass finished
    bool finished = false;
    bool cancelled = false;
    sp_status status = SP_OK;
    std::string error;         // detail of a failure, handed to the waiting thread
    Clock::time_point t_submit, t_done;
    std::condition_variable cv;
};

struct GraphSlot {
    sp_graph g = nullptr;
    std::deque<sp_request> waiting;  // requests with chunks left, arrival order
    std::vector<sp::BatchWorkspace *> idle;
    std::vector<double *> free_parts;  // V-double chunk buffers for reuse
    Clock::time_point last_used;
};

struct sp_server_s {
    sp_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable work_cv;
    std::deque<GraphSlot> graphs;  // deque: references stay valid as graphs are added
    std::vector<std::thread> workers;
    bool stopping = false;
    size_t admitted = 0;  // bytes of workspaces held (idle + in use)
    int held = 0;         // workspaces taken by workers (being created or running)
    sp_server_stats stats{};
};

namespace sp {

static int32_t pending_sources(const sp_server_s *srv) {
    int64_t n = 0;
    for (const auto &gs : srv->graphs)
        for (auto *r : gs.waiting)
            n += std::max<int64_t>(0, (int64_t)r->sources.size() - (int64_t)r->next_chunk * r->chunk);
    return (int32_t)std::min<int64_t>(n, INT32_MAX);
}

static int32_t chunk_size(const sp_request_s *r, int32_t c) {
    return std::min<int32_t>(r->chunk, (int32_t)r->sources.size() - c * r->chunk);
}

// A request's next chunk may start: it has one, and at most n_streams chunks
// lie between the merge point and it (bounds its chunk buffers).
static bool can_start(const sp_server_s *srv, const sp_request_s *r) {
    return r->status >= 0 && r->next_chunk < r->n_chunks && r->next_chunk < r->merged + srv->cfg.n_streams;
}

// Pick the graph whose oldest request with a chunk that may start arrived first.
static int pick_graph(sp_server_s *srv) {
    int best = -1;
    Clock::time_point bt{};
    for (size_t i = 0; i < srv->graphs.size(); ++i)
        for (auto *r : srv->graphs[i].waiting) {
            if (!can_start(srv, r)) continue;
            if (best < 0 || r->t_submit < bt) {
                best = (int)i;
                bt = r->t_submit;
            }
            break;  // only the first eligible request of each graph matters
        }
    return best;
}

__global__ void k_add_f64(double *dst, const double *__restrict__ src, int32_t n) {
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) dst[v] += src[v];
}

// Make room for `need` more bytes by freeing idle workspaces of other graphs.
static bool admit(sp_server_s *srv, size_t need, int keep_graph) {
    for (size_t i = 0; i < srv->graphs.size() && srv->admitted + need > srv->cfg.memory_budget; ++i) {
        GraphSlot &o = srv->graphs[i];  // pooled chunk buffers go first
        while (!o.free_parts.empty() && srv->admitted + need > srv->cfg.memory_budget) {
            dev_free(o.free_parts.back());
            o.free_parts.pop_back();
            srv->admitted -= (size_t)std::max(o.g->n, 1) * 8;
        }
    }
    while (srv->admitted + need > srv->cfg.memory_budget) {
        int victim = -1;
        for (size_t i = 0; i < srv->graphs.size(); ++i) {
            if ((int)i == keep_graph || srv->graphs[i].idle.empty()) continue;
            if (victim < 0 || srv->graphs[i].last_used < srv->graphs[victim].last_used) victim = (int)i;
        }
        if (victim < 0) return false;
        BatchWorkspace *ws = srv->graphs[victim].idle.back();
        srv->graphs[victim].idle.pop_back();
        srv->admitted -= ws->bytes;
        srv->stats.workspaces_evicted++;
        batch_ws_destroy(*ws);
        delete ws;
    }
    return true;
}

static void finish_request(sp_server_s *srv, sp_request r, sp_status st) {
    r->status = st;
    r->t_done = Clock::now();
    __atomic_store_n(&r->finished, true, __ATOMIC_RELEASE);
    if (st < 0) srv->stats.failed++; else srv->stats.completed++;
    r->cv.notify_all();
}

// Fail the waiting requests at the front of gs's queue that have nothing on
// the device; their chunk buffers go back to the pool.
static void fail_idle_waiting(sp_server_s *srv, GraphSlot &gs, sp_status st, const std::string &why) {
    while (!gs.waiting.empty() && gs.waiting.front()->in_flight == 0) {
        sp_request r = gs.waiting.front();
        gs.waiting.pop_front();
        for (double *&b : r->part)
            if (b) {
                gs.free_parts.push_back(b);
                b = nullptr;
            }
        r->error = why;
        finish_request(srv, r, st);
    }
}

static void worker_main(sp_server_s *srv) {
    (void)hipSetDevice(srv->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        int gi = -1;
        srv->work_cv.wait(lk, [&] {
            if (srv->stopping && pending_sources(srv) == 0) return true;
            gi = pick_graph(srv);
            return gi >= 0;
        });
        if (gi < 0) break;  // stopping and drained
        GraphSlot &gs = srv->graphs[gi];
        sp_graph g = gs.g;
        int32_t width = 0;
        BatchRunOpts o = resolve_batch(g, nullptr, &width);
        width = srv->cfg.max_batch;  // passes are filled with whole chunks of up to max_batch
        // Workers launch level chunks directly: a hipGraph capture on one
        // worker's stream while other workers launch and allocate has failed
        // their calls (the runtime's legacy-stream dependency check), and
        // capture saves little here (deep road passes run the blocks engine,
        // which captures nothing).
        o.chunk_levels = -std::max(1, std::abs(o.chunk_levels));
        // Workspace: reuse an idle one of this graph, else admit a new one.
        BatchWorkspace *ws = nullptr;
        if (!gs.idle.empty()) {
            ws = gs.idle.back();
            gs.idle.pop_back();
            srv->held++;
        } else {
            const size_t need = batch_ws_bytes(g, initial_qcap(g->n, kSlots), kSlots, o.engine);
            if (!admit(srv, need, gi)) {
                // Memory is held by other workers: wait for one to return it.
                // With none held every workspace is idle and freeable, so
                // admission only fails if one pass exceeds the budget, which
                // submit already rejects; fail defensively.
                if (srv->held == 0) {
                    fail_idle_waiting(srv, gs, SP_ERR_OUT_OF_MEMORY,
                                      "a pass's workspace does not fit the server's memory budget");
                    continue;
                }
                srv->work_cv.wait(lk);
                continue;
            }
            srv->admitted += need;
            srv->held++;
            srv->stats.workspaces_created++;
            srv->stats.admitted_bytes = srv->admitted;
            srv->stats.peak_admitted_bytes = std::max(srv->stats.peak_admitted_bytes, srv->admitted);
            lk.unlock();
            ws = new (std::nothrow) BatchWorkspace;
            sp_status st = ws ? batch_ws_create(g, initial_qcap(g->n, kSlots), kSlots, o.engine, *ws)
                              : SP_ERR_OUT_OF_MEMORY;
            lk.lock();
            if (st < 0) {
                if (ws) {
                    batch_ws_destroy(*ws);
                    delete ws;
                }
                srv->admitted -= need;
                srv->held--;
                fail_idle_waiting(srv, gs, st, sp_last_error());
                srv->work_cv.notify_all();
                continue;
            }
            ws->bytes = need;
        }
        // Fill the pass with whole chunks of this graph's waiting requests, in
        // arrival order (a chunk that does not fit the room left is skipped).
        std::vector<int32_t> srcs;
        std::vector<double *> outs;
        struct Part {
            sp_request r;
            int32_t c;      // chunk index
            int32_t count;  // its sources (= its slots in this pass)
            double *dst;    // its accumulation buffer
        };
        std::vector<Part> parts;
        bool no_buffer = false;
        for (auto *r : gs.waiting) {
            while (can_start(srv, r)) {
                const int32_t c = r->next_chunk, cnt = chunk_size(r, c);
                if ((int32_t)srcs.size() + cnt > width) break;
                double *dst = r->out_bc;
                if (c > 0) {
                    // A pooled buffer, else a new one admitted against the
                    // budget; over budget only when the pass has nothing
                    // else to run (so every request keeps making progress).
                    const size_t pb = (size_t)std::max(g->n, 1) * 8;
                    if (!gs.free_parts.empty()) {
                        dst = gs.free_parts.back();
                        gs.free_parts.pop_back();
                    } else if ((admit(srv, pb, gi) || srcs.empty()) &&
                               dev_alloc((void **)&dst, pb) == SP_OK) {
                        srv->admitted += pb;
                        srv->stats.peak_admitted_bytes = std::max(srv->stats.peak_admitted_bytes, srv->admitted);
                    } else {
                        no_buffer = true;
                        break;
                    }
                    r->part[c] = dst;
                }
                parts.push_back({r, c, cnt, dst});
                for (int32_t k = 0; k < cnt; ++k) {
                    srcs.push_back(r->sources[c * r->chunk + k]);
                    outs.push_back(dst);
                }
                r->next_chunk++;
                r->in_flight++;
            }
            if ((int32_t)srcs.size() >= width || no_buffer) break;
        }
        if (srcs.empty()) {  // nothing fits now (taken by another worker, or no buffer memory)
            gs.idle.push_back(ws);
            srv->held--;
            if (no_buffer) srv->work_cv.wait_for(lk, std::chrono::milliseconds(1));
            srv->work_cv.notify_all();
            continue;
        }
        // Requests whose every chunk is now assigned leave the waiting list.
        gs.waiting.erase(std::remove_if(gs.waiting.begin(), gs.waiting.end(),
                                        [](sp_request r) { return r->next_chunk >= r->n_chunks; }),
                         gs.waiting.end());
        srv->stats.in_flight++;
        srv->stats.passes++;
        srv->stats.slots_used += (int64_t)srcs.size();
        srv->stats.queue_depth = pending_sources(srv);
        lk.unlock();

        sp_status st = SP_OK;
        clear_error();
        for (auto &p : parts)  // every chunk sums into a buffer that starts at zero
            if (st >= 0) st = launch_fill_f64(p.dst, g->n, 0.0, stream);
        BatchResult res;
        if (st >= 0) st = batch_run(g, *ws, srcs.data(), (int32_t)srcs.size(), outs.data(), o, stream, &res);
        if (st >= 0 && hipStreamSynchronize(stream) != hipSuccess) {
            set_error("serving pass: stream synchronisation failed");
            st = SP_ERR_DEVICE;
        }
        const std::string err = st < 0 ? std::string(sp_last_error()) : std::string();

        lk.lock();
        srv->stats.in_flight--;
        srv->held--;
        if (ws->bytes != batch_ws_bytes(g, ws->qcap, ws->width, ws->engine)) {  // the queue grew
            const size_t now = batch_ws_bytes(g, ws->qcap, ws->width, ws->engine);
            srv->admitted = srv->admitted - ws->bytes + now;
            ws->bytes = now;
            srv->stats.peak_admitted_bytes = std::max(srv->stats.peak_admitted_bytes, srv->admitted);
        }
        gs.idle.push_back(ws);
        gs.last_used = Clock::now();
        int32_t slot0 = 0;  // the part's slots are [slot0, slot0 + count)
        std::vector<sp_request> touched;
        for (auto &p : parts) {
            sp_request r = p.r;
            r->in_flight--;
            r->chunk_done[p.c] = 1;
            const unsigned long long mine =
                (p.count >= 64 ? ~0ull : ((1ull << p.count) - 1ull)) << slot0;
            slot0 += p.count;
            if (st < 0) {
                if (r->status >= 0) r->error = err;
                r->status = st;
            } else if (r->status >= 0 && (res.flagged_mask & mine)) {
                r->status |= SP_WARN_SIGMA_LARGE;  // only the request that owns the slot
            }
            srv->stats.edges_traversed += (int64_t)p.count * (g->nnz / 2);
            if (std::find(touched.begin(), touched.end(), r) == touched.end()) touched.push_back(r);
        }
        // Add finished chunks into each touched request's output in chunk
        // order; finish the request when all are in (or, after a failure,
        // when none is left on the device).
        for (sp_request r : touched) {
            if (r->status < 0)
                gs.waiting.erase(std::remove(gs.waiting.begin(), gs.waiting.end(), r), gs.waiting.end());
            if (!r->merging) {
                r->merging = true;
                while (r->status >= 0 && r->merged < r->n_chunks && r->chunk_done[r->merged]) {
                    const int32_t c = r->merged;
                    if (c > 0) {
                        double *src = r->part[c];
                        lk.unlock();
                        hipLaunchKernelGGL(k_add_f64, dim3(grid_for(g->n, 256, 2048)), dim3(256), 0, stream,
                                           r->out_bc, (const double *)src, g->n);
                        hipError_t e = hipGetLastError();
                        if (e == hipSuccess) e = hipStreamSynchronize(stream);
                        lk.lock();
                        if (e != hipSuccess) {
                            r->error = "serving: adding a chunk's BC failed";
                            r->status = SP_ERR_DEVICE;
                            break;
                        }
                        gs.free_parts.push_back(src);
                        r->part[c] = nullptr;
                    }
                    r->merged++;
                }
                r->merging = false;
            }
            const bool complete = r->status >= 0 && r->merged == r->n_chunks;
            const bool failed_and_idle = r->status < 0 && r->in_flight == 0 && !r->merging;
            if ((complete || failed_and_idle) && !r->finished) {
                for (double *&b : r->part)
                    if (b) {
                        gs.free_parts.push_back(b);
                        b = nullptr;
                    }
                finish_request(srv, r, r->status);
            }
        }
        srv->stats.admitted_bytes = srv->admitted;
        srv->work_cv.notify_all();
    }
    lk.unlock();
    (void)hipStreamDestroy(stream);
}

}  // namespace sp

using namespace sp;

extern "C" {

sp_status sp_server_create(const sp_server_config *cfg, sp_server *out) {
    try {
        clear_error();
        if (!out) return SP_ERR_INVALID_ARGUMENT;
        sp_server_config c{};
        if (cfg) c = *cfg;
        for (int r : c.reserved)
            if (r) {
                set_error("reserved fields must be zero");
                return SP_ERR_INVALID_ARGUMENT;
            }
        if (c.max_batch < 0 || c.max_batch > kSlots || c.n_streams < 0 || c.n_streams > 8) {
            set_error("max_batch must be 0..64 and n_streams 0..8");
            return SP_ERR_INVALID_ARGUMENT;
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            set_error("no HIP device");
            return SP_ERR_NOT_SUPPORTED;
        }
        if (!c.max_batch) c.max_batch = kSlots;
        if (!c.n_streams) c.n_streams = 4;
        if (!c.memory_budget) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return SP_ERR_DEVICE;
            c.memory_budget = fr / 4;
        }
        auto *srv = new sp_server_s;
        srv->cfg = c;
        srv->device = dev;
        for (int i = 0; i < c.n_streams; ++i) srv->workers.emplace_back(worker_main, srv);
        *out = srv;
        return SP_OK;
    } catch (...) {
        set_error("server creation failed");
        return SP_ERR_OUT_OF_MEMORY;
    }
}

sp_status sp_server_add_graph(sp_server srv, sp_graph g, int32_t *graph_id) {
    if (!srv || !g || !graph_id) return SP_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return SP_ERR_REJECTED;
    GraphSlot gs;
    gs.g = g;
    gs.last_used = Clock::now();
    srv->graphs.push_back(std::move(gs));
    *graph_id = (int32_t)srv->graphs.size() - 1;
    return SP_OK;
}

sp_status sp_stream_submit(sp_server srv, int32_t graph_id, const int32_t *sources, int32_t n_sources,
                           double *out_bc, sp_request *out_req) {
    try {
        clear_error();
        if (!srv || !out_req || n_sources < 0 || (n_sources > 0 && !sources)) {
            set_error("sp_stream_submit: bad arguments");
            return SP_ERR_INVALID_ARGUMENT;
        }
        std::unique_lock<std::mutex> lk(srv->mu);
        if (graph_id < 0 || graph_id >= (int32_t)srv->graphs.size()) {
            set_error("unknown graph id %d", graph_id);
            return SP_ERR_INVALID_ARGUMENT;
        }
        sp_graph g = srv->graphs[graph_id].g;
        if (g->n > 0 && !out_bc) {
            set_error("null output");
            return SP_ERR_INVALID_ARGUMENT;
        }
        for (int32_t i = 0; i < n_sources; ++i)
            if (sources[i] < 0 || sources[i] >= g->n) {
                set_error("sources[%d] = %d outside [0, %d)", i, sources[i], g->n);
                return SP_ERR_INVALID_ARGUMENT;
            }
        if (srv->stopping) {
            srv->stats.rejected++;
            set_error("server is shutting down");
            return SP_ERR_REJECTED;
        }
        int32_t width = 0;
        const BatchRunOpts o = resolve_batch(g, nullptr, &width);
        const size_t need = batch_ws_bytes(g, initial_qcap(g->n, kSlots), kSlots, o.engine);
        if (need > srv->cfg.memory_budget) {
            srv->stats.rejected++;
            set_error("one pass on this graph needs %zu bytes, budget is %zu", need,
                      srv->cfg.memory_budget);
            return SP_ERR_REJECTED;
        }
        auto *r = new sp_request_s;
        r->srv = srv;
        r->graph_id = graph_id;
        r->sources.assign(sources, sources + n_sources);
        r->out_bc = out_bc;
        r->chunk = srv->cfg.max_batch;
        r->n_chunks = (n_sources + r->chunk - 1) / r->chunk;
        r->part.assign(r->n_chunks, nullptr);
        r->chunk_done.assign(r->n_chunks, 0);
        r->t_submit = Clock::now();
        srv->stats.submitted++;
        if (n_sources == 0 || g->n == 0) {
            lk.unlock();
            sp_status st = SP_OK;
            if (g->n > 0) {
                st = launch_fill_f64(out_bc, g->n, 0.0, nullptr);
                if (st >= 0 && hipDeviceSynchronize() != hipSuccess) st = SP_ERR_DEVICE;
            }
            lk.lock();
            finish_request(srv, r, st);
        } else {
            srv->graphs[graph_id].waiting.push_back(r);
            srv->stats.queue_depth = pending_sources(srv);
            srv->work_cv.notify_all();
        }
        *out_req = r;
        return SP_OK;
    } catch (...) {
        set_error("submit failed");
        return SP_ERR_OUT_OF_MEMORY;
    }
}

sp_status sp_request_wait(sp_request r, int64_t timeout_us, sp_status *result) {
    if (!r) return SP_ERR_INVALID_ARGUMENT;
    if (!__atomic_load_n(&r->finished, __ATOMIC_ACQUIRE)) {
        std::unique_lock<std::mutex> lk(r->srv->mu);
        auto ready = [&] { return r->finished; };
        if (timeout_us < 0) {
            r->cv.wait(lk, ready);
        } else if (!r->cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
            return SP_ERR_TIMEOUT;
        }
    }
    if (result) *result = r->cancelled ? SP_ERR_CANCELLED : r->status;
    if (!r->cancelled && r->status < 0 && !r->error.empty()) set_error("%s", r->error.c_str());
    return SP_OK;
}

sp_status sp_request_cancel(sp_request r) {
    if (!r) return SP_ERR_INVALID_ARGUMENT;
    if (__atomic_load_n(&r->finished, __ATOMIC_ACQUIRE)) return SP_ERR_REJECTED;
    sp_server_s *srv = r->srv;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (r->next_chunk > 0 || r->finished) return SP_ERR_REJECTED;
    auto &w = srv->graphs[r->graph_id].waiting;
    w.erase(std::remove(w.begin(), w.end(), r), w.end());
    r->cancelled = true;
    r->status = SP_ERR_CANCELLED;
    r->t_done = Clock::now();
    srv->stats.cancelled++;
    __atomic_store_n(&r->finished, true, __ATOMIC_RELEASE);
    r->cv.notify_all();
    return SP_OK;
}

sp_status sp_request_poll(sp_request r, int32_t *done, sp_status *result) {
    if (!r || !done) return SP_ERR_INVALID_ARGUMENT;
    const bool f = __atomic_load_n(&r->finished, __ATOMIC_ACQUIRE);
    *done = f ? 1 : 0;
    if (f && result) *result = r->cancelled ? SP_ERR_CANCELLED : r->status;
    if (f && !r->cancelled && r->status < 0 && !r->error.empty()) set_error("%s", r->error.c_str());
    return SP_OK;
}

sp_status sp_request_latency_us(sp_request r, double *latency_us) {
    if (!r || !latency_us) return SP_ERR_INVALID_ARGUMENT;
    if (!__atomic_load_n(&r->finished, __ATOMIC_ACQUIRE)) return SP_ERR_TIMEOUT;
    *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    return SP_OK;
}

sp_status sp_request_release(sp_request r) {
    if (!r) return SP_OK;
    if (!__atomic_load_n(&r->finished, __ATOMIC_ACQUIRE)) {
        set_error("request still running");
        return SP_ERR_INVALID_ARGUMENT;
    }
    delete r;
    return SP_OK;
}

sp_status sp_server_get_stats(sp_server srv, sp_server_stats *out) {
    if (!srv || !out) return SP_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.queue_depth = pending_sources(srv);
    srv->stats.admitted_bytes = srv->admitted;
    *out = srv->stats;
    return SP_OK;
}

sp_status sp_server_destroy(sp_server srv) {
    if (!srv) return SP_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->work_cv.notify_all();
    }
    for (auto &t : srv->workers) t.join();
    (void)hipSetDevice(srv->device);
    for (auto &gs : srv->graphs) {
        for (auto *ws : gs.idle) {
            batch_ws_destroy(*ws);
            delete ws;
        }
        for (double *b : gs.free_parts) dev_free(b);
    }
    delete srv;
    return SP_OK;
}

}  // extern "C"
