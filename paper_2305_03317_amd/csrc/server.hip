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
// Result independence: a request never has two passes in flight, its sources
// occupy slots in list order, and the BC reduction adds slots in ascending
// order per vertex, so every request's BC is accumulated per vertex in its
// own source-list order whatever else shares its passes.  Each slot's delta
// depends only on its own source (batch_path.hip), so a request's result is
// bit-identical alone and in a mix.
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
    int32_t next = 0;          // first source not yet given to a pass
    int32_t done_sources = 0;  // sources whose pass finished
    bool in_flight = false;
    bool started = false;      // output zeroed, first pass issued
    bool finished = false;
    bool cancelled = false;
    sp_status status = SP_OK;
    std::string error;         // detail of a failure, handed to the waiting thread
    Clock::time_point t_submit, t_done;
    std::condition_variable cv;
};

struct GraphSlot {
    sp_graph g = nullptr;
    std::deque<sp_request> waiting;  // requests with sources left, arrival order
    std::vector<sp::BatchWorkspace *> idle;
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
        for (auto *r : gs.waiting) n += (int64_t)r->sources.size() - r->next;
    return (int32_t)std::min<int64_t>(n, INT32_MAX);
}

// Pick the graph whose oldest waiting request (not in flight) arrived first.
static int pick_graph(sp_server_s *srv) {
    int best = -1;
    Clock::time_point bt{};
    for (size_t i = 0; i < srv->graphs.size(); ++i)
        for (auto *r : srv->graphs[i].waiting) {
            if (r->in_flight) continue;
            if (best < 0 || r->t_submit < bt) {
                best = (int)i;
                bt = r->t_submit;
            }
            break;  // only the first eligible request of each graph matters
        }
    return best;
}

// Make room for `need` more bytes by freeing idle workspaces of other graphs.
static bool admit(sp_server_s *srv, size_t need, int keep_graph) {
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
        const BatchRunOpts o = resolve_batch(g, nullptr, &width);
        width = std::min(width, srv->cfg.max_batch);
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
                    while (!gs.waiting.empty() && !gs.waiting.front()->in_flight) {
                        sp_request r = gs.waiting.front();
                        gs.waiting.pop_front();
                        r->error = "a pass's workspace does not fit the server's memory budget";
                        finish_request(srv, r, SP_ERR_OUT_OF_MEMORY);
                    }
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
                while (!gs.waiting.empty() && !gs.waiting.front()->in_flight) {
                    sp_request r = gs.waiting.front();
                    gs.waiting.pop_front();
                    r->error = sp_last_error();
                    finish_request(srv, r, st);
                }
                srv->work_cv.notify_all();
                continue;
            }
            ws->bytes = need;
        }
        // Fill the pass: waiting requests of this graph in arrival order.
        std::vector<int32_t> srcs;
        std::vector<double *> outs;
        struct Part {
            sp_request r;
            int32_t count;
            bool first;
        };
        std::vector<Part> parts;
        for (auto *r : gs.waiting) {
            if ((int32_t)srcs.size() >= width) break;
            if (r->in_flight) continue;
            const int32_t take = std::min<int32_t>(width - (int32_t)srcs.size(),
                                                   (int32_t)r->sources.size() - r->next);
            if (take <= 0) continue;
            parts.push_back({r, take, !r->started});
            for (int32_t k = 0; k < take; ++k) {
                srcs.push_back(r->sources[r->next + k]);
                outs.push_back(r->out_bc);
            }
            r->next += take;
            r->in_flight = true;
            r->started = true;
        }
        if (srcs.empty()) {  // another worker took these sources while we allocated
            gs.idle.push_back(ws);
            srv->held--;
            srv->work_cv.notify_all();
            continue;
        }
        // Requests whose every source is now assigned leave the waiting list.
        gs.waiting.erase(std::remove_if(gs.waiting.begin(), gs.waiting.end(),
                                        [](sp_request r) { return r->next >= (int32_t)r->sources.size(); }),
                         gs.waiting.end());
        srv->stats.in_flight++;
        srv->stats.passes++;
        srv->stats.slots_used += (int64_t)srcs.size();
        srv->stats.queue_depth = pending_sources(srv);
        lk.unlock();

        sp_status st = SP_OK;
        clear_error();
        for (auto &p : parts)
            if (p.first && st >= 0) st = launch_fill_f64(p.r->out_bc, g->n, 0.0, stream);
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
        for (auto &p : parts) {
            sp_request r = p.r;
            r->in_flight = false;
            r->done_sources += p.count;
            const unsigned long long mine =
                (p.count >= 64 ? ~0ull : ((1ull << p.count) - 1ull)) << slot0;
            slot0 += p.count;
            if (st < 0) {
                r->status = st;
                r->error = err;
            } else if (r->status >= 0 && (res.flagged_mask & mine)) {
                r->status |= SP_WARN_SIGMA_LARGE;  // only the request that owns the slot
            }
            srv->stats.edges_traversed += (int64_t)p.count * (g->nnz / 2);
            if (r->done_sources >= (int32_t)r->sources.size() || r->status < 0) {
                if (r->status < 0)
                    gs.waiting.erase(std::remove(gs.waiting.begin(), gs.waiting.end(), r), gs.waiting.end());
                if (!r->finished) finish_request(srv, r, r->status);
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
        if (!c.n_streams) c.n_streams = 2;
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
    if (r->started || r->finished) return SP_ERR_REJECTED;
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
    for (auto &gs : srv->graphs)
        for (auto *ws : gs.idle) {
            batch_ws_destroy(*ws);
            delete ws;
        }
    delete srv;
    return SP_OK;
}

}  // extern "C"
