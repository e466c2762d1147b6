// PageRank, pull form, double buffered (paper Appendix, Fig. "PR computation
// in StarPlat").  Every vertex starts at 1/N; an iteration computes
//     val[v] = (1 - delta) / N + delta * sum over in-neighbours u of pr[u] / outdeg(u)
// from the previous iteration's values, and the run stops once the sum over
// vertices of |val - pr| is at most beta or max_iter iterations have run
// (the absolute difference is this library's reading of the paper's `diff`).
// A vertex's in-neighbours are its row on an undirected graph and its row of
// the reversed graph on a directed one; outdeg is always the outgoing row's
// length, and a vertex without outgoing arcs passes nothing on.
//
// Design: each iteration is one streaming pass over the CSR.  The producer of
// a value also stores share = val / outdeg, so the gather reads one double
// per adjacency entry.  A wave takes 64 consecutive vertices: rows of at most
// 8 entries are summed in row order by their own lane, longer ones by the
// wave in chunks of 8 aligned at the row start (wave_chunk_sum); either way a
// vertex's sum depends only on its row, so results are reproducible.  Rows
// longer than kHubDeg are cut by row eighths into 8m pieces of at most
// kHubChunk entries (split_piece), which waves reduce into partials, one XCD
// per eighth; a finishing kernel adds a row's partials in row order.  The
// stopping test sums |val - pr| per block in a fixed order and adds the block
// sums as fixed-point integers, so the total and the decision do not depend on
// scheduling.  The last working block of an iteration's last kernel closes it;
// chunks of iterations are captured as HIP graphs and replayed until the
// device reports done.
#include "capture.h"
#include "common.h"
#include "devutil.h"
#include "levels.h"

namespace sp {

// Rows of at most this many entries are summed by their own lane.
constexpr int kPrShortRow = 8;

__device__ __forceinline__ unsigned long long diff_fixed(double x) {
    return (unsigned long long)__double2ll_rn(x * 0x1p60);
}

// Block-uniform read of the iteration state (iteration * 2 + done).
__device__ __forceinline__ int32_t read_pr_state(PrCtl *c) {
    __shared__ int32_t s_state;
    if (threadIdx.x == 0) s_state = ld_agent(&c->state);
    __syncthreads();
    return s_state;
}

// Sum of the block's per-thread |change| in a fixed order, added to the
// iteration's total as a fixed-point integer.
template <int BS>
__device__ __forceinline__ void add_block_diff(PrCtl *c, double x, double *lds) {
    x = wave_sum_f64(x);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < BS / kWave; ++w) s += lds[w];
        if (s > 0.0) atomicAdd(&c->diff_.v, diff_fixed(s));
    }
}

// End of an iteration (one thread of the last working block).
__device__ void close_iteration(PrCtl *c) {
    const int32_t it = (c->state >> 1) + 1;
    const double diff = (double)ld_agent(&c->diff_.v) * 0x1p-60;
    c->diff_.v = 0;
    c->last_diff = diff;
    const bool done = !(diff > c->beta && it < c->max_iter);
    __hip_atomic_store(&c->state, it * 2 + (done ? 1 : 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_pr_init(PrCtl *c, const int32_t *__restrict__ rp, double *pr, double *share,
                          int32_t n, double beta, int32_t max_iter) {
    const double x = 1.0 / (double)n;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t deg = rp[v + 1] - rp[v];
        pr[v] = x;
        share[v] = deg > 0 ? x / (double)deg : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->state = 0;
        c->max_iter = max_iter;
        c->beta = beta;
        c->last_diff = 0.0;
        c->diff_.v = 0;
        c->blocks_done_.v = 0;
    }
}

// One iteration's gather.  blockIdx.y == 0: each wave takes 64 consecutive
// vertices (hubs excluded) and writes val, share and the block's |change|.
// blockIdx.y == 1: a wave per hub chunk writes the chunk's partial sum.
// Without hubs this kernel closes the iteration.  Bounded to eight waves per
// SIMD (some registers spilled): more gathers in flight, rmat-22 1.23 -> 1.13
// ms per iteration against six waves without spills.
template <int BS>
__global__ __launch_bounds__(BS, 8) void k_pr_pull(PrCtl *c, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const int32_t *__restrict__ rpo, double *pr0,
                                                double *pr1, double *sh0, double *sh1,
                                                double *partial, const HubEntry *__restrict__ hs,
                                                const int32_t *__restrict__ os, int32_t n,
                                                int32_t nch, double teleport, double delta,
                                                int32_t closes, int32_t parity,
                                                unsigned long long *prof) {
    const int32_t st = read_pr_state(c);
    if ((st & 1) || ((st >> 1) & 1) != parity) return;
    __shared__ int32_t s_coff[BS], s_beg[BS], s_deg[BS];
    __shared__ double s_acc[BS], s_w[BS / kWave];
    __shared__ unsigned long long s_red[1];
    const double *pr = parity ? pr1 : pr0;
    const double *sh = parity ? sh1 : sh0;
    double *pr_n = parity ? pr0 : pr1;
    double *sh_n = parity ? sh0 : sh1;
    const int lane = lane_id();
    const int wbase = threadIdx.x - lane;
    unsigned long long my_items = 0, my_edges = 0;
    double my_diff = 0.0;
    if (blockIdx.y == 0) {
        const WaveScratch ws{s_coff + wbase, s_beg + wbase, s_deg + wbase, s_acc + wbase, nullptr};
        for (int32_t b = blockIdx.x * BS + wbase; b < n; b += gridDim.x * BS) {
            const int32_t v = b + lane;
            int32_t beg = 0, deg = 0, dout = 0;
            if (v < n) {
                beg = rp[v];
                deg = rp[v + 1] - beg;
                dout = rpo == rp ? deg : rpo[v + 1] - rpo[v];
            }
            const bool hub = deg > kHubDeg, shortrow = deg <= kPrShortRow;
            // short rows: the lane's own row, all loads issued before the
            // in-order sum; longer rows: the wave's chunked sum
            double sum = 0.0;
            if (shortrow) {
                int32_t u[kPrShortRow];
                double x[kPrShortRow];
#pragma unroll
                for (int j = 0; j < kPrShortRow; ++j) u[j] = j < deg ? ci[beg + j] : 0;
#pragma unroll
                for (int j = 0; j < kPrShortRow; ++j) x[j] = j < deg ? sh[u[j]] : 0.0;
#pragma unroll
                for (int j = 0; j < kPrShortRow; ++j)
                    if (j < deg) sum += x[j];
            }
            const double chunked = wave_chunk_sum(beg, hub || shortrow ? 0 : deg, ws,
                                                  [&](int32_t e, int32_t) { return sh[ci[e]]; });
            if (!shortrow) sum = chunked;
            if (v < n && !hub) {
                const double val = teleport + delta * sum;
                my_diff += fabs(val - pr[v]);
                pr_n[v] = val;
                sh_n[v] = dout > 0 ? val / (double)dout : 0.0;
                ++my_items;
                my_edges += (unsigned long long)deg;
            }
        }
        add_block_diff<BS>(c, my_diff, s_w);
    } else {
        // with a grid that is a multiple of 8, block (x, 1) runs on XCD x mod 8
        for_xcd_chunks<BS>(nch, [&](int64_t k) {
            const HubEntry h = hs[os[k]];
            const int32_t rb = rp[h.v];
            int32_t beg, end;
            split_piece(rb, rp[h.v + 1] - rb, h.nchunks, (int32_t)k - h.chunk_base, beg, end);
            hub_chunk((int32_t)k, beg, end, partial, [&](int32_t e) { return sh[ci[e]]; });
            my_edges += lane == 0 ? (unsigned long long)(end - beg) : 0ull;
        });
    }
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
    if (closes && last_block(c, working_blocks((int64_t)n, BS)) && threadIdx.x == 0) close_iteration(c);
}

// Hubs of one iteration from their chunk sums, in row order (a thread per
// hub); closes the iteration.
__global__ void k_pr_hub_fin(PrCtl *c, const int32_t *__restrict__ rpo, double *pr0, double *pr1,
                             double *sh0, double *sh1, const double *__restrict__ partial,
                             const HubEntry *__restrict__ hs, int32_t nh, double teleport,
                             double delta, int32_t parity) {
    const int32_t st = read_pr_state(c);
    if ((st & 1) || ((st >> 1) & 1) != parity) return;
    __shared__ double s_w[256 / kWave];
    const double *pr = parity ? pr1 : pr0;
    double *pr_n = parity ? pr0 : pr1;
    double *sh_n = parity ? sh0 : sh1;
    double my_diff = 0.0;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nh; j += stride) {
        const HubEntry h = hs[j];
        const double val = teleport + delta * sum_split_chunks(partial, h.chunk_base, h.nchunks);
        my_diff += fabs(val - pr[h.v]);
        pr_n[h.v] = val;
        const int32_t dout = rpo[h.v + 1] - rpo[h.v];  // outgoing row (may be empty when directed)
        sh_n[h.v] = dout > 0 ? val / (double)dout : 0.0;
    }
    add_block_diff<256>(c, my_diff, s_w);
    if (last_block(c, working_blocks((int64_t)nh, 256)) && threadIdx.x == 0) close_iteration(c);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
sp_status pr_ws_create(sp_graph g, PrWorkspace &ws) {
    const size_t n = (size_t)std::max(g->n, 1);
    SP_HIP(hipGetDevice(&ws.device));
    sp_status st = SP_OK;
    for (int p = 0; p < 2 && st == SP_OK; ++p) {
        st = dev_alloc((void **)&ws.pr[p], sizeof(double) * n);
        if (st == SP_OK) st = dev_alloc((void **)&ws.share[p], sizeof(double) * n);
    }
    if (st == SP_OK) st = dev_alloc((void **)&ws.partial, sizeof(double) * ((size_t)g->pr_chunks + 1));
    if (st == SP_OK) st = dev_alloc((void **)&ws.ctl, sizeof(PrCtl));
    if (st != SP_OK) {
        pr_ws_destroy(ws);
        return st;
    }
    if (hipHostMalloc((void **)&ws.ctl_host, sizeof(PrCtl), hipHostMallocDefault) != hipSuccess) {
        ws.ctl_host = nullptr;
        pr_ws_destroy(ws);
        set_error("pinned host allocation failed");
        return SP_ERR_OUT_OF_MEMORY;
    }
    if (hipEventCreate(&ws.ev0) != hipSuccess || hipEventCreate(&ws.ev1) != hipSuccess) {
        pr_ws_destroy(ws);
        set_error("hipEventCreate failed");
        return SP_ERR_DEVICE;
    }
    return SP_OK;
}

void pr_ws_destroy(PrWorkspace &ws) {
    if (ws.iters.exec) (void)hipGraphExecDestroy(ws.iters.exec);
    if (ws.cap_stream) (void)hipStreamDestroy(ws.cap_stream);
    for (int p = 0; p < 2; ++p) {
        dev_free(ws.pr[p]);
        dev_free(ws.share[p]);
    }
    dev_free(ws.partial);
    dev_free(ws.ctl);
    if (ws.ctl_host) (void)hipHostFree(ws.ctl_host);
    if (ws.ev0) (void)hipEventDestroy(ws.ev0);
    if (ws.ev1) (void)hipEventDestroy(ws.ev1);
    ws = PrWorkspace{};
}

// `count` iterations starting at an even iteration (parity = k & 1).
template <int BS>
static void enqueue_iterations(sp_graph g, PrWorkspace &ws, int count, int grid, int fin_grid,
                               double teleport, double delta, hipStream_t s) {
    const bool hubs = g->pr_n_hubs > 0;
    for (int k = 0; k < count; ++k) {
        const int32_t parity = k & 1;
        {
            ProfScope ps(P_PR_PULL, s);
            hipLaunchKernelGGL(k_pr_pull<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s, ws.ctl,
                               (const int32_t *)g->rp_in, (const int32_t *)g->ci_in,
                               (const int32_t *)g->row_ptr, ws.pr[0],
                               ws.pr[1], ws.share[0], ws.share[1], ws.partial,
                               (const HubEntry *)g->pr_hubs, (const int32_t *)g->pr_owner, g->n,
                               (int32_t)g->pr_chunks, teleport, delta, (int32_t)!hubs, parity,
                               prof_counters(P_PR_PULL));
        }
        if (hubs) {
            ProfScope ps(P_PR_HUB, s);
            hipLaunchKernelGGL(k_pr_hub_fin, dim3(fin_grid), dim3(256), 0, s, ws.ctl,
                               (const int32_t *)g->row_ptr, ws.pr[0], ws.pr[1], ws.share[0], ws.share[1],
                               (const double *)ws.partial, (const HubEntry *)g->pr_hubs, g->pr_n_hubs,
                               teleport, delta, parity);
        }
    }
}

static long long bits_of(double x) {
    long long b;
    std::memcpy(&b, &x, sizeof(b));
    return b;
}

template <int BS>
static sp_status pr_run_bs(sp_graph g, PrWorkspace &ws, double beta, double delta, int32_t max_iter,
                           double *out_pr, const PrOpts &o, hipStream_t s, PrResult *res) {
    const int32_t n = g->n;
    const int maxb = device_cu_count() * 8;
    const int grid = grid_for((int64_t)n, BS, maxb);
    const int fin_grid = grid_for((int64_t)g->pr_n_hubs, 256, maxb);
    const double teleport = (1.0 - delta) / (double)n;
    hipLaunchKernelGGL(k_pr_init, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.ctl,
                       (const int32_t *)g->row_ptr, ws.pr[0], ws.share[0], n, beta, max_iter);
    SP_HIP(hipGetLastError());
    const bool capture = o.chunk_iters > 0 && !prof_enabled();
    const int base = std::max(1, std::abs(o.chunk_iters));
    const int chunk = base + (base & 1);  // even: every chunk starts at an even iteration
    int32_t enqueued = 0, graph_launches = 0;
    for (;;) {
        if (capture) {
            const std::array<long long, 12> key = {
                BS, grid, fin_grid, chunk, (long long)(intptr_t)ws.pr[0], (long long)(intptr_t)ws.ctl,
                (long long)(intptr_t)g->pr_hubs, bits_of(teleport),
                bits_of(delta), g->pr_n_hubs, 0, 0};
            SP_TRY(replay_captured(&ws.cap_stream, ws.iters, key,
                                   [&](hipStream_t cs) {
                                       enqueue_iterations<BS>(g, ws, chunk, grid, fin_grid, teleport, delta, cs);
                                   },
                                   s));
            ++graph_launches;
        } else {
            enqueue_iterations<BS>(g, ws, chunk, grid, fin_grid, teleport, delta, s);
            SP_HIP(hipGetLastError());
        }
        enqueued += chunk;
        SP_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(PrCtl), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        if (ws.ctl_host->state & 1) break;
        if (enqueued >= max_iter + chunk) {
            set_error("PageRank did not stop after %d iterations", enqueued);
            return SP_ERR_DEVICE;
        }
    }
    const int32_t iters = ws.ctl_host->state >> 1;
    SP_HIP(hipMemcpyAsync(out_pr, ws.pr[iters & 1], sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (res) {
        res->iterations = iters;
        res->diff = ws.ctl_host->last_diff;
        res->graph_launches = graph_launches;
    }
    return SP_OK;
}

sp_status pr_run(sp_graph g, PrWorkspace &ws, double beta, double delta, int32_t max_iter,
                 double *out_pr, const PrOpts &o, hipStream_t s, PrResult *res) {
    switch (o.block) {
        case 128: return pr_run_bs<128>(g, ws, beta, delta, max_iter, out_pr, o, s, res);
        case 512: return pr_run_bs<512>(g, ws, beta, delta, max_iter, out_pr, o, s, res);
        default: return pr_run_bs<256>(g, ws, beta, delta, max_iter, out_pr, o, s, res);
    }
}

}  // namespace sp
