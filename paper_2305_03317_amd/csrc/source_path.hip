// Per-source Brandes pass on the GPU: one source at a time.
//
// Forward (paper Section 2.3.2 "iterateInBFS", Appendix Fig. "BC computation
// in StarPlat"): levels are expanded one after another.  A level is
//   discover: the next frontier F_{l+1} = unreached vertices adjacent to F_l,
//             either top-down (scan the adjacency of F_l, claim with a CAS on
//             dist) or bottom-up (every unreached vertex scans its own
//             adjacency and stops at the first neighbour in F_l);
//   sigma:    every w in F_{l+1} sums sigma over its DAG parents (neighbours
//             at level l) -- a pull, so no floating-point atomics and a fixed
//             summation order;
//   advance:  one thread moves the frontier window and picks the direction of
//             the next level from the frontier's and the unreached vertices'
//             adjacency sizes.
// The queue holds the vertices in level order; level_off[l] is where level l
// starts, so the reverse pass replays the levels without a second BFS.
//
// Reverse ("iterateInReverse"): for l = L-1 down to 1 each v in F_l sums
// (sigma[v] / sigma[w]) * (1 + delta[w]) over its DAG children w (level l+1),
// in CSR order for vertices handled by one lane, and adds delta[v] to BC[v].
// The source (level 0) is skipped.
//
// Level loops run on the device: the host enqueues a chunk of levels, whose
// kernels return at once after the control block says `done`, and reads the
// control block back once per chunk.
#include "common.h"
#include "devutil.h"

namespace sp {

// ---------------------------------------------------------------------------
// Fills
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

sp_status launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return SP_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    SP_HIP(hipGetLastError());
    return SP_OK;
}

sp_status launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return SP_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    SP_HIP(hipGetLastError());
    return SP_OK;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_src_init(LevelCtl *c, int32_t *dist, double *sigma, int32_t *queue,
                           int32_t *level_off, const int32_t *rp, int32_t src, int32_t n,
                           long long nnz, double alpha, double beta) {
    const int32_t deg = rp[src + 1] - rp[src];
    c->level = 0;
    c->lo = 0;
    c->hi = 1;
    c->tail = 1;
    c->done = 0;
    c->mode = MODE_TOPDOWN;
    c->overflow = 0;
    c->front_deg = (unsigned long long)deg;
    c->next_deg = 0;
    c->unset_deg = (unsigned long long)(nnz - deg);
    c->sigma_max_bits = (unsigned long long)__double_as_longlong(1.0);
    c->flagged_slots = 0;
    c->alpha = alpha;
    c->beta = beta;
    c->n_vertices = n;
    c->topdown_levels = 0;
    c->bottomup_levels = 0;
    dist[src] = 0;
    sigma[src] = 1.0;
    queue[0] = src;
    level_off[0] = 0;
    level_off[1] = 1;
}

// Top-down discovery: the block takes BS frontier vertices, scans their
// degrees, and walks the concatenated adjacency BS entries at a time, so
// every lane has one edge regardless of the degree mix.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_topdown(LevelCtl *c, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, int32_t *dist,
                                                    int32_t *queue) {
    if (c->done || c->mode != MODE_TOPDOWN) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_scan[BS / kWave + 1];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lo = c->lo, hi = c->hi, nl = c->level + 1, n = c->n_vertices;
    for (int32_t b = lo + blockIdx.x * BS; b < hi; b += gridDim.x * BS) {
        const int32_t i = b + threadIdx.x;
        int32_t beg = 0, deg = 0;
        if (i < hi) {
            const int32_t v = queue[i];
            beg = rp[v];
            deg = rp[v + 1] - beg;
        }
        int32_t total;
        const int32_t off = block_excl_scan<BS>(deg, s_scan, &total);
        s_beg[threadIdx.x] = beg;
        s_off[threadIdx.x] = off;
        __syncthreads();
        for (int32_t k0 = 0; k0 < total; k0 += BS) {
            const int32_t k = k0 + threadIdx.x;
            bool claim = false;
            int32_t w = 0;
            if (k < total) {
                int32_t a = 0, z = BS - 1;  // last j with s_off[j] <= k
                while (a < z) {
                    const int32_t mid = (a + z + 1) >> 1;
                    if (s_off[mid] <= k) a = mid; else z = mid - 1;
                }
                w = ci[s_beg[a] + (k - s_off[a])];
                if (dist[w] < 0) claim = atomicCAS(&dist[w], -1, nl) == -1;
            }
            q.stage(claim, w, &c->tail, queue, n, &c->overflow);
        }
        __syncthreads();
    }
    q.finish(&c->tail, queue, n, &c->overflow);
}

// Bottom-up discovery: each unreached vertex looks for any neighbour on the
// current level and stops at the first one.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_bottomup(LevelCtl *c, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, int32_t *dist,
                                                     int32_t *queue) {
    if (c->done || c->mode != MODE_BOTTOMUP) return;
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lvl = c->level, n = c->n_vertices;
    for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
        const int32_t v = b + threadIdx.x;
        bool found = false;
        if (v < n && dist[v] < 0) {
            const int32_t end = rp[v + 1];
            for (int32_t e = rp[v]; e < end; ++e)
                if (dist[ci[e]] == lvl) {
                    found = true;
                    break;
                }
        }
        if (found) dist[v] = lvl + 1;
        q.stage(found, v, &c->tail, queue, n, &c->overflow);
    }
    q.finish(&c->tail, queue, n, &c->overflow);
}

// Path counts of the new frontier: sigma[w] = sum of sigma[u] over neighbours
// u on the current level.  A lane owns a vertex of small degree and sums in
// CSR order; larger vertices are summed by the whole wave.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_sigma(LevelCtl *c, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const int32_t *__restrict__ queue,
                                                  const int32_t *__restrict__ dist, double *sigma) {
    if (c->done) return;
    __shared__ unsigned long long s_red[1];
    const int32_t lvl = c->level, hi = c->hi, tail = c->tail;
    const int lane = lane_id();
    unsigned long long my_deg = 0;
    double my_max = 0.0;
    bool large = false;
    for (int32_t b = hi + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < tail;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        int32_t w = -1, beg = 0, end = 0;
        if (i < tail) {
            w = queue[i];
            beg = rp[w];
            end = rp[w + 1];
        }
        const bool big = (end - beg) > kWave;
        double s = 0.0;
        if (w >= 0 && !big)
            for (int32_t e = beg; e < end; ++e) {
                const int32_t u = ci[e];
                if (dist[u] == lvl) s += sigma[u];
            }
        unsigned long long bm = __ballot(w >= 0 && big);
        while (bm) {
            const int j = __ffsll((long long)bm) - 1;
            bm &= bm - 1;
            const int32_t bj = shfl_i32(beg, j), ej = shfl_i32(end, j);
            double part = 0.0;
            for (int32_t e = bj + lane; e < ej; e += kWave) {
                const int32_t u = ci[e];
                if (dist[u] == lvl) part += sigma[u];
            }
            part = wave_sum_f64(part);
            if (lane == j) s = part;
        }
        if (w >= 0) {
            sigma[w] = s;
            my_deg += (unsigned long long)(end - beg);
            my_max = fmax(my_max, s);
            large |= sigma_is_large(s);
        }
    }
    my_max = wave_max_f64(my_max);
    if (lane == 0) atomic_max_nonneg_f64(&c->sigma_max_bits, my_max);
    if (__ballot(large) && lane == 0) atomicOr(&c->flagged_slots, 1ull);
    block_add_u64<BS>(my_deg, s_red, &c->next_deg);
}

__global__ void k_src_advance(LevelCtl *c, int32_t *level_off) {
    if (c->done) return;
    if (c->mode == MODE_TOPDOWN) c->topdown_levels++; else c->bottomup_levels++;
    const int32_t nf = c->tail - c->hi;
    if (nf <= 0) {
        c->done = 1;
        return;
    }
    level_off[c->level + 2] = c->tail;
    c->front_deg = c->next_deg;
    c->unset_deg -= c->next_deg;
    c->next_deg = 0;
    c->lo = c->hi;
    c->hi = c->tail;
    c->level += 1;
    if (c->mode == MODE_TOPDOWN) {
        if ((double)c->front_deg * c->alpha > (double)c->unset_deg) c->mode = MODE_BOTTOMUP;
    } else {
        if ((double)nf * c->beta < (double)c->n_vertices) c->mode = MODE_TOPDOWN;
    }
}

// Reverse sweep over one level.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_delta(const int32_t *__restrict__ level_off, int32_t lvl,
                                                  const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const int32_t *__restrict__ queue,
                                                  const int32_t *__restrict__ dist,
                                                  const double *__restrict__ sigma, double *delta,
                                                  double *bc) {
    const int32_t lo = level_off[lvl], hi = level_off[lvl + 1], nl = lvl + 1;
    const int lane = lane_id();
    for (int32_t b = lo + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < hi;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        int32_t v = -1, beg = 0, end = 0;
        double sv = 0.0;
        if (i < hi) {
            v = queue[i];
            beg = rp[v];
            end = rp[v + 1];
            sv = sigma[v];
        }
        const bool big = (end - beg) > kWave;
        double acc = 0.0;
        if (v >= 0 && !big)
            for (int32_t e = beg; e < end; ++e) {
                const int32_t w = ci[e];
                if (dist[w] == nl) acc += (sv / sigma[w]) * (1.0 + delta[w]);
            }
        unsigned long long bm = __ballot(v >= 0 && big);
        while (bm) {
            const int j = __ffsll((long long)bm) - 1;
            bm &= bm - 1;
            const int32_t bj = shfl_i32(beg, j), ej = shfl_i32(end, j);
            const double svj = shfl_f64(sv, j);
            double part = 0.0;
            for (int32_t e = bj + lane; e < ej; e += kWave) {
                const int32_t w = ci[e];
                if (dist[w] == nl) part += (svj / sigma[w]) * (1.0 + delta[w]);
            }
            part = wave_sum_f64(part);
            if (lane == j) acc = part;
        }
        if (v >= 0) {
            delta[v] = acc;
            if (bc) bc[v] += acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
sp_status source_ws_create(sp_graph g, SourceWorkspace &ws) {
    ws.device = g->device;
    ws.n = g->n;
    const size_t n = (size_t)std::max(g->n, 1);
    SP_TRY(dev_alloc((void **)&ws.dist, n * sizeof(int32_t)));
    SP_TRY(dev_alloc((void **)&ws.sigma, n * sizeof(double)));
    SP_TRY(dev_alloc((void **)&ws.delta, n * sizeof(double)));
    SP_TRY(dev_alloc((void **)&ws.queue, n * sizeof(int32_t)));
    ws.level_cap = (int32_t)n + 2;
    SP_TRY(dev_alloc((void **)&ws.level_off, (size_t)ws.level_cap * sizeof(int32_t)));
    SP_TRY(dev_alloc((void **)&ws.ctl, sizeof(LevelCtl)));
    SP_HIP(hipHostMalloc((void **)&ws.ctl_host, sizeof(LevelCtl), hipHostMallocDefault));
    SP_HIP(hipEventCreate(&ws.ev0));
    SP_HIP(hipEventCreate(&ws.ev1));
    return SP_OK;
}

void source_ws_destroy(SourceWorkspace &ws) {
    dev_free(ws.dist);
    dev_free(ws.sigma);
    dev_free(ws.delta);
    dev_free(ws.queue);
    dev_free(ws.level_off);
    dev_free(ws.ctl);
    if (ws.ctl_host) (void)hipHostFree(ws.ctl_host);
    if (ws.ev0) (void)hipEventDestroy(ws.ev0);
    if (ws.ev1) (void)hipEventDestroy(ws.ev1);
    ws = SourceWorkspace{};
}

template <int BS>
static sp_status source_run_bs(sp_graph g, SourceWorkspace &ws, int32_t src, double *bc,
                               bool with_backward, const SourceRunOpts &o, hipStream_t s,
                               SourceResult *res) {
    const int32_t n = g->n;
    const int grid_frontier = grid_for((int64_t)n, BS, device_cu_count() * 8);
    SP_TRY(launch_fill_i32(ws.dist, n, -1, s));
    hipLaunchKernelGGL(k_src_init, dim3(1), dim3(1), 0, s, ws.ctl, ws.dist, ws.sigma, ws.queue,
                       ws.level_off, (const int32_t *)g->row_ptr, src, n, (long long)g->nnz, o.alpha,
                       o.beta);
    SP_HIP(hipGetLastError());
    int32_t enqueued = 0;
    for (;;) {
        const int chunk = std::max(1, o.chunk_levels);
        for (int k = 0; k < chunk; ++k) {
            hipLaunchKernelGGL(k_src_topdown<BS>, dim3(grid_frontier), dim3(BS), 0, s, ws.ctl,
                               g->row_ptr, g->col_idx, ws.dist, ws.queue);
            hipLaunchKernelGGL(k_src_bottomup<BS>, dim3(grid_frontier), dim3(BS), 0, s, ws.ctl,
                               g->row_ptr, g->col_idx, ws.dist, ws.queue);
            hipLaunchKernelGGL(k_src_sigma<BS>, dim3(grid_frontier), dim3(BS), 0, s, ws.ctl,
                               g->row_ptr, g->col_idx, ws.queue, ws.dist, ws.sigma);
            hipLaunchKernelGGL(k_src_advance, dim3(1), dim3(1), 0, s, ws.ctl, ws.level_off);
        }
        SP_HIP(hipGetLastError());
        enqueued += chunk;
        SP_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(LevelCtl), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        if (ws.ctl_host->done) break;
        if (enqueued > n + 2) {
            set_error("BFS did not terminate after %d levels", enqueued);
            return SP_ERR_DEVICE;
        }
    }
    const LevelCtl &c = *ws.ctl_host;
    const int32_t levels = c.level + 1;
    if (with_backward && levels > 1) {
        std::vector<int32_t> off(levels + 1);
        SP_HIP(hipMemcpyAsync(off.data(), ws.level_off, sizeof(int32_t) * (levels + 1),
                              hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        for (int32_t l = levels - 1; l >= 1; --l) {
            const int32_t cnt = off[l + 1] - off[l];
            const int grid = grid_for((int64_t)cnt, BS, device_cu_count() * 8);
            hipLaunchKernelGGL(k_src_delta<BS>, dim3(grid), dim3(BS), 0, s, ws.level_off, l,
                               g->row_ptr, g->col_idx, ws.queue, ws.dist, ws.sigma, ws.delta, bc);
        }
        SP_HIP(hipGetLastError());
    }
    if (res) {
        res->levels = levels;
        res->reached = c.hi;
        std::memcpy(&res->sigma_max, &c.sigma_max_bits, sizeof(double));
        res->flagged = c.flagged_slots != 0;
        res->td = c.topdown_levels;
        res->bu = c.bottomup_levels;
    }
    return SP_OK;
}

sp_status source_run(sp_graph g, SourceWorkspace &ws, int32_t src, double *bc, bool with_backward,
                     const SourceRunOpts &o, hipStream_t s, SourceResult *res) {
    switch (o.block) {
        case 128: return source_run_bs<128>(g, ws, src, bc, with_backward, o, s, res);
        case 512: return source_run_bs<512>(g, ws, src, bc, with_backward, o, s, res);
        default: return source_run_bs<256>(g, ws, src, bc, with_backward, o, s, res);
    }
}

}  // namespace sp
