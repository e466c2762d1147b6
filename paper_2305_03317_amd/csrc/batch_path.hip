// Batched multi-source Brandes pass: up to 64 sources advance level by level
// together.  Each vertex carries 64-bit source bitmaps (bit i = batch slot i):
//   seen[v]   slots that have reached v at some level so far,
//   nxt[v]    slots discovering v at the level being built,
//   front[p]  per level parity p, {mask, level tag} of v's entry at that level.
// A (vertex, mask) pair per level is an "entry"; entries of one level are
// contiguous in `queue`/`qmask`, and level_off[l] is where level l starts.
//
// Per-source arithmetic is exactly the per-source path's (paper Appendix,
// Fig. "BC computation in StarPlat"; DAG semantics of Section 2.3.2): lane s
// of a wave owns slot s, so sigma[w][s] sums sigma[u][s] over u with s in
// front(l)[u] in CSR order, and delta[v][s] sums
// (sigma[v][s] / sigma[w][s]) * (1 + delta[w][s]) over w with s in
// front(l+1)[w] in CSR order.  sigma and delta rows are vertex-major
// (64 doubles per vertex), so one wave reads a neighbour's row with one
// coalesced access for all its slots.
//
// Forward level:  discover (top-down: expand the entries of level l, OR the
//                 new slots into nxt[w] and claim w on the first OR;
//                 bottom-up: every vertex with unsettled slots ORs the level-l
//                 masks of its neighbours and stops when all are found)
//                 -> sigma (wave per new entry) -> advance (one thread).
// Reverse level:  one kernel per level, wave per entry; it also re-publishes
//                 the entry's {mask, level} in front(l) for the next step.
// BC:             per vertex, slots in ascending order, skipping the slot
//                 whose source is the vertex itself.
#include "common.h"
#include "devutil.h"

namespace sp {

struct SlotTable {
    double *out[kSlots];
};

__device__ __forceinline__ unsigned long long mask_of(uint4 f) {
    return (unsigned long long)f.x | ((unsigned long long)f.y << 32);
}

__device__ __forceinline__ uint4 make_front(unsigned long long m, uint32_t tag) {
    return make_uint4((uint32_t)m, (uint32_t)(m >> 32), tag, 0u);
}

constexpr uint32_t kNoTag = 0xFFFFFFFFu;

__global__ void k_ms_clear(unsigned long long *seen, unsigned long long *nxt, uint4 *f0, uint4 *f1,
                           int32_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint4 z = make_front(0, kNoTag);
    for (; i < n; i += stride) {
        seen[i] = 0;
        nxt[i] = 0;
        f0[i] = z;
        f1[i] = z;
    }
}

// Level 0: entries [0, n0) hold the distinct source vertices and their slots.
__global__ void k_ms_init(LevelCtl *c, const int32_t *__restrict__ rp, const int32_t *queue,
                          const unsigned long long *qmask, int32_t n0, unsigned long long *seen,
                          uint4 *front0, double *sigma, int32_t *level_off, int32_t n,
                          long long nnz, unsigned long long active, double alpha, double beta) {
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    for (int32_t i = wv; i < n0; i += blockDim.x / kWave) {
        const int32_t v = queue[i];
        const unsigned long long m = qmask[i];
        if ((m >> lane) & 1ull) sigma[(int64_t)v * kSlots + lane] = 1.0;
        if (lane == 0) {
            seen[v] = m;
            front0[v] = make_front(m, 0u);
        }
    }
    if (threadIdx.x == 0) {
        unsigned long long fdeg = 0, settled = 0;
        for (int32_t i = 0; i < n0; ++i) {
            const int32_t v = queue[i];
            const unsigned long long d = (unsigned long long)(rp[v + 1] - rp[v]);
            fdeg += d;
            if (qmask[i] == active) settled += d;
        }
        c->level = 0;
        c->lo = 0;
        c->hi = n0;
        c->tail = n0;
        c->done = 0;
        c->mode = MODE_TOPDOWN;
        c->overflow = 0;
        c->front_deg = fdeg;
        c->next_deg = 0;
        c->settled_deg = 0;
        c->reached_pairs = 0;
        for (int32_t i = 0; i < n0; ++i) c->reached_pairs += __popcll(qmask[i]);
        c->unset_deg = (unsigned long long)nnz - settled;
        c->sigma_max_bits = (unsigned long long)__double_as_longlong(1.0);
        c->flagged_slots = 0;
        c->alpha = alpha;
        c->beta = beta;
        c->n_vertices = n;
        c->topdown_levels = 0;
        c->bottomup_levels = 0;
        level_off[0] = 0;
        level_off[1] = n0;
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ms_topdown(LevelCtl *c, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, int32_t *queue,
                                                   const unsigned long long *__restrict__ qmask,
                                                   const unsigned long long *__restrict__ seen,
                                                   unsigned long long *nxt, long long qcap) {
    if (c->done || c->mode != MODE_TOPDOWN) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_scan[BS / kWave + 1];
    __shared__ unsigned long long s_mask[BS];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lo = c->lo, hi = c->hi;
    for (int32_t b = lo + blockIdx.x * BS; b < hi; b += gridDim.x * BS) {
        const int32_t i = b + threadIdx.x;
        int32_t beg = 0, deg = 0;
        unsigned long long fm = 0;
        if (i < hi) {
            const int32_t v = queue[i];
            fm = qmask[i];
            beg = rp[v];
            deg = rp[v + 1] - beg;
        }
        int32_t total;
        const int32_t off = block_excl_scan<BS>(deg, s_scan, &total);
        s_beg[threadIdx.x] = beg;
        s_off[threadIdx.x] = off;
        s_mask[threadIdx.x] = fm;
        __syncthreads();
        for (int32_t k0 = 0; k0 < total; k0 += BS) {
            const int32_t k = k0 + threadIdx.x;
            bool claim = false;
            int32_t w = 0;
            if (k < total) {
                int32_t a = 0, z = BS - 1;
                while (a < z) {
                    const int32_t mid = (a + z + 1) >> 1;
                    if (s_off[mid] <= k) a = mid; else z = mid - 1;
                }
                w = ci[s_beg[a] + (k - s_off[a])];
                const unsigned long long nm = s_mask[a] & ~seen[w];
                if (nm && (nm & ~*(volatile unsigned long long *)&nxt[w]))
                    claim = atomicOr(&nxt[w], nm) == 0ull;
            }
            q.stage(claim, w, &c->tail, queue, qcap, &c->overflow);
        }
        __syncthreads();
    }
    q.finish(&c->tail, queue, qcap, &c->overflow);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ms_bottomup(LevelCtl *c, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const unsigned long long *__restrict__ seen,
                                                    unsigned long long *nxt,
                                                    const uint4 *__restrict__ front_cur,
                                                    int32_t *queue, unsigned long long active,
                                                    long long qcap) {
    if (c->done || c->mode != MODE_BOTTOMUP) return;
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const uint32_t lvl = (uint32_t)c->level;
    const int32_t n = c->n_vertices;
    for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
        const int32_t v = b + threadIdx.x;
        bool found = false;
        if (v < n) {
            const unsigned long long uns = active & ~seen[v];
            if (uns) {
                unsigned long long acc = 0;
                const int32_t end = rp[v + 1];
                for (int32_t e = rp[v]; e < end; ++e) {
                    const uint4 f = front_cur[ci[e]];
                    if (f.z == lvl) {
                        acc |= mask_of(f) & uns;
                        if (acc == uns) break;
                    }
                }
                if (acc) {
                    nxt[v] = acc;
                    found = true;
                }
            }
        }
        q.stage(found, v, &c->tail, queue, qcap, &c->overflow);
    }
    q.finish(&c->tail, queue, qcap, &c->overflow);
}

// Path counts of the new entries; wave per entry, lane = slot.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_sigma(LevelCtl *c, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ queue,
                                                 unsigned long long *qmask, unsigned long long *seen,
                                                 unsigned long long *nxt,
                                                 const uint4 *__restrict__ front_cur,
                                                 uint4 *front_nxt, double *sigma,
                                                 unsigned long long active, long long qcap) {
    if (c->done) return;
    __shared__ unsigned long long s_red[1];
    const uint32_t lvl = (uint32_t)c->level;
    const int32_t hi = c->hi;
    const int32_t tail = (int32_t)min((long long)c->tail, qcap);
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * BS + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * BS / kWave;
    unsigned long long my_deg = 0, my_settled = 0, my_flag = 0, my_pairs = 0;
    double my_max = 0.0;
    for (int64_t i = hi + wave0; i < tail; i += nwaves) {
        const int32_t w = queue[i];
        const unsigned long long m = nxt[w];
        const int32_t beg = rp[w], end = rp[w + 1];
        double acc = 0.0;
        for (int32_t e0 = beg; e0 < end; e0 += kWave) {
            const int32_t e = e0 + lane;
            int32_t u = 0;
            unsigned long long f = 0;
            if (e < end) {
                u = ci[e];
                const uint4 fu = front_cur[u];
                if (fu.z == lvl) f = mask_of(fu) & m;
            }
            unsigned long long nz = __ballot(f != 0ull);
            while (nz) {
                const int j = __ffsll((long long)nz) - 1;
                nz &= nz - 1;
                const int32_t uj = shfl_i32(u, j);
                const unsigned long long fj = shfl_u64(f, j);
                if ((fj >> lane) & 1ull) acc += sigma[(int64_t)uj * kSlots + lane];
            }
        }
        const bool mine = (m >> lane) & 1ull;
        if (mine) {
            sigma[(int64_t)w * kSlots + lane] = acc;
            my_max = fmax(my_max, acc);
        }
        my_flag |= __ballot(mine && sigma_is_large(acc));
        if (lane == 0) {
            qmask[i] = m;
            nxt[w] = 0;
            const unsigned long long now = seen[w] | m;
            seen[w] = now;
            front_nxt[w] = make_front(m, lvl + 1);
            const unsigned long long d = (unsigned long long)(end - beg);
            my_deg += d;
            my_pairs += (unsigned long long)__popcll(m);
            if (now == active) my_settled += d;
        }
    }
    my_max = wave_max_f64(my_max);
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits, my_max);
        if (my_flag) atomicOr(&c->flagged_slots, my_flag);
    }
    block_add_u64<BS>(my_deg, s_red, &c->next_deg);
    __syncthreads();
    block_add_u64<BS>(my_settled, s_red, &c->settled_deg);
    __syncthreads();
    block_add_u64<BS>(my_pairs, s_red, &c->reached_pairs);
}

__global__ void k_ms_advance(LevelCtl *c, int32_t *level_off, long long qcap) {
    if (c->done) return;
    if (c->mode == MODE_TOPDOWN) c->topdown_levels++; else c->bottomup_levels++;
    if ((long long)c->tail > qcap || c->overflow) {
        c->overflow = 1;
        c->done = 1;
        return;
    }
    const int32_t nf = c->tail - c->hi;
    if (nf <= 0) {
        c->done = 1;
        return;
    }
    level_off[c->level + 2] = c->tail;
    c->front_deg = c->next_deg;
    c->unset_deg -= c->settled_deg;
    c->next_deg = 0;
    c->settled_deg = 0;
    c->lo = c->hi;
    c->hi = c->tail;
    c->level += 1;
    if (c->mode == MODE_TOPDOWN) {
        if ((double)c->front_deg * c->alpha > (double)c->unset_deg) c->mode = MODE_BOTTOMUP;
    } else {
        if ((double)nf * c->beta < (double)c->n_vertices) c->mode = MODE_TOPDOWN;
    }
}

// Reverse sweep of one level; wave per entry, lane = slot.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_delta(const int32_t *__restrict__ level_off, int32_t lvl,
                                                 int32_t deepest, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ queue,
                                                 const unsigned long long *__restrict__ qmask,
                                                 const uint4 *__restrict__ front_rd,
                                                 uint4 *front_wr, const double *__restrict__ sigma,
                                                 double *delta) {
    const int32_t lo = level_off[lvl], hi = level_off[lvl + 1];
    const uint32_t nl = (uint32_t)lvl + 1;
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * BS + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * BS / kWave;
    for (int64_t i = lo + wave0; i < hi; i += nwaves) {
        const int32_t v = queue[i];
        const unsigned long long m = qmask[i];
        const bool mine = (m >> lane) & 1ull;
        if (lane == 0) front_wr[v] = make_front(m, (uint32_t)lvl);
        double acc = 0.0;
        if (!deepest) {
            const double sv = mine ? sigma[(int64_t)v * kSlots + lane] : 0.0;
            const int32_t beg = rp[v], end = rp[v + 1];
            for (int32_t e0 = beg; e0 < end; e0 += kWave) {
                const int32_t e = e0 + lane;
                int32_t w = 0;
                unsigned long long g = 0;
                if (e < end) {
                    w = ci[e];
                    const uint4 fw = front_rd[w];
                    if (fw.z == nl) g = mask_of(fw) & m;
                }
                unsigned long long nz = __ballot(g != 0ull);
                while (nz) {
                    const int j = __ffsll((long long)nz) - 1;
                    nz &= nz - 1;
                    const int32_t wj = shfl_i32(w, j);
                    const unsigned long long gj = shfl_u64(g, j);
                    if ((gj >> lane) & 1ull) {
                        const int64_t o = (int64_t)wj * kSlots + lane;
                        acc += (sv / sigma[o]) * (1.0 + delta[o]);
                    }
                }
            }
        }
        if (mine) delta[(int64_t)v * kSlots + lane] = acc;
    }
}

// BC[v] += delta[v][s] for slots in ascending order; consecutive slots with
// the same output array are summed in a register.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_bc(int32_t n, const unsigned long long *__restrict__ seen,
                                              const double *__restrict__ delta,
                                              const int32_t *__restrict__ slot_src, int32_t nslots,
                                              SlotTable tbl) {
    __shared__ int32_t s_src[kSlots];
    if (threadIdx.x < kSlots) s_src[threadIdx.x] = threadIdx.x < nslots ? slot_src[threadIdx.x] : -1;
    __syncthreads();
    for (int32_t v = blockIdx.x * BS + threadIdx.x; v < n; v += gridDim.x * BS) {
        const unsigned long long sm = seen[v];
        if (!sm) continue;
        const double *row = delta + (int64_t)v * kSlots;
        double *cur = nullptr;
        double acc = 0.0;
        for (int32_t s = 0; s < nslots; ++s) {
            double *out = tbl.out[s];
            if (!out) continue;
            if (out != cur) {
                if (cur) cur[v] = acc;
                cur = out;
                acc = out[v];
            }
            if (((sm >> s) & 1ull) && s_src[s] != v) acc += row[s];
        }
        if (cur) cur[v] = acc;
    }
}

// Per-slot results of one level into source-major arrays (for checks).
__global__ void k_ms_extract(const int32_t *__restrict__ queue,
                             const unsigned long long *__restrict__ qmask, int32_t lo, int32_t hi,
                             int32_t lvl, int32_t n, const double *__restrict__ sigma,
                             const double *__restrict__ delta, int32_t *out_dist,
                             double *out_sigma, double *out_delta) {
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = lo + wave0; i < hi; i += nwaves) {
        const int32_t v = queue[i];
        if (!((qmask[i] >> lane) & 1ull)) continue;
        const int64_t o = (int64_t)lane * n + v, r = (int64_t)v * kSlots + lane;
        out_dist[o] = lvl;
        if (out_sigma) out_sigma[o] = sigma[r];
        if (out_delta) out_delta[o] = lvl > 0 ? delta[r] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
size_t batch_ws_bytes(int32_t n, int64_t qcap, int32_t level_cap) {
    const size_t V = (size_t)std::max(n, 1);
    return V * (8 + 8 + 16 + 16) + V * kSlots * 16 + (size_t)qcap * 12 +
           (size_t)level_cap * 4 + kSlots * 4 + sizeof(LevelCtl);
}

sp_status batch_ws_create(sp_graph g, int64_t qcap, BatchWorkspace &ws) {
    ws.device = g->device;
    ws.n = g->n;
    const size_t V = (size_t)std::max(g->n, 1);
    ws.qcap = qcap;
    ws.level_cap = (int32_t)std::min<int64_t>((int64_t)V + 2, (int64_t)INT32_MAX);
    SP_TRY(dev_alloc((void **)&ws.seen, V * 8));
    SP_TRY(dev_alloc((void **)&ws.nxt, V * 8));
    SP_TRY(dev_alloc((void **)&ws.front[0], V * 16));
    SP_TRY(dev_alloc((void **)&ws.front[1], V * 16));
    SP_TRY(dev_alloc((void **)&ws.sigma, V * kSlots * 8));
    SP_TRY(dev_alloc((void **)&ws.delta, V * kSlots * 8));
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    SP_TRY(dev_alloc((void **)&ws.level_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.slot_src, kSlots * 4));
    SP_TRY(dev_alloc((void **)&ws.ctl, sizeof(LevelCtl)));
    SP_HIP(hipHostMalloc((void **)&ws.ctl_host, sizeof(LevelCtl), hipHostMallocDefault));
    SP_HIP(hipHostMalloc((void **)&ws.staging, kSlots * (4 + 8 + 4), hipHostMallocDefault));
    SP_HIP(hipEventCreate(&ws.ev0));
    SP_HIP(hipEventCreate(&ws.ev1));
    ws.bytes = batch_ws_bytes(g->n, qcap, ws.level_cap);
    return SP_OK;
}

void batch_ws_destroy(BatchWorkspace &ws) {
    dev_free(ws.seen);
    dev_free(ws.nxt);
    dev_free(ws.front[0]);
    dev_free(ws.front[1]);
    dev_free(ws.sigma);
    dev_free(ws.delta);
    dev_free(ws.queue);
    dev_free(ws.qmask);
    dev_free(ws.level_off);
    dev_free(ws.slot_src);
    dev_free(ws.ctl);
    if (ws.ctl_host) (void)hipHostFree(ws.ctl_host);
    if (ws.staging) (void)hipHostFree(ws.staging);
    if (ws.ev0) (void)hipEventDestroy(ws.ev0);
    if (ws.ev1) (void)hipEventDestroy(ws.ev1);
    ws = BatchWorkspace{};
}

static sp_status grow_queue(BatchWorkspace &ws, int64_t qcap) {
    dev_free(ws.queue);
    dev_free(ws.qmask);
    ws.queue = nullptr;
    ws.qmask = nullptr;
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    ws.qcap = qcap;
    ws.bytes = batch_ws_bytes(ws.n, qcap, ws.level_cap);
    return SP_OK;
}

template <int BS>
static sp_status batch_forward(sp_graph g, BatchWorkspace &ws, int32_t n0, unsigned long long active,
                               const BatchRunOpts &o, hipStream_t s) {
    const int32_t n = g->n;
    const int grid = grid_for((int64_t)n, BS, device_cu_count() * 8);
    hipLaunchKernelGGL(k_ms_clear, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.seen, ws.nxt,
                       ws.front[0], ws.front[1], n);
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(256), 0, s, ws.ctl, (const int32_t *)g->row_ptr,
                       (const int32_t *)ws.queue, (const unsigned long long *)ws.qmask, n0, ws.seen,
                       ws.front[0], ws.sigma, ws.level_off, n, (long long)g->nnz, active, o.alpha,
                       o.beta);
    SP_HIP(hipGetLastError());
    int64_t enqueued = 0;
    for (;;) {
        const int chunk = std::max(1, o.chunk_levels);
        for (int k = 0; k < chunk; ++k) {
            const int64_t l = enqueued + k;  // level this group expands
            uint4 *fcur = ws.front[l & 1], *fnxt = ws.front[(l + 1) & 1];
            hipLaunchKernelGGL(k_ms_topdown<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                               g->col_idx, ws.queue, ws.qmask, ws.seen, ws.nxt, (long long)ws.qcap);
            hipLaunchKernelGGL(k_ms_bottomup<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                               g->col_idx, ws.seen, ws.nxt, fcur, ws.queue, active,
                               (long long)ws.qcap);
            hipLaunchKernelGGL(k_ms_sigma<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                               g->col_idx, ws.queue, ws.qmask, ws.seen, ws.nxt, fcur, fnxt,
                               ws.sigma, active, (long long)ws.qcap);
            hipLaunchKernelGGL(k_ms_advance, dim3(1), dim3(1), 0, s, ws.ctl, ws.level_off,
                               (long long)ws.qcap);
        }
        SP_HIP(hipGetLastError());
        enqueued += chunk;
        SP_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(LevelCtl), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        if (ws.ctl_host->done) break;
        if (enqueued > (int64_t)n + 2) {
            set_error("multi-source BFS did not terminate after %lld levels", (long long)enqueued);
            return SP_ERR_DEVICE;
        }
    }
    return SP_OK;
}

template <int BS>
static sp_status batch_run_bs(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                              double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s,
                              BatchResult *res, bool keep_levels) {
    const int32_t n = g->n;
    const unsigned long long active = nslots >= 64 ? ~0ull : ((1ull << nslots) - 1ull);
    // Level 0: distinct source vertices with the mask of their slots.
    int32_t *h_q = (int32_t *)ws.staging;
    unsigned long long *h_m = (unsigned long long *)(h_q + kSlots);
    int32_t *h_src = (int32_t *)(h_m + kSlots);
    int32_t n0 = 0;
    for (int32_t i = 0; i < kSlots; ++i) h_src[i] = i < nslots ? srcs[i] : -1;
    for (int32_t i = 0; i < nslots; ++i) {
        int32_t j = 0;
        while (j < n0 && h_q[j] != srcs[i]) ++j;
        if (j == n0) {
            h_q[n0] = srcs[i];
            h_m[n0] = 0;
            ++n0;
        }
        h_m[j] |= 1ull << i;
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        SP_HIP(hipMemcpyAsync(ws.queue, h_q, n0 * 4, hipMemcpyHostToDevice, s));
        SP_HIP(hipMemcpyAsync(ws.qmask, h_m, n0 * 8, hipMemcpyHostToDevice, s));
        SP_HIP(hipMemcpyAsync(ws.slot_src, h_src, kSlots * 4, hipMemcpyHostToDevice, s));
        SP_TRY(batch_forward<BS>(g, ws, n0, active, o, s));
        if (!ws.ctl_host->overflow) break;
        if (attempt == 1) {
            set_error("multi-source queue overflow at capacity %lld", (long long)ws.qcap);
            return SP_ERR_DEVICE;
        }
        // Every vertex holds at most one entry per slot, so this always fits.
        SP_TRY(grow_queue(ws, (int64_t)std::max(n, 1) * nslots + kSlots));
    }
    const LevelCtl c = *ws.ctl_host;
    const int32_t levels = c.level + 1;
    std::vector<int32_t> off(levels + 1);
    SP_HIP(hipMemcpyAsync(off.data(), ws.level_off, sizeof(int32_t) * (levels + 1),
                          hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
    const int maxb = device_cu_count() * 8;
    for (int32_t l = levels - 1; l >= 1; --l) {
        const int64_t cnt = off[l + 1] - off[l];
        const int grid = grid_for(cnt * kWave, BS, maxb);
        const int32_t lvl_par = l & 1;
        hipLaunchKernelGGL(k_ms_delta<BS>, dim3(grid), dim3(BS), 0, s, ws.level_off, l,
                           (int32_t)(l == levels - 1), g->row_ptr, g->col_idx, ws.queue, ws.qmask,
                           ws.front[(l + 1) & 1], ws.front[lvl_par], ws.sigma, ws.delta);
    }
    SP_HIP(hipGetLastError());
    bool any_out = false;
    SlotTable tbl{};
    for (int32_t i = 0; i < kSlots; ++i) {
        tbl.out[i] = (bc_of_slot && i < nslots) ? bc_of_slot[i] : nullptr;
        any_out |= tbl.out[i] != nullptr;
    }
    if (any_out) {
        hipLaunchKernelGGL(k_ms_bc<BS>, dim3(grid_for(n, BS, maxb)), dim3(BS), 0, s, n, ws.seen,
                           ws.delta, ws.slot_src, nslots, tbl);
        SP_HIP(hipGetLastError());
    }
    if (res) {
        res->levels = levels;
        res->reached = (int64_t)c.reached_pairs;
        std::memcpy(&res->sigma_max, &c.sigma_max_bits, sizeof(double));
        res->flagged = __builtin_popcountll(c.flagged_slots);
        res->td = c.topdown_levels;
        res->bu = c.bottomup_levels;
        res->entries = off[levels];
    }
    if (keep_levels) ws.kept_off = std::move(off);
    return SP_OK;
}

sp_status batch_run(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                    double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s,
                    BatchResult *res, bool keep_levels) {
    if (nslots < 1 || nslots > kSlots) {
        set_error("batch of %d sources (1..64 allowed)", nslots);
        return SP_ERR_INVALID_ARGUMENT;
    }
    switch (o.block) {
        case 128: return batch_run_bs<128>(g, ws, srcs, nslots, bc_of_slot, o, s, res, keep_levels);
        case 512: return batch_run_bs<512>(g, ws, srcs, nslots, bc_of_slot, o, s, res, keep_levels);
        default: return batch_run_bs<256>(g, ws, srcs, nslots, bc_of_slot, o, s, res, keep_levels);
    }
}

sp_status batch_extract(sp_graph g, BatchWorkspace &ws, int32_t nslots, int32_t *out_dist,
                        double *out_sigma, double *out_delta, hipStream_t s) {
    const int64_t total = (int64_t)nslots * g->n;
    SP_TRY(launch_fill_i32(out_dist, total, -1, s));
    if (out_sigma) SP_TRY(launch_fill_f64(out_sigma, total, 0.0, s));
    if (out_delta) SP_TRY(launch_fill_f64(out_delta, total, 0.0, s));
    const std::vector<int32_t> &off = ws.kept_off;
    for (size_t l = 0; l + 1 < off.size(); ++l) {
        const int64_t cnt = off[l + 1] - off[l];
        if (cnt <= 0) continue;
        hipLaunchKernelGGL(k_ms_extract, dim3(grid_for(cnt * kWave, 256, 4096)), dim3(256), 0, s,
                           ws.queue, ws.qmask, off[l], off[l + 1], (int32_t)l, g->n, ws.sigma,
                           ws.delta, out_dist, out_sigma, out_delta);
    }
    SP_HIP(hipGetLastError());
    return SP_OK;
}

}  // namespace sp
