// Per-source Brandes pass on the GPU: one source at a time.
//
// Forward (paper Section 2.3.2 "iterateInBFS", Appendix Fig. "BC computation
// in StarPlat"): levels are expanded one after another.  A level is
//   discover: the next frontier F_{l+1} = unreached vertices adjacent to F_l,
//             either top-down (scan the adjacency of F_l, claim with a CAS on
//             dist) or bottom-up (every unreached vertex scans its own
//             adjacency and stops once it finds a neighbour in F_l);
//   sigma:    every w in F_{l+1} sums sigma over its DAG parents (neighbours
//             at level l) -- a pull, so no floating-point atomics;
//   advance:  one thread moves the frontier window and picks the direction of
//             the next level from the frontier's and the unreached vertices'
//             adjacency sizes;
//   sigma_hub: path counts of the new level's hubs (see kHubDeg), chunk by
//             chunk.
// The queue holds the vertices in level order; level_off[l] is where level l
// starts, so the reverse pass replays the levels without a second BFS.
//
// Reverse ("iterateInReverse"): for l = L-1 down to 1 each v in F_l sums
// (sigma[v] / sigma[w]) * (1 + delta[w]) over its DAG children w (level l+1)
// and adds delta[v] to BC[v]; the source (level 0) is skipped.  Sums are
// formed chunk by chunk in a fixed order (wave_chunk_sum), so every vertex's
// value is independent of where it sits in the queue.
//
// Level loops run on the device: the host enqueues a chunk of levels, whose
// kernels return at once after the control block says `done`, and reads the
// control block back once per chunk.
#include "common.h"
#include "devutil.h"
#include "levels.h"

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
// Directed graphs: register a vertex of the level being built whose incoming
// row is longer than the hub threshold (list rebuilt every level).
__device__ __forceinline__ void in_hub_register(LevelCtl *c, HubEntry *list, long long cap, int32_t v,
                                                int32_t entry, int32_t deg) {
    hub_register(&c->in_hub_pack_.v, list, cap, 0, v, entry, deg);
}

// A hub of the level being built (split chunking, see split_hub_nchunks).
__device__ __forceinline__ void out_hub_register(LevelCtl *c, HubEntry *list, long long cap,
                                                 int32_t v, int32_t entry, int32_t deg) {
    hub_register(&c->hub_pack_.v, list, cap, c->hub_next, v, entry, deg);
}

__global__ void k_src_init(LevelCtl *c, int32_t *dist, double *sigma, int32_t *queue,
                           int32_t *level_off, HubEntry *hub_list, int32_t *hub_off,
                           int32_t *hub_lvl_chunks, const int32_t *rp, int32_t src, int32_t n,
                           long long nnz, double alpha, double beta, int32_t hub_deg) {
    const int32_t deg = rp[src + 1] - rp[src];
    c->level = 0;
    c->lo = 0;
    c->hi = 1;
    c->tail_.v = 1;
    c->done = 0;
    c->mode = MODE_TOPDOWN;
    c->overflow_.v = 0;
    c->front_deg = (unsigned long long)deg;
    c->next_deg_.v = 0;
    c->unset_deg = (unsigned long long)(nnz - deg);
    c->reached_pairs = 1;
    c->sigma_max_bits_.v = (unsigned long long)__double_as_longlong(1.0);
    c->flagged_slots_.v = 0;
    c->settled_deg_.v = 0;
    c->alpha = alpha;
    c->beta = beta;
    c->n_vertices = n;
    c->topdown_levels = 0;
    c->bottomup_levels = 0;
    const bool hub = deg > hub_deg;
    const int32_t nch = hub ? split_hub_nchunks(deg) : 0;
    if (hub) hub_list[0] = HubEntry{src, 0, 0, nch};
    c->hub_pack_.v = 0;
    c->in_hub_n = 0;
    c->in_hub_nchunks = 0;
    c->in_hub_pack_.v = 0;
    c->hub_lo = 0;
    c->hub_hi = hub ? 1 : 0;
    c->hub_nchunks = nch;
    c->hub_next = c->hub_hi;
    hub_off[0] = 0;
    hub_off[1] = c->hub_hi;
    hub_lvl_chunks[0] = nch;
    dist[src] = 0;
    sigma[src] = 1.0;
    queue[0] = src;
    level_off[0] = 0;
    level_off[1] = 1;
}

// Top-down discovery.  blockIdx.y == 0: the block takes BS frontier vertices
// (hubs excluded), scans their degrees, and walks the concatenated adjacency BS
// entries at a time, one entry per lane.  blockIdx.y == 1: blocks walk the
// chunks of the frontier's hubs.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_topdown(LevelCtl *c, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, int32_t *dist,
                                                    int32_t *queue,
                                                    const HubEntry *__restrict__ hub_list,
                                                    unsigned long long *prof, int32_t hub_deg) {
    if (c->done || c->mode != MODE_TOPDOWN) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_scan[BS / kWave + 1];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ unsigned long long s_red[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lo = c->lo, hi = c->hi, nl = c->level + 1, n = c->n_vertices;
    unsigned long long my_items = 0, my_edges = 0;
    if (blockIdx.y == 0) {
        for (int32_t b = lo + blockIdx.x * BS; b < hi; b += gridDim.x * BS) {
            const int32_t i = b + threadIdx.x;
            int32_t beg = 0, deg = 0;
            if (i < hi) {
                const int32_t v = queue[i];
                beg = rp[v];
                deg = rp[v + 1] - beg;
                if (deg > hub_deg) deg = 0;  // chunks handled by blockIdx.y == 1
                ++my_items;
                my_edges += deg;
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
                q.stage(claim, w, &c->tail_.v, queue, n, &c->overflow_.v);
            }
            __syncthreads();
        }
    } else {
        const int32_t hlo = c->hub_lo, hhi = c->hub_hi, nch = c->hub_nchunks;
        for (int32_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const HubEntry h = hub_list[hub_find(hub_list, hlo, hhi, k)];
            int32_t beg, end;
            if (!hub_chunk_range(h, k, rp, beg, end)) continue;
            my_edges += (threadIdx.x == 0) ? (unsigned long long)(end - beg) : 0ull;
            for (int32_t e0 = beg; e0 < end; e0 += BS) {
                const int32_t e = e0 + threadIdx.x;
                bool claim = false;
                int32_t w = 0;
                if (e < end) {
                    w = ci[e];
                    if (dist[w] < 0) claim = atomicCAS(&dist[w], -1, nl) == -1;
                }
                q.stage(claim, w, &c->tail_.v, queue, n, &c->overflow_.v);
            }
        }
    }
    q.finish(&c->tail_.v, queue, n, &c->overflow_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// Bottom-up discovery: every unreached vertex looks for a neighbour on the
// current level, 8 entries per lane group, and stops once it finds one.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_bottomup(LevelCtl *c, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, int32_t *dist,
                                                     int32_t *queue, unsigned long long *prof) {
    if (c->done || c->mode != MODE_BOTTOMUP) return;
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ int32_t s_coff[BS], s_beg[BS], s_deg[BS];
    __shared__ double s_acc[BS];
    __shared__ unsigned long long s_red[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int wbase = threadIdx.x & ~(kWave - 1);
    const WaveScratch ws{s_coff + wbase, s_beg + wbase, s_deg + wbase, s_acc + wbase, nullptr};
    const int32_t lvl = c->level, n = c->n_vertices;
    unsigned long long my_items = 0, my_edges = 0;
    for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
        const int32_t v = b + threadIdx.x;
        int32_t beg = 0, deg = 0;
        if (v < n && dist[v] < 0) {
            beg = rp[v];
            deg = rp[v + 1] - beg;
            ++my_items;
        }
        const bool found = wave_chunk_any(beg, deg, ws, [&](int32_t e, int32_t) {
            ++my_edges;
            return dist[ci[e]] == lvl;
        });
        if (found) dist[v] = lvl + 1;
        q.stage(found, v, &c->tail_.v, queue, n, &c->overflow_.v);
    }
    q.finish(&c->tail_.v, queue, n, &c->overflow_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// Path counts of the new frontier: sigma[w] = sum of sigma[u] over neighbours
// u on the current level.  Hubs are registered for k_src_sigma_hub.
template <int BS>
__global__ __launch_bounds__(BS) void k_src_sigma(LevelCtl *c, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const int32_t *__restrict__ queue,
                                                  const int32_t *__restrict__ dist, double *sigma,
                                                  HubEntry *hub_list, long long hub_cap,
                                                  unsigned long long *prof, int32_t hub_deg,
                                                  const int32_t *__restrict__ rp_out,
                                                  HubEntry *in_list, long long in_cap) {
    if (c->done) return;
    __shared__ int32_t s_coff[BS], s_beg[BS], s_deg[BS];
    __shared__ double s_acc[BS];
    __shared__ unsigned long long s_red[1];
    const int wbase = threadIdx.x & ~(kWave - 1);
    const WaveScratch ws{s_coff + wbase, s_beg + wbase, s_deg + wbase, s_acc + wbase, nullptr};
    const int32_t lvl = c->level, hi = c->hi, tail = min(c->tail_.v, c->n_vertices);
    const int lane = lane_id();
    unsigned long long my_deg = 0, my_items = 0, my_pairs = 0, my_scan = 0;
    double my_max = 0.0;
    bool large = false;
    for (int32_t b = hi + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < tail;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        int32_t w = -1, beg = 0, deg = 0;
        if (i < tail) {
            w = queue[i];
            beg = rp[w];
            deg = rp[w + 1] - beg;
        }
        const bool hub = deg > hub_deg;
        const double s = wave_chunk_sum(beg, hub ? 0 : deg, ws, [&](int32_t e, int32_t) {
            const int32_t u = ci[e];
            if (dist[u] != lvl) return 0.0;
            ++my_pairs;
            return sigma[u];
        });
        if (w >= 0) {
            my_deg += (unsigned long long)deg;
            ++my_items;
            if (in_list) {
                // directed: rows walked by discovery and delta are the
                // outgoing ones; the chunked path counts use in_list
                const int32_t dout = rp_out[w + 1] - rp_out[w];
                if (dout > hub_deg) out_hub_register(c, hub_list, hub_cap, w, i, dout);
                if (hub) in_hub_register(c, in_list, in_cap, w, i, deg);
            } else if (hub) {
                out_hub_register(c, hub_list, hub_cap, w, i, deg);
            }
            if (!hub) {
                my_scan += (unsigned long long)deg;
                sigma[w] = s;
                my_max = fmax(my_max, s);
                large |= sigma_is_large(s);
            }
        }
    }
    my_max = wave_max_f64(my_max);
    if (lane == 0) atomic_max_nonneg_f64(&c->sigma_max_bits_.v, my_max);
    if (__ballot(large) && lane == 0) atomicOr(&c->flagged_slots_.v, 1ull);
    block_add_u64<BS>(my_deg, s_red, &c->next_deg_.v);
    flush_counters<BS>(prof, my_items, my_scan, my_pairs, s_red);
}

__global__ void k_src_advance(LevelCtl *c, int32_t *level_off, int32_t *hub_off,
                              int32_t *hub_lvl_chunks) {
    if (c->done) return;
    if (c->mode == MODE_TOPDOWN) c->topdown_levels++; else c->bottomup_levels++;
    const int32_t nf = c->tail_.v - c->hi;
    if (nf <= 0) {
        c->done = 1;
        return;
    }
    const int32_t nl = c->level + 1;
    level_off[nl + 1] = c->tail_.v;
    const unsigned long long hp = c->hub_pack_.v;
    c->hub_lo = c->hub_next;
    c->hub_hi = c->hub_next + (int32_t)(hp >> 40);
    c->hub_nchunks = (int32_t)(hp & ((1ull << 40) - 1));
    c->hub_next = c->hub_hi;
    c->hub_pack_.v = 0;
    hub_off[nl + 1] = c->hub_hi;
    hub_lvl_chunks[nl] = c->hub_nchunks;
    const unsigned long long ip = c->in_hub_pack_.v;
    c->in_hub_n = (int32_t)(ip >> 40);
    c->in_hub_nchunks = (int32_t)(ip & ((1ull << 40) - 1));
    c->in_hub_pack_.v = 0;
    c->front_deg = c->next_deg_.v;
    c->unset_deg -= c->next_deg_.v;
    c->next_deg_.v = 0;
    c->reached_pairs += (unsigned long long)nf;
    c->lo = c->hi;
    c->hi = c->tail_.v;
    c->level = nl;
    if (c->mode == MODE_TOPDOWN) {
        if ((double)c->front_deg * c->alpha > (double)c->unset_deg) c->mode = MODE_BOTTOMUP;
    } else {
        if ((double)nf * c->beta < (double)c->n_vertices) c->mode = MODE_TOPDOWN;
    }
}

// Path counts of the current level's hubs (parents one level up).
template <int BS>
__global__ __launch_bounds__(BS) void k_src_sigma_hub(LevelCtl *c, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const int32_t *__restrict__ dist,
                                                      double *sigma, const HubEntry *hub_list,
                                                      unsigned int *hub_cnt, double *partial,
                                                      unsigned long long *prof, int32_t use_in) {
    if (c->done) return;
    // undirected: the level's hub segment; directed: the incoming-row list
    const int32_t hlo = use_in ? 0 : c->hub_lo, hhi = use_in ? c->in_hub_n : c->hub_hi;
    const int32_t nch = use_in ? c->in_hub_nchunks : c->hub_nchunks, pl = c->level - 1;
    __shared__ unsigned long long s_red[1];
    unsigned long long my_edges = 0, my_pairs = 0;
    for_xcd_chunks<BS>(nch, [&](int64_t k) {
        const HubEntry h = hub_list[hub_find(hub_list, hlo, hhi, (int32_t)k)];
        int32_t beg, end;
        if (!hub_chunk_range(h, k, rp, beg, end)) return;
        if (lane_id() == 0) my_edges += (unsigned long long)(end - beg);
        hub_chunk((int32_t)k, beg, end, partial, [&](int32_t e) {
            const int32_t u = ci[e];
            if (dist[u] != pl) return 0.0;
            ++my_pairs;
            return sigma[u];
        });
    });
    flush_counters<BS>(prof, 0, my_edges, my_pairs, s_red);
    (void)hub_cnt;
}

// Path counts of the current level's hubs from their chunk sums (a thread per hub).
__global__ void k_src_sigma_hub_fin(LevelCtl *c, double *sigma, const HubEntry *__restrict__ hub_list,
                                    const double *__restrict__ partial, int32_t use_in) {
    if (c->done) return;
    const int32_t hlo = use_in ? 0 : c->hub_lo, hhi = use_in ? c->in_hub_n : c->hub_hi;
    for (int64_t j = hlo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < hhi;
         j += (int64_t)gridDim.x * blockDim.x) {
        const HubEntry h = hub_list[j];
        const double s = sum_hub_chunks(partial, h.chunk_base, h.nchunks);
        sigma[h.v] = s;
        atomic_max_nonneg_f64(&c->sigma_max_bits_.v, s);
        if (sigma_is_large(s)) atomicOr(&c->flagged_slots_.v, 1ull);
    }
}

// Reverse sweep over one level (hubs excluded; see k_src_delta_hub).
template <int BS>
__global__ __launch_bounds__(BS) void k_src_delta(const int32_t *__restrict__ level_off, int32_t lvl,
                                                  const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const int32_t *__restrict__ queue,
                                                  const int32_t *__restrict__ dist,
                                                  const double *__restrict__ sigma, double *delta,
                                                  double *bc, unsigned long long *prof, int32_t hub_deg) {
    __shared__ int32_t s_coff[BS], s_beg[BS], s_deg[BS];
    __shared__ double s_acc[BS], s_val[BS];
    __shared__ unsigned long long s_red[1];
    const int wbase = threadIdx.x & ~(kWave - 1);
    const WaveScratch ws{s_coff + wbase, s_beg + wbase, s_deg + wbase, s_acc + wbase, s_val + wbase};
    const int32_t lo = level_off[lvl], hi = level_off[lvl + 1], nl = lvl + 1;
    const int lane = lane_id();
    unsigned long long my_items = 0, my_edges = 0, my_pairs = 0;
    for (int32_t b = lo + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < hi;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        int32_t v = -1, beg = 0, deg = 0;
        double sv = 0.0;
        if (i < hi) {
            v = queue[i];
            beg = rp[v];
            deg = rp[v + 1] - beg;
            sv = sigma[v];
        }
        const bool hub = deg > hub_deg;
        ws.val[lane] = sv;
        const double acc = wave_chunk_sum(beg, hub ? 0 : deg, ws, [&](int32_t e, int32_t a) {
            const int32_t w = ci[e];
            if (dist[w] != nl) return 0.0;
            ++my_pairs;
            return (ws.val[a] / sigma[w]) * (1.0 + delta[w]);
        });
        if (v >= 0 && !hub) {
            delta[v] = acc;
            if (bc) bc[v] += acc;
            ++my_items;
            my_edges += deg;
        }
    }
    flush_counters<BS>(prof, my_items, my_edges, my_pairs, s_red);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_src_delta_hub(
    const int32_t *__restrict__ hub_off, const int32_t *__restrict__ hub_lvl_chunks, int32_t lvl,
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const int32_t *__restrict__ dist,
    const double *__restrict__ sigma, double *delta, double *bc, const HubEntry *hub_list,
    unsigned int *hub_cnt, double *partial, unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    unsigned long long my_edges = 0, my_pairs = 0;
    const int32_t hlo = hub_off[lvl], hhi = hub_off[lvl + 1], nch = hub_lvl_chunks[lvl];
    const int32_t nl = lvl + 1;
    for_xcd_chunks<BS>(nch, [&](int64_t k) {
        const HubEntry h = hub_list[hub_find(hub_list, hlo, hhi, (int32_t)k)];
        int32_t beg, end;
        if (!hub_chunk_range(h, k, rp, beg, end)) return;
        const double sv = sigma[h.v];
        if (lane_id() == 0) my_edges += (unsigned long long)(end - beg);
        hub_chunk((int32_t)k, beg, end, partial, [&](int32_t e) {
            const int32_t w = ci[e];
            if (dist[w] != nl) return 0.0;
            ++my_pairs;
            return (sv / sigma[w]) * (1.0 + delta[w]);
        });
    });
    flush_counters<BS>(prof, 0, my_edges, my_pairs, s_red);
    (void)hub_cnt;
    (void)bc;
}

// Dependencies of one level's hubs from their chunk sums (a thread per hub).
__global__ void k_src_delta_hub_fin(const int32_t *__restrict__ hub_off, int32_t lvl, double *delta,
                                    double *bc, const HubEntry *__restrict__ hub_list,
                                    const double *__restrict__ partial) {
    const int32_t hlo = hub_off[lvl], hhi = hub_off[lvl + 1];
    for (int64_t j = hlo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < hhi;
         j += (int64_t)gridDim.x * blockDim.x) {
        const HubEntry h = hub_list[j];
        const double s = sum_hub_chunks(partial, h.chunk_base, h.nchunks);
        delta[h.v] = s;
        if (bc) bc[h.v] += s;
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
    SP_TRY(dev_alloc((void **)&ws.hub_off, (size_t)ws.level_cap * sizeof(int32_t)));
    SP_TRY(dev_alloc((void **)&ws.hub_lvl_chunks, (size_t)ws.level_cap * sizeof(int32_t)));
    SP_TRY(dev_alloc((void **)&ws.hub_list, ((size_t)g->n_hubs + 1) * sizeof(HubEntry)));
    SP_TRY(dev_alloc((void **)&ws.in_hub_list, ((size_t)g->n_hubs_in + 1) * sizeof(HubEntry)));
    SP_TRY(dev_alloc((void **)&ws.hub_cnt, ((size_t)g->n_hubs + 1) * sizeof(unsigned int)));
    SP_TRY(dev_alloc((void **)&ws.partial,
                     ((size_t)std::max(g->split_hub_chunks, g->split_hub_chunks_in) + 1) * sizeof(double)));
    SP_HIP(hipMemset(ws.hub_cnt, 0, ((size_t)g->n_hubs + 1) * sizeof(unsigned int)));
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
    dev_free(ws.hub_off);
    dev_free(ws.hub_lvl_chunks);
    dev_free(ws.hub_list);
    dev_free(ws.in_hub_list);
    dev_free(ws.hub_cnt);
    dev_free(ws.partial);
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
    const int maxb = device_cu_count() * 8;
    const int grid = grid_for((int64_t)n, BS, maxb);
    // Hub rows: discovery and the reverse pass walk outgoing rows, the path
    // counts incoming ones.  On an undirected graph they are the same rows and
    // one hub list serves all passes; a directed graph keeps a second list of
    // the level's long incoming rows for the path counts.
    const bool hubs = g->n_hubs > 0;
    const bool hubs_in = g->n_hubs_in > 0;
    const bool directed = g->directed;
    const int32_t hub_deg = kHubDeg;
    const bool may_pull = o.alpha > 0 && g->max_degree > 8;  // sparse meshes never pull
    SP_TRY(launch_fill_i32(ws.dist, n, -1, s));
    hipLaunchKernelGGL(k_src_init, dim3(1), dim3(1), 0, s, ws.ctl, ws.dist, ws.sigma, ws.queue,
                       ws.level_off, ws.hub_list, ws.hub_off, ws.hub_lvl_chunks,
                       (const int32_t *)g->row_ptr, src, n, (long long)g->nnz,
                       may_pull ? o.alpha : 0.0, o.beta, hub_deg);  // alpha 0: never switch to bottom-up
    SP_HIP(hipGetLastError());
    int32_t enqueued = 0;
    for (;;) {
        const int chunk = std::max(1, std::abs(o.chunk_levels));
        for (int k = 0; k < chunk; ++k) {
            {
                ProfScope ps(P_SRC_TOPDOWN, s);
                hipLaunchKernelGGL(k_src_topdown<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s,
                                   ws.ctl, g->row_ptr, g->col_idx, ws.dist, ws.queue,
                                   (const HubEntry *)ws.hub_list, prof_counters(P_SRC_TOPDOWN), hub_deg);
            }
            if (may_pull) {
                ProfScope ps(P_SRC_BOTTOMUP, s);
                hipLaunchKernelGGL(k_src_bottomup<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->rp_in,
                                   g->ci_in, ws.dist, ws.queue, prof_counters(P_SRC_BOTTOMUP));
            }
            {
                ProfScope ps(P_SRC_SIGMA, s);
                hipLaunchKernelGGL(k_src_sigma<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->rp_in,
                                   g->ci_in, ws.queue, ws.dist, ws.sigma, ws.hub_list,
                                   (long long)g->n_hubs + 1, prof_counters(P_SRC_SIGMA), hub_deg,
                                   (const int32_t *)g->row_ptr, directed ? ws.in_hub_list : nullptr,
                                   (long long)g->n_hubs_in + 1);
            }
            hipLaunchKernelGGL(k_src_advance, dim3(1), dim3(1), 0, s, ws.ctl, ws.level_off,
                               ws.hub_off, ws.hub_lvl_chunks);
            if (hubs_in) {
                ProfScope ps(P_SRC_SIGMA_HUB, s);
                const HubEntry *plist = directed ? ws.in_hub_list : ws.hub_list;
                const int hub_grid = xcd_grid(grid_for(g->split_hub_chunks_in * kWave, BS, maxb), maxb);
                hipLaunchKernelGGL(k_src_sigma_hub<BS>, dim3(hub_grid), dim3(BS), 0, s,
                                   ws.ctl, g->rp_in, g->ci_in, ws.dist, ws.sigma, plist, ws.hub_cnt,
                                   ws.partial, prof_counters(P_SRC_SIGMA_HUB), (int32_t)directed);
                hipLaunchKernelGGL(k_src_sigma_hub_fin, dim3(grid_for(g->n_hubs_in, 256, maxb)), dim3(256), 0,
                                   s, ws.ctl, ws.sigma, plist, (const double *)ws.partial, (int32_t)directed);
            }
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
    // Reverse pass, deepest level first.  The level offsets and hub chunk
    // counts that size its launches come back to the host a window of
    // kRevWindow levels at a time, into fixed buffers (no host allocation per
    // call; one synchronisation per window).
    constexpr int32_t kRevWindow = 1024;
    int32_t off_w[kRevWindow + 1], hch_w[kRevWindow];
    for (int32_t top = with_backward ? levels - 1 : 0; top >= 1; top -= kRevWindow) {
        const int32_t lo = std::max(1, top - kRevWindow + 1);  // window: levels lo..top
        SP_HIP(hipMemcpyAsync(off_w, ws.level_off + lo, sizeof(int32_t) * (top - lo + 2),
                              hipMemcpyDeviceToHost, s));
        SP_HIP(hipMemcpyAsync(hch_w, ws.hub_lvl_chunks + lo, sizeof(int32_t) * (top - lo + 1),
                              hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        const int32_t *off = off_w - lo;      // off[l] for l in [lo, top + 1]
        const int32_t *hchunks = hch_w - lo;  // hchunks[l] for l in [lo, top]
        for (int32_t l = top; l >= lo; --l) {
            const int32_t cnt = off[l + 1] - off[l];
            {
                ProfScope ps(P_SRC_DELTA, s);
                hipLaunchKernelGGL(k_src_delta<BS>, dim3(grid_for((int64_t)cnt, BS, maxb)), dim3(BS), 0, s,
                                   ws.level_off, l, g->row_ptr, g->col_idx, ws.queue, ws.dist,
                                   ws.sigma, ws.delta, bc, prof_counters(P_SRC_DELTA), hub_deg);
            }
            if (hubs && hchunks[l] > 0) {
                ProfScope ps(P_SRC_DELTA_HUB, s);
                hipLaunchKernelGGL(k_src_delta_hub<BS>,
                                   dim3(xcd_grid(grid_for((int64_t)hchunks[l] * kWave, BS, maxb), maxb)),
                                   dim3(BS), 0, s, (const int32_t *)ws.hub_off,
                                   (const int32_t *)ws.hub_lvl_chunks, l, g->row_ptr, g->col_idx,
                                   ws.dist, ws.sigma, ws.delta, bc, (const HubEntry *)ws.hub_list,
                                   ws.hub_cnt, ws.partial, prof_counters(P_SRC_DELTA_HUB));
                hipLaunchKernelGGL(k_src_delta_hub_fin, dim3(grid_for(g->n_hubs, 256, maxb)), dim3(256), 0, s,
                                   (const int32_t *)ws.hub_off, l, ws.delta, bc,
                                   (const HubEntry *)ws.hub_list, (const double *)ws.partial);
            }
        }
        SP_HIP(hipGetLastError());
    }
    if (res) {
        res->levels = levels;
        res->reached = c.hi;
        std::memcpy(&res->sigma_max, &c.sigma_max_bits_.v, sizeof(double));
        res->flagged = c.flagged_slots_.v != 0;
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
