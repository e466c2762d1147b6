// Batched multi-source Brandes pass: up to 64 sources advance level by level
// together.  Each vertex carries 64-bit source bitmaps (bit i = batch slot i):
//   seen[v]   slots that have reached v at some level so far,
//   nxt[v]    slots discovering v at the level being built,
//   front[p]  per level parity p, {mask, level tag} of v's entry at that level.
// A (vertex, mask) pair per level is an "entry"; entries of one level are
// contiguous in `queue`/`qmask`, and level_off[l] is where level l starts.
//
// Per-source arithmetic is exactly the per-source path's (paper Appendix,
// Fig. "BC computation in StarPlat"; DAG semantics of Section 2.3.2): for
// slot s, sigma[w][s] sums sigma[u][s] over neighbours u with s in
// front(l)[u], and delta[v][s] sums (sigma[v][s] / sigma[w][s]) *
// (1 + delta[w][s]) over neighbours w with s in front(l+1)[w], both in CSR
// order.  sigma and delta rows are vertex-major (64 doubles per vertex).
//
// An entry is reduced one of three ways:
//   dense  (many slots): one wave, lane = slot; the wave reads the neighbours'
//          masks 64 at a time and then up to 8 neighbour rows at once, each a
//          single coalesced access for all slots;
//   sparse (<= kSparseSlots slots, degree <= kSparseDeg): one lane walks the
//          adjacency for each of its slots (road-like graphs);
//   hub    (degree > kHubDeg): chunks of kHubChunk entries reduced by separate
//          waves into partial rows, summed in chunk order by the last one.
// Dense and sparse sums are sequential in CSR order per slot, so they give the
// same bits; every result is independent of batch composition and scheduling.
//
// Forward level:  discover (top-down: expand the entries of level l, OR the
//                 new slots into nxt[w] and claim w on the first OR;
//                 bottom-up: every vertex with unsettled slots ORs the level-l
//                 masks of its neighbours, 8 at a time per lane group, and stops
//                 when all are found) -> sigma -> advance -> sigma_hub.
// Reverse level:  delta (also re-publishes every entry's {mask, level} in
//                 front(l) for the next step) -> delta_hub.
// BC:             per vertex, slots in ascending order, skipping the slot
//                 whose source is the vertex itself.
#include "common.h"
#include "devutil.h"
#include "levels.h"

namespace sp {

struct SlotTable {
    double *out[kSlots];
};

constexpr int kSparseSlots = 2;
constexpr int32_t kSparseDeg = 64;
constexpr uint32_t kNoTag = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long mask_of(uint4 f) {
    return (unsigned long long)f.x | ((unsigned long long)f.y << 32);
}

__device__ __forceinline__ uint4 make_front(unsigned long long m, uint32_t tag) {
    return make_uint4((uint32_t)m, (uint32_t)(m >> 32), tag, 0u);
}

__device__ __forceinline__ int32_t rl_i32(int32_t v, int j) { return __builtin_amdgcn_readlane(v, j); }

__device__ __forceinline__ unsigned long long rl_u64(unsigned long long v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

// lane = slot: sum over adjacency entries [beg, end) of sigma[u][lane] for
// neighbours u whose level-`tag` mask (restricted to m) holds the lane.
__device__ __forceinline__ double dense_sigma(int32_t beg, int32_t end, unsigned long long m,
                                              uint32_t tag, const int32_t *__restrict__ ci,
                                              const uint4 *__restrict__ front,
                                              const double *__restrict__ sigma,
                                              unsigned long long &pairs) {
    const int lane = lane_id();
    double acc = 0.0;
    for (int32_t e0 = beg; e0 < end; e0 += kWave) {
        const int32_t e = e0 + lane;
        int32_t u = 0;
        unsigned long long f = 0;
        if (e < end) {
            u = ci[e];
            const uint4 fu = front[u];
            if (fu.z == tag) f = mask_of(fu) & m;
        }
        unsigned long long nz = __ballot(f != 0ull);
        while (nz) {
            int32_t uj[8];
            unsigned long long fj[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (nz) {
                    const int j = __ffsll((long long)nz) - 1;
                    nz &= nz - 1;
                    uj[t] = rl_i32(u, j);
                    fj[t] = rl_u64(f, j);
                } else {
                    uj[t] = 0;
                    fj[t] = 0;
                }
            }
            double x[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                x[t] = ((fj[t] >> lane) & 1ull) ? sigma[(int64_t)uj[t] * kSlots + lane] : 0.0;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if ((fj[t] >> lane) & 1ull) acc += x[t];
                pairs += (unsigned long long)__popcll(fj[t]);
            }
        }
    }
    return acc;
}

// lane = slot: sum over [beg, end) of (sv / sigma[w][lane]) * (1 + delta[w][lane])
// for neighbours w whose level-`tag` mask (restricted to m) holds the lane.
__device__ __forceinline__ double dense_delta(int32_t beg, int32_t end, unsigned long long m,
                                              uint32_t tag, double sv,
                                              const int32_t *__restrict__ ci,
                                              const uint4 *__restrict__ front,
                                              const double *__restrict__ sigma,
                                              const double *__restrict__ delta,
                                              unsigned long long &pairs) {
    const int lane = lane_id();
    double acc = 0.0;
    for (int32_t e0 = beg; e0 < end; e0 += kWave) {
        const int32_t e = e0 + lane;
        int32_t w = 0;
        unsigned long long g = 0;
        if (e < end) {
            w = ci[e];
            const uint4 fw = front[w];
            if (fw.z == tag) g = mask_of(fw) & m;
        }
        unsigned long long nz = __ballot(g != 0ull);
        while (nz) {
            int32_t wj[8];
            unsigned long long gj[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (nz) {
                    const int j = __ffsll((long long)nz) - 1;
                    nz &= nz - 1;
                    wj[t] = rl_i32(w, j);
                    gj[t] = rl_u64(g, j);
                } else {
                    wj[t] = 0;
                    gj[t] = 0;
                }
            }
            double sg[8], dl[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const bool on = (gj[t] >> lane) & 1ull;
                const int64_t o = (int64_t)wj[t] * kSlots + lane;
                sg[t] = on ? sigma[o] : 1.0;
                dl[t] = on ? delta[o] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if ((gj[t] >> lane) & 1ull) acc += (sv / sg[t]) * (1.0 + dl[t]);
                pairs += (unsigned long long)__popcll(gj[t]);
            }
        }
    }
    return acc;
}

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
                          uint4 *front0, double *sigma, int32_t *level_off, HubEntry *hub_list,
                          int32_t *hub_off, int32_t *hub_lvl_chunks, int32_t n, long long nnz,
                          unsigned long long active, double alpha, double beta) {
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
        unsigned long long fdeg = 0, settled = 0, pairs = 0;
        int32_t nh = 0, nch = 0;
        for (int32_t i = 0; i < n0; ++i) {
            const int32_t v = queue[i];
            const int32_t d = rp[v + 1] - rp[v];
            fdeg += (unsigned long long)d;
            pairs += (unsigned long long)__popcll(qmask[i]);
            if (qmask[i] == active) settled += (unsigned long long)d;
            if (d > kHubDeg) {
                const int32_t k = (d + kHubChunk - 1) / kHubChunk;
                hub_list[nh++] = HubEntry{v, i, nch, k};
                nch += k;
            }
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
        c->reached_pairs = pairs;
        c->unset_deg = (unsigned long long)nnz - settled;
        c->sigma_max_bits = (unsigned long long)__double_as_longlong(1.0);
        c->flagged_slots = 0;
        c->alpha = alpha;
        c->beta = beta;
        c->n_vertices = n;
        c->topdown_levels = 0;
        c->bottomup_levels = 0;
        c->hub_pack = 0;
        c->hub_lo = 0;
        c->hub_hi = nh;
        c->hub_nchunks = nch;
        c->hub_next = nh;
        hub_off[0] = 0;
        hub_off[1] = nh;
        hub_lvl_chunks[0] = nch;
        level_off[0] = 0;
        level_off[1] = n0;
    }
}

// Top-down discovery.  blockIdx.y == 0: block gather over the frontier's
// entries (hubs excluded), one adjacency entry per lane.  blockIdx.y == 1:
// the chunks of the frontier's hubs.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_topdown(LevelCtl *c, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, int32_t *queue,
                                                   const unsigned long long *__restrict__ qmask,
                                                   const unsigned long long *__restrict__ seen,
                                                   unsigned long long *nxt,
                                                   const HubEntry *__restrict__ hub_list,
                                                   long long qcap, unsigned long long *prof) {
    if (c->done || c->mode != MODE_TOPDOWN) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_scan[BS / kWave + 1];
    __shared__ unsigned long long s_mask[BS];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ unsigned long long s_red[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lo = c->lo, hi = c->hi;
    unsigned long long my_items = 0, my_edges = 0;
    auto visit = [&](int32_t w, unsigned long long fm) {
        const unsigned long long nm = fm & ~seen[w];
        if (nm && (nm & ~*(volatile unsigned long long *)&nxt[w])) return atomicOr(&nxt[w], nm) == 0ull;
        return false;
    };
    if (blockIdx.y == 0) {
        for (int32_t b = lo + blockIdx.x * BS; b < hi; b += gridDim.x * BS) {
            const int32_t i = b + threadIdx.x;
            int32_t beg = 0, deg = 0;
            unsigned long long fm = 0;
            if (i < hi) {
                const int32_t v = queue[i];
                fm = qmask[i];
                beg = rp[v];
                deg = rp[v + 1] - beg;
                if (deg > kHubDeg) deg = 0;
                ++my_items;
                my_edges += deg;
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
                    claim = visit(w, s_mask[a]);
                }
                q.stage(claim, w, &c->tail, queue, qcap, &c->overflow);
            }
            __syncthreads();
        }
    } else {
        const int32_t hlo = c->hub_lo, hhi = c->hub_hi, nch = c->hub_nchunks;
        for (int32_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const HubEntry h = hub_list[hub_find(hub_list, hlo, hhi, k)];
            const unsigned long long fm = qmask[h.entry];
            const int32_t beg = rp[h.v] + (k - h.chunk_base) * kHubChunk;
            const int32_t end = min(rp[h.v + 1], beg + kHubChunk);
            my_edges += (threadIdx.x == 0) ? (unsigned long long)(end - beg) : 0ull;
            for (int32_t e0 = beg; e0 < end; e0 += BS) {
                const int32_t e = e0 + threadIdx.x;
                bool claim = false;
                int32_t w = 0;
                if (e < end) {
                    w = ci[e];
                    claim = visit(w, fm);
                }
                q.stage(claim, w, &c->tail, queue, qcap, &c->overflow);
            }
        }
    }
    q.finish(&c->tail, queue, qcap, &c->overflow);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// Bottom-up discovery: every vertex with unsettled slots ORs the level-l masks
// of its neighbours, 8 entries per lane group, until all its unsettled slots
// are found.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_bottomup(LevelCtl *c, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const unsigned long long *__restrict__ seen,
                                                    unsigned long long *nxt,
                                                    const uint4 *__restrict__ front_cur,
                                                    int32_t *queue, unsigned long long active,
                                                    long long qcap, unsigned long long *prof) {
    if (c->done || c->mode != MODE_BOTTOMUP) return;
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ int32_t s_coff[BS], s_beg[BS], s_deg[BS];
    __shared__ unsigned long long s_acc[BS], s_uns[BS];
    __shared__ unsigned long long s_red[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int lane = lane_id();
    const int wb = threadIdx.x & ~(kWave - 1);
    int32_t *coff = s_coff + wb, *bg = s_beg + wb, *dg = s_deg + wb;
    unsigned long long *acc = s_acc + wb, *uns = s_uns + wb;
    const uint32_t lvl = (uint32_t)c->level;
    const int32_t n = c->n_vertices;
    const int g = lane >> 3, j = lane & 7;
    unsigned long long my_items = 0, my_edges = 0;
    for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
        const int32_t v = b + threadIdx.x;
        int32_t beg = 0, deg = 0;
        unsigned long long u_s = 0;
        if (v < n) {
            u_s = active & ~seen[v];
            if (u_s) {
                beg = rp[v];
                deg = rp[v + 1] - beg;
                ++my_items;
            }
        }
        const int32_t nch = (deg + 7) >> 3;
        const int32_t incl = wave_incl_scan(nch);
        const int32_t total = __shfl(incl, kWave - 1, kWave);
        coff[lane] = incl - nch;
        bg[lane] = beg;
        dg[lane] = deg;
        acc[lane] = 0;
        uns[lane] = u_s;
        __builtin_amdgcn_wave_barrier();
        for (int32_t t0 = 0; t0 < total; t0 += 8) {
            const int32_t k = t0 + g;
            int32_t a = -1;
            unsigned long long x = 0;
            if (k < total) {
                int32_t lo = 0, hi = kWave - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (coff[mid] <= k) lo = mid; else hi = mid - 1;
                }
                a = lo;
                const int32_t off = (k - coff[a]) * 8 + j;
                const unsigned long long want = uns[a];
                if (off < dg[a] && acc[a] != want) {
                    const uint4 f = front_cur[ci[bg[a] + off]];
                    if (f.z == lvl) x = mask_of(f) & want;
                    ++my_edges;
                }
            }
            x |= __shfl_xor(x, 1, kWave);
            x |= __shfl_xor(x, 2, kWave);
            x |= __shfl_xor(x, 4, kWave);
            if (j == 0 && x) atomicOr(&acc[a], x);  // LDS; OR is order-free
            __builtin_amdgcn_wave_barrier();
            const bool open = deg > 0 && acc[lane] != u_s;
            if (!__ballot(open)) break;
        }
        __builtin_amdgcn_wave_barrier();
        const unsigned long long found = acc[lane];
        if (found) nxt[v] = found;
        q.stage(found != 0ull, v, &c->tail, queue, qcap, &c->overflow);
    }
    q.finish(&c->tail, queue, qcap, &c->overflow);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// Path counts of the new entries [hi, tail).  Wave takes 64 entries; sparse
// ones are reduced by their own lane, dense ones by the whole wave in turn,
// hubs are registered for k_ms_sigma_hub.  Every entry's bookkeeping (qmask,
// nxt reset, seen, front of the new level) is done here.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_sigma(LevelCtl *c, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ queue,
                                                 unsigned long long *qmask, unsigned long long *seen,
                                                 unsigned long long *nxt,
                                                 const uint4 *__restrict__ front_cur,
                                                 uint4 *front_nxt, double *sigma,
                                                 HubEntry *hub_list, long long hub_cap,
                                                 unsigned long long active, long long qcap,
                                                 unsigned long long *prof) {
    if (c->done) return;
    __shared__ unsigned long long s_red[1];
    const uint32_t lvl = (uint32_t)c->level;
    const int32_t hi = c->hi;
    const int32_t tail = (int32_t)min((long long)c->tail, qcap);
    const int lane = lane_id();
    unsigned long long my_deg = 0, my_settled = 0, my_flag = 0, my_pairs = 0, my_items = 0,
                       my_dag = 0;
    double my_max = 0.0;
    for (int32_t b = hi + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < tail;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        int32_t w = 0, beg = 0, end = 0;
        unsigned long long m = 0;
        if (i < tail) {
            w = queue[i];
            m = nxt[w];
            beg = rp[w];
            end = rp[w + 1];
        }
        const int32_t deg = end - beg;
        const int pc = __popcll(m);
        const bool valid = i < tail;
        const bool hub = valid && deg > kHubDeg;
        const bool sparse = valid && !hub && pc <= kSparseSlots && deg <= kSparseDeg;
        const bool dense = valid && !hub && !sparse;
        if (sparse) {
            unsigned long long bits = m;
            while (bits) {
                const int s = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                double acc = 0.0;
                for (int32_t e = beg; e < end; ++e) {
                    const int32_t u = ci[e];
                    const uint4 fu = front_cur[u];
                    if (fu.z == lvl && ((mask_of(fu) >> s) & 1ull)) {
                        acc += sigma[(int64_t)u * kSlots + s];
                        ++my_dag;
                    }
                }
                sigma[(int64_t)w * kSlots + s] = acc;
                my_max = fmax(my_max, acc);
                if (sigma_is_large(acc)) my_flag |= 1ull << s;
            }
        }
        unsigned long long dm = __ballot(dense);
        while (dm) {
            const int jl = __ffsll((long long)dm) - 1;
            dm &= dm - 1;
            const int32_t wj = rl_i32(w, jl), bj = rl_i32(beg, jl), ej = rl_i32(end, jl);
            const unsigned long long mj = rl_u64(m, jl);
            unsigned long long pr = 0;
            const double acc = dense_sigma(bj, ej, mj, lvl, ci, front_cur, sigma, pr);
            if (lane == 0) my_dag += pr;
            if ((mj >> lane) & 1ull) {
                sigma[(int64_t)wj * kSlots + lane] = acc;
                my_max = fmax(my_max, acc);
            }
            my_flag |= __ballot(((mj >> lane) & 1ull) && sigma_is_large(acc));
        }
        if (hub) hub_register(c, hub_list, hub_cap, w, i, deg);
        if (valid) {
            qmask[i] = m;
            nxt[w] = 0;
            const unsigned long long now = seen[w] | m;
            seen[w] = now;
            front_nxt[w] = make_front(m, lvl + 1);
            my_deg += (unsigned long long)deg;
            my_pairs += (unsigned long long)pc;
            ++my_items;
            if (now == active) my_settled += (unsigned long long)deg;
        }
    }
    my_max = wave_max_f64(my_max);
    for (int o = 32; o > 0; o >>= 1) my_flag |= __shfl_xor(my_flag, o, kWave);
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits, my_max);
        if (my_flag) atomicOr(&c->flagged_slots, my_flag);
    }
    block_add_u64<BS>(my_deg, s_red, &c->next_deg);
    __syncthreads();
    block_add_u64<BS>(my_settled, s_red, &c->settled_deg);
    __syncthreads();
    block_add_u64<BS>(my_pairs, s_red, &c->reached_pairs);
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_deg, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_dag, s_red, prof + 2);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 3);
    }
}

__global__ void k_ms_advance(LevelCtl *c, int32_t *level_off, int32_t *hub_off,
                             int32_t *hub_lvl_chunks, long long qcap, long long hub_cap) {
    if (c->done) return;
    if (c->mode == MODE_TOPDOWN) c->topdown_levels++; else c->bottomup_levels++;
    const unsigned long long hp = c->hub_pack;
    if ((long long)c->tail > qcap || c->overflow ||
        (long long)c->hub_next + (long long)(hp >> 40) > hub_cap) {
        c->overflow = 1;
        c->done = 1;
        return;
    }
    const int32_t nf = c->tail - c->hi;
    if (nf <= 0) {
        c->done = 1;
        return;
    }
    const int32_t nl = c->level + 1;
    level_off[nl + 1] = c->tail;
    c->hub_lo = c->hub_next;
    c->hub_hi = c->hub_next + (int32_t)(hp >> 40);
    c->hub_nchunks = (int32_t)(hp & ((1ull << 40) - 1));
    c->hub_next = c->hub_hi;
    c->hub_pack = 0;
    hub_off[nl + 1] = c->hub_hi;
    hub_lvl_chunks[nl] = c->hub_nchunks;
    c->front_deg = c->next_deg;
    c->unset_deg -= c->settled_deg;
    c->next_deg = 0;
    c->settled_deg = 0;
    c->lo = c->hi;
    c->hi = c->tail;
    c->level = nl;
    if (c->mode == MODE_TOPDOWN) {
        if ((double)c->front_deg * c->alpha > (double)c->unset_deg) c->mode = MODE_BOTTOMUP;
    } else {
        if ((double)nf * c->beta < (double)c->n_vertices) c->mode = MODE_TOPDOWN;
    }
}

// One chunk of a hub, lane = slot: partial row of 64 doubles.  The last chunk
// of the hub to finish sums the rows in chunk order and hands the result to
// fin(lane_sum) (all lanes).
template <class Row, class Final>
__device__ __forceinline__ void ms_hub_chunk(const HubEntry &h, int32_t k, double *partial,
                                             unsigned int *cnt, Row row, Final fin) {
    const int lane = lane_id();
    const double x = row();
    partial[(int64_t)k * kSlots + lane] = x;
    __threadfence();
    unsigned int old = 0;
    if (lane == 0) old = atomicAdd(cnt, 1u);
    old = __shfl(old, 0, kWave);
    if (old == (unsigned int)h.nchunks - 1) {
        __threadfence();
        const volatile double *vp = partial;
        double s = 0.0;
        for (int32_t q = 0; q < h.nchunks; ++q) s += vp[(int64_t)(h.chunk_base + q) * kSlots + lane];
        if (lane == 0) *cnt = 0;
        fin(s);
    }
}

// Path counts of the current level's hubs (after advance), chunk by chunk.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_sigma_hub(LevelCtl *c, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const unsigned long long *__restrict__ qmask,
                                                     const uint4 *__restrict__ front_par,
                                                     double *sigma, const HubEntry *hub_list,
                                                     unsigned int *hub_cnt, double *partial,
                                                     unsigned long long *prof) {
    if (c->done) return;
    __shared__ unsigned long long s_red[1];
    const int32_t hlo = c->hub_lo, hhi = c->hub_hi, nch = c->hub_nchunks;
    const uint32_t pl = (uint32_t)c->level - 1;
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * BS + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * BS / kWave;
    unsigned long long my_dag = 0, my_edges = 0, my_flag = 0;
    double my_max = 0.0;
    for (int64_t k = wave0; k < nch; k += nwaves) {
        const int32_t jh = hub_find(hub_list, hlo, hhi, (int32_t)k);
        const HubEntry h = hub_list[jh];
        const unsigned long long m = qmask[h.entry];
        const int32_t beg = rp[h.v] + ((int32_t)k - h.chunk_base) * kHubChunk;
        const int32_t end = min(rp[h.v + 1], beg + kHubChunk);
        if (lane == 0) my_edges += (unsigned long long)(end - beg);
        unsigned long long pr = 0;
        ms_hub_chunk(h, (int32_t)k, partial, hub_cnt + (jh - hlo),
                     [&] { return dense_sigma(beg, end, m, pl, ci, front_par, sigma, pr); },
                     [&](double s) {
                         if ((m >> lane) & 1ull) {
                             sigma[(int64_t)h.v * kSlots + lane] = s;
                             my_max = fmax(my_max, s);
                         }
                         my_flag |= __ballot(((m >> lane) & 1ull) && sigma_is_large(s));
                     });
        if (lane == 0) my_dag += pr;
    }
    my_max = wave_max_f64(my_max);
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits, my_max);
        if (my_flag) atomicOr(&c->flagged_slots, my_flag);
    }
    if (prof) {
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_dag, s_red, prof + 2);
    }
}

// Reverse sweep of one level.  Every entry re-publishes {mask, level} in
// front(l); dense and sparse entries get delta here, hubs in k_ms_delta_hub.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_delta(const int32_t *__restrict__ level_off, int32_t lvl,
                                                 int32_t deepest, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ queue,
                                                 const unsigned long long *__restrict__ qmask,
                                                 const uint4 *__restrict__ front_rd,
                                                 uint4 *front_wr, const double *__restrict__ sigma,
                                                 double *delta, unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    const int32_t lo = level_off[lvl], hi = level_off[lvl + 1];
    const uint32_t nl = (uint32_t)lvl + 1;
    const int lane = lane_id();
    unsigned long long my_items = 0, my_edges = 0, my_pairs = 0, my_slots = 0;
    for (int32_t b = lo + (int32_t)(blockIdx.x * BS + threadIdx.x) - lane; b < hi;
         b += gridDim.x * BS) {
        const int32_t i = b + lane;
        const bool valid = i < hi;
        int32_t v = 0, beg = 0, end = 0;
        unsigned long long m = 0;
        if (valid) {
            v = queue[i];
            m = qmask[i];
            beg = rp[v];
            end = rp[v + 1];
            front_wr[v] = make_front(m, (uint32_t)lvl);
            ++my_items;
            my_slots += (unsigned long long)__popcll(m);
        }
        const int32_t deg = end - beg;
        if (deepest) {  // no children: delta is zero
            unsigned long long bits = m;
            while (bits) {
                const int s = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                delta[(int64_t)v * kSlots + s] = 0.0;
            }
            continue;
        }
        const bool hub = valid && deg > kHubDeg;
        const bool sparse = valid && !hub && __popcll(m) <= kSparseSlots && deg <= kSparseDeg;
        const bool dense = valid && !hub && !sparse;
        if (sparse) {
            my_edges += (unsigned long long)deg;
            unsigned long long bits = m;
            while (bits) {
                const int s = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                const double sv = sigma[(int64_t)v * kSlots + s];
                double acc = 0.0;
                for (int32_t e = beg; e < end; ++e) {
                    const int32_t w = ci[e];
                    const uint4 fw = front_rd[w];
                    if (fw.z == nl && ((mask_of(fw) >> s) & 1ull)) {
                        const int64_t o = (int64_t)w * kSlots + s;
                        acc += (sv / sigma[o]) * (1.0 + delta[o]);
                        ++my_pairs;
                    }
                }
                delta[(int64_t)v * kSlots + s] = acc;
            }
        }
        unsigned long long dm = __ballot(dense);
        while (dm) {
            const int jl = __ffsll((long long)dm) - 1;
            dm &= dm - 1;
            const int32_t vj = rl_i32(v, jl), bj = rl_i32(beg, jl), ej = rl_i32(end, jl);
            const unsigned long long mj = rl_u64(m, jl);
            const bool mine = (mj >> lane) & 1ull;
            const double sv = mine ? sigma[(int64_t)vj * kSlots + lane] : 0.0;
            unsigned long long pr = 0;
            const double acc = dense_delta(bj, ej, mj, nl, sv, ci, front_rd, sigma, delta, pr);
            if (lane == 0) {
                my_pairs += pr;
                my_edges += (unsigned long long)(ej - bj);
            }
            if (mine) delta[(int64_t)vj * kSlots + lane] = acc;
        }
    }
    if (prof) {
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
        __syncthreads();
        block_add_u64<BS>(my_slots, s_red, prof + 3);
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_ms_delta_hub(
    const int32_t *__restrict__ hub_off, const int32_t *__restrict__ hub_lvl_chunks, int32_t lvl,
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const unsigned long long *__restrict__ qmask, const uint4 *__restrict__ front_rd,
    const double *__restrict__ sigma, double *delta, const HubEntry *hub_list,
    unsigned int *hub_cnt, double *partial, unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    const int32_t hlo = hub_off[lvl], hhi = hub_off[lvl + 1], nch = hub_lvl_chunks[lvl];
    const uint32_t nl = (uint32_t)lvl + 1;
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * BS + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * BS / kWave;
    unsigned long long my_edges = 0, my_pairs = 0;
    for (int64_t k = wave0; k < nch; k += nwaves) {
        const int32_t jh = hub_find(hub_list, hlo, hhi, (int32_t)k);
        const HubEntry h = hub_list[jh];
        const unsigned long long m = qmask[h.entry];
        const int32_t beg = rp[h.v] + ((int32_t)k - h.chunk_base) * kHubChunk;
        const int32_t end = min(rp[h.v + 1], beg + kHubChunk);
        const bool mine = (m >> lane) & 1ull;
        const double sv = mine ? sigma[(int64_t)h.v * kSlots + lane] : 0.0;
        if (lane == 0) my_edges += (unsigned long long)(end - beg);
        unsigned long long pr = 0;
        ms_hub_chunk(h, (int32_t)k, partial, hub_cnt + (jh - hlo),
                     [&] { return dense_delta(beg, end, m, nl, sv, ci, front_rd, sigma, delta, pr); },
                     [&](double s) {
                         if (mine) delta[(int64_t)h.v * kSlots + lane] = s;
                     });
        if (lane == 0) my_pairs += pr;
    }
    if (prof) {
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
    }
}

// BC[v] += delta[v][s] for slots in ascending order; consecutive slots with
// the same output array are summed in a register.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_bc(int32_t n, const unsigned long long *__restrict__ seen,
                                              const double *__restrict__ delta,
                                              const int32_t *__restrict__ slot_src, int32_t nslots,
                                              SlotTable tbl, unsigned long long *prof) {
    __shared__ int32_t s_src[kSlots];
    __shared__ unsigned long long s_red[1];
    if (threadIdx.x < kSlots) s_src[threadIdx.x] = threadIdx.x < nslots ? slot_src[threadIdx.x] : -1;
    __syncthreads();
    unsigned long long my_items = 0, my_slots = 0;
    for (int32_t v = blockIdx.x * BS + threadIdx.x; v < n; v += gridDim.x * BS) {
        const unsigned long long sm = seen[v];
        if (!sm) continue;
        ++my_items;
        my_slots += (unsigned long long)__popcll(sm);
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
    if (prof) {
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_slots, s_red, prof + 3);
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
static int64_t hub_capacity(sp_graph g) { return (int64_t)g->n_hubs * kSlots + kSlots; }

size_t batch_ws_bytes(sp_graph g, int64_t qcap) {
    const size_t V = (size_t)std::max(g->n, 1);
    return V * (8 + 8 + 16 + 16) + V * kSlots * 16 + (size_t)qcap * 12 + (V + 2) * 12 +
           kSlots * 4 + (size_t)hub_capacity(g) * sizeof(HubEntry) + ((size_t)g->n_hubs + 1) * 4 +
           ((size_t)g->hub_chunks + 1) * kSlots * 8 + sizeof(LevelCtl);
}

sp_status batch_ws_create(sp_graph g, int64_t qcap, BatchWorkspace &ws) {
    ws.device = g->device;
    ws.n = g->n;
    const size_t V = (size_t)std::max(g->n, 1);
    ws.qcap = qcap;
    ws.level_cap = (int32_t)std::min<int64_t>((int64_t)V + 2, (int64_t)INT32_MAX);
    ws.hub_cap = hub_capacity(g);
    SP_TRY(dev_alloc((void **)&ws.seen, V * 8));
    SP_TRY(dev_alloc((void **)&ws.nxt, V * 8));
    SP_TRY(dev_alloc((void **)&ws.front[0], V * 16));
    SP_TRY(dev_alloc((void **)&ws.front[1], V * 16));
    SP_TRY(dev_alloc((void **)&ws.sigma, V * kSlots * 8));
    SP_TRY(dev_alloc((void **)&ws.delta, V * kSlots * 8));
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    SP_TRY(dev_alloc((void **)&ws.level_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_lvl_chunks, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_list, (size_t)ws.hub_cap * sizeof(HubEntry)));
    SP_TRY(dev_alloc((void **)&ws.hub_cnt, ((size_t)g->n_hubs + 1) * 4));
    SP_TRY(dev_alloc((void **)&ws.partial, ((size_t)g->hub_chunks + 1) * kSlots * 8));
    SP_HIP(hipMemset(ws.hub_cnt, 0, ((size_t)g->n_hubs + 1) * 4));
    SP_TRY(dev_alloc((void **)&ws.slot_src, kSlots * 4));
    SP_TRY(dev_alloc((void **)&ws.ctl, sizeof(LevelCtl)));
    SP_HIP(hipHostMalloc((void **)&ws.ctl_host, sizeof(LevelCtl), hipHostMallocDefault));
    SP_HIP(hipHostMalloc((void **)&ws.staging, kSlots * (4 + 8 + 4), hipHostMallocDefault));
    SP_HIP(hipEventCreate(&ws.ev0));
    SP_HIP(hipEventCreate(&ws.ev1));
    ws.bytes = batch_ws_bytes(g, qcap);
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
    dev_free(ws.hub_off);
    dev_free(ws.hub_lvl_chunks);
    dev_free(ws.hub_list);
    dev_free(ws.hub_cnt);
    dev_free(ws.partial);
    dev_free(ws.slot_src);
    dev_free(ws.ctl);
    if (ws.ctl_host) (void)hipHostFree(ws.ctl_host);
    if (ws.staging) (void)hipHostFree(ws.staging);
    if (ws.ev0) (void)hipEventDestroy(ws.ev0);
    if (ws.ev1) (void)hipEventDestroy(ws.ev1);
    ws = BatchWorkspace{};
}

static sp_status grow_queue(sp_graph g, BatchWorkspace &ws, int64_t qcap) {
    dev_free(ws.queue);
    dev_free(ws.qmask);
    ws.queue = nullptr;
    ws.qmask = nullptr;
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    ws.qcap = qcap;
    ws.bytes = batch_ws_bytes(g, qcap);
    return SP_OK;
}

template <int BS>
static sp_status batch_forward(sp_graph g, BatchWorkspace &ws, int32_t n0, unsigned long long active,
                               const BatchRunOpts &o, hipStream_t s) {
    const int32_t n = g->n;
    const int maxb = device_cu_count() * 8;
    const int grid = grid_for((int64_t)n, BS, maxb);
    const bool hubs = g->n_hubs > 0;
    const bool may_pull = o.alpha > 0 && g->max_degree > 8;  // sparse meshes never pull
    const int hub_grid = grid_for((int64_t)g->hub_chunks * kWave, BS, maxb);
    hipLaunchKernelGGL(k_ms_clear, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.seen, ws.nxt,
                       ws.front[0], ws.front[1], n);
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(256), 0, s, ws.ctl, (const int32_t *)g->row_ptr,
                       (const int32_t *)ws.queue, (const unsigned long long *)ws.qmask, n0, ws.seen,
                       ws.front[0], ws.sigma, ws.level_off, ws.hub_list, ws.hub_off,
                       ws.hub_lvl_chunks, n, (long long)g->nnz, active,
                       may_pull ? o.alpha : 0.0, o.beta);  // alpha 0: never switch to bottom-up
    SP_HIP(hipGetLastError());
    int64_t enqueued = 0;
    for (;;) {
        const int chunk = std::max(1, o.chunk_levels);
        for (int k = 0; k < chunk; ++k) {
            const int64_t l = enqueued + k;  // level this group expands
            uint4 *fcur = ws.front[l & 1], *fnxt = ws.front[(l + 1) & 1];
            {
                ProfScope ps(P_MS_TOPDOWN, s);
                hipLaunchKernelGGL(k_ms_topdown<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s, ws.ctl,
                                   g->row_ptr, g->col_idx, ws.queue, ws.qmask, ws.seen, ws.nxt,
                                   (const HubEntry *)ws.hub_list, (long long)ws.qcap,
                                   prof_counters(P_MS_TOPDOWN));
            }
            if (may_pull) {
                ProfScope ps(P_MS_BOTTOMUP, s);
                hipLaunchKernelGGL(k_ms_bottomup<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                                   g->col_idx, ws.seen, ws.nxt, fcur, ws.queue, active,
                                   (long long)ws.qcap, prof_counters(P_MS_BOTTOMUP));
            }
            {
                ProfScope ps(P_MS_SIGMA, s);
                hipLaunchKernelGGL(k_ms_sigma<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                                   g->col_idx, ws.queue, ws.qmask, ws.seen, ws.nxt, fcur, fnxt,
                                   ws.sigma, ws.hub_list, (long long)ws.hub_cap, active,
                                   (long long)ws.qcap, prof_counters(P_MS_SIGMA));
            }
            hipLaunchKernelGGL(k_ms_advance, dim3(1), dim3(1), 0, s, ws.ctl, ws.level_off,
                               ws.hub_off, ws.hub_lvl_chunks, (long long)ws.qcap,
                               (long long)ws.hub_cap);
            if (hubs) {
                ProfScope ps(P_MS_SIGMA, s);
                hipLaunchKernelGGL(k_ms_sigma_hub<BS>, dim3(hub_grid), dim3(BS), 0, s, ws.ctl,
                                   g->row_ptr, g->col_idx, (const unsigned long long *)ws.qmask,
                                   (const uint4 *)fcur, ws.sigma, (const HubEntry *)ws.hub_list,
                                   ws.hub_cnt, ws.partial, prof_counters(P_MS_SIGMA));
            }
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
        SP_TRY(grow_queue(g, ws, (int64_t)std::max(n, 1) * nslots + kSlots));
    }
    const LevelCtl c = *ws.ctl_host;
    const int32_t levels = c.level + 1;
    std::vector<int32_t> off(levels + 1), hch(levels);
    SP_HIP(hipMemcpyAsync(off.data(), ws.level_off, sizeof(int32_t) * (levels + 1),
                          hipMemcpyDeviceToHost, s));
    SP_HIP(hipMemcpyAsync(hch.data(), ws.hub_lvl_chunks, sizeof(int32_t) * levels,
                          hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
    const int maxb = device_cu_count() * 8;
    for (int32_t l = levels - 1; l >= 1; --l) {
        const int64_t cnt = off[l + 1] - off[l];
        const bool deepest = l == levels - 1;
        uint4 *frd = ws.front[(l + 1) & 1], *fwr = ws.front[l & 1];
        {
            ProfScope ps(P_MS_DELTA, s);
            hipLaunchKernelGGL(k_ms_delta<BS>, dim3(grid_for(cnt, BS, maxb)), dim3(BS), 0, s,
                               ws.level_off, l, (int32_t)deepest, g->row_ptr, g->col_idx, ws.queue,
                               ws.qmask, (const uint4 *)frd, fwr, ws.sigma, ws.delta,
                               prof_counters(P_MS_DELTA));
        }
        if (!deepest && hch[l] > 0) {
            ProfScope ps(P_MS_DELTA, s);
            hipLaunchKernelGGL(k_ms_delta_hub<BS>, dim3(grid_for((int64_t)hch[l] * kWave, BS, maxb)),
                               dim3(BS), 0, s, (const int32_t *)ws.hub_off,
                               (const int32_t *)ws.hub_lvl_chunks, l, g->row_ptr, g->col_idx,
                               (const unsigned long long *)ws.qmask, (const uint4 *)frd, ws.sigma,
                               ws.delta, (const HubEntry *)ws.hub_list, ws.hub_cnt, ws.partial,
                               prof_counters(P_MS_DELTA));
        }
    }
    SP_HIP(hipGetLastError());
    bool any_out = false;
    SlotTable tbl{};
    for (int32_t i = 0; i < kSlots; ++i) {
        tbl.out[i] = (bc_of_slot && i < nslots) ? bc_of_slot[i] : nullptr;
        any_out |= tbl.out[i] != nullptr;
    }
    if (any_out) {
        ProfScope ps(P_MS_BC, s);
        hipLaunchKernelGGL(k_ms_bc<BS>, dim3(grid_for(n, BS, maxb)), dim3(BS), 0, s, n, ws.seen,
                           ws.delta, ws.slot_src, nslots, tbl, prof_counters(P_MS_BC));
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
