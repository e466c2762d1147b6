// Single-source shortest paths on a weighted graph (paper Section 2.2, Fig.
// "SSSP computation in StarPlat"; the pull form in the Appendix).
//
// The paper's method is a Bellman-Ford variant driven by a `modified` flag:
// in each round every vertex modified in the previous round relaxes its edges
// with an atomic Min (push), or every vertex takes the Min over its modified
// neighbours (pull), until a round modifies nothing.  Here:
//
//   * the `modified` set of a round is a frontier queue (push reads it) and a
//     stamp per vertex (pull reads it): ds[v] = {dist, stamp}, where stamp is
//     the last round whose frontier holds v.  One 8-byte load gives a
//     neighbour's distance and its membership;
//   * a push relaxation lowers dist[u] with atomicMin; the first thread in a
//     round whose atomicMin lowered it raises u's stamp to the next round with
//     atomicMax and appends u to the next frontier, so a vertex joins a
//     frontier at most once per round;
//   * a pull round walks every vertex's row, takes the least candidate over
//     neighbours whose stamp is at least the current round (in the current
//     frontier, or lowered earlier in this round), and stores it when lower;
//   * rows longer than kHubDeg entries ("hubs") are cut into chunks of
//     kHubChunk entries that blocks take one at a time: in push rounds the
//     frontier's hubs (registered when they join it), in pull rounds every
//     hub of the graph (a fixed list built with the weights);
//   * adjacency entries are packed {neighbour, weight}; one load per entry;
//   * each round is one kernel per direction.  The direction is chosen on the
//     device: a round pulls when its frontier's adjacency entries times alpha
//     exceed the graph's; the other direction's kernel returns at once.  The
//     last working block of a round's kernel closes the round, so chunks of
//     rounds are captured once as HIP graphs and replayed until a round
//     lowers nothing.
//
// Every round only lowers distances toward the same least fixed point, so
// the result does not depend on scheduling: it is the shortest-path distance
// (INT32_MAX where unreached), bit for bit.
#include "capture.h"
#include "common.h"
#include "devutil.h"
#include "levels.h"

namespace sp {

namespace {
constexpr int32_t kInf = INT32_MAX;
}

// d + w, or kInf with `ovf` set when the sum reaches INT32_MAX.  d and w lie
// in [0, INT32_MAX), so the unsigned sum cannot wrap.  A saturated candidate
// lowers nothing (kInf is the unreached mark).  It only matters if it is the
// sole way to reach a vertex, which the check after the last round decides
// (k_sssp_unfit), so `ovf` merely asks for that check.
__device__ __forceinline__ int32_t candidate(int32_t d, int32_t w, bool &ovf) {
    const uint32_t s = (uint32_t)d + (uint32_t)w;
    if (s >= (uint32_t)kInf) {
        ovf = true;
        return kInf;
    }
    return (int32_t)s;
}

// Push relaxation of u to nd in round r.  True for exactly one caller per
// vertex and round: the first whose atomicMin lowered u's distance in this
// round; it puts u into the next frontier.  A stale plain read can only be
// too large, so skipping on it is safe.
__device__ __forceinline__ bool relax_push(int2 *ds, int32_t u, int32_t nd, int32_t r, bool &lowered) {
    lowered = false;
    if (nd >= ds[u].x) return false;
    const int32_t old = atomicMin(&ds[u].x, nd);
    if (nd >= old) return false;
    lowered = true;
    return atomicMax(&ds[u].y, r + 1) < r + 1;
}

// Entries of a block's local frontier (see k_sssp_push).
constexpr int kLocalCap = 512;

// The round state word (SsspCtl::state).
struct RoundState {
    int32_t cnt;      // frontier size
    int32_t chunks;   // chunks of the frontier's hubs
    int32_t parity;   // round & 1
    bool pull, done;
};

__device__ __forceinline__ unsigned long long pack_state(int32_t cnt, int32_t chunks, int32_t round,
                                                         int32_t mode, bool done) {
    return (unsigned long long)(uint32_t)cnt | ((unsigned long long)(uint32_t)chunks << 31) |
           ((unsigned long long)(round & 1) << 55) | ((unsigned long long)(mode == SSSP_PULL) << 56) |
           ((unsigned long long)done << 57);
}

__device__ __forceinline__ RoundState unpack_state(unsigned long long w) {
    return RoundState{(int32_t)(w & 0x7fffffffull), (int32_t)((w >> 31) & 0xffffffull),
                      (int32_t)((w >> 55) & 1ull), ((w >> 56) & 1ull) != 0, ((w >> 57) & 1ull) != 0};
}

// Largest frontier hub chunk count the state word holds (24 bits).
constexpr int64_t kMaxStateChunks = (1 << 24) - 1;

// Block-uniform snapshot of the round state: one load by thread 0, shared
// through LDS.  A block of round r's kernel that starts after the round was
// closed sees round r + 1, whose parity differs from the kernel's: it returns.
__device__ __forceinline__ RoundState read_state(SsspCtl *c) {
    __shared__ unsigned long long s_state;
    if (threadIdx.x == 0) s_state = ld_agent(&c->state);
    __syncthreads();
    return unpack_state(s_state);
}

// Bookkeeping of a vertex that joined the next frontier: its adjacency
// entries count toward the next round's direction choice, and a hub is
// registered for the next round's chunk blocks (list entry plus the owner of
// each of its chunks).
__device__ __forceinline__ void joined(SsspCtl *c, const int32_t *__restrict__ rp, HubEntry *hn,
                                       int32_t *on, int32_t hub_cap, int32_t chunk_cap, int32_t u,
                                       unsigned long long &my_deg) {
    const int32_t deg = rp[u + 1] - rp[u];
    my_deg += (unsigned long long)deg;
    if (deg > kHubDeg) {
        const int32_t nch = (deg + kHubChunk - 1) / kHubChunk;
        const unsigned long long old =
            atomicAdd(&c->hub_pack_.v, (1ull << 40) | (unsigned long long)nch);
        const int64_t idx = (int64_t)(old >> 40);
        const int64_t base = (int64_t)(old & ((1ull << 40) - 1));
        if (idx >= hub_cap || base + nch > chunk_cap) {
            atomicOr(&c->capacity_.v, 1);
            return;
        }
        hn[idx] = HubEntry{u, 0, (int32_t)base, nch};
        for (int32_t q = 0; q < nch; ++q) on[base + q] = (int32_t)idx;
    }
}

// Last j with off[j] <= k (off ascending, off[0] = 0).
template <int BS>
__device__ __forceinline__ int32_t owner_of(const int32_t *off, int32_t k) {
    int32_t a = 0, z = BS - 1;
    while (a < z) {
        const int32_t mid = (a + z + 1) >> 1;
        if (off[mid] <= k) a = mid; else z = mid - 1;
    }
    return a;
}

template <int BS>
__device__ __forceinline__ int32_t block_min_i32(int32_t x, int32_t *lds) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
    if (lane_id() == 0) lds[threadIdx.x / kWave] = x;
    __syncthreads();
    int32_t m = lds[0];
    for (int w = 1; w < BS / kWave; ++w) m = min(m, lds[w]);
    __syncthreads();
    return m;
}

// End of a round (one thread of the last working block): the next frontier
// becomes current, its hubs' chunks become the chunk work, the direction of
// the next round is chosen, or the run ends.  The state word is stored last.
__device__ void close_round(SsspCtl *c, int32_t mode, int32_t n, int32_t hub_cap, int32_t chunk_cap) {
    if (mode == SSSP_PUSH) c->push_rounds++; else c->pull_rounds++;
    const int32_t tail = ld_agent(&c->tail_.v);
    const unsigned long long hp = ld_agent(&c->hub_pack_.v);
    const int64_t nh = (int64_t)(hp >> 40), nch = (int64_t)(hp & ((1ull << 40) - 1));
    const unsigned long long deg = ld_agent(&c->next_deg_.v);
    const int32_t r = c->round + 1;
    c->round = r;
    c->tail_.v = 0;
    c->next_deg_.v = 0;
    c->hub_pack_.v = 0;
    if (tail > n || nh > hub_cap || nch > chunk_cap || nch > kMaxStateChunks) c->capacity_.v = 1;
    const bool done = tail <= 0 || c->capacity_.v;
    int32_t next = SSSP_PUSH;
    if (c->forced >= 0) next = c->forced;
    else if ((double)deg * c->alpha > (double)c->nnz) next = SSSP_PULL;
    c->done = done;
    __hip_atomic_store(&c->state, pack_state(done ? 0 : tail, done ? 0 : (int32_t)nch, r, next, done),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_sssp_fill(int2 *ds, int32_t n) {
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) ds[v] = make_int2(kInf, -1);
}

__global__ void k_sssp_init(SsspCtl *c, const int32_t *__restrict__ rp, int2 *ds, int32_t *q0,
                            HubEntry *h0, int32_t *o0, int32_t src, int32_t n, long long nnz,
                            int32_t forced, double alpha, int32_t static_chunks) {
    const int32_t deg = rp[src + 1] - rp[src];
    ds[src] = make_int2(0, 0);
    q0[0] = src;
    c->round = 0;
    c->done = 0;
    c->n_vertices = n;
    c->forced = forced;
    c->push_rounds = 0;
    c->pull_rounds = 0;
    c->static_chunks = static_chunks;
    c->nnz = nnz;
    c->alpha = alpha;
    const int32_t nch = deg > kHubDeg ? (deg + kHubChunk - 1) / kHubChunk : 0;
    if (nch) h0[0] = HubEntry{src, 0, 0, nch};
    for (int32_t q = 0; q < nch; ++q) o0[q] = 0;
    c->tail_.v = 0;
    c->overflow_.v = 0;
    c->capacity_.v = 0;
    c->next_deg_.v = 0;
    c->hub_pack_.v = 0;
    c->blocks_done_.v = 0;
    c->reached_.v = 0;
    int32_t mode = SSSP_PUSH;
    if (forced >= 0) mode = forced;
    else if ((double)deg * alpha > (double)nnz) mode = SSSP_PULL;
    c->state = pack_state(1, nch, 0, mode, false);
}

// Push round.  blockIdx.y == 0: a block takes BS frontier vertices (hubs
// excluded), scans their row lengths and walks the concatenated rows BS
// entries at a time, one entry per lane.  blockIdx.y == 1: blocks take the
// chunks of the frontier's hubs.
//
// With HOPS > 0 (graphs of short rows, where rounds are many and small) a
// block also follows its own lowerings for up to HOPS more hops inside the
// round: every vertex it lowered goes, with the distance it wrote, into an
// LDS list, and the list is expanded the same way.  Every lowering still
// puts its vertex into the next frontier (first lowering in the round) or
// finds it there already, so the next round expands it with its current
// distance whatever happened locally; the local hops only add relaxations
// from valid path lengths, and the improvements travel up to HOPS + 1 edges
// per round instead of one.
template <int BS, int HOPS>
__global__ __launch_bounds__(BS) void k_sssp_push(SsspCtl *c, const int32_t *__restrict__ rp,
                                                  const int2 *__restrict__ adj, int2 *ds,
                                                  int32_t *q0, int32_t *q1, HubEntry *h0,
                                                  HubEntry *h1, int32_t *o0, int32_t *o1,
                                                  int32_t hub_cap, int32_t chunk_cap, int32_t n,
                                                  int32_t parity, unsigned long long *prof) {
    const RoundState st = read_state(c);
    if (st.done || st.pull || st.parity != parity) return;
    constexpr int kLists = HOPS > 0 ? 2 : 1, kCap = HOPS > 0 ? kLocalCap : 1;
    __shared__ int32_t s_beg[BS], s_off[BS], s_d[BS], s_scan[BS / kWave + 1];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ int32_t s_lv[kLists][kCap], s_ld[kLists][kCap], s_ln[2];
    __shared__ unsigned long long s_red[1];
    const int32_t r = c->round, cnt = st.cnt, nch = st.chunks;
    const int32_t *qc = parity ? q1 : q0;
    int32_t *qn = parity ? q0 : q1;
    const HubEntry *hc = parity ? h1 : h0;
    HubEntry *hn = parity ? h0 : h1;
    const int32_t *oc = parity ? o1 : o0;
    int32_t *on = parity ? o0 : o1;
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    unsigned long long my_deg = 0, my_items = 0, my_edges = 0;
    bool ovf = false;
    const int nb0 = working_blocks(cnt, BS);
    const int nb1 = (int)min((int64_t)gridDim.x, (int64_t)nch);
    // Expands the rows held by the block's threads (row start, length, the
    // distance to extend): scan, walk one entry per lane, relax; lowered
    // vertices go to local list `dst` when dst >= 0.  All threads call it.
    auto walk = [&](int32_t beg, int32_t deg, int32_t d, int dst) {
        int32_t total;
        const int32_t off = block_excl_scan<BS>(deg, s_scan, &total);
        s_beg[threadIdx.x] = beg;
        s_off[threadIdx.x] = off;
        s_d[threadIdx.x] = d;
        __syncthreads();
        for (int32_t k0 = 0; k0 < total; k0 += BS) {
            const int32_t k = k0 + threadIdx.x;
            bool take = false;
            int32_t u = 0;
            if (k < total) {
                const int32_t a = owner_of<BS>(s_off, k);
                const int2 e = adj[s_beg[a] + (k - s_off[a])];
                u = e.x;
                const int32_t nd = candidate(s_d[a], e.y, ovf);
                bool lowered;
                take = relax_push(ds, u, nd, r, lowered);
                if (take) joined(c, rp, hn, on, hub_cap, chunk_cap, u, my_deg);
                if (HOPS > 0 && dst >= 0 && lowered) {
                    const int32_t at = atomicAdd(&s_ln[dst], 1);
                    if (at < kCap) {
                        s_lv[dst][at] = u;
                        s_ld[dst][at] = nd;
                    }
                }
            }
            q.stage(take, u, &c->tail_.v, qn, n, &c->capacity_.v);
        }
        __syncthreads();
    };
    bool working;
    if (blockIdx.y == 0) {
        working = (int)blockIdx.x < nb0;
        for (int32_t b = blockIdx.x * BS; b < cnt; b += gridDim.x * BS) {
            const int32_t i = b + threadIdx.x;
            int32_t beg = 0, deg = 0, d = 0;
            if (i < cnt) {
                const int32_t v = qc[i];
                beg = rp[v];
                deg = rp[v + 1] - beg;
                if (deg > kHubDeg) deg = 0;  // its chunks are taken by blockIdx.y == 1
                d = ds[v].x;
                ++my_items;
                my_edges += (unsigned long long)deg;
            }
            if (HOPS > 0 && threadIdx.x == 0) s_ln[0] = 0;  // seen after the scan's barrier
            walk(beg, deg, d, HOPS > 0 ? 0 : -1);
            int cur = 0;
            for (int hop = 0; hop < HOPS; ++hop) {
                const int32_t ln = min(s_ln[cur], kCap);
                if (ln == 0) break;
                const int nxt = cur ^ 1;
                if (threadIdx.x == 0) s_ln[nxt] = 0;
                for (int32_t lb = 0; lb < ln; lb += BS) {
                    const int32_t j = lb + threadIdx.x;
                    int32_t lbeg = 0, ldeg = 0, ld = 0;
                    if (j < ln) {
                        const int32_t v = s_lv[cur][j];
                        ld = s_ld[cur][j];
                        lbeg = rp[v];
                        ldeg = rp[v + 1] - lbeg;
                        if (ldeg > kHubDeg) ldeg = 0;  // already in the next frontier
                        ++my_items;
                        my_edges += (unsigned long long)ldeg;
                    }
                    walk(lbeg, ldeg, ld, hop + 1 < HOPS ? nxt : -1);
                }
                cur = nxt;
            }
        }
    } else {
        working = (int)blockIdx.x < nb1;
        for (int32_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const HubEntry h = hc[oc[k]];
            const int32_t beg = rp[h.v] + (k - h.chunk_base) * kHubChunk;
            const int32_t end = min(rp[h.v + 1], beg + kHubChunk);
            const int32_t d = ds[h.v].x;
            my_edges += threadIdx.x == 0 ? (unsigned long long)(end - beg) : 0ull;
            for (int32_t e0 = beg; e0 < end; e0 += BS) {
                const int32_t e = e0 + threadIdx.x;
                bool take = false;
                int32_t u = 0;
                if (e < end) {
                    const int2 x = adj[e];
                    u = x.x;
                    bool lowered;
                    take = relax_push(ds, u, candidate(d, x.y, ovf), r, lowered);
                    if (take) joined(c, rp, hn, on, hub_cap, chunk_cap, u, my_deg);
                }
                q.stage(take, u, &c->tail_.v, qn, n, &c->capacity_.v);
            }
        }
    }
    q.finish(&c->tail_.v, qn, n, &c->capacity_.v);
    if (__ballot(ovf) && lane_id() == 0) atomicOr(&c->overflow_.v, 1);
    block_add_u64<BS>(my_deg, s_red, &c->next_deg_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
    if (last_working_block(&c->blocks_done_.v, working, nb0 + nb1) && threadIdx.x == 0)
        close_round(c, SSSP_PUSH, n, hub_cap, chunk_cap);
}

// Pull round.  blockIdx.y == 0: a block takes BS consecutive vertices (hubs
// excluded), walks their concatenated rows one entry per lane, and folds each
// entry's candidate into its vertex's LDS minimum; each vertex then stores
// the minimum when it is lower (only its own thread writes it).
// blockIdx.y == 1: blocks take the chunks of every hub of the graph, reduce a
// chunk to its minimum and lower the hub with atomicMin.
template <int BS>
__global__ __launch_bounds__(BS) void k_sssp_pull(SsspCtl *c, const int32_t *__restrict__ rp,
                                                  const int2 *__restrict__ adj, int2 *ds,
                                                  int32_t *q0, int32_t *q1, HubEntry *h0,
                                                  HubEntry *h1, int32_t *o0, int32_t *o1,
                                                  int32_t hub_cap, int32_t chunk_cap, int32_t n,
                                                  const HubEntry *__restrict__ hs,
                                                  const int32_t *__restrict__ os, int32_t parity,
                                                  unsigned long long *prof) {
    const RoundState st = read_state(c);
    if (st.done || !st.pull || st.parity != parity) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_best[BS], s_scan[BS / kWave + 1];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2], s_min[BS / kWave];
    __shared__ unsigned long long s_red[1];
    const int32_t r = c->round, nch = c->static_chunks;
    int32_t *qn = parity ? q0 : q1;
    HubEntry *hn = parity ? h0 : h1;
    int32_t *on = parity ? o0 : o1;
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    unsigned long long my_deg = 0, my_items = 0, my_edges = 0;
    bool ovf = false;
    const int nb0 = working_blocks(n, BS);
    const int nb1 = (int)min((int64_t)gridDim.x, (int64_t)nch);
    bool working;
    if (blockIdx.y == 0) {
        working = (int)blockIdx.x < nb0;
        for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
            const int32_t v = b + threadIdx.x;
            int32_t beg = 0, deg = 0;
            if (v < n) {
                beg = rp[v];
                deg = rp[v + 1] - beg;
                if (deg > kHubDeg) deg = 0;  // its chunks are taken by blockIdx.y == 1
                ++my_items;
                my_edges += (unsigned long long)deg;
            }
            int32_t total;
            const int32_t off = block_excl_scan<BS>(deg, s_scan, &total);
            s_beg[threadIdx.x] = beg;
            s_off[threadIdx.x] = off;
            s_best[threadIdx.x] = kInf;
            __syncthreads();
            for (int32_t k0 = 0; k0 < total; k0 += BS) {
                const int32_t k = k0 + threadIdx.x;
                if (k < total) {
                    const int32_t a = owner_of<BS>(s_off, k);
                    const int2 e = adj[s_beg[a] + (k - s_off[a])];
                    const int2 su = ds[e.x];
                    if (su.y >= r) {
                        const int32_t nd = candidate(su.x, e.y, ovf);
                        if (nd < s_best[a]) atomicMin(&s_best[a], nd);
                    }
                }
            }
            __syncthreads();
            bool take = false;
            if (deg > 0) {
                const int32_t best = s_best[threadIdx.x];
                if (best < ds[v].x) {
                    ds[v] = make_int2(best, r + 1);
                    take = true;
                    joined(c, rp, hn, on, hub_cap, chunk_cap, v, my_deg);
                }
            }
            q.stage(take, v, &c->tail_.v, qn, n, &c->capacity_.v);
        }
    } else {
        working = (int)blockIdx.x < nb1;
        for (int32_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const HubEntry h = hs[os[k]];
            const int32_t beg = rp[h.v] + (k - h.chunk_base) * kHubChunk;
            const int32_t end = min(rp[h.v + 1], beg + kHubChunk);
            my_edges += threadIdx.x == 0 ? (unsigned long long)(end - beg) : 0ull;
            int32_t m = kInf;
            for (int32_t e = beg + threadIdx.x; e < end; e += BS) {
                const int2 x = adj[e];
                const int2 su = ds[x.x];
                if (su.y >= r) m = min(m, candidate(su.x, x.y, ovf));
            }
            m = block_min_i32<BS>(m, s_min);
            bool take = false;
            if (threadIdx.x == 0 && m < ds[h.v].x) {
                const int32_t old = atomicMin(&ds[h.v].x, m);
                take = m < old && atomicMax(&ds[h.v].y, r + 1) < r + 1;
                if (take) joined(c, rp, hn, on, hub_cap, chunk_cap, h.v, my_deg);
            }
            q.stage(take, h.v, &c->tail_.v, qn, n, &c->capacity_.v);
        }
    }
    q.finish(&c->tail_.v, qn, n, &c->capacity_.v);
    if (__ballot(ovf) && lane_id() == 0) atomicOr(&c->overflow_.v, 1);
    block_add_u64<BS>(my_deg, s_red, &c->next_deg_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
    if (last_working_block(&c->blocks_done_.v, working, nb0 + nb1) && threadIdx.x == 0)
        close_round(c, SSSP_PULL, n, hub_cap, chunk_cap);
}

// After the rounds, when some candidate saturated: a reached vertex with an
// unreached neighbour means that neighbour's distance is INT32_MAX or more
// (every relaxation into it saturated), which int32 cannot hold.
__global__ void k_sssp_unfit(SsspCtl *c, const int32_t *__restrict__ rp,
                             const int2 *__restrict__ adj, const int2 *__restrict__ ds, int32_t n) {
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        if (ds[u].x == kInf) continue;
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
            if (ds[adj[e].x].x == kInf) {
                atomicOr(&c->capacity_.v, 2);
                return;
            }
    }
}

// Distances to the caller's buffer, and the count of reached vertices.
__global__ void k_sssp_export(SsspCtl *c, const int2 *__restrict__ ds, int32_t *out, int32_t n) {
    __shared__ unsigned long long s_red[1];
    unsigned long long reached = 0;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t d = ds[v].x;
        out[v] = d;
        reached += d != kInf;
    }
    block_add_u64<256>(reached, s_red, &c->reached_.v);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
sp_status sssp_ws_create(sp_graph g, SsspWorkspace &ws) {
    const int32_t n = std::max(g->n, 1);
    const size_t hubs = (size_t)g->n_hubs + 1, chunks = (size_t)g->hub_chunks + 1;
    ws.n = g->n;
    SP_HIP(hipGetDevice(&ws.device));
    auto fail = [&](sp_status st) {
        sssp_ws_destroy(ws);
        return st;
    };
    sp_status st = dev_alloc((void **)&ws.ds, sizeof(int2) * (size_t)n);
    if (st == SP_OK) st = dev_alloc((void **)&ws.queue[0], sizeof(int32_t) * (size_t)n);
    if (st == SP_OK) st = dev_alloc((void **)&ws.queue[1], sizeof(int32_t) * (size_t)n);
    if (st == SP_OK) st = dev_alloc((void **)&ws.hubs[0], sizeof(HubEntry) * hubs);
    if (st == SP_OK) st = dev_alloc((void **)&ws.hubs[1], sizeof(HubEntry) * hubs);
    if (st == SP_OK) st = dev_alloc((void **)&ws.owner[0], sizeof(int32_t) * chunks);
    if (st == SP_OK) st = dev_alloc((void **)&ws.owner[1], sizeof(int32_t) * chunks);
    if (st == SP_OK) st = dev_alloc((void **)&ws.ctl, sizeof(SsspCtl));
    if (st != SP_OK) return fail(st);
    if (hipHostMalloc((void **)&ws.ctl_host, sizeof(SsspCtl), hipHostMallocDefault) != hipSuccess) {
        ws.ctl_host = nullptr;
        set_error("pinned host allocation failed");
        return fail(SP_ERR_OUT_OF_MEMORY);
    }
    if (hipEventCreate(&ws.ev0) != hipSuccess || hipEventCreate(&ws.ev1) != hipSuccess) {
        set_error("hipEventCreate failed");
        return fail(SP_ERR_DEVICE);
    }
    return SP_OK;
}

void sssp_ws_destroy(SsspWorkspace &ws) {
    if (ws.rounds_short.exec) (void)hipGraphExecDestroy(ws.rounds_short.exec);
    if (ws.rounds_long.exec) (void)hipGraphExecDestroy(ws.rounds_long.exec);
    if (ws.cap_stream) (void)hipStreamDestroy(ws.cap_stream);
    dev_free(ws.ds);
    dev_free(ws.queue[0]);
    dev_free(ws.queue[1]);
    dev_free(ws.hubs[0]);
    dev_free(ws.hubs[1]);
    dev_free(ws.owner[0]);
    dev_free(ws.owner[1]);
    dev_free(ws.ctl);
    if (ws.ctl_host) (void)hipHostFree(ws.ctl_host);
    if (ws.ev0) (void)hipEventDestroy(ws.ev0);
    if (ws.ev1) (void)hipEventDestroy(ws.ev1);
    ws = SsspWorkspace{};
}

// `rounds` rounds starting at an even round: each round launches its push
// and/or pull kernel with the round's parity, and a kernel runs only while the
// control block is at a round of that parity.  A block of round r's kernel
// that starts after the round was closed therefore sees round r + 1 and
// returns, instead of taking part in a round that is not its own.
template <int BS, int HOPS>
static void enqueue_rounds(sp_graph g, SsspWorkspace &ws, int rounds, int grid, bool hubs,
                           bool may_pull, bool may_push, hipStream_t s) {
    const int32_t hub_cap = g->n_hubs + 1, chunk_cap = (int32_t)g->hub_chunks + 1, n = g->n;
    for (int k = 0; k < rounds; ++k) {
        const int32_t parity = k & 1;
        if (may_push) {
            ProfScope ps(P_SSSP_PUSH, s);
            hipLaunchKernelGGL((k_sssp_push<BS, HOPS>), dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s, ws.ctl,
                               (const int32_t *)g->row_ptr, (const int2 *)g->adjw, ws.ds, ws.queue[0],
                               ws.queue[1], ws.hubs[0], ws.hubs[1], ws.owner[0], ws.owner[1],
                               hub_cap, chunk_cap, n, parity, prof_counters(P_SSSP_PUSH));
        }
        if (may_pull) {
            ProfScope ps(P_SSSP_PULL, s);
            hipLaunchKernelGGL(k_sssp_pull<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s, ws.ctl,
                               (const int32_t *)g->row_ptr, (const int2 *)g->adjw, ws.ds, ws.queue[0],
                               ws.queue[1], ws.hubs[0], ws.hubs[1], ws.owner[0], ws.owner[1],
                               hub_cap, chunk_cap, n, (const HubEntry *)g->hub_static,
                               (const int32_t *)g->owner_static, parity, prof_counters(P_SSSP_PULL));
        }
    }
}

template <int BS, int HOPS>
static sp_status sssp_run_bs(sp_graph g, SsspWorkspace &ws, int32_t src, int32_t *out_dist,
                             const SsspOpts &o, hipStream_t s, SsspResult *res) {
    const int32_t n = g->n;
    const int maxb = o.max_blocks > 0 ? o.max_blocks : device_cu_count() * 8;
    const int grid = grid_for((int64_t)n, BS, maxb);
    const bool hubs = g->n_hubs > 0;
    // Automatic choice never pulls on sparse meshes (every row at most 8 long),
    // nor when alpha <= 1 (a frontier's entries never exceed the graph's).
    const bool may_pull = o.forced == SSSP_PULL || (o.forced < 0 && o.alpha > 1.0 && g->max_degree > 8);
    const bool may_push = o.forced != SSSP_PULL;
    const int forced = may_pull ? o.forced : SSSP_PUSH;
    hipLaunchKernelGGL(k_sssp_fill, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.ds, n);
    hipLaunchKernelGGL(k_sssp_init, dim3(1), dim3(1), 0, s, ws.ctl, (const int32_t *)g->row_ptr,
                       ws.ds, ws.queue[0], ws.hubs[0], ws.owner[0], src, n, (long long)g->nnz,
                       forced, o.alpha, (int32_t)g->hub_chunks);
    SP_HIP(hipGetLastError());
    const bool capture = o.chunk_rounds > 0 && !prof_enabled();
    int32_t enqueued = 0, chunks = 0, graph_launches = 0;
    for (;;) {
        const bool deep = chunks >= 4;
        const int base = std::max(1, std::abs(o.chunk_rounds));
        const int chunk = (base + (base & 1)) * (deep ? 4 : 1);  // even: parity holds
        if (capture) {
            const std::array<long long, 12> key = {
                BS * 16 + HOPS, grid, hubs, may_pull, may_push, chunk, (long long)(intptr_t)ws.ds,
                (long long)(intptr_t)g->adjw, (long long)(intptr_t)g->hub_static,
                (long long)(intptr_t)g->owner_static, (long long)(intptr_t)ws.ctl, g->n_hubs};
            SP_TRY(replay_captured(&ws.cap_stream, deep ? ws.rounds_long : ws.rounds_short, key,
                                   [&](hipStream_t cs) {
                                       enqueue_rounds<BS, HOPS>(g, ws, chunk, grid, hubs, may_pull, may_push, cs);
                                   },
                                   s));
            ++graph_launches;
        } else {
            enqueue_rounds<BS, HOPS>(g, ws, chunk, grid, hubs, may_pull, may_push, s);
            SP_HIP(hipGetLastError());
        }
        enqueued += chunk;
        ++chunks;
        SP_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(SsspCtl), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        if (ws.ctl_host->done) break;
        // Round k leaves every distance of a shortest path of at most k + 1
        // edges final, so n + 1 rounds always suffice.
        if (enqueued > n + 2 + chunk) {
            set_error("SSSP did not converge after %d rounds", enqueued);
            return SP_ERR_DEVICE;
        }
    }
    const SsspCtl &c = *ws.ctl_host;
    if (res) {
        res->rounds = c.push_rounds + c.pull_rounds;
        res->push_rounds = c.push_rounds;
        res->pull_rounds = c.pull_rounds;
        res->graph_launches = graph_launches;
    }
    if (c.capacity_.v) {
        set_error("SSSP frontier capacity exceeded (internal error)");
        return SP_ERR_DEVICE;
    }
    if (c.overflow_.v) {
        hipLaunchKernelGGL(k_sssp_unfit, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.ctl,
                           (const int32_t *)g->row_ptr, (const int2 *)g->adjw, (const int2 *)ws.ds, n);
        SP_HIP(hipGetLastError());
        int32_t unfit = 0;
        SP_HIP(hipMemcpyAsync(&unfit, &ws.ctl->capacity_.v, sizeof(unfit), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        if (unfit) {
            if (res) res->overflow = true;
            set_error("a shortest-path length reaches INT32_MAX; distances do not fit in int32");
            return SP_ERR_NOT_SUPPORTED;
        }
    }
    hipLaunchKernelGGL(k_sssp_export, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.ctl,
                       (const int2 *)ws.ds, out_dist, n);
    SP_HIP(hipGetLastError());
    if (res) {
        unsigned long long reached = 0;
        SP_HIP(hipMemcpyAsync(&reached, &ws.ctl->reached_.v, sizeof(reached), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        res->reached = (int32_t)reached;
    }
    return SP_OK;
}

template <int HOPS>
static sp_status sssp_run_hops(sp_graph g, SsspWorkspace &ws, int32_t src, int32_t *out_dist,
                               const SsspOpts &o, hipStream_t s, SsspResult *res) {
    switch (o.block) {
        case 128: return sssp_run_bs<128, HOPS>(g, ws, src, out_dist, o, s, res);
        case 512: return sssp_run_bs<512, HOPS>(g, ws, src, out_dist, o, s, res);
        default: return sssp_run_bs<256, HOPS>(g, ws, src, out_dist, o, s, res);
    }
}

int sssp_local_hops(sp_graph g, int requested) {
    if (requested < 0) return 0;
    if (requested > 0) return requested;
    // automatic: graphs of short rows only (many small rounds); hub rows
    // never go through the local lists
    // (measured on road-4096: 4 hops 98 ms per source, 8: 73, 16: 51, 32: 43,
    // 64: 44, 128: 52; on rmat-22 any local hops cost time)
    return (g->max_degree <= 8 && g->n_hubs == 0) ? 32 : 0;
}

sp_status sssp_run(sp_graph g, SsspWorkspace &ws, int32_t src, int32_t *out_dist, const SsspOpts &o,
                   hipStream_t s, SsspResult *res) {
    switch (sssp_local_hops(g, o.local_hops)) {
        case 0: return sssp_run_hops<0>(g, ws, src, out_dist, o, s, res);
        case 1: return sssp_run_hops<1>(g, ws, src, out_dist, o, s, res);
        case 2: return sssp_run_hops<2>(g, ws, src, out_dist, o, s, res);
        case 4: return sssp_run_hops<4>(g, ws, src, out_dist, o, s, res);
        case 8: return sssp_run_hops<8>(g, ws, src, out_dist, o, s, res);
        case 16: return sssp_run_hops<16>(g, ws, src, out_dist, o, s, res);
        case 32: return sssp_run_hops<32>(g, ws, src, out_dist, o, s, res);
        case 64: return sssp_run_hops<64>(g, ws, src, out_dist, o, s, res);
        default: return sssp_run_hops<128>(g, ws, src, out_dist, o, s, res);
    }
}

}  // namespace sp
