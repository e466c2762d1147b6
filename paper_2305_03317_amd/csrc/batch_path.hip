// Batched multi-source Brandes pass: up to 64 sources advance level by level
// together.  Each vertex carries 64-bit source bitmaps (bit i = batch slot i):
//   seen[v]   slots that have reached v at some level so far,
//   nxt[v]    slots discovering v at the level being built,
//   front[p]  per level parity p, {mask, level tag} of v's entry at that level.
// A (vertex, mask) pair per level is an "entry"; entries of one level are
// contiguous in `queue`/`qmask`, and level_off[l] is where level l starts.
//
// Per slot s the arithmetic is Brandes' (paper Appendix, Fig. "BC computation
// in StarPlat"; DAG semantics of Section 2.3.2): sigma_s(w) sums sigma_s(u)
// over neighbours u whose level-l entry holds s, in CSR order.  The reverse
// sum is regrouped: with rho_s(w) = (1 + delta_s(w)) / sigma_s(w),
//   delta_s(v) = sum_w (sigma_s(v) / sigma_s(w)) (1 + delta_s(w))
//              = sigma_s(v) * sum_w rho_s(w),
// so a child contributes one stored value instead of two (same sum, a few
// ulps apart).  Values are stored per entry, compactly: slot s of entry
// (v, level, m) lives at val[vb + rank_m(s)] and the front record carries vb,
// so a neighbour's values for the slots it shares are one short contiguous
// read.  delta also goes to vertex-major rows dlt[v][64] for the BC sums.
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
#include "capture.h"
#include "levels.h"

namespace sp {

constexpr int kSparseSlots = 2;
constexpr int32_t kSparseDeg = 64;
constexpr uint32_t kNoTag = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long mask_of(uint4 f) {
    return (unsigned long long)f.x | ((unsigned long long)f.y << 32);
}

// {mask lo, mask hi, level tag, value base}
__device__ __forceinline__ uint4 make_front(unsigned long long m, uint32_t tag, uint32_t vb) {
    return make_uint4((uint32_t)m, (uint32_t)(m >> 32), tag, vb);
}

__device__ __forceinline__ int32_t rl_i32(int32_t v, int j) { return __builtin_amdgcn_readlane(v, j); }

__device__ __forceinline__ unsigned long long rl_u64(unsigned long long v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

__device__ __forceinline__ int rank_in(unsigned long long m, int s) {
    return __popcll(m & ((1ull << s) - 1ull));
}

// lane = slot: sum over adjacency entries [beg, end) of the value of slot
// `lane` of each neighbour's level-`tag` entry, for neighbours whose entry
// holds the lane and m holds it too.  The sum runs in CSR order, one window
// of kWave entries at a time; within a window up to 16 neighbour values are
// loaded at once.  Forward: parents' sigma.  Reverse: children's rho.
//
// Latency: a window needs three dependent loads (column ids, front records,
// values).  The loop keeps them in flight together: while the values of
// window k are loaded, the front records of window k+1 and the column ids of
// window k+2 are already on their way (issued first, so waiting for the
// values does not wait for more than they need).

// A value every lane holds alike, moved into scalar registers, so that the
// mask arithmetic on it below runs once per wave.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

// Whether the lane's slot is in the wave-uniform mask m (m used as the exec
// mask itself).
__device__ __forceinline__ bool lane_in(unsigned long long m) {
    return __builtin_amdgcn_inverse_ballot_w64(m);
}

// rank_in(m, lane) for a wave-uniform m: set bits of m below the lane.
__device__ __forceinline__ int lane_rank(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One window: add the values of the matching neighbours whose front records
// are `fu` (lane i holds the record of the window's i-th entry); m is
// wave-uniform.  Sixteen matched neighbours' value loads go out at a time
// (rmat-22: 8 -> 16 took a step from 302 to 298 ms; 4 gave 314).  A neighbour's mask and value base are read into scalar
// registers, so per neighbour a lane only computes its rank and loads; lanes
// whose slot the neighbour lacks add +0.0, which leaves their sum (never
// negative) unchanged bit for bit.
__device__ __forceinline__ void window_acc(uint4 fu, unsigned long long m, uint32_t tag,
                                           const double *__restrict__ val, double &acc,
                                           unsigned long long &pairs) {
    unsigned long long mu = 0;
    uint32_t vb = 0;
    if (fu.z == tag) {
        mu = mask_of(fu);
        vb = fu.w;
    }
    unsigned long long nz = __ballot((mu & m) != 0ull);
    while (nz) {
        unsigned long long mj[16];
        uint32_t vj[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            if (nz) {
                const int j = __ffsll((long long)nz) - 1;
                nz &= nz - 1;
                mj[t] = rl_u64(mu, j);
                vj[t] = (uint32_t)rl_i32((int32_t)vb, j);
            } else {
                mj[t] = 0;
                vj[t] = 0;
            }
        }
        double x[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            x[t] = 0.0;
            if (lane_in(mj[t] & m)) x[t] = val[(int64_t)vj[t] + lane_rank(mj[t])];
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            acc += x[t];
            pairs += (unsigned long long)__popcll(mj[t] & m);
        }
    }
}

__device__ __forceinline__ uint4 no_front() { return make_uint4(0u, 0u, kNoTag, 0u); }

// dense_sum given the records `f` of the first window (entries [beg, beg+kWave)).
__device__ __forceinline__ double dense_sum_from(uint4 f, int32_t beg, int32_t end,
                                                 unsigned long long m, uint32_t tag,
                                                 const int32_t *__restrict__ ci,
                                                 const uint4 *__restrict__ front,
                                                 const double *__restrict__ val,
                                                 unsigned long long &pairs) {
    const int lane = lane_id();
    double acc = 0.0;
    m = uniform_u64(m);  // one entry's slots: the same in every lane
    int32_t un = beg + kWave + lane < end ? ci[beg + kWave + lane] : -1;
    for (int32_t e0 = beg; e0 < end; e0 += kWave) {
        const uint4 fn = un >= 0 ? front[un] : no_front();  // window k+1
        const int32_t e2 = e0 + 2 * kWave + lane;
        un = e2 < end ? ci[e2] : -1;                         // window k+2
        window_acc(f, m, tag, val, acc, pairs);
        f = fn;
    }
    return acc;
}

__device__ __forceinline__ double dense_sum(int32_t beg, int32_t end, unsigned long long m,
                                            uint32_t tag, const int32_t *__restrict__ ci,
                                            const uint4 *__restrict__ front,
                                            const double *__restrict__ val,
                                            unsigned long long &pairs) {
    const int lane = lane_id();
    const int32_t u = beg + lane < end ? ci[beg + lane] : -1;
    return dense_sum_from(u >= 0 ? front[u] : no_front(), beg, end, m, tag, ci, front, val, pairs);
}

// dense_sum for every lane j set in dm, one after another in lane order
// (lane j's vertex: entries [beg_j, end_j), slots m_j), calling
// fin(j, sum, pairs) for each.  The next vertex's first window is fetched
// while the current one is summed, and the column ids of the one after it.
template <class Fin>
__device__ __forceinline__ void dense_each(unsigned long long dm, int32_t beg, int32_t end,
                                           unsigned long long m, uint32_t tag,
                                           const int32_t *__restrict__ ci,
                                           const uint4 *__restrict__ front,
                                           const double *__restrict__ val, Fin fin) {
    const int lane = lane_id();
    auto take = [&](int32_t &j, int32_t &b, int32_t &e, int32_t &u) {
        if (!dm) {
            j = -1;
            u = -1;
            return;
        }
        j = __ffsll((long long)dm) - 1;
        dm &= dm - 1;
        b = rl_i32(beg, j);
        e = rl_i32(end, j);
        u = b + lane < e ? ci[b + lane] : -1;
    };
    int32_t jl, bl = 0, el = 0, ul;
    int32_t jn, bn = 0, en = 0, un;
    take(jl, bl, el, ul);
    take(jn, bn, en, un);
    uint4 fl = ul >= 0 ? front[ul] : no_front();
    while (jl >= 0) {
        const uint4 fn = un >= 0 ? front[un] : no_front();
        int32_t jm, bm = 0, em = 0, um;
        take(jm, bm, em, um);
        unsigned long long pr = 0;
        const double acc = dense_sum_from(fl, bl, el, rl_u64(m, jl), tag, ci, front, val, pr);
        fin(jl, acc, pr);
        jl = jn;
        bl = bn;
        el = en;
        fl = fn;
        jn = jm;
        bn = bm;
        en = em;
        un = um;
    }
}

// Dense entries with rows of at most kPackDeg entries go through packed_each,
// which loads the values of kPackBatch matches at a time.
constexpr int32_t kPackDeg = 64;
constexpr int kPackBatch = 8;

// dense_sum for every lane j set in pm, with short rows packed: the rows of
// the set lanes, in lane order, are laid end to end and walked 64 entries per
// window (lane k of a window finds its entry by binary search over the row
// offsets in LDS), so one window's loads serve several entries.  Matches are
// taken in window order, which is entry order and CSR order inside an entry;
// a running sum is handed to fin(j, sum, pairs) when the entry changes, and
// an entry without a match gets fin(j, 0.0, 0).  Each entry's sum therefore
// adds the same terms in the same order as dense_sum: the same bits.  The
// column ids two windows ahead and the front records one window ahead are
// loaded while a window is summed.  s_off/s_beg: 64 ints of LDS for the wave.
template <class Fin>
__device__ __forceinline__ void packed_each(unsigned long long pm, int32_t beg, int32_t end,
                                            unsigned long long m, uint32_t tag,
                                            const int32_t *__restrict__ ci,
                                            const uint4 *__restrict__ front,
                                            const double *__restrict__ val, int32_t *s_off,
                                            int32_t *s_beg, Fin fin) {
    if (!pm) return;
    const int lane = lane_id();
    const int32_t d = ((pm >> lane) & 1ull) ? end - beg : 0;
    const int32_t incl = wave_incl_scan(d);
    const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
    s_off[lane] = incl - d;
    s_beg[lane] = beg;
    __builtin_amdgcn_wave_barrier();
    // entry (lane index) and neighbour of virtual position p, or -1 past the end
    auto locate = [&](int32_t p, int32_t &e, int32_t &u) {
        e = -1;
        u = -1;
        if (p < total) {
            int32_t a = 0, z = kWave - 1;
            while (a < z) {
                const int32_t mid = (a + z + 1) >> 1;
                if (s_off[mid] <= p) a = mid; else z = mid - 1;
            }
            e = a;
            u = ci[s_beg[a] + (p - s_off[a])];
        }
    };
    int32_t e0, u0, e1, u1;
    locate(lane, e0, u0);
    locate(kWave + lane, e1, u1);
    uint4 f = u0 >= 0 ? front[u0] : no_front();
    int32_t cur = -1;
    double acc = 0.0;
    unsigned long long pairs = 0, done = 0;
    for (int32_t p0 = 0; p0 < total; p0 += kWave) {
        const uint4 fn = u1 >= 0 ? front[u1] : no_front();  // window k+1
        int32_t e2, u2;
        locate(p0 + 2 * kWave + lane, e2, u2);               // window k+2
        // the slots of the lane's entry, read from the entry's lane; every
        // lane takes part in the shuffle (a lane switched off would hand
        // zero to the lanes reading from it)
        const int src = e0 >= 0 ? e0 : 0;
        const uint32_t me_lo = (uint32_t)__shfl((int)(uint32_t)m, src, kWave);
        const uint32_t me_hi = (uint32_t)__shfl((int)(uint32_t)(m >> 32), src, kWave);
        const unsigned long long me =
            e0 >= 0 ? ((unsigned long long)me_lo | ((unsigned long long)me_hi << 32)) : 0ull;
        unsigned long long mu = 0;
        uint32_t vbu = 0;
        if (f.z == tag) {
            mu = mask_of(f);
            vbu = f.w;
        }
        unsigned long long nz = __ballot((mu & me) != 0ull);
        while (nz) {
            int32_t ej[kPackBatch];
            unsigned long long mj[kPackBatch], bj[kPackBatch];
            uint32_t vj[kPackBatch];
#pragma unroll
            for (int t = 0; t < kPackBatch; ++t) {
                if (nz) {
                    const int j = __ffsll((long long)nz) - 1;
                    nz &= nz - 1;
                    ej[t] = rl_i32(e0, j);
                    mj[t] = rl_u64(mu, j);
                    vj[t] = (uint32_t)rl_i32((int32_t)vbu, j);
                    bj[t] = mj[t] & rl_u64(m, ej[t]);
                } else {  // past the last match: adds +0.0 to no entry
                    ej[t] = -1;
                    mj[t] = 0;
                    vj[t] = 0;
                    bj[t] = 0;
                }
            }
            double x[kPackBatch];
#pragma unroll
            for (int t = 0; t < kPackBatch; ++t) {
                x[t] = 0.0;
                if (lane_in(bj[t])) x[t] = val[(int64_t)vj[t] + lane_rank(mj[t])];
            }
#pragma unroll
            for (int t = 0; t < kPackBatch; ++t) {
                if (ej[t] >= 0 && ej[t] != cur) {
                    if (cur >= 0) {
                        fin(cur, acc, pairs);
                        done |= 1ull << cur;
                    }
                    cur = ej[t];
                    acc = 0.0;
                    pairs = 0;
                }
                acc += x[t];
                pairs += (unsigned long long)__popcll(bj[t]);
            }
        }
        f = fn;
        e0 = e1;
        e1 = e2;
        u1 = u2;
    }
    if (cur >= 0) {
        fin(cur, acc, pairs);
        done |= 1ull << cur;
    }
    for (unsigned long long rest = pm & ~done; rest; rest &= rest - 1)
        fin(__ffsll((long long)rest) - 1, 0.0, 0ull);
    __builtin_amdgcn_wave_barrier();  // the wave's LDS rows are free again
}

// One lane, one slot s: the same sum as dense_sum for slot s alone.  Four
// adjacency entries are in flight at a time (their column ids, then their
// front records, then the values), and added in CSR order.
__device__ __forceinline__ double sparse_sum(int32_t beg, int32_t end, int s, uint32_t tag,
                                             const int32_t *__restrict__ ci,
                                             const uint4 *__restrict__ front,
                                             const double *__restrict__ val,
                                             unsigned long long &pairs) {
    double acc = 0.0;
    for (int32_t e0 = beg; e0 < end; e0 += 4) {
        int32_t u[4];
        uint4 f[4];
        double x[4];
        bool hit[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) u[t] = e0 + t < end ? ci[e0 + t] : -1;
#pragma unroll
        for (int t = 0; t < 4; ++t) f[t] = u[t] >= 0 ? front[u[t]] : make_uint4(0u, 0u, kNoTag, 0u);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const unsigned long long mu = mask_of(f[t]);
            hit[t] = f[t].z == tag && ((mu >> s) & 1ull);
            x[t] = hit[t] ? val[(int64_t)f[t].w + rank_in(mu, s)] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (hit[t]) {
                acc += x[t];
                ++pairs;
            }
    }
    return acc;
}

__global__ void k_ms_clear(unsigned long long *seen, unsigned long long *nxt, uint4 *f0, uint4 *f1,
                           int32_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint4 z = make_front(0, kNoTag, 0u);
    for (; i < n; i += stride) {
        seen[i] = 0;
        nxt[i] = 0;
        f0[i] = z;
        f1[i] = z;
    }
}

// Level 0: entries [0, n0) hold the distinct source vertices and their slots.
__global__ void k_ms_init(LevelCtl *c, const int32_t *__restrict__ rp, const int32_t *queue,
                          const unsigned long long *qmask, uint32_t *qvb, int32_t n0,
                          unsigned long long *seen, uint4 *front0, double *val, int32_t *level_off,
                          HubEntry *hub_list, int32_t *hub_off, int32_t *hub_lvl_chunks,
                          int32_t *owner, int32_t *chunk_off, int32_t n,
                          long long nnz, unsigned long long active, double alpha, double beta) {
    __shared__ uint32_t s_vb[kSlots + 1];
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int32_t i = 0; i < n0; ++i) {
            s_vb[i] = run;
            run += (uint32_t)__popcll(qmask[i]);
        }
        s_vb[n0] = run;
    }
    __syncthreads();
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    for (int32_t i = wv; i < n0; i += blockDim.x / kWave) {
        const int32_t v = queue[i];
        const unsigned long long m = qmask[i];
        const uint32_t vb = s_vb[i];
        if ((m >> lane) & 1ull) val[vb + rank_in(m, lane)] = 1.0;
        if (lane == 0) {
            seen[v] = m;
            front0[v] = make_front(m, 0u, vb);
            qvb[i] = vb;
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
            if (d > kHubDeg) {  // at most kSlots hubs; split hubs start at a multiple of kXcds
                const int32_t k = split_hub_nchunks(d);
                const int32_t base = k >= kXcds ? (nch + kXcds - 1) & ~(kXcds - 1) : nch;
                for (int32_t q = nch; q < base + k; ++q) owner[q] = nh;
                hub_list[nh++] = HubEntry{v, i, base, k};
                nch = base + k;
            }
        }
        c->level = 0;
        c->lo = 0;
        c->hi = n0;
        c->tail_.v = n0;
        c->done = 0;
        c->mode = MODE_TOPDOWN;
        c->overflow_.v = 0;
        c->front_deg = fdeg;
        c->next_deg_.v = 0;
        c->settled_deg_.v = 0;
        c->reached_pairs = pairs;  // = s_vb[n0]
        c->val_lo = 0;
        c->vtail_.v = s_vb[n0];
        c->unset_deg = (unsigned long long)nnz - settled;
        c->sigma_max_bits_.v = (unsigned long long)__double_as_longlong(1.0);
        c->flagged_slots_.v = 0;
        c->live = active;  // every slot's level-0 frontier holds its source
        c->active = active;
        c->nlive_.v = 0;
        c->blocks_done_.v = 0;
        c->alpha = alpha;
        c->beta = beta;
        c->n_vertices = n;
        c->topdown_levels = 0;
        c->bottomup_levels = 0;
        c->hub_pack_.v = 0;
        c->in_hub_pack_.v = 0;
        c->in_hub_n = 0;
        c->in_hub_nchunks = 0;
        c->pull_cost_.v = 0;
        c->sigma_push = 0;
        c->hub_lo = 0;
        c->hub_hi = nh;
        c->hub_nchunks = nch;
        c->hub_next = nh;
        hub_off[0] = 0;
        hub_off[1] = nh;
        hub_lvl_chunks[0] = nch;
        chunk_off[0] = 0;
        c->chunk_next = nch;
        level_off[0] = 0;
        level_off[1] = n0;
    }
}

// Top-down discovery.  blockIdx.y == 0: block gather over the frontier's
// entries (hubs excluded), one adjacency entry per lane.  blockIdx.y == 1:
// the chunks of the frontier's hubs.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_topdown(LevelCtl *c, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const int32_t *__restrict__ rpi, int32_t *queue,
                                                   const unsigned long long *__restrict__ qmask,
                                                   const unsigned long long *__restrict__ seen,
                                                   unsigned long long *nxt,
                                                   const HubEntry *__restrict__ hub_list,
                                                   const int32_t *__restrict__ owner,
                                                   const int32_t *__restrict__ chunk_off,
                                                   long long qcap, unsigned long long *prof) {
    if (c->done || c->mode != MODE_TOPDOWN) return;
    __shared__ int32_t s_beg[BS], s_off[BS], s_scan[BS / kWave + 1];
    __shared__ unsigned long long s_mask[BS];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ unsigned long long s_red[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    const int32_t lo = c->lo, hi = c->hi;
    unsigned long long my_items = 0, my_edges = 0, my_pull = 0;
    // claims a new vertex for the next level; its incoming row length is the
    // work a pull of its path counts would do (the push/pull choice)
    auto visit = [&](int32_t w, unsigned long long fm) {
        const unsigned long long nm = fm & ~seen[w];
        if (nm && (nm & ~*(volatile unsigned long long *)&nxt[w]) && atomicOr(&nxt[w], nm) == 0ull) {
            my_pull += (unsigned long long)(rpi[w + 1] - rpi[w]);
            return true;
        }
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
                q.stage(claim, w, &c->tail_.v, queue, qcap, &c->overflow_.v);
            }
            __syncthreads();
        }
    } else {
        const int32_t nch = c->hub_nchunks, obase = chunk_off[c->level];
        // block k takes chunk id k: with a grid that is a multiple of kXcds,
        // XCD x gets the ids congruent to x, as in the hub sum kernels
        for (int32_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const HubEntry h = hub_list[owner[obase + k]];
            int32_t beg, end;
            if (!hub_chunk_range(h, k, rp, beg, end)) continue;
            const unsigned long long fm = qmask[h.entry];
            my_edges += (threadIdx.x == 0) ? (unsigned long long)(end - beg) : 0ull;
            for (int32_t e0 = beg; e0 < end; e0 += BS) {
                const int32_t e = e0 + threadIdx.x;
                bool claim = false;
                int32_t w = 0;
                if (e < end) {
                    w = ci[e];
                    claim = visit(w, fm);
                }
                q.stage(claim, w, &c->tail_.v, queue, qcap, &c->overflow_.v);
            }
        }
    }
    q.finish(&c->tail_.v, queue, qcap, &c->overflow_.v);
    block_add_u64<BS>(my_pull, s_red, &c->pull_cost_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// Bottom-up discovery: every vertex with unsettled slots ORs the level-l masks
// of its neighbours, 8 * kBuPerLane entries per lane group and step, until
// all its unsettled slots are found.
constexpr int kBuPerLane = 4;
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_bottomup(LevelCtl *c, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const unsigned long long *__restrict__ seen,
                                                    unsigned long long *nxt,
                                                    const uint4 *__restrict__ front_cur,
                                                    int32_t *queue, long long qcap,
                                                    unsigned long long *prof) {
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
    unsigned long long my_items = 0, my_edges = 0, my_pull = 0;
    for (int32_t b = blockIdx.x * BS; b < n; b += gridDim.x * BS) {
        const int32_t v = b + threadIdx.x;
        int32_t beg = 0, deg = 0;
        unsigned long long u_s = 0;
        if (v < n) {
            u_s = c->live & ~seen[v];  // live only ever holds slots in use
            if (u_s) {
                beg = rp[v];
                deg = rp[v + 1] - beg;
                ++my_items;
            }
        }
        constexpr int32_t kChunk = 8 * kBuPerLane;  // a lane group's entries per step
        const int32_t nch = (deg + kChunk - 1) / kChunk;
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
                const int32_t off = (k - coff[a]) * kChunk + j, da = dg[a], ba = bg[a];
                const unsigned long long want = uns[a];
                if (off < da && acc[a] != want) {
                    // the lane's kBuPerLane entries (8 apart) loaded together,
                    // past the row's end from its last entry, then dropped
                    uint4 f[kBuPerLane];
#pragma unroll
                    for (int r = 0; r < kBuPerLane; ++r) f[r] = front_cur[ci[ba + min(off + 8 * r, da - 1)]];
#pragma unroll
                    for (int r = 0; r < kBuPerLane; ++r)
                        if (off + 8 * r < da) {
                            if (f[r].z == lvl) x |= mask_of(f[r]) & want;
                            ++my_edges;
                        }
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
        if (found) {
            nxt[v] = found;
            my_pull += (unsigned long long)deg;  // rows here are the incoming ones
        }
        q.stage(found != 0ull, v, &c->tail_.v, queue, qcap, &c->overflow_.v);
    }
    q.finish(&c->tail_.v, queue, qcap, &c->overflow_.v);
    block_add_u64<BS>(my_pull, s_red, &c->pull_cost_.v);
    flush_counters<BS>(prof, my_items, my_edges, 0, s_red);
}

// End of a forward level (one thread): close the new frontier, turn the hub
// registrations into the next level's hub segment, decide the next
// direction, or set `done`.
__device__ void advance_level(LevelCtl *c, int32_t *level_off, int32_t *hub_off,
                              int32_t *hub_lvl_chunks, long long qcap, long long hub_cap,
                              int32_t *chunk_off, long long owner_cap, int32_t push) {
    if (c->done) return;
    c->sigma_push = push;  // how the level being closed gets its path counts
    c->pull_cost_.v = 0;
    if (c->mode == MODE_TOPDOWN) c->topdown_levels++; else c->bottomup_levels++;
    const int32_t tail = ld_agent(&c->tail_.v);
    const unsigned long long hp = ld_agent(&c->hub_pack_.v);
    const long long nchk = (long long)(hp & ((1ull << 40) - 1));
    if ((long long)tail > qcap || ld_agent(&c->overflow_.v) ||
        (long long)c->hub_next + (long long)(hp >> 40) > hub_cap ||
        (long long)c->chunk_next + nchk > owner_cap) {
        c->overflow_.v = 1;
        c->done = 1;
        return;
    }
    const int32_t nf = tail - c->hi;
    if (nf <= 0) {
        c->done = 1;
        return;
    }
    const int32_t nl = c->level + 1;
    level_off[nl + 1] = tail;
    c->hub_lo = c->hub_next;
    c->hub_hi = c->hub_next + (int32_t)(hp >> 40);
    c->hub_nchunks = (int32_t)(hp & ((1ull << 40) - 1));
    c->hub_next = c->hub_hi;
    c->hub_pack_.v = 0;
    hub_off[nl + 1] = c->hub_hi;
    hub_lvl_chunks[nl] = c->hub_nchunks;
    chunk_off[nl] = c->chunk_next;  // where this level's registrations put their chunk owners
    c->chunk_next += c->hub_nchunks;
    const unsigned long long ip = ld_agent(&c->in_hub_pack_.v);  // directed: incoming-row hubs
    c->in_hub_n = (int32_t)(ip >> 40);
    c->in_hub_nchunks = (int32_t)(ip & ((1ull << 40) - 1));
    c->in_hub_pack_.v = 0;
    c->front_deg = ld_agent(&c->next_deg_.v);
    c->unset_deg -= ld_agent(&c->settled_deg_.v);
    c->next_deg_.v = 0;
    c->settled_deg_.v = 0;
    c->val_lo = c->reached_pairs;  // the new level's values: [val_lo, reached_pairs)
    c->reached_pairs = ld_agent(&c->vtail_.v);  // every reached (slot, vertex) pair owns one value
    c->live = ld_agent(&c->nlive_.v);
    c->nlive_.v = 0;
    c->lo = c->hi;
    c->hi = tail;
    c->level = nl;
    if (c->mode == MODE_TOPDOWN) {
        if ((double)c->front_deg * c->alpha > (double)c->unset_deg) c->mode = MODE_BOTTOMUP;
    } else {
        if ((double)nf * c->beta < (double)c->n_vertices) c->mode = MODE_TOPDOWN;
    }
}

// Push threshold: the parents' outgoing entries must be fewer than the new
// entries' incoming ones by this factor (an atomic add per (slot, DAG edge)
// costs more than the load a pull makes instead).  Measured on RMAT-22 with
// 64-source batches: 2 -> 339 ms per 1,024 sources, 3 -> 332, 4 -> 327,
// 6 -> 327, 10 -> 328, never -> 342.
constexpr double kPushFactor = 4.0;

// Whether the level being built gets its path counts pushed (see k_ms_sigma).
__device__ __forceinline__ bool push_sigma(const LevelCtl *c, int32_t max_deg) {
    const double smax = __longlong_as_double((long long)ld_agent(&c->sigma_max_bits_.v));
    const bool exact = smax * (double)max_deg < 9007199254740992.0;  // 2^53
    const double pull = (double)ld_agent(&c->pull_cost_.v);
    return exact && (double)c->front_deg * kPushFactor < pull;
}

// Path counts of the new entries [hi, tail).  Wave takes 64 entries, gives
// each its value range, then: sparse entries are reduced by their own lane,
// dense ones by the whole wave in turn, hubs are registered for
// k_ms_sigma_hub.  Every entry's bookkeeping (qmask, value base, nxt reset,
// seen, front of the new level) is done here.  Six waves per SIMD, with some
// registers spilled, beat fewer waves without spills (rmat-22, 64-source
// batches, per 1,024 sources: 4 waves 55.4 ms in this kernel, 5: 56.1,
// 6: 53.1).
template <int BS>
__global__ __launch_bounds__(BS, 6) void k_ms_sigma(LevelCtl *c, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ rpi,
                                                 const int32_t *__restrict__ cii,
                                                 HubEntry *in_hub_list, long long in_hub_cap,
                                                 const int32_t *__restrict__ queue,
                                                 unsigned long long *qmask, uint32_t *qvb,
                                                 unsigned long long *seen, unsigned long long *nxt,
                                                 const uint4 *__restrict__ front_cur,
                                                 uint4 *front_nxt, double *val, long long vcap,
                                                 HubEntry *hub_list, long long hub_cap,
                                                 long long qcap, int32_t track_deg, int32_t *level_off,
                                                 int32_t *hub_off, int32_t *hub_lvl_chunks,
                                                 int32_t *owner, long long owner_cap,
                                                 int32_t *chunk_off, int32_t max_deg,
                                                 unsigned long long *prof) {
    if (c->done) return;
    const unsigned long long active = c->active;
    __shared__ unsigned long long s_red[1], s_base[1], s_or[1];
    __shared__ int32_t s_scan[BS / kWave + 1], s_poff[BS], s_pbeg[BS];
    const uint32_t lvl = (uint32_t)c->level;
    // Path counts of the new level by pull (each new entry sums its parents
    // over its incoming row) or by push (k_ms_sigma_push: each parent adds
    // its values into its children with float atomics), whichever reads
    // fewer adjacency entries: the new entries' incoming rows (counted by
    // discovery) against the parents' outgoing rows.  The push is taken only
    // while every sum it builds stays an exact integer -- below 2^53 with
    // at most max_deg terms of at most the largest path count so far -- so
    // the order of the atomics cannot change a bit: both ways give the same
    // values.  Every block of the grid computes the same decision from
    // control-block fields this kernel does not change before its last block
    // closes the level.
    const bool push = push_sigma(c, max_deg);
    const int32_t hi = c->hi;
    const int32_t tail = (int32_t)min((long long)c->tail_.v, qcap);
    const int lane = lane_id();
    if (threadIdx.x == 0) s_or[0] = 0;
    __syncthreads();
    unsigned long long my_deg = 0, my_settled = 0, my_flag = 0, my_pairs = 0, my_items = 0,
                       my_dag = 0, my_or = 0, my_scan = 0;
    double my_max = 0.0;
    for (int32_t b = hi + (int32_t)(blockIdx.x * BS); b < tail; b += gridDim.x * BS) {
        const int32_t i = b + (int32_t)threadIdx.x;
        const bool valid = i < tail;
        int32_t w = 0, beg = 0, end = 0, dout = 0;
        unsigned long long m = 0;
        if (valid) {
            w = queue[i];
            m = nxt[w];
            beg = rpi[w];  // parents: incoming row
            end = rpi[w + 1];
            dout = in_hub_list ? rp[w + 1] - rp[w] : end - beg;
        }
        const int32_t deg = end - beg;
        const int pc = __popcll(m);
        // value range of this entry: block scan + one atomic per block
        int32_t btotal;
        const int32_t excl = block_excl_scan<BS>(pc, s_scan, &btotal);
        if (threadIdx.x == 0) s_base[0] = btotal ? atomicAdd(&c->vtail_.v, (unsigned long long)btotal) : 0ull;
        __syncthreads();
        const unsigned long long vb64 = s_base[0] + (unsigned long long)excl;
        __syncthreads();
        const bool fits = vb64 + (unsigned long long)pc <= (unsigned long long)vcap;
        const uint32_t vb = (uint32_t)vb64;
        if (valid && !fits) atomicOr(&c->overflow_.v, 1);
        const bool hub = valid && fits && deg > kHubDeg;
        const bool sparse = !push && valid && fits && !hub && pc <= kSparseSlots && deg <= kSparseDeg;
        const bool dense = !push && valid && fits && !hub && !sparse;
        if (push && valid && fits)  // the parents add into these values
            for (int r = 0; r < pc; ++r) val[vb + r] = 0.0;
        if (sparse) {
            unsigned long long bits = m;
            while (bits) {
                const int s = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                const double acc = sparse_sum(beg, end, s, lvl, cii, front_cur, val, my_dag);
                val[vb + rank_in(m, s)] = acc;
                my_max = fmax(my_max, acc);
                if (sigma_is_large(acc)) my_flag |= 1ull << s;
            }
        }
        auto fin = [&](int jl, double acc, unsigned long long pr) {
            const uint32_t vbj = (uint32_t)rl_i32((int32_t)vb, jl);
            const unsigned long long mj = rl_u64(m, jl);
            if (lane == 0) my_dag += pr;
            const bool mine = lane_in(mj);
            if (mine) {
                val[vbj + lane_rank(mj)] = acc;
                my_max = fmax(my_max, acc);
            }
            my_flag |= __ballot(mine && sigma_is_large(acc));
        };
        const bool packed = dense && deg <= kPackDeg;
        packed_each(__ballot(packed), beg, end, m, lvl, cii, front_cur, val,
                    s_poff + (threadIdx.x & ~(kWave - 1)), s_pbeg + (threadIdx.x & ~(kWave - 1)), fin);
        dense_each(__ballot(dense && !packed), beg, end, m, lvl, cii, front_cur, val, fin);
        // Hub chunks of the level's outgoing rows (discovery, reverse pass)
        // are kept for the whole pass; on a directed graph the path counts
        // chunk the incoming rows, listed afresh for this level only.
        if (in_hub_list) {
            if (hub && !push) hub_register(&c->in_hub_pack_.v, in_hub_list, in_hub_cap, 0, w, i, deg);
            if (valid && fits && dout > kHubDeg)
                hub_register(&c->hub_pack_.v, hub_list, hub_cap, c->hub_next, w, i, dout, owner,
                             c->chunk_next, owner_cap);
        } else if (hub) {
            hub_register(&c->hub_pack_.v, hub_list, hub_cap, c->hub_next, w, i, deg, owner,
                         c->chunk_next, owner_cap);
        }
        if (sparse || dense) my_scan += (unsigned long long)deg;  // hubs: k_ms_sigma_hub
        if (valid) {
            qmask[i] = m;
            qvb[i] = vb;
            nxt[w] = 0;
            const unsigned long long now = seen[w] | m;
            seen[w] = now;
            front_nxt[w] = make_front(m, lvl + 1, vb);
            my_deg += (unsigned long long)dout;  // the next frontier's outgoing entries
            my_pairs += (unsigned long long)pc;
            my_or |= m;
            ++my_items;
            if (now == active) my_settled += (unsigned long long)deg;  // incoming: bottom-up's scan
        }
    }
    my_max = wave_max_f64(my_max);
    for (int o = 32; o > 0; o >>= 1) {
        my_flag |= __shfl_xor(my_flag, o, kWave);
        my_or |= __shfl_xor(my_or, o, kWave);
    }
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits_.v, my_max);
        if (my_flag) atomicOr(&c->flagged_slots_.v, my_flag);
        if (my_or) atomicOr(&s_or[0], my_or);  // LDS
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_or[0]) {
        // bits are only added during a level: a stale read is a subset of the
        // current value, so skipping when it already holds our bits is safe
        const unsigned long long cur = *(volatile unsigned long long *)&c->nlive_.v;
        if ((cur | s_or[0]) != cur) atomicOr(&c->nlive_.v, s_or[0]);
    }
    block_add_u64<BS>(my_deg, s_red, &c->next_deg_.v);  // direction switch and push choice
    if (track_deg) {  // only the direction switch needs this one
        __syncthreads();
        block_add_u64<BS>(my_settled, s_red, &c->settled_deg_.v);
    }
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_scan, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_dag, s_red, prof + 2);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 3);
    }
    // the last block to finish closes the level
    if (last_block(c, working_blocks((int64_t)tail - hi, BS)) && threadIdx.x == 0)
        advance_level(c, level_off, hub_off, hub_lvl_chunks, qcap, hub_cap, chunk_off, owner_cap, push);
}


// One forward level in one kernel, for sparse graphs (maximum degree
// kExpandDeg or less, so never bottom-up and no hubs; road-like): discovery of
// the next frontier and its path counts.  A thread takes one frontier entry
// and walks its row; for a neighbour x with new slots, the thread that raises
// x's claim tag to this level first (atomicMax on `claim`, which only grows)
// owns x's entry and puts x on the block's LDS list.  Then each thread takes
// one owned vertex: it gathers the slots of all x's parents on the current
// level (pulling over x's row, so the mask is complete whichever parent got
// there first), sums each slot's parents' sigma in CSR order (sparse_sum: the
// same order as k_ms_sigma, so the results are the same bits) and writes the
// entry.  Other threads reaching x see either its updated `seen` or a lost
// claim.  The frontier's own qmask/qvb are filled here from its front records
// (an owner appends only the vertex).  The last working block closes the level.
constexpr int kExpandDeg = 8;

template <int BS>
__global__ __launch_bounds__(BS) void k_ms_expand(
    LevelCtl *c, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t *queue,
    unsigned long long *qmask, uint32_t *qvb, unsigned long long *seen, int32_t *claim,
    const uint4 *__restrict__ front_cur, uint4 *front_nxt, double *val, long long vcap,
    long long qcap, int32_t *level_off, int32_t *hub_off, int32_t *hub_lvl_chunks, long long hub_cap,
    int32_t *chunk_off, long long owner_cap, int32_t parity, unsigned long long *prof) {
    // This kernel ends its level in its last working block.  A block that
    // starts only after that (the grid need not fit on the chip at once)
    // must not take part in the next level: the launch carries its level's
    // parity, the block reads done and level once (shared by the block), and
    // the level's entry range comes from level_off, which no later level
    // rewrites.
    __shared__ int32_t s_ctl[2];
    if (threadIdx.x == 0) {
        s_ctl[0] = ld_agent(&c->done);
        s_ctl[1] = ld_agent(&c->level);
    }
    __syncthreads();
    if (s_ctl[0] || (s_ctl[1] & 1) != parity) return;
    const unsigned long long active = c->active;
    __shared__ int32_t s_own[kExpandDeg * BS], s_cnt[1], s_scan[BS / kWave + 1];
    __shared__ int32_t s_qbuf[4 * BS], s_meta[2];
    __shared__ unsigned long long s_red[1], s_base[1], s_or[1];
    StagedQueue<BS, 4 * BS> q;
    q.init(s_qbuf, s_meta);
    if (threadIdx.x == 0) {
        s_or[0] = 0;
        s_cnt[0] = 0;
    }
    __syncthreads();
    const uint32_t lvl = (uint32_t)s_ctl[1];
    const int32_t lo = level_off[lvl], hi = level_off[lvl + 1];
    const int32_t nl = (int32_t)lvl + 1;
    const int lane = lane_id();
    unsigned long long my_items = 0, my_edges = 0, my_pairs = 0, my_pull = 0, my_flag = 0, my_or = 0;
    double my_max = 0.0;
    for (int32_t b = lo + blockIdx.x * BS; b < hi; b += gridDim.x * BS) {
        // claims: one frontier entry per thread, its row four entries at a time
        const int32_t i = b + threadIdx.x;
        if (i < hi) {
            const int32_t v = queue[i];
            const uint4 f = front_cur[v];
            const unsigned long long fm = mask_of(f);
            qmask[i] = fm;
            qvb[i] = f.w;
            const int32_t beg = rp[v], end = rp[v + 1];
            ++my_items;
            my_edges += (unsigned long long)(end - beg);
            for (int32_t e0 = beg; e0 < end; e0 += 4) {
                int32_t x[4];
                unsigned long long sx[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) x[t] = e0 + t < end ? ci[e0 + t] : -1;
#pragma unroll
                for (int t = 0; t < 4; ++t) sx[t] = x[t] >= 0 ? seen[x[t]] : ~0ull;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if ((fm & ~sx[t]) && atomicMax(&claim[x[t]], nl) < nl)
                        s_own[atomicAdd(&s_cnt[0], 1)] = x[t];
            }
        }
        __syncthreads();
        const int32_t n_own = s_cnt[0];
        // owned vertices: one per thread
        for (int32_t t0 = 0; t0 < n_own; t0 += BS) {
            const int32_t t = t0 + threadIdx.x;
            const bool own = t < n_own;
            int32_t x = 0;
            unsigned long long sx = 0, mx = 0;
            uint4 fu[kExpandDeg];  // x's row's front records, kept for the sums below
            if (own) {
                x = s_own[t];
                sx = seen[x];
                const int32_t xb = rp[x], xe = rp[x + 1];
                int32_t u[kExpandDeg];
#pragma unroll
                for (int k = 0; k < kExpandDeg; ++k) u[k] = xb + k < xe ? ci[xb + k] : -1;
#pragma unroll
                for (int k = 0; k < kExpandDeg; ++k) {
                    fu[k] = u[k] >= 0 ? front_cur[u[k]] : no_front();
                    if (fu[k].z == lvl) mx |= mask_of(fu[k]);
                }
                mx &= active & ~sx;
                my_pull += (unsigned long long)(xe - xb);
            }
            const int32_t pc = __popcll(mx);
            int32_t btotal;
            const int32_t excl = block_excl_scan<BS>(pc, s_scan, &btotal);
            if (threadIdx.x == 0)
                s_base[0] = btotal ? atomicAdd(&c->vtail_.v, (unsigned long long)btotal) : 0ull;
            __syncthreads();
            const unsigned long long vb64 = s_base[0] + (unsigned long long)excl;
            const bool fits = vb64 + (unsigned long long)pc <= (unsigned long long)vcap;
            if (own && mx && !fits) atomicOr(&c->overflow_.v, 1);
            const bool take = own && mx != 0ull && fits;
            if (take) {
                const uint32_t vb = (uint32_t)vb64;
                unsigned long long bits = mx;
                while (bits) {  // per slot: parents' sigma in CSR order (as sparse_sum)
                    const int sl = __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    double xv[kExpandDeg];
#pragma unroll
                    for (int k = 0; k < kExpandDeg; ++k) {
                        const unsigned long long mu = mask_of(fu[k]);
                        xv[k] = (fu[k].z == lvl && ((mu >> sl) & 1ull))
                                    ? val[(int64_t)fu[k].w + rank_in(mu, sl)] : 0.0;
                    }
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < kExpandDeg; ++k) {
                        const unsigned long long mu = mask_of(fu[k]);
                        if (fu[k].z == lvl && ((mu >> sl) & 1ull)) {
                            acc += xv[k];
                            ++my_pairs;
                        }
                    }
                    val[vb + rank_in(mx, sl)] = acc;
                    my_max = fmax(my_max, acc);
                    if (sigma_is_large(acc)) my_flag |= 1ull << sl;
                }
                front_nxt[x] = make_front(mx, (uint32_t)nl, vb);
                seen[x] = sx | mx;
                my_or |= mx;
            }
            q.stage(take, x, &c->tail_.v, queue, qcap, &c->overflow_.v);
        }
        if (threadIdx.x == 0) s_cnt[0] = 0;
        __syncthreads();
    }
    q.finish(&c->tail_.v, queue, qcap, &c->overflow_.v);
    my_max = wave_max_f64(my_max);
    for (int o = 32; o > 0; o >>= 1) {
        my_flag |= __shfl_xor(my_flag, o, kWave);
        my_or |= __shfl_xor(my_or, o, kWave);
    }
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits_.v, my_max);
        if (my_flag) atomicOr(&c->flagged_slots_.v, my_flag);
        if (my_or) atomicOr(&s_or[0], my_or);  // LDS
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_or[0]) atomicOr(&c->nlive_.v, s_or[0]);
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
        __syncthreads();
        block_add_u64<BS>(my_pull, s_red, prof + 3);
    }
    if (last_block(c, working_blocks((int64_t)hi - lo, BS)) && threadIdx.x == 0)
        advance_level(c, level_off, hub_off, hub_lvl_chunks, qcap, hub_cap, chunk_off, owner_cap, 0);
}

// Hubs, lane = slot: each chunk of kHubChunk adjacency entries is reduced by
// its own wave into a row of `partial` (64 doubles); a second kernel adds a
// hub's rows in chunk order.  The kernel boundary between them makes the rows
// visible without fences inside either kernel.  The chunk kernels are bounded
// to eight waves per SIMD (their scalar registers otherwise allow seven):
// rmat-22, per 1,024 sources, k_ms_delta_hub 108.1 -> 106.8 ms and
// k_ms_sigma_hub 48.1 -> 47.0 ms.
__device__ __forceinline__ double sum_rows(const double *__restrict__ partial, int32_t base,
                                           int32_t n) {
    const int lane = lane_id();
    double s = 0.0;
    int32_t q = 0;
    for (; q + 8 <= n; q += 8) {  // eight rows in flight, added in chunk order
        double x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = partial[(int64_t)(base + q + t) * kSlots + lane];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += x[t];
    }
    for (; q < n; ++q) s += partial[(int64_t)(base + q) * kSlots + lane];
    return s;
}

// A hub's chunk rows added in row order (split_id for a split hub).
__device__ __forceinline__ double sum_hub_rows(const double *__restrict__ partial,
                                               const HubEntry &h) {
    if (h.nchunks < kXcds) return sum_rows(partial, h.chunk_base, h.nchunks);
    const int lane = lane_id();
    double s = 0.0;
    for (int32_t r = 0; r < h.nchunks; r += 8) {  // nchunks is a multiple of 8
        double x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            x[t] = partial[(int64_t)(h.chunk_base + split_id(h.nchunks, r + t)) * kSlots + lane];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += x[t];
    }
    return s;
}

// Path counts of the current level's hubs (after advance), chunk by chunk.
// Undirected: the level's segment of the pass's hub list, through the owner
// map; directed (in_hub_list set): the level's incoming-row hubs, found by
// binary search over their chunk bases.
template <int BS>
__global__ __launch_bounds__(BS, 8) void k_ms_sigma_hub(LevelCtl *c, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const unsigned long long *__restrict__ qmask,
                                                     const uint32_t *__restrict__ qvb,
                                                     const uint4 *__restrict__ front_par,
                                                     double *val, const HubEntry *hub_list,
                                                     const int32_t *__restrict__ owner,
                                                     const int32_t *__restrict__ chunk_off,
                                                     const HubEntry *in_hub_list,
                                                     double *partial, unsigned long long *prof) {
    if (c->done || c->sigma_push) return;  // pushed: k_ms_sigma_push
    __shared__ unsigned long long s_red[1];
    const bool in = in_hub_list != nullptr;
    const int32_t nch = in ? c->in_hub_nchunks : c->hub_nchunks;
    const int32_t obase = in ? 0 : chunk_off[c->level], in_n = in ? c->in_hub_n : 0;
    const uint32_t pl = (uint32_t)c->level - 1;
    const int lane = lane_id();
    unsigned long long my_dag = 0, my_edges = 0;
    for_xcd_chunks<BS>(nch, [&](int64_t k) {
        const HubEntry h = in ? in_hub_list[hub_find(in_hub_list, 0, in_n, (int32_t)k)]
                              : hub_list[owner[obase + k]];
        int32_t beg, end;
        if (!hub_chunk_range(h, k, rp, beg, end)) return;
        const unsigned long long m = qmask[h.entry];
        if (lane == 0) my_edges += (unsigned long long)(end - beg);
        unsigned long long pr = 0;
        partial[k * kSlots + lane] = dense_sum(beg, end, m, pl, ci, front_par, val, pr);
        if (lane == 0) my_dag += pr;
    });
    if (prof) {
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_dag, s_red, prof + 2);
    }
}

// Path counts of the current level's hubs: each hub's chunk rows added in
// chunk order (one wave per hub entry).
__global__ void k_ms_sigma_hub_fin(LevelCtl *c, const unsigned long long *__restrict__ qmask,
                                   const uint32_t *__restrict__ qvb, double *val,
                                   const HubEntry *__restrict__ hub_list,
                                   const double *__restrict__ partial,
                                   const HubEntry *__restrict__ in_hub_list) {
    if (c->done || c->sigma_push) return;
    if (in_hub_list) hub_list = in_hub_list;  // directed: the level's incoming-row hubs
    const int32_t hlo = in_hub_list ? 0 : c->hub_lo, hhi = in_hub_list ? c->in_hub_n : c->hub_hi;
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    unsigned long long my_flag = 0;
    double my_max = 0.0;
    for (int64_t j = hlo + wave0; j < hhi; j += nwaves) {
        const HubEntry h = hub_list[j];
        const unsigned long long m = qmask[h.entry];
        const double s = sum_hub_rows(partial, h);
        const bool mine = (m >> lane) & 1ull;
        if (mine) {
            val[qvb[h.entry] + rank_in(m, lane)] = s;
            my_max = fmax(my_max, s);
        }
        my_flag |= __ballot(mine && sigma_is_large(s));
    }
    my_max = wave_max_f64(my_max);
    if (lane == 0) {
        atomic_max_nonneg_f64(&c->sigma_max_bits_.v, my_max);
        if (my_flag) atomicOr(&c->flagged_slots_.v, my_flag);
    }
}

// Pushed path counts, for a level whose sigma_push k_ms_sigma set: every
// entry of the parent level adds its value of each slot into the entries of
// its children (outgoing row, next level) that hold that slot, with float
// atomics; k_ms_sigma zeroed the children's values.  The sums are exact
// integers whenever the push is taken, so they equal the pulled ones bit for
// bit whatever order the atomics land in.

// One window of a parent's row, lane = slot: lane i holds the front record
// `fu` of the window's i-th child; every lane of a slot in both masks adds
// the parent's value `sig` of that slot into the child's value of it.  m is
// wave-uniform.
__device__ __forceinline__ void push_window(uint4 fu, unsigned long long m, uint32_t tag,
                                            double sig, double *val, unsigned long long &pairs) {
    unsigned long long mu = 0;
    uint32_t vb = 0;
    if (fu.z == tag) {
        mu = mask_of(fu);
        vb = fu.w;
    }
    unsigned long long nz = __ballot((mu & m) != 0ull);
    while (nz) {
        const int j = __ffsll((long long)nz) - 1;
        nz &= nz - 1;
        const unsigned long long mj = rl_u64(mu, j);
        const uint32_t vj = (uint32_t)rl_i32((int32_t)vb, j);
        if (lane_in(mj & m)) unsafeAtomicAdd(&val[(int64_t)vj + lane_rank(mj)], sig);
        pairs += (unsigned long long)__popcll(mj & m);
    }
}

// A wave pushes one parent over row entries [beg, end) (lane = slot, parent
// mask m, `sig` = the parent's value of the lane's slot).  The column ids of
// the window after next and the records of the next one are loaded while the
// current window is pushed.
__device__ __forceinline__ void push_row(int32_t beg, int32_t end, unsigned long long m,
                                         uint32_t tag, double sig,
                                         const int32_t *__restrict__ ci,
                                         const uint4 *__restrict__ front, double *val,
                                         unsigned long long &pairs) {
    const int lane = lane_id();
    m = uniform_u64(m);
    const int32_t u = beg + lane < end ? ci[beg + lane] : -1;
    uint4 f = u >= 0 ? front[u] : no_front();
    int32_t un = beg + kWave + lane < end ? ci[beg + kWave + lane] : -1;
    for (int32_t e0 = beg; e0 < end; e0 += kWave) {
        const uint4 fn = un >= 0 ? front[un] : no_front();
        const int32_t e2 = e0 + 2 * kWave + lane;
        un = e2 < end ? ci[e2] : -1;
        push_window(f, m, tag, sig, val, pairs);
        f = fn;
    }
}

// Parents with at most this many slots push lane = row entry
// (push_row_lanes): one pass over the window per parent slot beats one per
// matching child.
constexpr int kPushLaneSlots = 16;

// A wave pushes one parent with few slots over row entries [beg, end), lane
// = entry: for each of the parent's slots in turn (value `pv` of lane r =
// the parent's r-th value), every lane whose child holds that slot adds the
// parent's value of it.  m is wave-uniform.
__device__ __forceinline__ void push_row_lanes(int32_t beg, int32_t end, unsigned long long m,
                                               double pv, uint32_t tag,
                                               const int32_t *__restrict__ ci,
                                               const uint4 *__restrict__ front, double *val,
                                               unsigned long long &pairs) {
    const int lane = lane_id();
    m = uniform_u64(m);
    const int32_t u = beg + lane < end ? ci[beg + lane] : -1;
    uint4 f = u >= 0 ? front[u] : no_front();
    int32_t un = beg + kWave + lane < end ? ci[beg + kWave + lane] : -1;
    for (int32_t e0 = beg; e0 < end; e0 += kWave) {
        const uint4 fn = un >= 0 ? front[un] : no_front();
        const int32_t e2 = e0 + 2 * kWave + lane;
        un = e2 < end ? ci[e2] : -1;
        const unsigned long long mu = f.z == tag ? mask_of(f) & m : 0ull;
        if (__ballot(mu != 0ull)) {
            unsigned long long rest = m;
            for (int r = 0; rest; ++r) {
                const int sl = __ffsll((long long)rest) - 1;
                rest &= rest - 1;
                const double x = __longlong_as_double(
                    (long long)rl_u64((unsigned long long)__double_as_longlong(pv), r));
                if ((mu >> sl) & 1ull) {
                    unsafeAtomicAdd(&val[(int64_t)f.w + rank_in(mask_of(f), sl)], x);
                    ++pairs;
                }
            }
        }
        f = fn;
    }
}

// One lane pushes a parent with at most kSparseSlots slots over its short
// row, four entries in flight.
__device__ __forceinline__ void push_sparse(int32_t beg, int32_t end, unsigned long long m,
                                            uint32_t vb, uint32_t tag,
                                            const int32_t *__restrict__ ci,
                                            const uint4 *__restrict__ front, double *val,
                                            unsigned long long &pairs) {
    double pv[kSparseSlots];
#pragma unroll
    for (int r = 0; r < kSparseSlots; ++r) pv[r] = r < __popcll(m) ? val[vb + r] : 0.0;
    for (int32_t e0 = beg; e0 < end; e0 += 4) {
        int32_t u[4];
        uint4 f[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) u[t] = e0 + t < end ? ci[e0 + t] : -1;
#pragma unroll
        for (int t = 0; t < 4; ++t) f[t] = u[t] >= 0 ? front[u[t]] : no_front();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (f[t].z != tag) continue;
            const unsigned long long mu = mask_of(f[t]);
            unsigned long long both = mu & m;
            while (both) {
                const int sl = __ffsll((long long)both) - 1;
                both &= both - 1;
                const int r = rank_in(m, sl);
                unsafeAtomicAdd(&val[(int64_t)f[t].w + rank_in(mu, sl)], r == 0 ? pv[0] : pv[1]);
                ++pairs;
            }
        }
    }
}

// A wave pushes one parent (wave-uniform mask m and value base vb) over row
// entries [beg, end), lane = entry for few slots, else lane = slot.  `pairs`
// counts in lane 0 only.
__device__ __forceinline__ void push_parent(int32_t beg, int32_t end, unsigned long long m,
                                            uint32_t vb, uint32_t tag,
                                            const int32_t *__restrict__ ci,
                                            const uint4 *__restrict__ front, double *val,
                                            unsigned long long &pairs) {
    const int lane = lane_id();
    m = uniform_u64(m);
    const int pc = __popcll(m);
    unsigned long long pr = 0;
    if (pc <= kPushLaneSlots) {
        const double pv = lane < pc ? val[vb + lane] : 0.0;
        push_row_lanes(beg, end, m, pv, tag, ci, front, val, pr);
        for (int o = 32; o > 0; o >>= 1) pr += __shfl_xor(pr, o, kWave);
    } else {
        const double sig = lane_in(m) ? val[vb + lane_rank(m)] : 0.0;
        push_row(beg, end, m, tag, sig, ci, front, val, pr);
    }
    if (lane == 0) pairs += pr;
}

// blockIdx.y == 0: the parent level's entries without a hub row, like
// k_ms_sigma's (a lane alone for few slots and a short row, else the wave in
// turn); blockIdx.y == 1: the chunks of the parents' hub rows, one wave each.
template <int BS>
__global__ __launch_bounds__(BS) void k_ms_sigma_push(LevelCtl *c,
                                                      const int32_t *__restrict__ level_off,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const int32_t *__restrict__ queue,
                                                      const unsigned long long *__restrict__ qmask,
                                                      const uint32_t *__restrict__ qvb,
                                                      const uint4 *__restrict__ front_child,
                                                      double *val, const HubEntry *hub_list,
                                                      const int32_t *__restrict__ owner,
                                                      const int32_t *__restrict__ chunk_off,
                                                      const int32_t *__restrict__ hub_lvl_chunks,
                                                      unsigned long long *prof) {
    if (c->done || !c->sigma_push) return;
    __shared__ unsigned long long s_red[1];
    const int32_t pl = c->level - 1;  // parents
    const uint32_t tag = (uint32_t)c->level;
    const int lane = lane_id();
    unsigned long long my_items = 0, my_edges = 0, my_pairs = 0;
    if (blockIdx.y == 0) {
        const int32_t plo = level_off[pl], phi = level_off[pl + 1];
        for (int32_t b = plo + (int32_t)(blockIdx.x * BS); b < phi; b += gridDim.x * BS) {
            const int32_t i = b + (int32_t)threadIdx.x;
            const bool valid = i < phi;
            int32_t beg = 0, end = 0;
            unsigned long long m = 0;
            uint32_t vb = 0;
            if (valid) {
                const int32_t v = queue[i];
                m = qmask[i];
                vb = qvb[i];
                beg = rp[v];
                end = rp[v + 1];
            }
            const int32_t deg = end - beg;
            const bool hub = deg > kHubDeg;  // blockIdx.y == 1
            const bool sparse = valid && !hub && __popcll(m) <= kSparseSlots && deg <= kSparseDeg;
            const bool dense = valid && !hub && !sparse;
            unsigned long long pr = 0;
            if (sparse) push_sparse(beg, end, m, vb, tag, ci, front_child, val, pr);
            my_pairs += pr;
            unsigned long long dm = __ballot(dense);
            while (dm) {
                const int j = __ffsll((long long)dm) - 1;
                dm &= dm - 1;
                const unsigned long long mj = rl_u64(m, j);
                const uint32_t vbj = (uint32_t)rl_i32((int32_t)vb, j);
                unsigned long long wp = 0;
                push_parent(rl_i32(beg, j), rl_i32(end, j), mj, vbj, tag, ci, front_child, val, wp);
                my_pairs += wp;
            }
            if (valid) {
                ++my_items;
                if (!hub) my_edges += (unsigned long long)deg;
            }
        }
    } else {
        const int32_t nch = hub_lvl_chunks[pl], obase = chunk_off[pl];
        for_xcd_chunks<BS>(nch, [&](int64_t k) {
            const HubEntry h = hub_list[owner[obase + k]];
            int32_t beg, end;
            if (!hub_chunk_range(h, k, rp, beg, end)) return;
            unsigned long long wp = 0;
            push_parent(beg, end, qmask[h.entry], qvb[h.entry], tag, ci, front_child, val, wp);
            my_pairs += wp;
            if (lane == 0) my_edges += (unsigned long long)(end - beg);
        });
    }
    flush_counters<BS>(prof, my_items, my_edges, my_pairs, s_red);
}

// Largest path count of a pushed level: one pass over its values
// [val_lo, reached_pairs), contiguous in the value store.  (Pushed sums are
// below 2^53, so no slot is flagged here.)
__global__ void k_ms_sigma_push_fin(LevelCtl *c, const double *__restrict__ val) {
    if (c->done || !c->sigma_push) return;
    const int64_t lo = (int64_t)c->val_lo, hi = (int64_t)c->reached_pairs;
    double my_max = 0.0;
    for (int64_t k = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < hi;
         k += (int64_t)gridDim.x * blockDim.x)
        my_max = fmax(my_max, val[k]);
    my_max = wave_max_f64(my_max);
    if (lane_id() == 0) atomic_max_nonneg_f64(&c->sigma_max_bits_.v, my_max);
}

// Finish slot `s` of an entry in the reverse pass: acc = sum of the
// children's rho; delta = sigma * acc goes to the BC rows, and the entry's
// value becomes rho = (1 + delta) / sigma for its parents.
__device__ __forceinline__ void finish_slot(double acc, double *vp, double *drow) {
    const double sg = *vp;
    const double d = sg * acc;
    *drow = d;
    *vp = (1.0 + d) / sg;
}

// Reverse sweep of one level.  Every entry re-publishes {mask, level, value
// base} in front(l); dense and sparse entries are finished here, hubs in
// k_ms_delta_hub.
template <int BS>
__global__ __launch_bounds__(BS, 6) void k_ms_delta(LevelCtl *c, int32_t step,
                                                 const int32_t *__restrict__ level_off,
                                                 const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const int32_t *__restrict__ queue,
                                                 const unsigned long long *__restrict__ qmask,
                                                 const uint32_t *__restrict__ qvb, uint4 *f0,
                                                 uint4 *f1, double *val, double *dlt,
                                                 int32_t parity, unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    __shared__ int32_t s_poff[BS], s_pbeg[BS];
    // The reverse sweep's level (0 = finished), read once by the block.  With
    // `step` this kernel moves the sweep up in its last working block; the
    // parity of the launch's step (levels swept before it) lets a block that
    // starts after that return instead of sweeping the next level.
    __shared__ int32_t s_ctl[2];
    if (threadIdx.x == 0) {
        s_ctl[0] = ld_agent(&c->bwd_level);
        s_ctl[1] = c->bwd_last;
    }
    __syncthreads();
    const int32_t lvl = s_ctl[0];
    if (lvl < 1 || ((s_ctl[1] - lvl) & 1) != parity) return;
    const bool deepest = lvl == s_ctl[1];
    const uint4 *__restrict__ front_rd = ((lvl + 1) & 1) ? f1 : f0;  // children's records
    uint4 *front_wr = (lvl & 1) ? f1 : f0;
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
        uint32_t vb = 0;
        if (valid) {
            v = queue[i];
            m = qmask[i];
            vb = qvb[i];
            beg = rp[v];
            end = rp[v + 1];
            front_wr[v] = make_front(m, (uint32_t)lvl, vb);
            ++my_items;
            my_slots += (unsigned long long)__popcll(m);
        }
        const int32_t deg = end - beg;
        if (deepest) {  // no children: delta = 0, rho = 1 / sigma
            unsigned long long bits = m;
            while (bits) {
                const int s = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                finish_slot(0.0, val + vb + rank_in(m, s), dlt + (int64_t)v * kSlots + s);
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
                const double acc = sparse_sum(beg, end, s, nl, ci, front_rd, val, my_pairs);
                finish_slot(acc, val + vb + rank_in(m, s), dlt + (int64_t)v * kSlots + s);
            }
        }
        auto fin = [&](int jl, double acc, unsigned long long pr) {
            const int32_t vj = rl_i32(v, jl);
            const uint32_t vbj = (uint32_t)rl_i32((int32_t)vb, jl);
            const unsigned long long mj = rl_u64(m, jl);
            if (lane == 0) {
                my_pairs += pr;
                my_edges += (unsigned long long)(rl_i32(end, jl) - rl_i32(beg, jl));
            }
            if (lane_in(mj))
                finish_slot(acc, val + vbj + lane_rank(mj), dlt + (int64_t)vj * kSlots + lane);
        };
        const bool packed = dense && deg <= kPackDeg;
        packed_each(__ballot(packed), beg, end, m, nl, ci, front_rd, val,
                    s_poff + (threadIdx.x & ~(kWave - 1)), s_pbeg + (threadIdx.x & ~(kWave - 1)), fin);
        dense_each(__ballot(dense && !packed), beg, end, m, nl, ci, front_rd, val, fin);
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
    // when no hub kernel follows, the last block moves the sweep one level up
    if (step && last_block(c, working_blocks((int64_t)hi - lo, BS)) && threadIdx.x == 0)
        c->bwd_level = lvl - 1;
}

template <int BS>
__global__ __launch_bounds__(BS, 8) void k_ms_delta_hub(
    const LevelCtl *c, const int32_t *__restrict__ hub_off,
    const int32_t *__restrict__ hub_lvl_chunks, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ ci, const unsigned long long *__restrict__ qmask,
    const uint4 *f0, const uint4 *f1, const double *val, const HubEntry *hub_list,
    const int32_t *__restrict__ owner, const int32_t *__restrict__ chunk_off, double *partial,
    unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    const int32_t lvl = c->bwd_level;
    if (lvl < 1) return;
    const uint4 *__restrict__ front_rd = ((lvl + 1) & 1) ? f1 : f0;
    const int32_t nch = lvl == c->bwd_last ? 0 : hub_lvl_chunks[lvl];  // deepest: no children
    const int32_t obase = chunk_off[lvl];
    const uint32_t nl = (uint32_t)lvl + 1;
    const int lane = lane_id();
    unsigned long long my_edges = 0, my_pairs = 0;
    for_xcd_chunks<BS>(nch, [&](int64_t k) {
        const HubEntry h = hub_list[owner[obase + k]];
        int32_t beg, end;
        if (!hub_chunk_range(h, k, rp, beg, end)) return;
        const unsigned long long m = qmask[h.entry];
        if (lane == 0) my_edges += (unsigned long long)(end - beg);
        unsigned long long pr = 0;
        partial[k * kSlots + lane] = dense_sum(beg, end, m, nl, ci, front_rd, val, pr);
        if (lane == 0) my_pairs += pr;
    });
    if (prof) {
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
    }
}

// Reverse sums of the swept level's hubs: chunk rows added in chunk order, then
// delta and rho as for other entries; the last working block moves the sweep
// one level up.
__global__ void k_ms_delta_hub_fin(LevelCtl *c, const int32_t *__restrict__ hub_off,
                                   const unsigned long long *__restrict__ qmask,
                                   const uint32_t *__restrict__ qvb, double *val, double *dlt,
                                   const HubEntry *__restrict__ hub_list,
                                   const double *__restrict__ partial, int32_t parity) {
    // Ends the reverse level in its last working block: guarded as k_ms_delta.
    __shared__ int32_t s_ctl[2];
    if (threadIdx.x == 0) {
        s_ctl[0] = ld_agent(&c->bwd_level);
        s_ctl[1] = c->bwd_last;
    }
    __syncthreads();
    const int32_t lvl = s_ctl[0];
    if (lvl < 1 || ((s_ctl[1] - lvl) & 1) != parity) return;
    const int32_t hlo = hub_off[lvl];
    const int32_t nh = lvl == s_ctl[1] ? 0 : hub_off[lvl + 1] - hlo;  // deepest: done in k_ms_delta
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t j = wave0; j < nh; j += nwaves) {
        const HubEntry h = hub_list[hlo + j];
        const unsigned long long m = qmask[h.entry];
        const double s = sum_hub_rows(partial, h);
        if ((m >> lane) & 1ull)
            finish_slot(s, val + qvb[h.entry] + rank_in(m, lane), dlt + (int64_t)h.v * kSlots + lane);
    }
    if (last_block(c, working_blocks((int64_t)nh * kWave, (int)blockDim.x)) && threadIdx.x == 0)
        c->bwd_level = lvl - 1;
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
        // The row is read a cache line (16 doubles) at a time, so each line is
        // fetched once and used whole; slots are still added one by one in order.
        for (int32_t s0 = 0; s0 < nslots; s0 += 16) {
            double x[16];
            const double2 *r2 = reinterpret_cast<const double2 *>(row + s0);  // inside the 64-slot row
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double2 p = r2[t];
                x[2 * t] = p.x;
                x[2 * t + 1] = p.y;
            }
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int32_t s = s0 + t;
                if (s >= nslots) break;
                double *out = tbl.out[s];
                if (!out) continue;
                if (out != cur) {
                    if (cur) cur[v] = acc;
                    cur = out;
                    acc = out[v];
                }
                if (((sm >> s) & 1ull) && s_src[s] != v) acc += x[t];
            }
        }
        if (cur) cur[v] = acc;
    }
    if (prof) {
        block_add_u64<BS>(my_items, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_slots, s_red, prof + 3);
    }
}

// Per-slot results of one level into source-major arrays (for checks):
// distance and sigma after the forward pass (values still hold sigma),
// delta after the reverse pass.
// Reverse-pass control: start at the deepest level; the last kernel of each
// reverse level moves it one level up.
__global__ void k_ms_bwd_init(LevelCtl *c) {
    c->bwd_level = c->level;
    c->bwd_last = c->level;
    c->blocks_done_.v = 0;
}

__global__ void k_ms_extract(const int32_t *__restrict__ queue,
                             const unsigned long long *__restrict__ qmask,
                             const uint32_t *__restrict__ qvb, int32_t lo, int32_t hi, int32_t lvl,
                             int32_t n, const double *__restrict__ val,
                             const double *__restrict__ dlt, int32_t *out_dist, double *out_sigma,
                             double *out_delta) {
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t i = lo + wave0; i < hi; i += nwaves) {
        const int32_t v = queue[i];
        const unsigned long long m = qmask[i];
        if (!((m >> lane) & 1ull)) continue;
        const int64_t o = (int64_t)lane * n + v;
        if (out_dist) out_dist[o] = lvl;
        if (out_sigma) out_sigma[o] = val[qvb[i] + rank_in(m, lane)];
        if (out_delta) out_delta[o] = lvl > 0 ? dlt[(int64_t)v * kSlots + lane] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int64_t hub_capacity(sp_graph g) { return (int64_t)g->n_hubs * kSlots + kSlots; }
// A hub has at most one entry per slot, so at most kSlots entries per pass.
static int64_t owner_capacity(sp_graph g) { return g->split_hub_chunks * kSlots + kSlots; }

static int64_t value_capacity(sp_graph g, int32_t width) {
    return (int64_t)std::max(g->n, 1) * width + kSlots;
}

// Hub chunk partial rows: the outgoing rows' chunks (reverse pass) or, on a
// directed graph, one level's incoming-row chunks (path counts), whichever
// needs more.
static int64_t partial_rows(sp_graph g) {
    return std::max(g->split_hub_chunks, g->directed ? g->split_hub_chunks_in : 0) + 1;
}

static int64_t in_hub_capacity(sp_graph g) { return g->directed ? (int64_t)g->n_hubs_in + 1 : 0; }

int32_t auto_engine(sp_graph g) {
    return g->n_hubs == 0 && g->n_hubs_in == 0 && g->max_degree <= kExpandDeg ? SP_ENGINE_BLOCKS
                                                                                : SP_ENGINE_BITMAP;
}

size_t batch_ws_bytes(sp_graph g, int64_t qcap, int32_t width, int32_t engine) {
    const size_t V = (size_t)std::max(g->n, 1);
    if (engine == SP_ENGINE_BLOCKS) return wg_ws_bytes(g, width) + kSlots * 4 + sizeof(LevelCtl);
    return V * (8 + 8 + 16 + 16) + V * kSlots * 8 + (size_t)value_capacity(g, width) * 8 +
           (size_t)qcap * 16 + (V + 2) * 12 + kSlots * 4 +
           (size_t)hub_capacity(g) * sizeof(HubEntry) + ((size_t)g->n_hubs + 1) * 4 +
           (size_t)in_hub_capacity(g) * sizeof(HubEntry) +
           (size_t)owner_capacity(g) * 4 + (V + 2) * 4 +
           (size_t)partial_rows(g) * kSlots * 8 + sizeof(LevelCtl);
}

sp_status batch_ws_create(sp_graph g, int64_t qcap, int32_t width, int32_t engine, BatchWorkspace &ws) {
    ws.device = g->device;
    ws.n = g->n;
    ws.width = width;
    ws.engine = engine;
    if (engine == SP_ENGINE_BLOCKS) {  // per-slot arrays only
        ws.qcap = 0;
        SP_TRY(wg_ws_alloc(g, width, ws));
        SP_TRY(dev_alloc((void **)&ws.slot_src, kSlots * 4));
        SP_HIP(hipHostMalloc((void **)&ws.staging, kSlots * (4 + 8 + 4), hipHostMallocDefault));
        ws.bytes = batch_ws_bytes(g, 0, width, engine);
        return SP_OK;
    }
    const size_t V = (size_t)std::max(g->n, 1);
    ws.qcap = qcap;
    ws.vcap = value_capacity(g, width);
    if (ws.vcap > (int64_t)UINT32_MAX) {
        set_error("graph too large for %d-slot passes (value bases are 32-bit)", width);
        return SP_ERR_NOT_SUPPORTED;
    }
    ws.level_cap = (int32_t)std::min<int64_t>((int64_t)V + 2, (int64_t)INT32_MAX);
    ws.hub_cap = hub_capacity(g);
    ws.owner_cap = owner_capacity(g);
    SP_TRY(dev_alloc((void **)&ws.owner, (size_t)ws.owner_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.chunk_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.seen, V * 8));
    SP_TRY(dev_alloc((void **)&ws.nxt, V * 8));
    SP_TRY(dev_alloc((void **)&ws.front[0], V * 16));
    SP_TRY(dev_alloc((void **)&ws.front[1], V * 16));
    SP_TRY(dev_alloc((void **)&ws.val, (size_t)ws.vcap * 8));
    SP_TRY(dev_alloc((void **)&ws.dlt, V * kSlots * 8));
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    SP_TRY(dev_alloc((void **)&ws.qvb, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.level_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_off, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_lvl_chunks, (size_t)ws.level_cap * 4));
    SP_TRY(dev_alloc((void **)&ws.hub_list, (size_t)ws.hub_cap * sizeof(HubEntry)));
    SP_TRY(dev_alloc((void **)&ws.hub_cnt, ((size_t)g->n_hubs + 1) * 4));
    SP_TRY(dev_alloc((void **)&ws.partial, (size_t)partial_rows(g) * kSlots * 8));
    ws.in_hub_cap = in_hub_capacity(g);
    if (ws.in_hub_cap) SP_TRY(dev_alloc((void **)&ws.in_hub_list, (size_t)ws.in_hub_cap * sizeof(HubEntry)));
    SP_HIP(hipMemset(ws.hub_cnt, 0, ((size_t)g->n_hubs + 1) * 4));
    SP_TRY(dev_alloc((void **)&ws.slot_src, kSlots * 4));
    SP_TRY(dev_alloc((void **)&ws.ctl, sizeof(LevelCtl)));
    SP_HIP(hipHostMalloc((void **)&ws.ctl_host, sizeof(LevelCtl), hipHostMallocDefault));
    SP_HIP(hipHostMalloc((void **)&ws.staging, kSlots * (4 + 8 + 4), hipHostMallocDefault));
    SP_HIP(hipEventCreate(&ws.ev0));
    SP_HIP(hipEventCreate(&ws.ev1));
    ws.bytes = batch_ws_bytes(g, qcap, width, engine);
    return SP_OK;
}

void batch_ws_destroy(BatchWorkspace &ws) {
    for (CapturedChunk *c : {&ws.fwd_short, &ws.fwd_long, &ws.bwd}) {
        if (c->exec) (void)hipGraphExecDestroy(c->exec);
        c->exec = nullptr;
    }
    if (ws.cap_stream) (void)hipStreamDestroy(ws.cap_stream);
    ws.cap_stream = nullptr;
    wg_ws_free(ws);
    dev_free(ws.seen);
    dev_free(ws.nxt);
    dev_free(ws.front[0]);
    dev_free(ws.front[1]);
    dev_free(ws.val);
    dev_free(ws.dlt);
    dev_free(ws.queue);
    dev_free(ws.qmask);
    dev_free(ws.qvb);
    dev_free(ws.level_off);
    dev_free(ws.hub_off);
    dev_free(ws.hub_lvl_chunks);
    dev_free(ws.hub_list);
    dev_free(ws.owner);
    dev_free(ws.chunk_off);
    dev_free(ws.hub_cnt);
    dev_free(ws.partial);
    dev_free(ws.in_hub_list);
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
    dev_free(ws.qvb);
    ws.queue = nullptr;
    ws.qmask = nullptr;
    ws.qvb = nullptr;
    SP_TRY(dev_alloc((void **)&ws.queue, (size_t)qcap * 4));
    SP_TRY(dev_alloc((void **)&ws.qmask, (size_t)qcap * 8));
    SP_TRY(dev_alloc((void **)&ws.qvb, (size_t)qcap * 4));
    ws.qcap = qcap;
    ws.bytes = batch_ws_bytes(g, qcap, ws.width, ws.engine);
    return SP_OK;
}

// The kernels of `count` forward levels starting at level `first`.  Every
// kernel reads the level it works on from the control block, so the same
// launches serve any chunk whose first level has the same parity.
template <int BS>
static void enqueue_levels(sp_graph g, BatchWorkspace &ws, int64_t first, int count, int grid,
                           int hub_grid, bool may_pull, hipStream_t s) {
    // Outgoing-row hubs (discovery, reverse pass); path-count hubs: the same
    // rows when undirected, the incoming rows' own list when directed.
    const bool hubs = g->n_hubs > 0;
    const bool sigma_hubs = g->directed ? g->n_hubs_in > 0 : hubs;
    const HubEntry *in_list = g->directed ? (const HubEntry *)ws.in_hub_list : nullptr;
    const int hub_fin_grid = grid_for((int64_t)std::max(g->n_hubs, g->n_hubs_in) * kWave, 256,
                                      device_cu_count() * 8);
    for (int k = 0; k < count; ++k) {
        const int64_t l = first + k;  // level this group expands
        uint4 *fcur = ws.front[l & 1], *fnxt = ws.front[(l + 1) & 1];
        if (!hubs && !may_pull && g->max_degree <= kExpandDeg && !g->directed) {  // road-like: one kernel per level
            // A road-like level holds a few thousand entries, and the kernel
            // walks them grid-stride: one block per CU covers any frontier
            // without dispatching the thousands of idle blocks a grid sized
            // for V would start (and retire) every level.
            ProfScope ps(P_MS_EXPAND, s);
            hipLaunchKernelGGL(k_ms_expand<BS>, dim3(std::min(grid, device_cu_count())), dim3(BS), 0, s,
                               ws.ctl, g->row_ptr,
                               g->col_idx, ws.queue, ws.qmask, ws.qvb, ws.seen, (int32_t *)ws.nxt,
                               (const uint4 *)fcur, fnxt, ws.val, (long long)ws.vcap,
                               (long long)ws.qcap, ws.level_off, ws.hub_off, ws.hub_lvl_chunks,
                               (long long)ws.hub_cap, ws.chunk_off, (long long)ws.owner_cap,
                               (int32_t)(l & 1), prof_counters(P_MS_EXPAND));
            continue;
        }
        {
            ProfScope ps(P_MS_TOPDOWN, s);
            hipLaunchKernelGGL(k_ms_topdown<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s, ws.ctl,
                               g->row_ptr, g->col_idx, (const int32_t *)g->rp_in, ws.queue, ws.qmask, ws.seen, ws.nxt,
                               (const HubEntry *)ws.hub_list, (const int32_t *)ws.owner,
                               (const int32_t *)ws.chunk_off, (long long)ws.qcap,
                               prof_counters(P_MS_TOPDOWN));
        }
        if (may_pull) {
            ProfScope ps(P_MS_BOTTOMUP, s);
            hipLaunchKernelGGL(k_ms_bottomup<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->rp_in,
                               g->ci_in, ws.seen, ws.nxt, fcur, ws.queue, (long long)ws.qcap,
                               prof_counters(P_MS_BOTTOMUP));
        }
        {
            ProfScope ps(P_MS_SIGMA, s);
            hipLaunchKernelGGL(k_ms_sigma<BS>, dim3(grid), dim3(BS), 0, s, ws.ctl, g->row_ptr,
                               (const int32_t *)g->rp_in, (const int32_t *)g->ci_in,
                               g->directed ? ws.in_hub_list : nullptr, (long long)ws.in_hub_cap,
                               ws.queue, ws.qmask, ws.qvb, ws.seen, ws.nxt, fcur, fnxt,
                               ws.val, (long long)ws.vcap, ws.hub_list, (long long)ws.hub_cap,
                               (long long)ws.qcap, (int32_t)may_pull, ws.level_off,
                               ws.hub_off, ws.hub_lvl_chunks, ws.owner, (long long)ws.owner_cap,
                               ws.chunk_off, (int32_t)g->max_degree, prof_counters(P_MS_SIGMA));
        }
        if (sigma_hubs) {
            ProfScope ps(P_MS_SIGMA_HUB, s);
            hipLaunchKernelGGL(k_ms_sigma_hub<BS>, dim3(hub_grid), dim3(BS), 0, s, ws.ctl,
                               g->rp_in, g->ci_in, (const unsigned long long *)ws.qmask,
                               (const uint32_t *)ws.qvb, (const uint4 *)fcur, ws.val,
                               (const HubEntry *)ws.hub_list, (const int32_t *)ws.owner,
                               (const int32_t *)ws.chunk_off, in_list, ws.partial,
                               prof_counters(P_MS_SIGMA_HUB));
            // (timed with the chunk kernel)
            hipLaunchKernelGGL(k_ms_sigma_hub_fin, dim3(hub_fin_grid), dim3(256), 0, s, ws.ctl,
                               (const unsigned long long *)ws.qmask, (const uint32_t *)ws.qvb,
                               ws.val, (const HubEntry *)ws.hub_list, (const double *)ws.partial,
                               in_list);
        }
        {
            ProfScope ps(P_MS_SIGMA_PUSH, s);
            hipLaunchKernelGGL(k_ms_sigma_push<BS>, dim3(grid, hubs ? 2 : 1), dim3(BS), 0, s,
                               ws.ctl, (const int32_t *)ws.level_off, g->row_ptr, g->col_idx,
                               (const int32_t *)ws.queue, (const unsigned long long *)ws.qmask,
                               (const uint32_t *)ws.qvb, (const uint4 *)fnxt, ws.val,
                               (const HubEntry *)ws.hub_list, (const int32_t *)ws.owner,
                               (const int32_t *)ws.chunk_off, (const int32_t *)ws.hub_lvl_chunks,
                               prof_counters(P_MS_SIGMA_PUSH));
            // (timed with the push kernel)
            hipLaunchKernelGGL(k_ms_sigma_push_fin, dim3(grid), dim3(256), 0, s, ws.ctl,
                               (const double *)ws.val);
        }
    }
}

// Replay `slot`'s captured graph on stream s, capturing it first (on the
// workspace's own stream, with enqueue(stream)) when absent or when its key
// differs from `key`.
template <class Enqueue>
static sp_status replay_chunk(BatchWorkspace &ws, CapturedChunk &slot,
                              const std::array<long long, 12> &key, Enqueue enqueue,
                              hipStream_t s) {
    return replay_captured(&ws.cap_stream, slot, key, enqueue, s);
}

// Forward levels.  With capture on (chunk_levels > 0) and kernel profiling
// off, chunks of levels run as replayed HIP graphs so the host submits one
// graph per chunk instead of four or five launches per level; after four
// chunks without reaching the end (a deep BFS, as on road graphs) the chunks
// grow fourfold.  Chunk lengths are even and every chunk starts at an even
// level, so the captured front-buffer parity holds for all of them.
template <int BS>
static sp_status batch_forward(sp_graph g, BatchWorkspace &ws, int32_t n0, unsigned long long active,
                               const BatchRunOpts &o, hipStream_t s, int32_t *graph_launches) {
    const int32_t n = g->n;
    const int maxb = device_cu_count() * 8;
    const int grid = grid_for((int64_t)n, BS, maxb);
    const bool may_pull = o.alpha > 0 && g->max_degree > 8;  // sparse meshes never pull
    const int hub_grid = xcd_grid(grid_for((partial_rows(g) - 1) * kWave, BS, maxb), maxb);
    hipLaunchKernelGGL(k_ms_clear, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, ws.seen, ws.nxt,
                       ws.front[0], ws.front[1], n);
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(256), 0, s, ws.ctl, (const int32_t *)g->row_ptr,
                       (const int32_t *)ws.queue, (const unsigned long long *)ws.qmask, ws.qvb, n0,
                       ws.seen, ws.front[0], ws.val, ws.level_off, ws.hub_list, ws.hub_off,
                       ws.hub_lvl_chunks, ws.owner, ws.chunk_off, n, (long long)g->nnz, active,
                       may_pull ? o.alpha : 0.0, o.beta);  // alpha 0: never switch to bottom-up
    SP_HIP(hipGetLastError());
    const bool capture = o.chunk_levels > 0 && !prof_enabled();  // events need direct launches
    const int req = std::abs(o.chunk_levels);
    const int short_chunk = o.chunk_levels > 0 ? std::max(2, req + (req & 1)) : std::max(1, req);
    int64_t enqueued = 0;
    for (int rounds = 0;; ++rounds) {
        const bool deep = rounds >= 4;
        const int chunk = deep ? 4 * short_chunk : short_chunk;
        if (capture) {
            // the slot set lives in the control block, so one capture serves every pass
            const std::array<long long, 12> key{BS, grid, hub_grid, chunk, 0, may_pull,
                                                (long long)(intptr_t)ws.queue, ws.qcap,
                                                (long long)(intptr_t)ws.val, ws.vcap, 0, 0};
            SP_TRY(replay_chunk(ws, deep ? ws.fwd_long : ws.fwd_short, key,
                                [&](hipStream_t cs) {
                                    enqueue_levels<BS>(g, ws, 0, chunk, grid, hub_grid, may_pull, cs);
                                },
                                s));
            ++*graph_launches;
        } else {
            enqueue_levels<BS>(g, ws, enqueued, chunk, grid, hub_grid, may_pull, s);
            SP_HIP(hipGetLastError());
        }
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

// `count` reverse levels: each step sweeps the control block's bwd_level
// (non-hub entries, then hub chunks; the last block of the step's last kernel
// moves it one level up); steps past level 1 return at once.
template <int BS>
static void enqueue_reverse(sp_graph g, BatchWorkspace &ws, int count, int grid_d, int grid_h,
                            bool hubs, hipStream_t s) {
    const int hub_fin_grid = grid_for((int64_t)g->n_hubs * kWave, 256, device_cu_count() * 8);
    for (int k = 0; k < count; ++k) {
        // callers start every group at an even step of the sweep
        const int32_t parity = k & 1;
        {
            ProfScope ps(P_MS_DELTA, s);
            hipLaunchKernelGGL(k_ms_delta<BS>, dim3(grid_d), dim3(BS), 0, s, ws.ctl, (int32_t)!hubs,
                               (const int32_t *)ws.level_off, g->row_ptr, g->col_idx, ws.queue,
                               ws.qmask, (const uint32_t *)ws.qvb, ws.front[0], ws.front[1], ws.val,
                               ws.dlt, parity, prof_counters(P_MS_DELTA));
        }
        if (hubs) {
            ProfScope ps(P_MS_DELTA_HUB, s);  // chunk and finishing kernels together
            {
                hipLaunchKernelGGL(k_ms_delta_hub<BS>, dim3(grid_h), dim3(BS), 0, s,
                                   (const LevelCtl *)ws.ctl, (const int32_t *)ws.hub_off,
                                   (const int32_t *)ws.hub_lvl_chunks, g->row_ptr, g->col_idx,
                                   (const unsigned long long *)ws.qmask, (const uint4 *)ws.front[0],
                                   (const uint4 *)ws.front[1], (const double *)ws.val,
                                   (const HubEntry *)ws.hub_list, (const int32_t *)ws.owner,
                                   (const int32_t *)ws.chunk_off, ws.partial,
                                   prof_counters(P_MS_DELTA_HUB));
            }
            hipLaunchKernelGGL(k_ms_delta_hub_fin, dim3(hub_fin_grid), dim3(256), 0, s, ws.ctl,
                               (const int32_t *)ws.hub_off, (const unsigned long long *)ws.qmask,
                               (const uint32_t *)ws.qvb, ws.val, ws.dlt,
                               (const HubEntry *)ws.hub_list, (const double *)ws.partial, parity);
        }
    }
}

static int pow2_at_least(int64_t x, int cap) {
    int p = 1;
    while (p < x && p < cap) p <<= 1;
    return std::min(p, cap);
}

static sp_status launch_extract(sp_graph g, BatchWorkspace &ws, const std::vector<int32_t> &off,
                                int32_t *dist, double *sigma, double *delta, hipStream_t s) {
    for (size_t l = 0; l + 1 < off.size(); ++l) {
        const int64_t cnt = off[l + 1] - off[l];
        if (cnt <= 0) continue;
        hipLaunchKernelGGL(k_ms_extract, dim3(grid_for(cnt * kWave, 256, 4096)), dim3(256), 0, s,
                           ws.queue, ws.qmask, ws.qvb, off[l], off[l + 1], (int32_t)l, g->n, ws.val,
                           ws.dlt, dist, sigma, delta);
    }
    SP_HIP(hipGetLastError());
    return SP_OK;
}

template <int BS>
static sp_status batch_run_bs(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                              double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s,
                              BatchResult *res, const BatchExtract *ex) {
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
    int32_t graph_launches = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        SP_HIP(hipMemcpyAsync(ws.queue, h_q, n0 * 4, hipMemcpyHostToDevice, s));
        SP_HIP(hipMemcpyAsync(ws.qmask, h_m, n0 * 8, hipMemcpyHostToDevice, s));
        SP_HIP(hipMemcpyAsync(ws.slot_src, h_src, kSlots * 4, hipMemcpyHostToDevice, s));
        SP_TRY(batch_forward<BS>(g, ws, n0, active, o, s, &graph_launches));
        if (!ws.ctl_host->overflow_.v) break;
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
    if (ex && (ex->dist || ex->sigma))
        SP_TRY(launch_extract(g, ws, off, ex->dist, ex->sigma, nullptr, s));
    // Reverse pass, device-driven: grids sized for the largest level (rounded
    // up to a power of two so that consecutive batches reuse one capture).
    const int maxb = device_cu_count() * 8;
    int64_t maxcnt = 1;
    int32_t maxh = 0;
    for (int32_t l = 1; l < levels; ++l) {
        maxcnt = std::max<int64_t>(maxcnt, off[l + 1] - off[l]);
        if (l < levels - 1) maxh = std::max(maxh, hch[l]);
    }
    const int grid_d = pow2_at_least(grid_for(maxcnt, BS, maxb), maxb);
    const int grid_h =
        xcd_grid(pow2_at_least(grid_for((int64_t)std::max(maxh, 1) * kWave, BS, maxb), maxb), maxb);
    const bool hubs = maxh > 0;
    hipLaunchKernelGGL(k_ms_bwd_init, dim3(1), dim3(1), 0, s, ws.ctl);
    const int32_t steps = levels - 1;  // levels L-1 .. 1
    const bool capture = o.chunk_levels > 0 && !prof_enabled();
    if (steps > 0 && capture) {
        constexpr int kBwdChunk = 8;
        const std::array<long long, 12> key{BS, grid_d, grid_h, kBwdChunk, hubs,
                                            (long long)(intptr_t)ws.queue, ws.qcap,
                                            (long long)(intptr_t)ws.val, ws.vcap, 0, 0, 0};
        // whole chunks from the graph, the remainder directly (no idle launches)
        const int32_t whole = steps / kBwdChunk * kBwdChunk;
        for (int32_t done = 0; done < whole; done += kBwdChunk) {
            SP_TRY(replay_chunk(ws, ws.bwd, key,
                                [&](hipStream_t cs) {
                                    enqueue_reverse<BS>(g, ws, kBwdChunk, grid_d, grid_h, hubs, cs);
                                },
                                s));
            ++graph_launches;
        }
        if (steps > whole) enqueue_reverse<BS>(g, ws, steps - whole, grid_d, grid_h, hubs, s);
    } else if (steps > 0) {
        enqueue_reverse<BS>(g, ws, steps, grid_d, grid_h, hubs, s);
    }
    SP_HIP(hipGetLastError());
    if (ex && ex->delta) SP_TRY(launch_extract(g, ws, off, nullptr, nullptr, ex->delta, s));
    bool any_out = false;
    SlotTable tbl{};
    for (int32_t i = 0; i < kSlots; ++i) {
        tbl.out[i] = (bc_of_slot && i < nslots) ? bc_of_slot[i] : nullptr;
        any_out |= tbl.out[i] != nullptr;
    }
    if (any_out) {
        ProfScope ps(P_MS_BC, s);
        hipLaunchKernelGGL(k_ms_bc<BS>, dim3(grid_for(n, BS, maxb)), dim3(BS), 0, s, n, ws.seen,
                           ws.dlt, ws.slot_src, nslots, tbl, prof_counters(P_MS_BC));
        SP_HIP(hipGetLastError());
    }
    if (res) {
        res->levels = levels;
        res->reached = (int64_t)c.reached_pairs;
        std::memcpy(&res->sigma_max, &c.sigma_max_bits_.v, sizeof(double));
        res->flagged = __builtin_popcountll(c.flagged_slots_.v);
        res->flagged_mask = c.flagged_slots_.v;
        res->td = c.topdown_levels;
        res->bu = c.bottomup_levels;
        res->entries = off[levels];
        res->graph_launches = graph_launches;
    }
    return SP_OK;
}

sp_status batch_run(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                    double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s,
                    BatchResult *res, const BatchExtract *ex) {
    if (nslots < 1 || nslots > ws.width) {
        set_error("batch of %d sources (1..%d allowed)", nslots, ws.width);
        return SP_ERR_INVALID_ARGUMENT;
    }
    if (o.engine != ws.engine) {
        set_error("internal: workspace built for engine %d, pass asks for %d", ws.engine, o.engine);
        return SP_ERR_DEVICE;
    }
    if (ws.engine == SP_ENGINE_BLOCKS) return wg_run(g, ws, srcs, nslots, bc_of_slot, o, s, res, ex);
    if (ex) {
        const int64_t total = (int64_t)nslots * g->n;
        if (ex->dist) SP_TRY(launch_fill_i32(ex->dist, total, -1, s));
        if (ex->sigma) SP_TRY(launch_fill_f64(ex->sigma, total, 0.0, s));
        if (ex->delta) SP_TRY(launch_fill_f64(ex->delta, total, 0.0, s));
    }
    switch (o.block) {
        case 128: return batch_run_bs<128>(g, ws, srcs, nslots, bc_of_slot, o, s, res, ex);
        case 512: return batch_run_bs<512>(g, ws, srcs, nslots, bc_of_slot, o, s, res, ex);
        default: return batch_run_bs<256>(g, ws, srcs, nslots, bc_of_slot, o, s, res, ex);
    }
}

}  // namespace sp
