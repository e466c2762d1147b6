// Batched BC with one workgroup per source ("workgroup engine"), for graphs
// of many short levels (road-like: no vertex of degree above kExpandDeg).
//
// The arithmetic is Brandes' per source (paper Appendix, Fig. "BC computation
// in StarPlat"; DAG semantics of Section 2.3.2), as on the per-source path:
//   sigma(w) = sum over parents u (incoming row, CSR order) of sigma(u),
//   delta(v) = sum over children w (outgoing row, CSR order) of
//              (sigma(v) / sigma(w)) * (1 + delta(w))
// (rows through the CSR offsets), or, regrouped as in the bitmap engine,
//   delta(v) = sigma(v) * sum over children w of rho(w),
//   rho(w) = (1 + delta(w)) / sigma(w)
// (fixed-width rows, below).
// What differs is the schedule.  On a road-like graph a source's BFS has
// thousands of levels of a few hundred vertices each; the bitmap engine runs
// the batch's sources in lockstep, one kernel per level for the whole batch,
// and each level pays the kernel's chain of dependent memory round trips and
// its grid-wide close.  Here each source's whole pass (forward levels, then
// reverse levels) runs inside one workgroup, the level barrier is the
// workgroup barrier, and the new frontier is appended with an LDS counter:
// the batch's sources advance independently, each on its own CU.
// (One thread block per source is the coarse-grained schedule of McLaughlin
// and Bader, "Scalable and high performance betweenness centrality on the
// GPU", SC 2014.)
//
// Layout, per slot s (source-major): a 16-byte record rec[s*V + v] = {level
// (-1: unreached), value}, delta[s*V + v], the BFS-order queue
// queue[s*V + i] and the level offsets loff[s*(V+2) + l] -- 32 bytes per
// vertex and slot.  Records are filled with level -1 before each pass; every
// other field is written before it is read.  The value is sigma after the
// forward pass; the fixed-width kernel replaces it by rho once the reverse
// pass has finished the vertex, so a neighbour costs one 16-byte load (level
// and value together).  sigma itself is written out only for sp_batch_levels
// (straight into the caller's array).
// BC: for each vertex, the slots' delta in ascending slot order, skipping
// unreached vertices and the vertex's own source (level <= 0).
//
// Only the slot's own workgroup touches its arrays during the pass, so the
// claim on a level is a workgroup-scope compare-and-swap, performed in the
// XCD's L2.  The CSR-offset kernel reads levels another wave may have
// claimed with workgroup-scope atomic loads; the fixed-width kernel reads
// records with plain loads and invalidates the CU's L1 after each level
// barrier instead.  Everything else is written with plain stores by waves of
// the same workgroup and read after a barrier.
//
// Memory-level parallelism: a thread takes kEntries queue entries at once
// and walks their rows kRowStep entries at a time; for all of them the
// column ids, then the neighbours' levels, then their values (or claims) are
// each issued together, so one step of a level costs a few dependent round
// trips for kEntries x kRowStep adjacency entries.  Sums still run in CSR
// order per vertex.
//
// Fixed-width rows: on a graph whose rows hold at most 8 entries the rows
// are copied once into a fixed-width layout (W = 4 or 8 ids per vertex, -1
// padding), so a vertex's neighbours come in one load instead of an offset
// load followed by an id load.  A discovery step is then queue entry -> row
// -> claim, a path-count step queue entry -> row -> the neighbours' records,
// and a reverse step queue entry -> row (and the vertex's own record) -> the
// neighbours' records; the record of a neighbour that turns out not to be a
// parent (child) is loaded and dropped.  Measured on a 2048 x 2048 grid
// (64 sources, one per workgroup): a level costs about 46 us and scales with
// the frontier, not with the chain of round trips -- the 64 workgroups'
// record and row lines (128 bytes fetched per 16 used) keep the memory
// system busy; spreading a source over 2 or 4 workgroups of one XCD, with a
// barrier between the groups' phases, was slower (201 and 339 ms against
// 181 ms for the whole pass).
#include "common.h"
#include "devutil.h"

namespace sp {

constexpr int kRowStep = 4;   // row entries per step (road-like rows hold at most 4)
constexpr int kEntries = 4;   // queue entries a thread works on at once

// Rows of the (up to) kEntries queue entries i0, i0 + BS, ... below `end`:
// [b[u], e[u]) in the rows `rows`; returns the longest row's length.
template <int BS>
__device__ __forceinline__ int32_t rows_of_bs(const int32_t *queue, int32_t i0, int32_t end,
                                              const int32_t *__restrict__ rows, int32_t *b, int32_t *e) {
    int32_t v[kEntries];
#pragma unroll
    for (int u = 0; u < kEntries; ++u) v[u] = i0 + u * BS < end ? queue[i0 + u * BS] : -1;
    int32_t len = 0;
#pragma unroll
    for (int u = 0; u < kEntries; ++u) {
        b[u] = v[u] >= 0 ? rows[v[u]] : 0;
        e[u] = v[u] >= 0 ? rows[v[u] + 1] : 0;
        len = max(len, e[u] - b[u]);
    }
    return len;
}

__device__ __forceinline__ int32_t ld_level(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// dist -1 -> lvl; returns the value found (-1 when this call claimed it).
__device__ __forceinline__ int32_t claim_level(int32_t *p, int32_t lvl) {
    int32_t expected = -1;
    __hip_atomic_compare_exchange_strong(p, &expected, lvl, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return expected;
}

__global__ void k_wg_fill(WgRec *rec, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        reinterpret_cast<int4 *>(rec + i)[0] = make_int4(-1, 0, 0, 0);  // level and value
}

// Fixed-width copy of the rows: ell[v * W + k] = k-th neighbour, -1 past the
// row's end (every row holds at most W entries).
template <int W>
__global__ void k_wg_ell(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t n,
                         int32_t *ell) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t b = rp[v], d = rp[v + 1] - b;
#pragma unroll
        for (int k = 0; k < W; ++k) ell[v * W + k] = k < d ? ci[b + k] : -1;
    }
}

// The loads below are issued unconditionally, from a valid address (row 0,
// vertex 0) when there is nothing to read, and their results dropped: a load
// under a branch of its own is waited for before the branch closes, which
// would turn a group of independent loads into a chain of round trips.

// queue[i] for i < end, else -1 (i < end for some lane of the call, end > 0).
__device__ __forceinline__ int32_t at_or_none(const int32_t *queue, int32_t i, int32_t end) {
    const int32_t x = queue[min(i, end - 1)];
    return i < end ? x : -1;
}

// Level barrier of the fixed-width kernel, whose records are read with plain
// loads: after the workgroup barrier the CU's L1 is invalidated, so the next
// phase sees in L2 the levels other waves claimed there with
// compare-and-swap and the values they stored.
__device__ __forceinline__ void sync_records() {
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// A record in one 16-byte load (the empty asm marks the pad word used, so
// the load is not narrowed into a 4-byte and an 8-byte one: two requests).
__device__ __forceinline__ WgRec load_rec(const WgRec *p) {
    int4 x = *reinterpret_cast<const int4 *>(p);
    asm("" : "+v"(x.y));
    WgRec r;
    r.dist = x.x;
    r.pad = x.y;
    r.val = __hiloint2double(x.w, x.z);
    return r;
}

// Append x to the queue where `take` holds: one LDS add per wave reserves
// the wave's entries, lanes in lane order.
__device__ __forceinline__ void append_wave(bool take, int32_t x, int32_t *queue, int32_t *s_tail) {
    const unsigned long long bal = __ballot(take);
    if (!bal) return;
    const int first = __ffsll((long long)bal) - 1;
    int32_t at = 0;
    if (lane_id() == first) at = atomicAdd(s_tail, __popcll(bal));  // LDS
    at = __shfl(at, first, kWave);
    const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (take) queue[at + r] = x;
}

// Row of v in the fixed-width layout (v < 0: an empty row).
template <int W>
__device__ __forceinline__ void ell_row(const int32_t *__restrict__ ell, int32_t v, int32_t (&nb)[W]) {
    const int4 *r = reinterpret_cast<const int4 *>(ell + (int64_t)max(v, 0) * W);
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
        const int4 x = r[q];
        nb[4 * q + 0] = v >= 0 ? x.x : -1;
        nb[4 * q + 1] = v >= 0 ? x.y : -1;
        nb[4 * q + 2] = v >= 0 ? x.z : -1;
        nb[4 * q + 3] = v >= 0 ? x.w : -1;
    }
}

// k_wg_bc over fixed-width rows (see the latency note above): the same sums
// in the same order.
template <int BS, int W>
__global__ __launch_bounds__(BS) void k_wg_bc_ell(const int32_t *__restrict__ ell,
                                                  const int32_t *__restrict__ ell_in,
                                                  const int32_t *__restrict__ slot_src, int32_t n,
                                                  WgRec *rec_all, double *delta_all, double *sigma_out,
                                                  int32_t *queue_all, int32_t *loff_all, WgSlotResult *res,
                                                  unsigned long long *prof) {
    constexpr int E = W == 8 ? 2 : kEntries;  // entries in flight per thread (registers)
    const int32_t slot = blockIdx.x;
    const int64_t base = (int64_t)slot * n;
    WgRec *rec = rec_all + base;
    double *delta = delta_all + base;
    double *sig_out = sigma_out ? sigma_out + base : nullptr;  // sp_batch_levels' sigma
    int32_t *queue = queue_all + base;
    int32_t *loff = loff_all + (int64_t)slot * ((int64_t)n + 2);
    const int32_t src = slot_src[slot];
    __shared__ int32_t s_tail, s_flag;
    __shared__ double s_max[BS / kWave];
    __shared__ unsigned long long s_red[1];
    if (threadIdx.x == 0) {
        rec[src].dist = 0;
        rec[src].val = 1.0;
        if (sig_out) sig_out[src] = 1.0;
        queue[0] = src;
        loff[0] = 0;
        loff[1] = 1;
        s_tail = 1;
        s_flag = 0;
    }
    sync_records();
    int32_t lo = 0, hi = 1, level = 0;
    double my_max = 1.0;
    unsigned long long my_edges = 0, my_pairs = 0;
    for (;;) {
        // Discovery of level + 1 from the frontier [lo, hi): the claim
        // (dist -1 -> level + 1) decides who appends the vertex; a wave
        // reserves its appends with one LDS add.
        for (int32_t i0 = lo + (int32_t)threadIdx.x; i0 < hi; i0 += BS * E) {
            int32_t v[E], nb[E][W], old[E][W];
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = at_or_none(queue, i0 + u * BS, hi);
#pragma unroll
            for (int u = 0; u < E; ++u) ell_row<W>(ell, v[u], nb[u]);
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int k = 0; k < W; ++k) old[u][k] = nb[u][k] >= 0 ? claim_level(&rec[nb[u][k]].dist, level + 1) : 0;
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if (nb[u][k] >= 0) ++my_edges;
                    append_wave(nb[u][k] >= 0 && old[u][k] == -1, nb[u][k], queue, &s_tail);
                }
        }
        sync_records();
        const int32_t tail = s_tail;
        if (tail == hi) break;  // block-uniform: every thread read the same tail
        // Path counts of the new vertices [hi, tail): parents over incoming
        // rows, added in row order; one record load per neighbour.
        for (int32_t j0 = hi + (int32_t)threadIdx.x; j0 < tail; j0 += BS * E) {
            int32_t w[E], p[E][W];
            WgRec r[E][W];
#pragma unroll
            for (int u = 0; u < E; ++u) w[u] = at_or_none(queue, j0 + u * BS, tail);
#pragma unroll
            for (int u = 0; u < E; ++u) ell_row<W>(ell_in, w[u], p[u]);
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int k = 0; k < W; ++k) r[u][k] = load_rec(&rec[max(p[u][k], 0)]);
#pragma unroll
            for (int u = 0; u < E; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < W; ++k)
                    if (p[u][k] >= 0 && r[u][k].dist == level) {
                        acc += r[u][k].val;
                        ++my_pairs;
                    }
                if (w[u] >= 0) {
                    rec[w[u]].val = acc;
                    if (sig_out) sig_out[w[u]] = acc;
                    my_max = fmax(my_max, acc);
                    if (sigma_is_large(acc)) s_flag = 1;
                }
            }
        }
        if (threadIdx.x == 0) loff[level + 2] = tail;
        sync_records();
        lo = hi;
        hi = tail;
        ++level;
    }
    // Reverse sweep from the deepest level up to level 1 (the deepest has no
    // children: its delta is 0); children over outgoing rows, in row order.
    // A finished vertex's record holds rho = (1 + delta) / sigma, so a parent
    // reads one record per neighbour: delta(v) = sigma(v) * sum of its
    // children's rho (the regrouping of the bitmap engine).
    for (int32_t l = level; l >= 1; --l) {
        const int32_t a = loff[l], z = loff[l + 1];
        for (int32_t j0 = a + (int32_t)threadIdx.x; j0 < z; j0 += BS * E) {
            int32_t v[E], nb[E][W];
            double sv[E];
            WgRec r[E][W];
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = at_or_none(queue, j0 + u * BS, z);
#pragma unroll
            for (int u = 0; u < E; ++u) {
                ell_row<W>(ell, v[u], nb[u]);
                sv[u] = rec[max(v[u], 0)].val;  // sigma(v)
            }
#pragma unroll
            for (int u = 0; u < E; ++u)
#pragma unroll
                for (int k = 0; k < W; ++k) r[u][k] = load_rec(&rec[max(nb[u][k], 0)]);
#pragma unroll
            for (int u = 0; u < E; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < W; ++k)
                    if (nb[u][k] >= 0 && r[u][k].dist == l + 1) {
                        acc += r[u][k].val;
                        ++my_pairs;
                    }
                if (v[u] >= 0) {
                    const double dv = sv[u] * acc;
                    delta[v[u]] = dv;
                    rec[v[u]].val = (1.0 + dv) / sv[u];
                }
            }
        }
        sync_records();
    }
    my_max = wave_max_f64(my_max);
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = my_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < BS / kWave; ++w) m = fmax(m, s_max[w]);
        res[slot] = WgSlotResult{level + 1, hi, m, s_flag};
    }
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(threadIdx.x == 0 ? (unsigned long long)hi : 0ull, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
    }
}

// One source per workgroup: blockIdx.x = slot.
template <int BS>
__global__ __launch_bounds__(BS) void k_wg_bc(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                              const int32_t *__restrict__ rpi,
                                              const int32_t *__restrict__ cii,
                                              const int32_t *__restrict__ slot_src, int32_t n,
                                              WgRec *rec_all, double *delta_all, double *sigma_out,
                                              int32_t *queue_all, int32_t *loff_all, WgSlotResult *res,
                                              unsigned long long *prof) {
    const int32_t slot = blockIdx.x;
    const int64_t base = (int64_t)slot * n;
    WgRec *rec = rec_all + base;
    double *delta = delta_all + base;
    double *sig_out = sigma_out ? sigma_out + base : nullptr;  // sp_batch_levels' sigma
    int32_t *queue = queue_all + base;
    int32_t *loff = loff_all + (int64_t)slot * ((int64_t)n + 2);
    const int32_t src = slot_src[slot];
    __shared__ int32_t s_tail, s_flag;
    __shared__ double s_max[BS / kWave];
    __shared__ unsigned long long s_red[1];
    if (threadIdx.x == 0) {
        rec[src].dist = 0;
        rec[src].val = 1.0;
        if (sig_out) sig_out[src] = 1.0;
        queue[0] = src;
        loff[0] = 0;
        loff[1] = 1;
        s_tail = 1;
        s_flag = 0;
    }
    __syncthreads();
    int32_t lo = 0, hi = 1, level = 0;
    double my_max = 1.0;
    unsigned long long my_edges = 0, my_pairs = 0;
    for (;;) {
        // Discovery of level + 1 from the frontier [lo, hi), outgoing rows;
        // the claim (dist -1 -> level + 1) decides who appends the vertex.
        for (int32_t i0 = lo + (int32_t)threadIdx.x; i0 < hi; i0 += BS * kEntries) {
            int32_t b[kEntries], e[kEntries];
            int32_t len = rows_of_bs<BS>(queue, i0, hi, rp, b, e);
            for (int32_t k0 = 0; k0 < len; k0 += kRowStep) {
                int32_t w[kEntries][kRowStep], d[kEntries][kRowStep], old[kEntries][kRowStep];
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) w[u][t] = b[u] + k0 + t < e[u] ? ci[b[u] + k0 + t] : -1;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) d[u][t] = w[u][t] >= 0 ? ld_level(&rec[w[u][t]].dist) : 0;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t)
                        old[u][t] = d[u][t] < 0 ? claim_level(&rec[w[u][t]].dist, level + 1) : 0;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t)
                        if (d[u][t] < 0 && old[u][t] == -1) queue[atomicAdd(&s_tail, 1)] = w[u][t];  // LDS
            }
#pragma unroll
            for (int u = 0; u < kEntries; ++u) my_edges += (unsigned long long)(e[u] - b[u]);
        }
        __syncthreads();
        const int32_t tail = s_tail;
        if (tail == hi) break;  // block-uniform: every thread read the same tail
        // Path counts of the new vertices [hi, tail): parents over incoming
        // rows, added in row order.
        for (int32_t j0 = hi + (int32_t)threadIdx.x; j0 < tail; j0 += BS * kEntries) {
            int32_t b[kEntries], e[kEntries];
            const int32_t len = rows_of_bs<BS>(queue, j0, tail, rpi, b, e);
            double acc[kEntries] = {};
            for (int32_t k0 = 0; k0 < len; k0 += kRowStep) {
                int32_t p[kEntries][kRowStep];
                bool par[kEntries][kRowStep];
                double x[kEntries][kRowStep];
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) p[u][t] = b[u] + k0 + t < e[u] ? cii[b[u] + k0 + t] : -1;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) par[u][t] = p[u][t] >= 0 && ld_level(&rec[p[u][t]].dist) == level;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) x[u][t] = par[u][t] ? rec[p[u][t]].val : 0.0;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t)
                        if (par[u][t]) {
                            acc[u] += x[u][t];
                            ++my_pairs;
                        }
            }
#pragma unroll
            for (int u = 0; u < kEntries; ++u) {
                const int32_t j = j0 + u * BS;
                if (j < tail) {
                    rec[queue[j]].val = acc[u];
                    if (sig_out) sig_out[queue[j]] = acc[u];
                    my_max = fmax(my_max, acc[u]);
                    if (sigma_is_large(acc[u])) s_flag = 1;
                }
            }
        }
        if (threadIdx.x == 0) loff[level + 2] = tail;
        __syncthreads();
        lo = hi;
        hi = tail;
        ++level;
    }
    // `level` is the deepest level; reverse sweep from it up to level 1
    // (the deepest has no children: its delta is 0).  Children over outgoing
    // rows, added in row order.
    for (int32_t l = level; l >= 1; --l) {
        const int32_t a = loff[l], z = loff[l + 1];
        for (int32_t j0 = a + (int32_t)threadIdx.x; j0 < z; j0 += BS * kEntries) {
            int32_t b[kEntries], e[kEntries], v[kEntries];
            double sv[kEntries], acc[kEntries] = {};
#pragma unroll
            for (int u = 0; u < kEntries; ++u) v[u] = j0 + u * BS < z ? queue[j0 + u * BS] : -1;
            int32_t len = 0;
#pragma unroll
            for (int u = 0; u < kEntries; ++u) {
                b[u] = v[u] >= 0 ? rp[v[u]] : 0;
                e[u] = v[u] >= 0 ? rp[v[u] + 1] : 0;
                sv[u] = v[u] >= 0 ? rec[v[u]].val : 0.0;
                len = max(len, e[u] - b[u]);
            }
            for (int32_t k0 = 0; k0 < len; k0 += kRowStep) {
                int32_t w[kEntries][kRowStep];
                bool ch[kEntries][kRowStep];
                double sw[kEntries][kRowStep], dw[kEntries][kRowStep];
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) w[u][t] = b[u] + k0 + t < e[u] ? ci[b[u] + k0 + t] : -1;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) ch[u][t] = w[u][t] >= 0 && ld_level(&rec[w[u][t]].dist) == l + 1;
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t) {
                        sw[u][t] = ch[u][t] ? rec[w[u][t]].val : 1.0;
                        dw[u][t] = ch[u][t] ? delta[w[u][t]] : 0.0;
                    }
#pragma unroll
                for (int u = 0; u < kEntries; ++u)
#pragma unroll
                    for (int t = 0; t < kRowStep; ++t)
                        if (ch[u][t]) {
                            acc[u] += (sv[u] / sw[u][t]) * (1.0 + dw[u][t]);
                            ++my_pairs;
                        }
            }
#pragma unroll
            for (int u = 0; u < kEntries; ++u)
                if (v[u] >= 0) delta[v[u]] = acc[u];
        }
        __syncthreads();
    }
    my_max = wave_max_f64(my_max);
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = my_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < BS / kWave; ++w) m = fmax(m, s_max[w]);
        res[slot] = WgSlotResult{level + 1, hi, m, s_flag};
    }
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(threadIdx.x == 0 ? (unsigned long long)hi : 0ull, s_red, prof + 0);
        __syncthreads();
        block_add_u64<BS>(my_edges, s_red, prof + 1);
        __syncthreads();
        block_add_u64<BS>(my_pairs, s_red, prof + 2);
    }
}

// BC[v] += delta of v for every slot that reached v from another vertex, in
// ascending slot order; consecutive slots with the same output array are
// summed in a register.
template <int BS>
__global__ __launch_bounds__(BS) void k_wg_bc_sum(int32_t n, int32_t nslots, const WgRec *__restrict__ rec,
                                                  const double *__restrict__ delta, SlotTable tbl,
                                                  unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    unsigned long long my_items = 0;
    for (int32_t v = blockIdx.x * BS + threadIdx.x; v < n; v += gridDim.x * BS) {
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
            const int64_t o = (int64_t)s * n + v;
            if (rec[o].dist > 0) {
                acc += delta[o];
                ++my_items;
            }
        }
        if (cur) cur[v] = acc;
    }
    if (prof) block_add_u64<BS>(my_items, s_red, prof + 3);
}

// Per-slot results into the caller's source-major arrays (sp_batch_levels):
// dist as is, sigma of reached vertices, delta of vertices below the source.
__global__ void k_wg_extract(int64_t count, const WgRec *__restrict__ rec, const double *__restrict__ delta,
                             int32_t *out_dist, double *out_sigma,
                             double *out_delta) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const int32_t d = rec[i].dist;
        if (out_dist) out_dist[i] = d;
        if (out_sigma && d < 0) out_sigma[i] = 0.0;  // reached: written by the pass
        if (out_delta) out_delta[i] = d > 0 ? delta[i] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Width of the fixed-width rows for g: 4 or 8 when every row fits, else 0.
static int32_t ell_width(sp_graph g) {
    return g->max_degree <= 4 ? 4 : g->max_degree <= 8 ? 8 : 0;
}

size_t wg_ws_bytes(sp_graph g, int32_t width) {
    const size_t V = (size_t)std::max(g->n, 1);
    const size_t ell = V * (size_t)ell_width(g) * 4 * (g->directed ? 2 : 1);
    return (size_t)width * (V * (sizeof(WgRec) + 8 + 4) + (V + 2) * 4) + (size_t)width * sizeof(WgSlotResult) + ell;
}

sp_status wg_ws_alloc(sp_graph g, int32_t width, BatchWorkspace &ws) {
    const size_t V = (size_t)std::max(g->n, 1), W = (size_t)width;
    SP_TRY(dev_alloc((void **)&ws.wg_rec, W * V * sizeof(WgRec)));
    SP_TRY(dev_alloc((void **)&ws.wg_delta, W * V * 8));
    SP_TRY(dev_alloc((void **)&ws.wg_queue, W * V * 4));
    SP_TRY(dev_alloc((void **)&ws.wg_loff, W * (V + 2) * 4));
    SP_TRY(dev_alloc((void **)&ws.wg_res, W * sizeof(WgSlotResult)));
    SP_HIP(hipHostMalloc((void **)&ws.wg_res_host, W * sizeof(WgSlotResult), hipHostMallocDefault));
    ws.wg_ell_w = ell_width(g);
    ws.wg_ell_built = false;
    if (ws.wg_ell_w) {
        const size_t cells = V * (size_t)ws.wg_ell_w;
        SP_TRY(dev_alloc((void **)&ws.wg_ell, cells * 4));
        if (g->directed) SP_TRY(dev_alloc((void **)&ws.wg_ell_in, cells * 4));
    }
    return SP_OK;
}

void wg_ws_free(BatchWorkspace &ws) {
    dev_free(ws.wg_rec);
    dev_free(ws.wg_delta);
    dev_free(ws.wg_queue);
    dev_free(ws.wg_loff);
    dev_free(ws.wg_res);
    dev_free(ws.wg_ell);
    dev_free(ws.wg_ell_in);
    ws.wg_ell = ws.wg_ell_in = nullptr;
    ws.wg_ell_w = 0;
    ws.wg_ell_built = false;
    if (ws.wg_res_host) (void)hipHostFree(ws.wg_res_host);
    ws.wg_rec = nullptr;
    ws.wg_delta = nullptr;
    ws.wg_queue = ws.wg_loff = nullptr;
    ws.wg_res = ws.wg_res_host = nullptr;
}

template <int BS>
static sp_status wg_run_bs(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                           double *const *bc_of_slot, hipStream_t s, BatchResult *res,
                           const BatchExtract *ex) {
    const int32_t n = g->n;
    const int64_t count = (int64_t)nslots * n;
    int32_t *h_src = (int32_t *)ws.staging;
    for (int32_t i = 0; i < kSlots; ++i) h_src[i] = i < nslots ? srcs[i] : -1;
    SP_HIP(hipMemcpyAsync(ws.slot_src, h_src, kSlots * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_wg_fill, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, ws.wg_rec, count);
    const int ew = ws.wg_ell_w;
    if (ew && !ws.wg_ell_built) {
        auto build = ew == 4 ? k_wg_ell<4> : k_wg_ell<8>;
        hipLaunchKernelGGL(build, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (const int32_t *)g->row_ptr,
                           (const int32_t *)g->col_idx, n, ws.wg_ell);
        if (g->directed)
            hipLaunchKernelGGL(build, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (const int32_t *)g->rp_in,
                               (const int32_t *)g->ci_in, n, ws.wg_ell_in);
        SP_HIP(hipGetLastError());
        ws.wg_ell_built = true;
    }
    {
        ProfScope ps(P_WG_BC, s);
        const int32_t *ell_in = g->directed ? ws.wg_ell_in : ws.wg_ell;
        if (ew == 4)
            hipLaunchKernelGGL((k_wg_bc_ell<BS, 4>), dim3(nslots), dim3(BS), 0, s, (const int32_t *)ws.wg_ell,
                               ell_in, (const int32_t *)ws.slot_src, n, ws.wg_rec, ws.wg_delta, ex ? ex->sigma : nullptr,
                               ws.wg_queue, ws.wg_loff, ws.wg_res, prof_counters(P_WG_BC));
        else if (ew == 8)
            hipLaunchKernelGGL((k_wg_bc_ell<BS, 8>), dim3(nslots), dim3(BS), 0, s, (const int32_t *)ws.wg_ell,
                               ell_in, (const int32_t *)ws.slot_src, n, ws.wg_rec, ws.wg_delta, ex ? ex->sigma : nullptr,
                               ws.wg_queue, ws.wg_loff, ws.wg_res, prof_counters(P_WG_BC));
        else
            hipLaunchKernelGGL(k_wg_bc<BS>, dim3(nslots), dim3(BS), 0, s, (const int32_t *)g->row_ptr,
                               (const int32_t *)g->col_idx, (const int32_t *)g->rp_in, (const int32_t *)g->ci_in,
                               (const int32_t *)ws.slot_src, n, ws.wg_rec, ws.wg_delta, ex ? ex->sigma : nullptr,
                               ws.wg_queue, ws.wg_loff, ws.wg_res, prof_counters(P_WG_BC));
    }
    SP_HIP(hipGetLastError());
    if (ex)
        hipLaunchKernelGGL(k_wg_extract, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, count,
                           (const WgRec *)ws.wg_rec, (const double *)ws.wg_delta, ex->dist, ex->sigma,
                           ex->delta);
    SlotTable tbl{};
    bool any_out = false;
    for (int32_t i = 0; i < kSlots; ++i) {
        tbl.out[i] = (bc_of_slot && i < nslots) ? bc_of_slot[i] : nullptr;
        any_out |= tbl.out[i] != nullptr;
    }
    if (any_out) {
        ProfScope ps(P_MS_BC, s);
        hipLaunchKernelGGL(k_wg_bc_sum<BS>, dim3(grid_for(n, BS, device_cu_count() * 8)), dim3(BS), 0, s, n,
                           nslots, (const WgRec *)ws.wg_rec, (const double *)ws.wg_delta, tbl,
                           prof_counters(P_MS_BC));
    }
    SP_HIP(hipGetLastError());
    SP_HIP(hipMemcpyAsync(ws.wg_res_host, ws.wg_res, (size_t)nslots * sizeof(WgSlotResult),
                          hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
    if (res) {
        *res = BatchResult{};
        for (int32_t i = 0; i < nslots; ++i) {
            const WgSlotResult &r = ws.wg_res_host[i];
            res->levels = std::max(res->levels, r.levels);
            res->reached += r.reached;
            res->entries += r.reached;
            res->sigma_max = std::max(res->sigma_max, r.sigma_max);
            if (r.flagged) {
                res->flagged++;
                res->flagged_mask |= 1ull << i;
            }
            res->td += r.levels - 1;  // every level expanded top-down
        }
    }
    return SP_OK;
}

sp_status wg_run(sp_graph g, BatchWorkspace &ws, const int32_t *srcs, int32_t nslots,
                 double *const *bc_of_slot, const BatchRunOpts &o, hipStream_t s, BatchResult *res,
                 const BatchExtract *ex) {
    switch (o.block) {
        case 128: return wg_run_bs<128>(g, ws, srcs, nslots, bc_of_slot, s, res, ex);
        case 256: return wg_run_bs<256>(g, ws, srcs, nslots, bc_of_slot, s, res, ex);
        case 512: return wg_run_bs<512>(g, ws, srcs, nslots, bc_of_slot, s, res, ex);
        default: return wg_run_bs<1024>(g, ws, srcs, nslots, bc_of_slot, s, res, ex);
    }
}

}  // namespace sp
