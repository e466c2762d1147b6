// Device-side helpers for wave64 (CDNA) kernels: lane queries, wave-level
// reductions in a fixed order, block scans, and an LDS-staged append buffer
// that turns per-vertex queue appends into one global atomic per flush.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ int32_t shfl_i32(int32_t v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long v, int src) {
    return __shfl(v, src, kWave);
}

__device__ __forceinline__ double shfl_f64(double v, int src) { return __shfl(v, src, kWave); }

// Number of set lanes of `m` below the calling lane.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    const int l = lane_id();
    return __popcll(m & ((l == 0) ? 0ull : (~0ull >> (64 - l))));
}

// Sum over the 64 lanes by a fixed xor butterfly: the same inputs give the
// same bits on every run.
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

// Inclusive prefix sum over the lanes of one wave.
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t y = __shfl_up(x, o, kWave);
        if (l >= o) x += y;
    }
    return x;
}

// Exclusive prefix sum over a block of BS threads; *total receives the sum.
// Uses BS / 64 + 1 ints of LDS at `scratch`.  All threads must call.
template <int BS>
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t *scratch, int32_t *total) {
    constexpr int NW = BS / kWave;
    const int w = threadIdx.x / kWave, l = lane_id();
    int32_t incl = wave_incl_scan(x);
    if (l == kWave - 1) scratch[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < NW; ++i) {
            int32_t t = scratch[i];
            scratch[i] = run;
            run += t;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    int32_t ex = scratch[w] + incl - x;
    *total = scratch[NW];
    __syncthreads();
    return ex;
}

// Non-negative doubles compare like their bit patterns (NaN above +inf), so a
// running maximum of sigma can use the integer atomic.
__device__ __forceinline__ void atomic_max_nonneg_f64(unsigned long long *bits, double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > *(volatile unsigned long long *)bits) atomicMax(bits, b);
}

__device__ __forceinline__ bool sigma_is_large(double s) { return !(s <= 1e300); }

// LDS-staged append buffer.  Threads stage values in LDS; the block moves
// them to the global queue with one atomic per flush.  Every thread of the
// block must call stage() and finish() the same number of times.
template <int BS, int CAP>
struct StagedQueue {
    static_assert(CAP >= 2 * BS, "capacity must hold two rounds");
    int32_t *buf;   // LDS, CAP entries
    int32_t *meta;  // LDS, 2 entries: [0] count, [1] global base

    __device__ void init(int32_t *lds_buf, int32_t *lds_meta) {
        buf = lds_buf;
        meta = lds_meta;
        if (threadIdx.x == 0) meta[0] = 0;
        __syncthreads();
    }

    __device__ void flush(int32_t *g_tail, int32_t *g_queue, int64_t qcap, int32_t *overflow) {
        // caller has synchronised; meta[0] is stable
        const int32_t cnt = meta[0];
        if (cnt == 0) return;
        if (threadIdx.x == 0) meta[1] = atomicAdd(g_tail, cnt);
        __syncthreads();
        const int32_t base = meta[1];
        for (int32_t i = threadIdx.x; i < cnt; i += BS) {
            int64_t p = (int64_t)base + i;
            if (p < qcap) g_queue[p] = buf[i];
        }
        if (threadIdx.x == 0) {
            if ((int64_t)base + cnt > qcap) *overflow = 1;
            meta[0] = 0;
        }
        __syncthreads();
    }

    // Stage `val` when `take`; flush if the next round might not fit.
    __device__ void stage(bool take, int32_t val, int32_t *g_tail, int32_t *g_queue, int64_t qcap,
                          int32_t *overflow) {
        unsigned long long m = __ballot(take);
        int32_t base = 0;
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            if (lane_id() == leader) base = atomicAdd(&meta[0], __popcll(m));
            base = shfl_i32(base, leader);
            if (take) buf[base + lanes_below(m)] = val;
        }
        __syncthreads();
        const int32_t staged = meta[0];
        __syncthreads();  // every thread has read the count before anyone stages again
        if (staged > CAP - BS) flush(g_tail, g_queue, qcap, overflow);
    }

    __device__ void finish(int32_t *g_tail, int32_t *g_queue, int64_t qcap, int32_t *overflow) {
        __syncthreads();
        flush(g_tail, g_queue, qcap, overflow);
    }
};

// Block-wide sum of a per-thread value, added to *dst by one atomic.
template <int BS>
__device__ __forceinline__ void block_add_u64(unsigned long long x, unsigned long long *lds2,
                                              unsigned long long *dst) {
    x = wave_sum_u64(x);
    if (threadIdx.x == 0) lds2[0] = 0;
    __syncthreads();
    if (lane_id() == 0 && x) atomicAdd(&lds2[0], x);
    __syncthreads();
    if (threadIdx.x == 0 && lds2[0]) atomicAdd(dst, lds2[0]);
}

}  // namespace sp

namespace sp {

// Per-wave LDS scratch for the chunked reductions below (64 entries each).
struct WaveScratch {
    int32_t *coff;  // first chunk index of each lane's vertex
    int32_t *beg;   // adjacency start
    int32_t *deg;   // adjacency length (0 = nothing to do)
    double *acc;    // running sum of each lane's vertex
    double *val;    // per-vertex operand the term may read (e.g. sigma[v])
};

// Wave-level sum over the adjacency of up to 64 vertices, one per lane.
// Every vertex's adjacency is cut into chunks of 8 entries aligned at its row
// start.  A step gives 8 chunks to 8 groups of 8 lanes (one entry per lane),
// folds each chunk with a fixed xor tree, and adds the chunk sums to the
// vertex's running sum in chunk order.  The result therefore depends only on
// the vertex's own adjacency, not on the lane or wave that handled it, and the
// lanes stay busy whatever the degree mix.  term(e, owner) is the
// contribution of adjacency entry e of the vertex held by lane `owner`.
template <class Term>
__device__ __forceinline__ double wave_chunk_sum(int32_t beg, int32_t deg, const WaveScratch &ws,
                                                 Term term) {
    const int lane = lane_id();
    const int32_t nch = (deg + 7) >> 3;
    const int32_t incl = wave_incl_scan(nch);
    const int32_t total = __shfl(incl, kWave - 1, kWave);
    ws.coff[lane] = incl - nch;
    ws.beg[lane] = beg;
    ws.deg[lane] = deg;
    ws.acc[lane] = 0.0;
    __builtin_amdgcn_wave_barrier();
    const int g = lane >> 3, j = lane & 7;
    for (int32_t t0 = 0; t0 < total; t0 += 8) {
        const int32_t k = t0 + g;
        int32_t a = -1;
        double x = 0.0;
        if (k < total) {
            int32_t lo = 0, hi = kWave - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (ws.coff[mid] <= k) lo = mid; else hi = mid - 1;
            }
            a = lo;
            const int32_t off = (k - ws.coff[a]) * 8 + j;
            if (off < ws.deg[a]) x = term(ws.beg[a] + off, a);
        }
        x += __shfl_xor(x, 1, kWave);
        x += __shfl_xor(x, 2, kWave);
        x += __shfl_xor(x, 4, kWave);
        int32_t ag[8];
        double xg[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            ag[q] = __shfl(a, q * 8, kWave);
            xg[q] = __shfl(x, q * 8, kWave);
        }
        const int32_t a_prev = __shfl(a, ((g + 7) & 7) * 8, kWave);
        if (j == 0 && a >= 0 && (g == 0 || a_prev != a)) {
            double s = ws.acc[a];
            bool run = true;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q >= g) {
                    if (run && ag[q] == a) s += xg[q];
                    else run = false;
                }
            ws.acc[a] = s;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    return ws.acc[lane];
}

// Wave-level "any": does some adjacency entry of each lane's vertex satisfy
// pred?  The lanes with entries are compacted; group g of 8 lanes takes them
// g, g+8, ... one at a time, 16 entries per step, and leaves a vertex in the
// step where an entry is found, so heavy vertices that are found early cost
// one or two steps however long their rows are.
template <class Pred>
__device__ __forceinline__ bool wave_chunk_any(int32_t beg, int32_t deg, const WaveScratch &ws,
                                               Pred pred) {
    const int lane = lane_id();
    const unsigned long long cm = __ballot(deg > 0);
    const int ncand = __popcll(cm);
    if (deg > 0) ws.coff[lanes_below(cm)] = lane;  // coff holds the candidate list here
    ws.beg[lane] = beg;
    ws.deg[lane] = deg;
    ws.acc[lane] = 0.0;  // 1.0 once found
    __builtin_amdgcn_wave_barrier();
    const int g = lane >> 3, j = lane & 7;
    int k = g;
    int a = k < ncand ? ws.coff[k] : -1;
    int32_t abeg = 0, adeg = 0, off = 0;
    if (a >= 0) {
        abeg = ws.beg[a];
        adeg = ws.deg[a];
    }
    while (__ballot(a >= 0)) {
        bool h0 = false, h1 = false;
        if (a >= 0) {
            const int32_t e0 = off + j, e1 = off + 8 + j;
            if (e0 < adeg) h0 = pred(abeg + e0, a);
            if (e1 < adeg) h1 = pred(abeg + e1, a);
        }
        const unsigned long long hb = __ballot(h0 || h1);
        const bool ghit = ((hb >> (g * 8)) & 0xffull) != 0ull;
        if (a >= 0) {
            off += 16;
            if (ghit || off >= adeg) {
                if (j == 0 && ghit) ws.acc[a] = 1.0;
                k += 8;
                off = 0;
                a = k < ncand ? ws.coff[k] : -1;
                if (a >= 0) {
                    abeg = ws.beg[a];
                    adeg = ws.deg[a];
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    return ws.acc[lane] != 0.0;
}

// One chunk of a hub: lanes stride over its entries, each summing in order,
// then a fixed xor tree; the chunk's sum goes to partial[k].  A finishing
// kernel adds a hub's chunk sums in chunk order (the kernel boundary makes
// them visible, so no fence is needed here).
template <class Term>
__device__ __forceinline__ void hub_chunk(int32_t k, int32_t beg, int32_t end, double *partial,
                                          Term term) {
    const int lane = lane_id();
    double x = 0.0;
    for (int32_t e = beg + lane; e < end; e += kWave) x += term(e);
    x = wave_sum_f64(x);
    if (lane == 0) partial[k] = x;
}

// Rows cut by row eighths (kXcds): a row of deg entries in nchunks = 8m
// near-equal pieces; chunk id offset t = 8g + x is piece x*m + g, in the x-th
// eighth of the row.  Workgroups are dispatched to the device's XCDs
// round-robin and each XCD has its own L2, so when the waves of block b take
// the ids congruent to b mod 8 (for_xcd_chunks) and every split row starts at
// an id that is a multiple of 8, each XCD gathers from one eighth of every
// such row: one eighth of the vertex ids when they are randomly numbered.
__device__ __forceinline__ void split_piece(int32_t rb, int32_t deg, int32_t nchunks, int32_t t,
                                            int32_t &beg, int32_t &end) {
    const int32_t m = nchunks / kXcds;
    const int64_t r = (int64_t)(t % kXcds) * m + t / kXcds;
    beg = rb + (int32_t)((int64_t)deg * r / nchunks);
    end = rb + (int32_t)((int64_t)deg * (r + 1) / nchunks);
}

// Chunk id offset of the piece at row position r (inverse of split_piece).
__device__ __forceinline__ int32_t split_id(int32_t nchunks, int32_t r) {
    const int32_t m = nchunks / kXcds;
    return (r % m) * kXcds + r / m;
}

// Wave loop over chunk ids [0, nch): the waves of block b take the ids
// congruent to b mod kXcds.  A grid that is not a multiple of kXcds walks the
// ids in plain wave order.  Either way every id is visited exactly once.
template <int BS, class F>
__device__ __forceinline__ void for_xcd_chunks(int64_t nch, F f) {
    constexpr int64_t wpb = BS / kWave;
    const int64_t w = threadIdx.x / kWave;
    if ((gridDim.x % kXcds) == 0) {
        const int64_t x = blockIdx.x % kXcds;
        const int64_t j = (int64_t)(blockIdx.x / kXcds) * wpb + w;
        for (int64_t k = x + kXcds * j; k < nch; k += (int64_t)gridDim.x * wpb) f(k);
    } else {
        for (int64_t k = (int64_t)blockIdx.x * wpb + w; k < nch; k += (int64_t)gridDim.x * wpb)
            f(k);
    }
}

// Sum of a split row's chunk sums in row order, eight loads in flight.
__device__ __forceinline__ double sum_split_chunks(const double *__restrict__ partial,
                                                   int32_t base, int32_t n) {
    double s = 0.0;
    for (int32_t r = 0; r < n; r += 8) {  // n is a multiple of 8
        double x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = partial[base + split_id(n, r + t)];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += x[t];
    }
    return s;
}

// Sum of partial[base .. base+n) in index order, eight loads in flight.
__device__ __forceinline__ double sum_chunks(const double *__restrict__ partial, int32_t base,
                                             int32_t n) {
    double s = 0.0;
    int32_t q = 0;
    for (; q + 8 <= n; q += 8) {
        double x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = partial[base + q + t];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += x[t];
    }
    for (; q < n; ++q) s += partial[base + q];
    return s;
}

// A hub's chunk sums in row order under the split chunking (hub_chunk_range).
__device__ __forceinline__ double sum_hub_chunks(const double *__restrict__ partial, int32_t base,
                                                 int32_t n) {
    return n < kXcds ? sum_chunks(partial, base, n) : sum_split_chunks(partial, base, n);
}

}  // namespace sp
