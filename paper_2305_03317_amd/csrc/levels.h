// Device helpers shared by the level and round kernels: hub registration on
// the level being built, the chunk-id lookup, coherent counter reads, the
// last-block election that ends a level inside its last kernel, and the
// profiling counter flush.
#pragma once

#include "common.h"
#include "devutil.h"

namespace sp {

// Register a hub of the level being built under the split chunking of
// split_hub_nchunks (rows over kHubSplitDeg cut by row eighths, first id aligned
// to kXcds): reserve split_hub_span(deg) chunk ids through the packed counter
// `pack` (list index in the high bits, chunk ids in the low 40) and store the
// entry at list[at + index].  `cap` is the list's capacity; an index past it
// is dropped and reported by `advance` as an overflow.  With an owner map
// (batched path), every reserved id, the alignment slack included, records
// the hub's list index at owner[owner_at + id], so chunk kernels find their
// hub with one load (hub_chunk_range turns the slack ids away); `advance`
// checks owner_cap.
__device__ __forceinline__ void hub_register(unsigned long long *pack, HubEntry *list,
                                             long long cap, int32_t at, int32_t v, int32_t entry,
                                             int32_t deg, int32_t *owner = nullptr,
                                             long long owner_at = 0, long long owner_cap = 0) {
    const int32_t nch = split_hub_nchunks(deg), span = split_hub_span(deg);
    const unsigned long long old = atomicAdd(pack, (1ull << 40) | (unsigned long long)span);
    const int32_t idx = (int32_t)(old >> 40);
    const int32_t base0 = (int32_t)(old & ((1ull << 40) - 1));
    const int32_t base = nch >= kXcds ? (base0 + kXcds - 1) & ~(kXcds - 1) : base0;
    if ((long long)at + idx < cap) list[at + idx] = HubEntry{v, entry, base, nch};
    if (owner)
        for (int32_t q = 0; q < span; ++q) {
            const long long p = owner_at + base0 + q;
            if (p < owner_cap) owner[p] = at + idx;
        }
}

// Adjacency range [beg, end) of chunk id k of hub h under the split chunking;
// false for an alignment slack id.  Hubs of fewer than kXcds chunks:
// consecutive kHubChunk pieces; split hubs: split_piece.
__device__ __forceinline__ bool hub_chunk_range(const HubEntry &h, int64_t k,
                                                const int32_t *__restrict__ rp, int32_t &beg,
                                                int32_t &end) {
    const int32_t t = (int32_t)k - h.chunk_base;
    if (t < 0 || t >= h.nchunks) return false;
    const int32_t rb = rp[h.v];
    if (h.nchunks < kXcds) {
        beg = rb + t * kHubChunk;
        end = min(rp[h.v + 1], beg + kHubChunk);
    } else {
        split_piece(rb, rp[h.v + 1] - rb, h.nchunks, t, beg, end);
    }
    return true;
}

// The hub whose chunk range holds chunk id k, in segment [lo, hi) sorted by
// chunk_base (the packed atomic hands out indices and bases in one order).
__device__ __forceinline__ int32_t hub_find(const HubEntry *list, int32_t lo, int32_t hi, int32_t k) {
    int32_t a = lo, z = hi - 1;
    while (a < z) {
        const int32_t mid = (a + z + 1) >> 1;
        if (list[mid].chunk_base <= k) a = mid; else z = mid - 1;
    }
    return a;
}

// Coherent read of a counter other blocks updated with device-scope atomics
// (relaxed: no cache invalidation is needed for the counters themselves).
template <class T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in exactly one of the `nb` blocks that call it with working = true
// (a block-uniform flag): the last of them to get here.  Every thread of a
// block calls it after the block's last atomic update of the control block;
// blocks without work return false at once, so only working blocks touch the
// counter, which is left at zero for the next kernel.  The chosen block reads
// only counters updated with device-scope atomics, so no cache write-back is
// needed: each wave waits until its own atomics are acknowledged (a barrier
// alone does not wait for them), then one thread counts the block.
__device__ __forceinline__ bool last_working_block(int32_t *blocks_done, bool working, int nb) {
    __shared__ int s_last;
    if (!working) return false;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int prev = atomicAdd(blocks_done, 1);
        s_last = prev == nb - 1;
        if (s_last) atomicExch(blocks_done, 0);
    }
    __syncthreads();
    return s_last != 0;
}

// One-dimensional grids whose working blocks are the first `nb`
// (blockIdx.x < nb); block 0 when nb is 0.
template <class Ctl>
__device__ __forceinline__ bool last_block(Ctl *c, int nb) {
    if (nb <= 0) return blockIdx.x == 0;
    return last_working_block(&c->blocks_done_.v, (int)blockIdx.x < nb, nb);
}

// Blocks of a grid-stride loop over `items` in steps of `per_block` that get
// at least one item.
__device__ __forceinline__ int working_blocks(int64_t items, int per_block) {
    if (items <= 0) return 0;
    return (int)min((int64_t)gridDim.x, (items + per_block - 1) / per_block);
}

template <int BS>
__device__ __forceinline__ void flush_counters(unsigned long long *prof, unsigned long long items,
                                               unsigned long long edges, unsigned long long pairs,
                                               unsigned long long *lds) {
    if (!prof) return;
    __syncthreads();
    block_add_u64<BS>(items, lds, prof + 0);
    __syncthreads();
    block_add_u64<BS>(edges, lds, prof + 1);
    __syncthreads();
    block_add_u64<BS>(pairs, lds, prof + 2);
    __syncthreads();
    block_add_u64<BS>(items, lds, prof + 3);
}

}  // namespace sp
