// Device helpers shared by the per-source and batched level kernels: hub
// registration on the level being built, the chunk-id lookup, and the
// profiling counter flush.
#pragma once

#include "common.h"
#include "devutil.h"

namespace sp {

// Register a hub of the level being built: reserve its chunk ids.
// `cap` is the list's capacity; an index past it is dropped and reported by
// `advance` as an overflow.  With an owner map (batched path), each of the
// hub's chunks also records the hub's list index at owner[chunk_next + id],
// so chunk kernels find their hub with one load; `advance` checks owner_cap.
__device__ __forceinline__ void hub_register(LevelCtl *c, HubEntry *list, long long cap, int32_t v,
                                             int32_t entry, int32_t deg, int32_t *owner = nullptr,
                                             long long owner_cap = 0) {
    const int32_t nch = (deg + kHubChunk - 1) / kHubChunk;
    const unsigned long long old = atomicAdd(&c->hub_pack_.v, (1ull << 40) | (unsigned long long)nch);
    const int32_t idx = (int32_t)(old >> 40);
    const int32_t base = (int32_t)(old & ((1ull << 40) - 1));
    if ((long long)c->hub_next + idx < cap) list[c->hub_next + idx] = HubEntry{v, entry, base, nch};
    if (owner)
        for (int32_t q = 0; q < nch; ++q) {
            const long long p = (long long)c->chunk_next + base + q;
            if (p < owner_cap) owner[p] = c->hub_next + idx;
        }
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
