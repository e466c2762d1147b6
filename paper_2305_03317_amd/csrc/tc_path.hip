// Triangle counting (paper Appendix, Fig. "TC computation in StarPlat").
//
// The paper's node iterator counts, for every vertex v, the adjacent pairs
// (u, w) of its neighbours with u < v < w, testing adjacency by binary search
// in a sorted row; each triangle is counted once.  Its work at a vertex is
// (neighbours below) x (neighbours above): quadratic in the degree of a
// high-degree vertex.  Here each triangle is instead counted once at its
// lowest-ranked edge, ranking vertices by (degree, id): N+(v) holds the
// neighbours of higher rank (a subsequence of v's sorted row, so sorted
// too), and for every v and u in N+(v) the triangles are the common entries
// of N+(v) and N+(u).  A vertex has at most sqrt(2m) neighbours of higher
// rank, so the work is bounded by O(m^1.5) whatever the degree mix.  The
// count is the same number the paper's loops produce.
//
// Kernels: the oriented rows are built once per graph (out-degree by rank,
// a two-level scan, a filtering copy that also records each oriented entry's
// row; rows longer than kHubDeg are counted and copied by a block each), then
// each oriented entry (v, u) intersects N+(v) and N+(u) (both sorted) by
// binary-searching the elements of the shorter list in the longer one: by
// its own lane when the shorter list is short, else by the whole wave.
// Lane counts are summed per block in a fixed order and added with one
// 64-bit atomic.
#include "common.h"
#include "devutil.h"
#include "levels.h"

namespace sp {

namespace {
constexpr int kScanTile = 1024;  // vertices per scan tile (256 threads x 4)
}

// rank(a) < rank(b): lower degree, ties broken by id.
__device__ __forceinline__ bool rank_below(int32_t da, int32_t a, int32_t db, int32_t b) {
    return da < db || (da == db && a < b);
}

// Out-degree under the rank order of every vertex whose row is at most
// kHubDeg long (a lane per vertex); longer rows are left to k_tc_hub_outdeg.
__global__ void k_tc_outdeg(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t n,
                            int32_t *odeg) {
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
        if (dv > kHubDeg) continue;
        int32_t d = 0;
        for (int32_t k = b; k < e; ++k) {
            const int32_t u = ci[k];
            d += rank_below(dv, v, rp[u + 1] - rp[u], u);
        }
        odeg[v] = d;
    }
}

// Out-degree of the hubs: a block per hub row.
__global__ __launch_bounds__(256) void k_tc_hub_outdeg(const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const HubEntry *__restrict__ hubs, int32_t nh,
                                                       int32_t *odeg) {
    __shared__ int32_t s_scan[256 / kWave + 1];
    for (int32_t j = blockIdx.x; j < nh; j += gridDim.x) {
        const int32_t v = hubs[j].v;
        const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
        int32_t d = 0;
        for (int32_t k = b + threadIdx.x; k < e; k += 256) {
            const int32_t u = ci[k];
            d += rank_below(dv, v, rp[u + 1] - rp[u], u);
        }
        int32_t total;
        (void)block_excl_scan<256>(d, s_scan, &total);
        if (threadIdx.x == 0) odeg[v] = total;
        __syncthreads();
    }
}

// Exclusive scan of the out-degrees within tiles of kScanTile vertices:
// odeg_off[v] = offset of v inside its tile; tile_sum[t] = the tile's total.
__global__ __launch_bounds__(256) void k_tc_scan_local(const int32_t *__restrict__ odeg, int32_t n,
                                                       int32_t *odeg_off, int32_t *tile_sum) {
    __shared__ int32_t s_scan[256 / kWave + 1];
    const int32_t v0 = blockIdx.x * kScanTile + threadIdx.x * 4;
    int32_t d[4];
    int32_t mine = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d[q] = v0 + q < n ? odeg[v0 + q] : 0;
        mine += d[q];
    }
    int32_t total;
    int32_t off = block_excl_scan<256>(mine, s_scan, &total);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (v0 + q < n) odeg_off[v0 + q] = off;
        off += d[q];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Exclusive scan of the tile totals in place (one block), and the entry count.
__global__ __launch_bounds__(256) void k_tc_scan_tiles(int32_t *tile_sum, int32_t ntiles,
                                                       int32_t *orp, int32_t n) {
    __shared__ int32_t s_scan[256 / kWave + 1];
    int32_t carry = 0;
    for (int32_t b = 0; b < ntiles; b += 256) {
        const int32_t i = b + threadIdx.x;
        const int32_t x = i < ntiles ? tile_sum[i] : 0;
        int32_t total;
        const int32_t off = block_excl_scan<256>(x, s_scan, &total);
        if (i < ntiles) tile_sum[i] = carry + off;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) orp[n] = carry;
}

// Oriented rows of the vertices with rows of at most kHubDeg entries (a lane
// per vertex): orp[v] = tile base + offset in tile; N+(v) copied in row
// order, with each entry's row in osrc.
__global__ void k_tc_fill(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t n,
                          const int32_t *__restrict__ odeg_off, const int32_t *__restrict__ tile_base,
                          int32_t *orp, int32_t *oci, int32_t *osrc) {
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        int32_t o = tile_base[v / kScanTile] + odeg_off[v];
        orp[v] = o;
        const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
        if (dv > kHubDeg) continue;
        for (int32_t k = b; k < e; ++k) {
            const int32_t u = ci[k];
            if (rank_below(dv, v, rp[u + 1] - rp[u], u)) {
                oci[o] = u;
                osrc[o] = v;
                ++o;
            }
        }
    }
}

// Oriented rows of the hubs: a block per hub compacts the row's
// higher-ranked entries in row order (block scan per 256 entries).
__global__ __launch_bounds__(256) void k_tc_hub_fill(const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const HubEntry *__restrict__ hubs, int32_t nh,
                                                     const int32_t *__restrict__ odeg_off,
                                                     const int32_t *__restrict__ tile_base,
                                                     int32_t *oci, int32_t *osrc) {
    __shared__ int32_t s_scan[256 / kWave + 1];
    for (int32_t j = blockIdx.x; j < nh; j += gridDim.x) {
        const int32_t v = hubs[j].v;
        const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
        int32_t o = tile_base[v / kScanTile] + odeg_off[v];
        for (int32_t k0 = b; k0 < e; k0 += 256) {
            const int32_t k = k0 + threadIdx.x;
            int32_t u = 0;
            bool keep = false;
            if (k < e) {
                u = ci[k];
                keep = rank_below(dv, v, rp[u + 1] - rp[u], u);
            }
            int32_t total;
            const int32_t off = block_excl_scan<256>((int32_t)keep, s_scan, &total);
            if (keep) {
                oci[o + off] = u;
                osrc[o + off] = v;
            }
            o += total;
            __syncthreads();
        }
    }
}

// First position in a[lo, hi) holding a value >= x.
__device__ __forceinline__ int32_t lower_bound(const int32_t *__restrict__ a, int32_t lo, int32_t hi,
                                               int32_t x) {
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// |N+(v) & N+(u)| for the oriented entries of a wave (64 consecutive
// entries, one per lane).  An entry whose shorter list has at most
// kTcLaneWork elements is intersected by its own lane, which walks the
// shorter list and binary-searches each element in the longer one, the
// window shrinking as the walk moves up.  Longer ones are taken by the whole
// wave in turn: lane j searches elements j, j + 64, ... of the shorter list
// in the whole longer one.  With `per` the three vertices of every triangle
// found get one count each.
constexpr int32_t kTcLaneWork = 32;

template <int BS>
__global__ __launch_bounds__(BS) void k_tc_count(const int32_t *__restrict__ orp,
                                                 const int32_t *__restrict__ oci,
                                                 const int32_t *__restrict__ osrc, int64_t m,
                                                 unsigned long long *total,
                                                 unsigned long long *per, unsigned long long *prof) {
    __shared__ unsigned long long s_red[1];
    const int lane = lane_id();
    unsigned long long mine = 0, probes = 0;
    auto hit = [&](int32_t v, int32_t u, int32_t w) {
        ++mine;
        if (per) {
            atomicAdd(&per[v], 1ull);
            atomicAdd(&per[u], 1ull);
            atomicAdd(&per[w], 1ull);
        }
    };
    const int64_t stride = (int64_t)gridDim.x * BS;
    for (int64_t e0 = (int64_t)blockIdx.x * BS + threadIdx.x - lane; e0 < m; e0 += stride) {
        const int64_t e = e0 + lane;
        int32_t v = 0, u = 0, sb = 0, se = 0, lb = 0, le = 0;
        if (e < m) {
            v = osrc[e];
            u = oci[e];
            sb = orp[v];
            se = orp[v + 1];
            lb = orp[u];
            le = orp[u + 1];
            if (se - sb > le - lb) {  // walk the shorter list
                int32_t t = sb; sb = lb; lb = t;
                t = se; se = le; le = t;
            }
        }
        const bool alone = se - sb <= kTcLaneWork;
        if (alone) {
            int32_t pos = lb;
            for (int32_t i = sb; i < se && pos < le; ++i) {
                const int32_t w = oci[i];
                pos = lower_bound(oci, pos, le, w);
                ++probes;
                if (pos < le && oci[pos] == w) {
                    hit(v, u, w);
                    ++pos;
                }
            }
        }
        unsigned long long big = __ballot(!alone);
        while (big) {
            const int src = __ffsll((long long)big) - 1;
            big &= big - 1;
            const int32_t bv = __shfl(v, src, kWave), bu = __shfl(u, src, kWave);
            const int32_t bsb = __shfl(sb, src, kWave), bse = __shfl(se, src, kWave);
            const int32_t blb = __shfl(lb, src, kWave), ble = __shfl(le, src, kWave);
            for (int32_t i = bsb + lane; i < bse; i += kWave) {
                const int32_t w = oci[i];
                const int32_t pos = lower_bound(oci, blb, ble, w);
                ++probes;
                if (pos < ble && oci[pos] == w) hit(bv, bu, w);
            }
        }
    }
    block_add_u64<BS>(mine, s_red, total);
    if (prof) {
        __syncthreads();
        block_add_u64<BS>(probes, s_red, prof + 1);
    }
}

__global__ void k_tc_zero(unsigned long long *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
sp_status ensure_oriented(sp_graph g, hipStream_t s) {
    SP_TRY(ensure_static_hubs(g, s));
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->tc_orp) return SP_OK;
    const int32_t n = g->n;
    const int32_t ntiles = std::max(1, (n + kScanTile - 1) / kScanTile);
    const int maxb = device_cu_count() * 8;
    int32_t *orp = nullptr, *oci = nullptr, *osrc = nullptr, *odeg = nullptr, *off = nullptr,
            *tiles = nullptr;
    auto fail = [&](sp_status st) {
        dev_free(orp);
        dev_free(oci);
        dev_free(osrc);
        dev_free(odeg);
        dev_free(off);
        dev_free(tiles);
        return st;
    };
    const size_t vn = (size_t)std::max(n, 1);
    sp_status st = dev_alloc((void **)&orp, sizeof(int32_t) * (vn + 1));
    if (st == SP_OK) st = dev_alloc((void **)&odeg, sizeof(int32_t) * vn);
    if (st == SP_OK) st = dev_alloc((void **)&off, sizeof(int32_t) * vn);
    if (st == SP_OK) st = dev_alloc((void **)&tiles, sizeof(int32_t) * (size_t)ntiles);
    if (st != SP_OK) return fail(st);
    if (n > 0) {
        hipLaunchKernelGGL(k_tc_outdeg, dim3(grid_for(n, 256, maxb)), dim3(256), 0, s,
                           (const int32_t *)g->row_ptr, (const int32_t *)g->col_idx, n, odeg);
        if (g->n_hubs > 0)
            hipLaunchKernelGGL(k_tc_hub_outdeg, dim3(std::min(g->n_hubs, maxb)), dim3(256), 0, s,
                               (const int32_t *)g->row_ptr, (const int32_t *)g->col_idx,
                               (const HubEntry *)g->hub_static, g->n_hubs, odeg);
        hipLaunchKernelGGL(k_tc_scan_local, dim3(ntiles), dim3(256), 0, s, (const int32_t *)odeg, n, off,
                           tiles);
    }
    hipLaunchKernelGGL(k_tc_scan_tiles, dim3(1), dim3(256), 0, s, tiles, n > 0 ? ntiles : 0, orp, n);
    SP_HIP(hipGetLastError());
    int32_t m = 0;
    SP_HIP(hipMemcpyAsync(&m, orp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
    if ((int64_t)m * 2 != g->nnz) {
        // a simple symmetric graph orients exactly one entry of each pair
        set_error("triangle counting needs a simple undirected CSR (%d oriented entries of %lld)", m,
                  (long long)g->nnz);
        return fail(SP_ERR_INVALID_ARGUMENT);
    }
    st = dev_alloc((void **)&oci, sizeof(int32_t) * (size_t)std::max(m, 1));
    if (st == SP_OK) st = dev_alloc((void **)&osrc, sizeof(int32_t) * (size_t)std::max(m, 1));
    if (st != SP_OK) return fail(st);
    if (n > 0) {
        hipLaunchKernelGGL(k_tc_fill, dim3(grid_for(n, 256, maxb)), dim3(256), 0, s,
                           (const int32_t *)g->row_ptr, (const int32_t *)g->col_idx, n, (const int32_t *)off,
                           (const int32_t *)tiles, orp, oci, osrc);
        if (g->n_hubs > 0)
            hipLaunchKernelGGL(k_tc_hub_fill, dim3(std::min(g->n_hubs, maxb)), dim3(256), 0, s,
                               (const int32_t *)g->row_ptr, (const int32_t *)g->col_idx,
                               (const HubEntry *)g->hub_static, g->n_hubs, (const int32_t *)off,
                               (const int32_t *)tiles, oci, osrc);
    }
    SP_HIP(hipGetLastError());
    SP_HIP(hipStreamSynchronize(s));
    dev_free(odeg);
    dev_free(off);
    dev_free(tiles);
    g->tc_orp = orp;
    g->tc_oci = oci;
    g->tc_osrc = osrc;
    g->tc_m = m;
    g->bytes += sizeof(int32_t) * (vn + 1 + 2 * (size_t)std::max(m, 1));
    return SP_OK;
}

sp_status tc_run(sp_graph g, unsigned long long *d_total, unsigned long long *per, hipStream_t s) {
    const int maxb = device_cu_count() * 8;
    hipLaunchKernelGGL(k_tc_zero, dim3(1), dim3(64), 0, s, d_total, (int64_t)1);
    if (per) hipLaunchKernelGGL(k_tc_zero, dim3(grid_for(g->n, 256, 4096)), dim3(256), 0, s, per, (int64_t)g->n);
    if (g->tc_m > 0) {
        ProfScope ps(P_TC_COUNT, s);
        hipLaunchKernelGGL(k_tc_count<256>, dim3(grid_for(g->tc_m, 256, maxb)), dim3(256), 0, s,
                           (const int32_t *)g->tc_orp, (const int32_t *)g->tc_oci,
                           (const int32_t *)g->tc_osrc, (int64_t)g->tc_m, d_total, per,
                           prof_counters(P_TC_COUNT));
    }
    SP_HIP(hipGetLastError());
    return SP_OK;
}

}  // namespace sp
