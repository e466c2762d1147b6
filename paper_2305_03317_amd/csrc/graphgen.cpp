// Seeded synthetic graph generators and the CSR builder (host C++, no GPU).
//
// This is the input side of the library: it turns a recipe and a seed into
// the simple undirected int32 CSR the BC path consumes (the paper stores
// graphs as CSR offsets plus neighbour lists, Section 2.3.1 "Data Types").
// It holds none of the traversal arithmetic, so tests may feed its graphs to
// both the GPU library and the CPU oracle.
//
// Recipes (stand-ins for the paper's input graphs of Section 5, Table
// "Input graphs", which are not available here):
//   uniform  n vertices, endpoints drawn uniformly, redrawn until exactly m
//            distinct non-loop undirected edges exist (the "uniform-random"
//            row).
//   rmat     2^scale vertices, edge_factor * 2^scale directed draws, each by
//            `scale` independent quadrant choices with probabilities
//            (a, b, c, 1-a-b-c) (the "rmat876" row used a = 0.57, b = c =
//            0.19), then a seeded uniform vertex relabelling.
//   road     W x W 4-neighbour grid; the minimum spanning tree under i.i.d.
//            uniform edge weights (Kruskal; a uniformly random edge order is
//            the same thing) plus a fraction of all grid edges drawn
//            uniformly without replacement from the non-tree ones; vertex id
//            row * W + col (the "usaroad"/"germany-osm" rows: high diameter,
//            degree <= 4).
// Every graph then goes through the same builder: self-loops dropped, each
// edge stored in both directions, rows sorted ascending, duplicates removed.
//
// Random numbers: xoshiro256** (Blackman & Vigna, 2018) seeded through
// splitmix64.  Work is cut into fixed chunks, each with its own stream, so the
// output does not depend on the number of threads.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_set>
#include <vector>

namespace {

struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

struct Xoshiro256ss {
    uint64_t s[4];
    explicit Xoshiro256ss(uint64_t seed) {
        SplitMix64 sm(seed);
        for (auto &x : s) x = sm.next();
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next() {
        const uint64_t result = rotl(s[1] * 5, 7) * 9;
        const uint64_t t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return result;
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
    // Unbiased integer in [0, bound) (Lemire's multiply-and-reject).
    uint64_t below(uint64_t bound) {
        unsigned __int128 m = (unsigned __int128)next() * bound;
        uint64_t lo = (uint64_t)m;
        if (lo < bound) {
            uint64_t thr = (0 - bound) % bound;
            while (lo < thr) {
                m = (unsigned __int128)next() * bound;
                lo = (uint64_t)m;
            }
        }
        return (uint64_t)(m >> 64);
    }
};

uint64_t stream_seed(uint64_t seed, uint64_t stream) {
    SplitMix64 sm(seed ^ (0xD1B54A32D192ED03ull * (stream + 1)));
    return sm.next();
}

int hw_threads() {
    const char *e = std::getenv("SPG_THREADS");
    if (e && std::atoi(e) > 0) return std::atoi(e);
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

template <class F>
void parallel_for(int64_t n, int64_t grain, F f) {
    int nt = hw_threads();
    if (n <= grain || nt <= 1) {
        if (n > 0) f(0, n);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (;;) {
                int64_t b = next.fetch_add(grain);
                if (b >= n) break;
                f(b, std::min(n, b + grain));
            }
        });
    for (auto &x : th) x.join();
}

struct Csr {
    int32_t n = 0;
    std::vector<int32_t> row_ptr;
    std::vector<int32_t> col_idx;
};

// Builder: undirected edge list -> simple symmetric CSR with sorted rows.
bool build_csr(int32_t n, const std::vector<int32_t> &src, const std::vector<int32_t> &dst, Csr &out) {
    const int64_t m = (int64_t)src.size();
    std::vector<std::atomic<int64_t>> deg(n);
    for (auto &d : deg) d.store(0, std::memory_order_relaxed);
    parallel_for(m, 1 << 18, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            if (src[i] == dst[i]) continue;
            deg[src[i]].fetch_add(1, std::memory_order_relaxed);
            deg[dst[i]].fetch_add(1, std::memory_order_relaxed);
        }
    });
    std::vector<int64_t> off(n + 1, 0);
    for (int32_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v].load(std::memory_order_relaxed);
    std::vector<int32_t> tmp;
    try { tmp.resize(off[n]); } catch (std::bad_alloc &) { return false; }
    std::vector<std::atomic<int64_t>> pos(n);
    for (int32_t v = 0; v < n; ++v) pos[v].store(off[v], std::memory_order_relaxed);
    parallel_for(m, 1 << 18, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            int32_t a = src[i], c = dst[i];
            if (a == c) continue;
            tmp[pos[a].fetch_add(1, std::memory_order_relaxed)] = c;
            tmp[pos[c].fetch_add(1, std::memory_order_relaxed)] = a;
        }
    });
    // Sort + dedupe each row in place; record the surviving length.
    std::vector<int64_t> keep(n, 0);
    parallel_for(n, 4096, [&](int64_t b, int64_t e) {
        for (int64_t v = b; v < e; ++v) {
            auto first = tmp.begin() + off[v], last = tmp.begin() + off[v + 1];
            std::sort(first, last);
            keep[v] = std::unique(first, last) - first;
        }
    });
    out.n = n;
    out.row_ptr.assign(n + 1, 0);
    int64_t total = 0;
    for (int32_t v = 0; v < n; ++v) {
        total += keep[v];
        if (total > INT32_MAX) return false;
        out.row_ptr[v + 1] = (int32_t)total;
    }
    try { out.col_idx.resize(total); } catch (std::bad_alloc &) { return false; }
    parallel_for(n, 4096, [&](int64_t b, int64_t e) {
        for (int64_t v = b; v < e; ++v)
            std::memcpy(out.col_idx.data() + out.row_ptr[v], tmp.data() + off[v],
                        sizeof(int32_t) * keep[v]);
    });
    return true;
}

struct UnionFind {
    std::vector<int32_t> parent, size;
    explicit UnionFind(int32_t n) : parent(n), size(n, 1) {
        for (int32_t i = 0; i < n; ++i) parent[i] = i;
    }
    int32_t find(int32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    }
    bool unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a == b) return false;
        if (size[a] < size[b]) std::swap(a, b);
        parent[b] = a;
        size[a] += size[b];
        return true;
    }
};

}  // namespace

extern "C" {

// Opaque result handle: the caller reads sizes, copies arrays out, releases.
struct spg_graph_s {
    Csr csr;
};
typedef struct spg_graph_s *spg_graph;

enum { SPG_OK = 0, SPG_BAD_ARG = -1, SPG_NO_MEMORY = -2 };

int spg_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, spg_graph *out) {
    if (!out || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return SPG_BAD_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return SPG_BAD_ARG;
    auto *g = new (std::nothrow) spg_graph_s;
    if (!g) return SPG_NO_MEMORY;
    std::vector<int32_t> s(src, src + m), d(dst, dst + m);
    if (!build_csr(n, s, d, g->csr)) {
        delete g;
        return SPG_NO_MEMORY;
    }
    *out = g;
    return SPG_OK;
}

int spg_uniform(int32_t n, int64_t m, uint64_t seed, spg_graph *out) {
    if (!out || n < 0 || m < 0) return SPG_BAD_ARG;
    if (m > (int64_t)n * (n - 1) / 2) return SPG_BAD_ARG;
    Xoshiro256ss rng(stream_seed(seed, 0));
    std::unordered_set<uint64_t> seen;
    seen.reserve((size_t)m * 2);
    std::vector<int32_t> src, dst;
    src.reserve(m);
    dst.reserve(m);
    while ((int64_t)src.size() < m) {
        int32_t a = (int32_t)rng.below((uint64_t)n);
        int32_t b = (int32_t)rng.below((uint64_t)n);
        if (a == b) continue;
        uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
        if (!seen.insert(key).second) continue;
        src.push_back(a);
        dst.push_back(b);
    }
    auto *g = new (std::nothrow) spg_graph_s;
    if (!g) return SPG_NO_MEMORY;
    if (!build_csr(n, src, dst, g->csr)) {
        delete g;
        return SPG_NO_MEMORY;
    }
    *out = g;
    return SPG_OK;
}

int spg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
             int32_t permute, spg_graph *out) {
    if (!out || scale < 1 || scale > 30 || edge_factor < 1) return SPG_BAD_ARG;
    if (!(a >= 0 && b >= 0 && c >= 0 && a + b + c <= 1.0)) return SPG_BAD_ARG;
    const int32_t n = (int32_t)1 << scale;
    const int64_t m = (int64_t)edge_factor << scale;
    std::vector<int32_t> src, dst;
    try {
        src.resize(m);
        dst.resize(m);
    } catch (std::bad_alloc &) {
        return SPG_NO_MEMORY;
    }
    const double ab = a + b, abc = a + b + c;
    const int64_t chunk = 1 << 16;
    parallel_for((m + chunk - 1) / chunk, 1, [&](int64_t cb, int64_t ce) {
        for (int64_t ci = cb; ci < ce; ++ci) {
            Xoshiro256ss rng(stream_seed(seed, 1 + (uint64_t)ci));
            int64_t e_end = std::min(m, (ci + 1) * chunk);
            for (int64_t e = ci * chunk; e < e_end; ++e) {
                uint32_t r = 0, col = 0;
                for (int32_t bit = scale - 1; bit >= 0; --bit) {
                    double u = rng.uniform();
                    if (u < a) {
                    } else if (u < ab) {
                        col |= 1u << bit;
                    } else if (u < abc) {
                        r |= 1u << bit;
                    } else {
                        r |= 1u << bit;
                        col |= 1u << bit;
                    }
                }
                src[e] = (int32_t)r;
                dst[e] = (int32_t)col;
            }
        }
    });
    if (permute) {
        std::vector<int32_t> perm(n);
        for (int32_t i = 0; i < n; ++i) perm[i] = i;
        Xoshiro256ss rng(stream_seed(seed, 0));
        for (int32_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[rng.below((uint64_t)i + 1)]);
        parallel_for(m, 1 << 18, [&](int64_t b0, int64_t e0) {
            for (int64_t i = b0; i < e0; ++i) {
                src[i] = perm[src[i]];
                dst[i] = perm[dst[i]];
            }
        });
    }
    auto *g = new (std::nothrow) spg_graph_s;
    if (!g) return SPG_NO_MEMORY;
    if (!build_csr(n, src, dst, g->csr)) {
        delete g;
        return SPG_NO_MEMORY;
    }
    *out = g;
    return SPG_OK;
}

int spg_road(int32_t W, double extra_fraction, uint64_t seed, spg_graph *out) {
    if (!out || W < 1 || W > 46340 || !(extra_fraction >= 0.0 && extra_fraction <= 1.0)) return SPG_BAD_ARG;
    const int32_t n = W * W;
    const int64_t n_h = (int64_t)W * (W - 1);   // horizontal edges come first
    const int64_t n_e = 2 * n_h;
    auto endpoints = [&](int64_t e, int32_t &x, int32_t &y) {
        if (e < n_h) {
            int64_t r = e / (W - 1), cc = e % (W - 1);
            x = (int32_t)(r * W + cc);
            y = x + 1;
        } else {
            int64_t f = e - n_h;
            x = (int32_t)f;   // (r, c) with r = f / W, c = f % W
            y = x + W;
        }
    };
    std::vector<int64_t> order(n_e);
    for (int64_t i = 0; i < n_e; ++i) order[i] = i;
    Xoshiro256ss rng(stream_seed(seed, 0));
    for (int64_t i = n_e - 1; i > 0; --i) std::swap(order[i], order[rng.below((uint64_t)i + 1)]);
    std::vector<uint8_t> in_tree(n_e, 0);
    UnionFind uf(n);
    std::vector<int32_t> src, dst;
    src.reserve(n + (size_t)(extra_fraction * n_e) + 1);
    dst.reserve(src.capacity());
    for (int64_t i = 0; i < n_e; ++i) {
        int32_t x, y;
        endpoints(order[i], x, y);
        if (uf.unite(x, y)) {
            in_tree[order[i]] = 1;
            src.push_back(x);
            dst.push_back(y);
        }
    }
    std::vector<int64_t>().swap(order);
    std::vector<int64_t> rest;
    rest.reserve(n_e - (n - 1));
    for (int64_t e = 0; e < n_e; ++e)
        if (!in_tree[e]) rest.push_back(e);
    int64_t k = (int64_t)std::llround(extra_fraction * (double)n_e);
    k = std::min<int64_t>(k, (int64_t)rest.size());
    Xoshiro256ss rng2(stream_seed(seed, 1));
    for (int64_t i = 0; i < k; ++i) {
        int64_t j = i + (int64_t)rng2.below((uint64_t)(rest.size() - i));
        std::swap(rest[i], rest[j]);
        int32_t x, y;
        endpoints(rest[i], x, y);
        src.push_back(x);
        dst.push_back(y);
    }
    auto *g = new (std::nothrow) spg_graph_s;
    if (!g) return SPG_NO_MEMORY;
    if (!build_csr(n, src, dst, g->csr)) {
        delete g;
        return SPG_NO_MEMORY;
    }
    *out = g;
    return SPG_OK;
}

int spg_size(spg_graph g, int32_t *n, int64_t *nnz) {
    if (!g || !n || !nnz) return SPG_BAD_ARG;
    *n = g->csr.n;
    *nnz = (int64_t)g->csr.col_idx.size();
    return SPG_OK;
}

int spg_copy(spg_graph g, int32_t *row_ptr, int32_t *col_idx) {
    if (!g || !row_ptr || (!col_idx && !g->csr.col_idx.empty())) return SPG_BAD_ARG;
    std::memcpy(row_ptr, g->csr.row_ptr.data(), sizeof(int32_t) * g->csr.row_ptr.size());
    if (!g->csr.col_idx.empty())
        std::memcpy(col_idx, g->csr.col_idx.data(), sizeof(int32_t) * g->csr.col_idx.size());
    return SPG_OK;
}

void spg_release(spg_graph g) { delete g; }

// Sources drawn without replacement, uniformly among vertices whose degree is
// at least min_degree, in draw order.  Fails if fewer candidates than count.
int spg_sources(int32_t n, const int32_t *row_ptr, int32_t count, int32_t min_degree, uint64_t seed,
                int32_t *out) {
    if (n < 0 || !row_ptr || count < 0 || (count > 0 && !out)) return SPG_BAD_ARG;
    std::vector<int32_t> cand;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] >= min_degree) cand.push_back(v);
    if ((int64_t)cand.size() < count) return SPG_BAD_ARG;
    Xoshiro256ss rng(stream_seed(seed, 0));
    for (int32_t i = 0; i < count; ++i) {
        size_t j = i + (size_t)rng.below(cand.size() - i);
        std::swap(cand[i], cand[j]);
        out[i] = cand[i];
    }
    return SPG_OK;
}

// Edge weights for the weighted algorithms (SSSP): one int32 per CSR entry,
// uniform on [lo, hi] (the paper draws weights uniformly from [1, 100] for
// graphs that have none, Section 5).  The weight of {u, v} is a hash of the
// seed and the unordered pair, so both stored directions get the same value
// and the result does not depend on the CSR's entry order.
int spg_weights(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t lo, int32_t hi,
                uint64_t seed, int32_t *out) {
    if (n < 0 || !row_ptr || lo > hi || (n > 0 && row_ptr[n] > 0 && (!col_idx || !out)))
        return SPG_BAD_ARG;
    const uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const uint32_t v = (uint32_t)col_idx[e];
            const uint64_t a = std::min((uint32_t)u, v), b = std::max((uint32_t)u, v);
            SplitMix64 sm(seed ^ ((a << 32) | b) * 0xD1B54A32D192ED03ull);
            out[e] = (int32_t)((int64_t)lo + (int64_t)(sm.next() % span));
        }
    return SPG_OK;
}

}  // extern "C"
