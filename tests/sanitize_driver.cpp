// Host-side sanitizer run: the C oracle (oracle/*.c) and the seeded graph
// generators (graphgen.cpp) built with AddressSanitizer and
// UndefinedBehaviorSanitizer and exercised here on small inputs.  Each
// check is an invariant or closed form the parity tests also pin:
//   generators   simple symmetric CSR (rows sorted, no loops, both
//                directions), sources distinct with degree >= min, weights
//                equal in both directions;
//   BC oracle    sum over v of BC(v) = sum over sources s and reached t of
//                (dist_s(t) - 1); path P_n: 2 i (n-1-i); star: centre
//                (n-1)(n-2); complete graph: 0;
//   SSSP oracle  unit weights give the BFS distances;
//   TC oracle    K_6 has 20 triangles; per-vertex counts sum to 3x the
//                total and match the one-vertex count.
// Any sanitizer report aborts the run (-fno-sanitize-recover=all); a failed
// check exits 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
int oracle_bc(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *sources, int32_t n_sources,
              double *bc, double *sigma_max);
int oracle_source_detail(int32_t n, const int32_t *rp, const int32_t *ci, int32_t src, int32_t *dist,
                         double *sigma, double *delta, int32_t *n_reached);
int oracle_sssp(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *w, int32_t src,
                int32_t *dist);
int oracle_tc(int32_t n, const int32_t *rp, const int32_t *ci, int64_t *out);
int oracle_tc_vertex(int32_t n, const int32_t *rp, const int32_t *ci, int32_t v, int64_t *out);
int oracle_tc_each(int32_t n, const int32_t *rp, const int32_t *ci, int64_t *out);

typedef struct spg_graph_s *spg_graph;
int spg_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, spg_graph *out);
int spg_uniform(int32_t n, int64_t m, uint64_t seed, spg_graph *out);
int spg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
             int32_t permute, spg_graph *out);
int spg_road(int32_t W, double extra_fraction, uint64_t seed, spg_graph *out);
int spg_size(spg_graph g, int32_t *n, int64_t *nnz);
int spg_copy(spg_graph g, int32_t *row_ptr, int32_t *col_idx);
void spg_release(spg_graph g);
int spg_sources(int32_t n, const int32_t *row_ptr, int32_t count, int32_t min_degree, uint64_t seed,
                int32_t *out);
int spg_weights(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t lo, int32_t hi,
                uint64_t seed, int32_t *out);
}

static int failures = 0;
#define CHECK(cond, ...)                        \
    do {                                        \
        if (!(cond)) {                          \
            std::printf("FAIL: " __VA_ARGS__);  \
            std::printf("\n");                  \
            ++failures;                         \
        }                                       \
    } while (0)

struct Graph {
    std::vector<int32_t> rp, ci;
    int32_t n() const { return (int32_t)rp.size() - 1; }
};

static Graph take(spg_graph h, const char *what) {
    Graph g;
    int32_t n = 0;
    int64_t nnz = 0;
    CHECK(spg_size(h, &n, &nnz) == 0, "%s: size", what);
    g.rp.resize((size_t)n + 1);
    g.ci.resize((size_t)(nnz > 0 ? nnz : 1));
    CHECK(spg_copy(h, g.rp.data(), g.ci.data()) == 0, "%s: copy", what);
    g.ci.resize((size_t)nnz);
    spg_release(h);
    return g;
}

static Graph from_edges(int32_t n, const std::vector<std::pair<int32_t, int32_t>> &e) {
    std::vector<int32_t> s, d;
    for (auto &p : e) {
        s.push_back(p.first);
        d.push_back(p.second);
    }
    spg_graph h = nullptr;
    CHECK(spg_from_edges(n, (int64_t)e.size(), s.data(), d.data(), &h) == 0, "from_edges");
    return take(h, "from_edges");
}

static void check_csr(const Graph &g, const char *what) {
    const int32_t n = g.n();
    CHECK(g.rp[0] == 0 && (size_t)g.rp[n] == g.ci.size(), "%s: offsets", what);
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = g.rp[v]; e < g.rp[v + 1]; ++e) {
            const int32_t w = g.ci[e];
            CHECK(w != v && w >= 0 && w < n, "%s: entry %d of row %d", what, e, v);
            CHECK(e == g.rp[v] || g.ci[e - 1] < w, "%s: row %d order", what, v);
            bool back = false;
            for (int32_t f = g.rp[w]; f < g.rp[w + 1] && !back; ++f) back = g.ci[f] == v;
            CHECK(back, "%s: %d->%d has no reverse", what, v, w);
        }
}

static void check_bc_sum(const Graph &g, const std::vector<int32_t> &src, const char *what) {
    const int32_t n = g.n();
    std::vector<double> bc((size_t)n), sigma((size_t)n), delta((size_t)n);
    std::vector<int32_t> dist((size_t)n);
    double smax = 0;
    CHECK(oracle_bc(n, g.rp.data(), g.ci.data(), src.data(), (int32_t)src.size(), bc.data(), &smax) == 0,
          "%s: oracle_bc", what);
    double total = 0, want = 0;
    for (double x : bc) total += x;
    for (int32_t s : src) {
        int32_t reached = 0;
        CHECK(oracle_source_detail(n, g.rp.data(), g.ci.data(), s, dist.data(), sigma.data(), delta.data(),
                                   &reached) == 0, "%s: detail", what);
        int32_t cnt = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (dist[v] >= 0) ++cnt;
            if (dist[v] > 0) want += dist[v] - 1;
        }
        CHECK(cnt == reached, "%s: reached count of source %d", what, s);
        // unit weights: Dijkstra gives the BFS distances
        std::vector<int32_t> w(g.ci.size(), 1), d2((size_t)n);
        CHECK(oracle_sssp(n, g.rp.data(), g.ci.data(), w.data(), s, d2.data()) == 0, "%s: sssp", what);
        for (int32_t v = 0; v < n; ++v)
            CHECK(d2[v] == (dist[v] < 0 ? INT32_MAX : dist[v]), "%s: sssp vs bfs at %d", what, v);
    }
    CHECK(std::fabs(total - want) <= 1e-9 * (want > 1 ? want : 1), "%s: global sum %.17g vs %.17g", what,
          total, want);
}

static std::vector<int32_t> all_vertices(int32_t n) {
    std::vector<int32_t> s((size_t)n);
    for (int32_t v = 0; v < n; ++v) s[v] = v;
    return s;
}

int main() {
    // generated graphs
    struct Gen {
        const char *name;
        spg_graph h;
        int32_t min_deg;
    } gens[3] = {{"uniform", nullptr, 0}, {"rmat", nullptr, 1}, {"road", nullptr, 0}};
    CHECK(spg_uniform(2048, 16384, 11, &gens[0].h) == 0, "uniform");
    CHECK(spg_rmat(11, 16, 0.57, 0.19, 0.19, 12, 1, &gens[1].h) == 0, "rmat");
    CHECK(spg_road(48, 0.02, 13, &gens[2].h) == 0, "road");
    for (auto &gen : gens) {
        if (!gen.h) continue;
        Graph g = take(gen.h, gen.name);
        check_csr(g, gen.name);
        std::vector<int32_t> src(24);
        CHECK(spg_sources(g.n(), g.rp.data(), 24, gen.min_deg, 14, src.data()) == 0, "%s: sources", gen.name);
        for (size_t i = 0; i < src.size(); ++i) {
            CHECK(src[i] >= 0 && src[i] < g.n(), "%s: source range", gen.name);
            CHECK(g.rp[src[i] + 1] - g.rp[src[i]] >= gen.min_deg, "%s: source degree", gen.name);
            for (size_t j = 0; j < i; ++j) CHECK(src[i] != src[j], "%s: repeated source", gen.name);
        }
        std::vector<int32_t> w(g.ci.size());
        CHECK(spg_weights(g.n(), g.rp.data(), g.ci.data(), 1, 100, 15, w.data()) == 0, "%s: weights", gen.name);
        for (int32_t v = 0; v < g.n(); ++v)
            for (int32_t e = g.rp[v]; e < g.rp[v + 1]; ++e) {
                const int32_t u = g.ci[e];
                CHECK(w[e] >= 1 && w[e] <= 100, "%s: weight range", gen.name);
                for (int32_t f = g.rp[u]; f < g.rp[u + 1]; ++f)
                    if (g.ci[f] == v) CHECK(w[f] == w[e], "%s: weight of {%d,%d}", gen.name, v, u);
            }
        check_bc_sum(g, src, gen.name);
    }
    // closed forms
    const int32_t n = 9;
    std::vector<std::pair<int32_t, int32_t>> path, star, k6, cyc;
    for (int32_t i = 0; i + 1 < n; ++i) path.push_back({i, i + 1});
    for (int32_t i = 1; i < n; ++i) star.push_back({0, i});
    for (int32_t i = 0; i < 6; ++i)
        for (int32_t j = i + 1; j < 6; ++j) k6.push_back({i, j});
    for (int32_t i = 0; i < 10; ++i) cyc.push_back({i, (i + 1) % 10});
    Graph P = from_edges(n, path), S = from_edges(n, star), K = from_edges(6, k6), C = from_edges(10, cyc);
    for (const Graph *g : {&P, &S, &K, &C}) check_csr(*g, "closed form");
    std::vector<double> bc(n);
    oracle_bc(n, P.rp.data(), P.ci.data(), all_vertices(n).data(), n, bc.data(), nullptr);
    for (int32_t i = 0; i < n; ++i) CHECK(bc[i] == 2.0 * i * (n - 1 - i), "path vertex %d: %g", i, bc[i]);
    oracle_bc(n, S.rp.data(), S.ci.data(), all_vertices(n).data(), n, bc.data(), nullptr);
    CHECK(bc[0] == (double)(n - 1) * (n - 2), "star centre %g", bc[0]);
    for (int32_t i = 1; i < n; ++i) CHECK(bc[i] == 0.0, "star leaf %d", i);
    std::vector<double> bk(6);
    oracle_bc(6, K.rp.data(), K.ci.data(), all_vertices(6).data(), 6, bk.data(), nullptr);
    for (double x : bk) CHECK(x == 0.0, "complete graph BC %g", x);
    std::vector<double> bcy(10);
    oracle_bc(10, C.rp.data(), C.ci.data(), all_vertices(10).data(), 10, bcy.data(), nullptr);
    for (double x : bcy) CHECK(std::fabs(x - 16.0) <= 1e-12, "even cycle BC %g (want ((n-2)/2)^2 = 16)", x);
    check_bc_sum(C, all_vertices(10), "cycle");
    // triangles
    int64_t t = 0;
    CHECK(oracle_tc(6, K.rp.data(), K.ci.data(), &t) == 0 && t == 20, "K_6 triangles %lld", (long long)t);
    Graph R = from_edges(2, {{0, 1}});
    {
        spg_graph h = nullptr;
        CHECK(spg_rmat(10, 16, 0.57, 0.19, 0.19, 16, 1, &h) == 0, "rmat-10");
        R = take(h, "rmat-10");
    }
    std::vector<int64_t> each((size_t)R.n());
    int64_t total = 0, sum = 0;
    CHECK(oracle_tc(R.n(), R.rp.data(), R.ci.data(), &total) == 0, "tc");
    CHECK(oracle_tc_each(R.n(), R.rp.data(), R.ci.data(), each.data()) == 0, "tc_each");
    for (int32_t v = 0; v < R.n(); ++v) {
        sum += each[v];
        if (v % 97 == 0) {
            int64_t one = -1;
            CHECK(oracle_tc_vertex(R.n(), R.rp.data(), R.ci.data(), v, &one) == 0 && one == each[v],
                  "tc_vertex %d", v);
        }
    }
    CHECK(sum == 3 * total, "per-vertex triangles %lld vs 3 x %lld", (long long)sum, (long long)total);
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitizer driver ok\n");
    return 0;
}
