// Kernel timing for measurement: HIP events recorded on the launch stream
// immediately before and after each launch of a kernel family
// (SP_PROFILE_TIMES), and device counters of the work each family did
// (SP_PROFILE_COUNTS).  The counters add reductions to the kernels, so the two
// are best taken in separate runs.  Off unless sp_profile_enable.
#include <atomic>
#include <vector>

#include "common.h"

namespace sp {

const char *const kProfNames[P_COUNT] = {
    "src_topdown", "src_bottomup", "src_sigma", "src_sigma_hub", "src_delta", "src_delta_hub",
    "ms_topdown", "ms_bottomup", "ms_sigma", "ms_sigma_hub", "ms_expand", "ms_delta", "ms_delta_hub",
    "ms_bc", "sssp_push", "sssp_pull", "pr_pull", "pr_hub", "tc_count", "wg_bc",
    "ms_sigma_push",
};

namespace {
std::atomic<int> g_on{0};  // SP_PROFILE_* bits
std::mutex g_mu;
struct Pending {
    int kind;
    hipEvent_t a, b;
};
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
long long g_launches[P_COUNT];
double g_ms[P_COUNT];
unsigned long long *g_counters[64];  // per device: P_COUNT x kProfCounters

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // Timing only: without the system-scope fence an event record does not
    // write back and invalidate the caches, which would slow the next kernel.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool prof_enabled() { return g_on.load(std::memory_order_relaxed) != 0; }

unsigned long long *prof_counters(int kind) {
    if (!(g_on.load(std::memory_order_relaxed) & SP_PROFILE_COUNTS)) return nullptr;
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_counters[d]) {
        void *p = nullptr;
        const size_t bytes = sizeof(unsigned long long) * P_COUNT * kProfCounters;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        if (hipMemset(p, 0, bytes) != hipSuccess) return nullptr;
        g_counters[d] = (unsigned long long *)p;
    }
    return g_counters[d] + (size_t)kind * kProfCounters;
}

ProfScope::ProfScope(int kind, hipStream_t s) : kind_(kind), s_(s) {
    const int on = g_on.load(std::memory_order_relaxed);
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_launches[kind]++;
    if (!(on & SP_PROFILE_TIMES)) return;
    a_ = take_event();
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (b && hipEventRecord(b, s_) == hipSuccess) g_pending.push_back({kind_, a_, b});
}

}  // namespace sp

using namespace sp;

extern "C" {

sp_status sp_profile_enable(int32_t what) {
    if (what & ~(int32_t)(SP_PROFILE_TIMES | SP_PROFILE_COUNTS)) {
        set_error("sp_profile_enable: unknown bits 0x%x", (unsigned)what);
        return SP_ERR_INVALID_ARGUMENT;
    }
    g_on.store(what);
    return SP_OK;
}

sp_status sp_profile_read(sp_kernel_profile *out, int32_t cap, int32_t *n_out) {
    if (!n_out || cap < 0 || (cap > 0 && !out)) {
        set_error("sp_profile_read: bad arguments");
        return SP_ERR_INVALID_ARGUMENT;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
            g_ms[p.kind] += ms;
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    unsigned long long cnt[P_COUNT * kProfCounters] = {0};
    int d = 0;
    if (hipGetDevice(&d) == hipSuccess && d >= 0 && d < 64 && g_counters[d]) {
        SP_HIP(hipDeviceSynchronize());
        SP_HIP(hipMemcpy(cnt, g_counters[d], sizeof cnt, hipMemcpyDeviceToHost));
        SP_HIP(hipMemset(g_counters[d], 0, sizeof cnt));
    }
    int32_t n = 0;
    for (int k = 0; k < P_COUNT; ++k) {
        if (!g_launches[k]) continue;
        if (n < cap) {
            sp_kernel_profile &o = out[n];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, kProfNames[k], sizeof o.name - 1);
            o.launches = g_launches[k];
            o.total_ms = g_ms[k];
            o.items = (int64_t)cnt[k * kProfCounters + 0];
            o.edges = (int64_t)cnt[k * kProfCounters + 1];
            o.pairs = (int64_t)cnt[k * kProfCounters + 2];
            o.item_slots = (int64_t)cnt[k * kProfCounters + 3];
        }
        ++n;
        g_launches[k] = 0;
        g_ms[k] = 0;
    }
    *n_out = std::min(n, cap);
    return SP_OK;
}

}  // extern "C"
