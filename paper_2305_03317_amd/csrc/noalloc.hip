// Allocation-free per-source BC: sp_bc's computation with its workspace in a
// fixed device array instead of memory the library allocates, for callers that
// cannot allocate device memory while they run.
//
// The array `scratch` is a file-scope device variable, so the code object
// loader places it in device memory once per GPU; it stays there until the
// process ends.  Host code never passes its name to a kernel (in host code the
// name is a host-side shadow, not a device address): the device address is
// looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_dev[device].
//
// The workspace carved from it is sp_bc's (distances, path counts,
// dependencies, BFS-order queue, level offsets, hub lists, hub chunk partial
// sums, level control block); the kernels are the same, so the results are
// bit-identical to sp_bc's.  Nothing in it has to start at zero: every pass
// initialises what it reads (distances filled with -1, the control block and
// first level written by the init kernel, every other value written before it
// is read), so the previous call's contents are never observed.
//
// One array per GPU serves every call on that GPU.  A per-device mutex held
// for the whole call (which synchronises its stream before returning) keeps
// calls from host threads on one GPU from overlapping.
#include "common.h"

namespace sp {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu[kMaxScratchDevices];
static unsigned char *g_scratch_dev[kMaxScratchDevices];  // device address, per device
static LevelCtl g_ctl_host[kMaxScratchDevices];           // host mirror of the control block

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves sp_bc's workspace for graph g from [base, base + kScratchBytes);
// returns the bytes it needs (base may be null to only measure).
static size_t carve(sp_graph g, unsigned char *base, SourceWorkspace &ws) {
    const size_t n = (size_t)std::max(g->n, 1);
    const size_t lv = n + 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return (void *)p;
    };
    ws.device = g->device;
    ws.n = g->n;
    ws.dist = (int32_t *)take(n * sizeof(int32_t));
    ws.sigma = (double *)take(n * sizeof(double));
    ws.delta = (double *)take(n * sizeof(double));
    ws.queue = (int32_t *)take(n * sizeof(int32_t));
    ws.level_cap = (int32_t)lv;
    ws.level_off = (int32_t *)take(lv * sizeof(int32_t));
    ws.hub_off = (int32_t *)take(lv * sizeof(int32_t));
    ws.hub_lvl_chunks = (int32_t *)take(lv * sizeof(int32_t));
    ws.hub_list = (HubEntry *)take(((size_t)g->n_hubs + 1) * sizeof(HubEntry));
    ws.in_hub_list = (HubEntry *)take(((size_t)g->n_hubs_in + 1) * sizeof(HubEntry));
    ws.hub_cnt = (unsigned int *)take(((size_t)g->n_hubs + 1) * sizeof(unsigned int));
    ws.partial = (double *)take(
        ((size_t)std::max(g->split_hub_chunks, g->split_hub_chunks_in) + 1) * sizeof(double));
    ws.ctl = (LevelCtl *)take(sizeof(LevelCtl));
    ws.ctl_host = nullptr;
    ws.ev0 = ws.ev1 = nullptr;  // no events: the call synchronises its stream instead
    return off;
}

// The device address of `scratch` on the current device (looked up on the
// first call there).  Caller holds g_scratch_mu[dev].
static sp_status scratch_address(int dev, unsigned char **out) {
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return SP_ERR_DEVICE;
        }
        g_scratch_dev[dev] = (unsigned char *)p;
    }
    *out = g_scratch_dev[dev];
    return SP_OK;
}

}  // namespace sp

using namespace sp;

extern "C" {

sp_status sp_bc_noalloc(sp_graph g, const int32_t *sources, int32_t n_sources, double *out_bc,
                        sp_stream s) {
    try {
        clear_error();
        SP_TRY(check_bc_args(g, sources, n_sources, out_bc, "sp_bc_noalloc"));
        sp_stats stats{};
        stats.n_sources = n_sources;
        if (g->n == 0) {
            tls_stats() = stats;
            return SP_OK;
        }
        SourceWorkspace ws;
        const size_t need = carve(g, nullptr, ws);
        if (need > kScratchBytes) {
            set_error("sp_bc_noalloc: graph needs %zu bytes of workspace, above the fixed %zu "
                      "(about 40 bytes per vertex; use sp_bc)", need, kScratchBytes);
            return SP_ERR_INVALID_ARGUMENT;
        }
        if (g->device < 0 || g->device >= kMaxScratchDevices) {
            set_error("sp_bc_noalloc: device %d outside [0, %d)", g->device, kMaxScratchDevices);
            return SP_ERR_NOT_SUPPORTED;
        }
        if (prof_enabled()) {  // kernel profiling creates events, i.e. allocates
            set_error("sp_bc_noalloc: not available while kernel profiling is on");
            return SP_ERR_NOT_SUPPORTED;
        }
        DeviceGuard dg(g->device);
        std::lock_guard<std::mutex> lk(g_scratch_mu[g->device]);
        unsigned char *base = nullptr;
        SP_TRY(scratch_address(g->device, &base));
        carve(g, base, ws);
        ws.ctl_host = &g_ctl_host[g->device];
        const sp_status rc = bc_per_source(g, ws, sources, n_sources, out_bc, (hipStream_t)s, &stats);
        if (rc >= 0) tls_stats() = stats;
        return rc;
    } catch (...) {
        set_error("unexpected C++ exception");
        return SP_ERR_DEVICE;
    }
}

}  // extern "C"
