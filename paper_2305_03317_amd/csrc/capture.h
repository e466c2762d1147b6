// Chunks of level or round kernels captured once as HIP graphs and replayed:
// the host submits one graph per chunk instead of a launch per kernel.
#pragma once

#include "common.h"

namespace sp {

// Replay `slot` on stream s, first capturing it (on the private stream
// *cap_stream, created on first use) when it is empty or was captured under
// another key.  enqueue(stream) issues the chunk's launches; the key holds
// every launch parameter the captured kernels depend on, so a stale graph is
// never replayed.
template <class Enqueue>
sp_status replay_captured(hipStream_t *cap_stream, CapturedChunk &slot,
                          const std::array<long long, 12> &key, Enqueue enqueue, hipStream_t s) {
    if (!slot.exec || slot.key != key) {
        if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        slot.exec = nullptr;
        if (!*cap_stream) SP_HIP(hipStreamCreateWithFlags(cap_stream, hipStreamNonBlocking));
        SP_HIP(hipStreamBeginCapture(*cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue(*cap_stream);
        const hipError_t el = hipGetLastError();
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(*cap_stream, &graph);
        hipError_t ei = hipSuccess;
        if (el == hipSuccess && ec == hipSuccess)
            ei = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (el != hipSuccess || ec != hipSuccess || ei != hipSuccess) {
            slot.exec = nullptr;
            set_error("capturing a chunk of kernels failed: %s",
                      hipGetErrorString(el != hipSuccess ? el : ec != hipSuccess ? ec : ei));
            return SP_ERR_DEVICE;
        }
        slot.key = key;
    }
    SP_HIP(hipGraphLaunch(slot.exec, s));
    return SP_OK;
}

}  // namespace sp
