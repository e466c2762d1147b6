// Serving loop: placeholder entry points (filled in by the continuous-batching
// scheduler).
#include "common.h"

using namespace sp;

extern "C" {

sp_status sp_autotune(sp_graph g, const int32_t *sources, int32_t n_sources, sp_batch_config *out,
                      sp_stream s) {
    (void)g; (void)sources; (void)n_sources; (void)out; (void)s;
    set_error("sp_autotune: not available yet");
    return SP_ERR_NOT_SUPPORTED;
}

sp_status sp_server_create(const sp_server_config *cfg, sp_server *out) {
    (void)cfg; (void)out;
    set_error("serving: not available yet");
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_server_add_graph(sp_server srv, sp_graph g, int32_t *graph_id) {
    (void)srv; (void)g; (void)graph_id;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_stream_submit(sp_server srv, int32_t graph_id, const int32_t *sources, int32_t n_sources,
                           double *out_bc, sp_request *out_req) {
    (void)srv; (void)graph_id; (void)sources; (void)n_sources; (void)out_bc; (void)out_req;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_request_wait(sp_request r, int64_t timeout_us, sp_status *result) {
    (void)r; (void)timeout_us; (void)result;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_request_poll(sp_request r, int32_t *done, sp_status *result) {
    (void)r; (void)done; (void)result;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_request_cancel(sp_request r) { (void)r; return SP_ERR_NOT_SUPPORTED; }
sp_status sp_request_latency_us(sp_request r, double *latency_us) {
    (void)r; (void)latency_us;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_request_release(sp_request r) { (void)r; return SP_ERR_NOT_SUPPORTED; }
sp_status sp_server_get_stats(sp_server srv, sp_server_stats *out) {
    (void)srv; (void)out;
    return SP_ERR_NOT_SUPPORTED;
}
sp_status sp_server_destroy(sp_server srv) { (void)srv; return SP_ERR_NOT_SUPPORTED; }

}  // extern "C"
