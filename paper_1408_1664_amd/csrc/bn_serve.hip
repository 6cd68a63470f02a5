// Serving entry points (filled in by the continuous-batching server).
#include <hip/hip_runtime.h>

#include "../../include/bn.h"

extern "C" {
bn_status bn_server_create(size_t, int32_t, void **server) {
    if (server) *server = nullptr;
    return BN_EINTERNAL;
}
bn_status bn_serve_submit(void *, const bn_problem *, bn_precision, uint64_t *) {
    return BN_EINTERNAL;
}
bn_status bn_serve_poll(void *, uint64_t, double *, bn_report *, int32_t) { return BN_EINTERNAL; }
bn_status bn_server_destroy(void *) { return BN_EINTERNAL; }
}
