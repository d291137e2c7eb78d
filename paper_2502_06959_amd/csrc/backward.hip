// Adjoint gradient of a probability-mass loss (placeholder).
#include <hip/hip_runtime.h>

#include "device.h"

namespace hsf {

size_t backward_workspace(const Plan& p, int64_t chunk) {
    (void)p;
    (void)chunk;
    return 0;
}

hsf_status backward(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, double* grad, int64_t n_params,
                    int64_t chunk, void* ws, size_t ws_bytes, hipStream_t stream) {
    (void)p; (void)d; (void)x; (void)nx; (void)grad; (void)n_params; (void)chunk; (void)ws; (void)ws_bytes;
    (void)stream;
    return fail(HSF_E_UNSUPPORTED, "hsf_backward not built yet");
}

}  // namespace hsf
