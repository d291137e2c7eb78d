// Split-BF16 x3 path sum (placeholder until the MFMA kernel lands).
#include <hip/hip_runtime.h>

#include "device.h"

namespace hsf {

hsf_status path_sum_bf16x3(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                           int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st) {
    (void)A; (void)ldA; (void)B; (void)ldB; (void)K; (void)M; (void)N; (void)out; (void)ldo; (void)accumulate;
    (void)ws; (void)st;
    return fail(HSF_E_UNSUPPORTED, "HSF_SUM_BF16X3 not built yet");
}

}  // namespace hsf
