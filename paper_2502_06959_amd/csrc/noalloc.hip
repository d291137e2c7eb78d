// hsf_amplitudes_full_noalloc: the path sum of hsf_amplitudes_full with its
// scratch (the split-BF16 planes of HSF_SUM_BF16X3) in a static device array
// of the library instead of a caller workspace, for callers that cannot
// allocate device memory (code under graph capture, serving loops).  Every
// call on one device shares that device's array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.h"

// The scratch array.  In host code its name is a host-side stand-in, not a
// device address: kernels and copies get the per-device address that
// hipGetSymbolAddress returns, never `scratch` itself.
static __device__ __align__(256) unsigned char scratch[HSF_NOALLOC_SCRATCH_BYTES];

namespace hsf {
namespace {

constexpr size_t kScratchBytes = HSF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per
// device with that device current.
hsf_status scratch_address(void** out) {
    int dev = 0;
    hsf_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (s != HSF_OK) return s;
    if (dev < 0 || dev >= kMaxDevices) return fail(HSF_E_DEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        s = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (s != HSF_OK) return s;
        if (!ptr) return fail(HSF_E_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HSF_OK;
}

}  // namespace
}  // namespace hsf

extern "C" {

hsf_status hsf_amplitudes_full_noalloc(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB,
                                       int64_t ldB, int64_t n_paths, int64_t row_begin, int64_t row_end, void* out,
                                       int64_t ldo, int32_t mode, int32_t accumulate, hsf_stream_t stream) {
    using namespace hsf;
    try {
        if (!plan) return fail(HSF_E_ARG, "null plan");
        if (mode == HSF_SUM_BF16X3_SPLIT)
            return fail(HSF_E_ARG, "HSF_SUM_BF16X3_SPLIT reads the caller's planes: use hsf_amplitudes_full");
        if (n_paths < 0) return fail(HSF_E_ARG, "negative path count");
        const Plan* p = reinterpret_cast<const Plan*>(plan);
        if (mode == HSF_SUM_BF16X3 && bf16x3_workspace(p->na, p->nb, n_paths) > kScratchBytes)
            return fail(HSF_E_ARG, "split-BF16 planes of n_paths x (2^n_a + 2^n_b) values exceed the static scratch (" +
                                       std::to_string(kScratchBytes >> 20) + " MiB): use hsf_amplitudes_full with a "
                                       "workspace, or fewer paths per call with accumulate = 1");
        void* ws = nullptr;
        hsf_status s = scratch_address(&ws);
        if (s != HSF_OK) return s;
        return amplitudes_full(plan, psiA, ldA, psiB, ldB, n_paths, row_begin, row_end, out, ldo, mode, accumulate,
                               ws, kScratchBytes, (hipStream_t)stream);
    } catch (const std::exception& e) {
        return fail(HSF_E_ARG, std::string("internal error: ") + e.what());
    }
}

}  // extern "C"
