// Device-side output epilogue of the MFMA path sums (HIP sources only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hsf {

// Epilogue shared by the FP32 and split-BF16 path sums: a 128 x 128 complex
// workgroup tile held as MFMA accumulators (4 waves in 2 x 2, each 2 x 2
// blocks of 32x32; accumulator r of a block sits at row (r/4)*8 +
// (lane/32)*4 + r%4, column lane%32) is stored straight from registers: each
// store writes two 256-byte row segments.  Rows >= M and columns >= N are
// skipped; accumulate adds the old contents.
using f32x16_t = float __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void store_tile_128(const f32x16_t (&cr)[2][2], const f32x16_t (&ci)[2][2],
                                               int64_t row0, int64_t col0, int64_t M, int64_t N,
                                               float2* __restrict__ out, int64_t ldo, int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t m0 = row0 + (w >> 1) * 64, n0 = col0 + (w & 1) * 64;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t col = n0 + b * 32 + li;
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + a * 32 + (r >> 2) * 8 + lk * 4 + (r & 3);
                if (row >= M) continue;
                float2 v = make_float2(cr[a][b][r], ci[a][b][r]);
                float2* o = out + row * ldo + col;
                if (accumulate) {
                    const float2 old = *o;
                    v.x += old.x;
                    v.y += old.y;
                }
                *o = v;
            }
        }
}

}  // namespace hsf
