// Path sum (Sec. II-B: Kronecker products of the two half-states, summed over
// paths).  With side a as rows and side b as columns the full state is the
// complex product C = PsiA^T PsiB (PsiA is paths x 2^n_a, PsiB paths x 2^n_b),
// so the sum is a dense contraction over the path index and runs on MFMA:
// real and imaginary parts are separate MFMA operands, accumulated in FP32
// (or FP64), and the epilogue writes interleaved complex output.  Also here:
// amplitudes of chosen bitstrings and FP64-accumulated norms.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "epilogue.h"

namespace hsf {

namespace {

using f32x16 = f32x16_t;
using f64x4 = double __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- FP32 ----
// Workgroup: 4 waves in a 2 x 2 grid, each wave 64 x 64 complex outputs made
// of 2 x 2 blocks of the 32x32x2 FP32 MFMA; per block four products:
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.  Operands stream straight from
// global memory: for one path index the 32 lanes of a half-wave read 32
// consecutive complex entries (256 contiguous bytes).
constexpr int F32_TILE = 128;

__device__ __forceinline__ void f32_tile(const float2* __restrict__ A, int64_t ldA, const float2* __restrict__ B,
                                         int64_t ldB, int64_t K, int64_t M, int64_t N, float2* __restrict__ out,
                                         int64_t ldo, int accumulate, int64_t row0, int64_t col0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t m0 = row0 + (w >> 1) * 64;
    const int64_t n0 = col0 + (w & 1) * 64;
    f32x16 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = (f32x16)0.0f;
            ci[a][b] = (f32x16)0.0f;
        }
    bool mok[2], nok[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        mok[a] = m0 + a * 32 + li < M;
        nok[a] = n0 + a * 32 + li < N;
    }
    auto load = [&](int64_t k, float2 (&av)[2], float2 (&bv)[2]) {
        const bool kok = k < K;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            av[a] = (kok && mok[a]) ? A[k * ldA + m0 + a * 32 + li] : make_float2(0.f, 0.f);
            bv[a] = (kok && nok[a]) ? B[k * ldB + n0 + a * 32 + li] : make_float2(0.f, 0.f);
        }
    };
    float2 av[2], bv[2];
    load(lk, av, bv);
    for (int64_t k0 = 0; k0 < K; k0 += 2) {
        float2 an[2], bn[2];
        load(k0 + 2 + lk, an, bn);   // prefetch the next path pair
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, -bv[b].y, cr[a][b], 0, 0, 0);
                ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
            }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            av[a] = an[a];
            bv[a] = bn[a];
        }
    }
    store_tile_128(cr, ci, row0, col0, M, N, out, ldo, accumulate);
}

// Persistent over 128 x 128 output tiles (see the split-BF16 kernel).
__global__ __launch_bounds__(256) void pathsum_f32(const float2* __restrict__ A, int64_t ldA,
                                                   const float2* __restrict__ B, int64_t ldB, int64_t K,
                                                   int64_t M, int64_t N, float2* __restrict__ out, int64_t ldo,
                                                   int accumulate, int64_t tiles_n, int64_t tiles) {
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
        f32_tile(A, ldA, B, ldB, K, M, N, out, ldo, accumulate, tm * F32_TILE, tn * F32_TILE);
    }
}

// Persistent over the union of all circuits' output tiles.
__global__ __launch_bounds__(256) void pathsum_f32_batch(const GemmDesc* __restrict__ d, int n, unsigned char* base,
                                                         int64_t tiles) {
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].tile_start <= tile) lo = mid;
            else hi = mid - 1;
        }
        const GemmDesc& g = d[lo];
        const int64_t local = tile - g.tile_start;
        const int64_t tm = local / g.tiles_n, tn = local - tm * g.tiles_n;
        f32_tile(reinterpret_cast<const float2*>(base + g.a_off), g.ldA,
                 reinterpret_cast<const float2*>(base + g.b_off), g.ldB, g.K, g.M, g.N, (float2*)g.out, g.ldo, 0,
                 tm * F32_TILE, tn * F32_TILE);
    }
}

// Row panels: at most 32 output rows (the first amplitudes of a large state)
// against every column.  The sum is then bound by reading PsiB once (each of
// its entries meets only the panel's rows), so the operands go straight from
// global memory into FP32 MFMAs, with no split planes and no LDS: each wave
// owns the panel x 32 columns as one 32x32x2 block per product (rows past M
// read as zero), its operands prefetched R_DEPTH path pairs ahead.
constexpr int R_COLS = 128;   // columns per workgroup (4 waves)
constexpr int R_DEPTH = 16;

__global__ __launch_bounds__(256) void pathsum_f32_rows(const float2* __restrict__ A, int64_t ldA,
                                                        const float2* __restrict__ B, int64_t ldB, int64_t K,
                                                        int64_t M, int64_t N, float2* __restrict__ out, int64_t ldo,
                                                        int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t n0 = (int64_t)blockIdx.x * R_COLS + w * 32;
    if (n0 >= N) return;
    const bool mok = li < M, nok = n0 + li < N;
    f32x16 cr = (f32x16)0.0f, ci = (f32x16)0.0f;
    float2 av[R_DEPTH], bv[R_DEPTH];
    const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
    for (int d = 0; d < R_DEPTH; ++d) {
        const int64_t k = 2 * d + lk;
        av[d] = (k < K && mok) ? A[k * ldA + li] : zero;
        bv[d] = (k < K && nok) ? B[k * ldB + n0 + li] : zero;
    }
    for (int64_t k0 = 0; k0 < K; k0 += 2 * R_DEPTH) {
#pragma unroll
        for (int d = 0; d < R_DEPTH; ++d) {
            const float2 a = av[d], b = bv[d];
            const int64_t kn = k0 + 2 * (d + R_DEPTH) + lk;
            av[d] = (kn < K && mok) ? A[kn * ldA + li] : zero;
            bv[d] = (kn < K && nok) ? B[kn * ldB + n0 + li] : zero;
            cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, -b.y, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, ci, 0, 0, 0);
        }
    }
    if (!nok) return;
    // accumulator r sits at row (r/4)*8 + (lane/32)*4 + r%4, column lane%32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t row = (r >> 2) * 8 + lk * 4 + (r & 3);
        if (row >= M) continue;
        float2 v = make_float2(cr[r], ci[r]);
        float2* o = out + row * ldo + n0 + li;
        if (accumulate) {
            const float2 old = *o;
            v.x += old.x;
            v.y += old.y;
        }
        *o = v;
    }
}

// Panels of at most 16 rows on the 16x16x4 FP32 MFMA (16 rows x 16 columns,
// four paths per instruction: half the MFMA work of a 32-row block): each
// wave owns 32 columns as two blocks, path quads prefetched R16_DEPTH ahead.
// Lane l supplies A row l%16 and B column l%16 of path l/16; accumulator r
// of a block sits at row 4 (l/16) + r, column l%16.
constexpr int R16_DEPTH = 16;
using f32x4 = float __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void pathsum_f32_rows16(const float2* __restrict__ A, int64_t ldA,
                                                          const float2* __restrict__ B, int64_t ldB, int64_t K,
                                                          int64_t M, int64_t N, float2* __restrict__ out,
                                                          int64_t ldo, int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t n0 = (int64_t)blockIdx.x * R_COLS + w * 32;
    if (n0 >= N) return;
    const bool mok = li < M;
    bool nok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) nok[b] = n0 + b * 16 + li < N;
    f32x4 cr[2], ci[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) cr[b] = ci[b] = (f32x4)0.0f;
    float2 av[R16_DEPTH], bv[R16_DEPTH][2];
    const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
    for (int d = 0; d < R16_DEPTH; ++d) {
        const int64_t k = 4 * d + lq;
        av[d] = (k < K && mok) ? A[k * ldA + li] : zero;
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[d][b] = (k < K && nok[b]) ? B[k * ldB + n0 + b * 16 + li] : zero;
    }
    for (int64_t k0 = 0; k0 < K; k0 += 4 * R16_DEPTH) {
#pragma unroll
        for (int d = 0; d < R16_DEPTH; ++d) {
            const float2 a = av[d], b0 = bv[d][0], b1 = bv[d][1];
            const int64_t kn = k0 + 4 * (d + R16_DEPTH) + lq;
            av[d] = (kn < K && mok) ? A[kn * ldA + li] : zero;
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[d][b] = (kn < K && nok[b]) ? B[kn * ldB + n0 + b * 16 + li] : zero;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float2 bb = b ? b1 : b0;
                cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, cr[b], 0, 0, 0);
                cr[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, -bb.y, cr[b], 0, 0, 0);
                ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.y, ci[b], 0, 0, 0);
                ci[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, ci[b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        if (!nok[b]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = 4 * lq + r;
            if (row >= M) continue;
            float2 v = make_float2(cr[b][r], ci[b][r]);
            float2* o = out + row * ldo + n0 + b * 16 + li;
            if (accumulate) {
                const float2 old = *o;
                v.x += old.x;
                v.y += old.y;
            }
            *o = v;
        }
    }
}

// ---------------------------------------------------------------- FP64 ----
// Same structure on the 16x16x4 FP64 MFMA: wave 32 x 32 outputs (2 x 2
// blocks), workgroup 64 x 64.  Inputs are c128, or c64 widened on load.
constexpr int F64_TILE = 64;

template <typename VIN>
__device__ __forceinline__ double2 widen(VIN v) {
    return make_double2((double)v.x, (double)v.y);
}

template <typename VIN>
__global__ __launch_bounds__(256) void pathsum_f64(const VIN* __restrict__ A, int64_t ldA,
                                                   const VIN* __restrict__ B, int64_t ldB, int64_t K,
                                                   int64_t M, int64_t N, double2* __restrict__ out,
                                                   int64_t ldo, int accumulate) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * F64_TILE + (w >> 1) * 32;
    const int64_t n0 = (int64_t)blockIdx.x * F64_TILE + (w & 1) * 32;
    f64x4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = (f64x4)0.0;
            ci[a][b] = (f64x4)0.0;
        }
    bool mok[2], nok[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        mok[a] = m0 + a * 16 + li < M;
        nok[a] = n0 + a * 16 + li < N;
    }
    for (int64_t k0 = 0; k0 < K; k0 += 4) {
        const int64_t k = k0 + lk;
        const bool kok = k < K;
        double2 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            av[a] = (kok && mok[a]) ? widen(A[k * ldA + m0 + a * 16 + li]) : make_double2(0.0, 0.0);
            bv[a] = (kok && nok[a]) ? widen(B[k * ldB + n0 + a * 16 + li]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, -bv[b].y, cr[a][b], 0, 0, 0);
                ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
            }
    }
    // accumulator r of a 16x16 FP64 block: row lane/16 + 4*r, column lane%16
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t col = n0 + b * 16 + li;
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + a * 16 + lk + 4 * r;
                if (row >= M) continue;
                double2 v = make_double2(cr[a][b][r], ci[a][b][r]);
                double2* o = out + row * ldo + col;
                if (accumulate) {
                    const double2 old = *o;
                    v.x += old.x;
                    v.y += old.y;
                }
                *o = v;
            }
        }
}

// ------------------------------------------------------------ gather-dot ----
// One wave per requested basis state; lanes stride over paths, FP64
// accumulation, fixed-order butterfly reduction (deterministic).
template <typename VIN>
__global__ __launch_bounds__(256) void gather_dot_kernel(const VIN* __restrict__ A, int64_t ldA,
                                                         const VIN* __restrict__ B, int64_t ldB, int64_t K,
                                                         int nb, int n, const uint64_t* __restrict__ x, int64_t nx,
                                                         double2* __restrict__ out, int accumulate, int64_t rsA,
                                                         int64_t rsB) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= nx) return;
    // copy blockIdx.y of replicated half-states (strides rsA, rsB elements), its own nx outputs
    A += (int64_t)blockIdx.y * rsA;
    B += (int64_t)blockIdx.y * rsB;
    out += (int64_t)blockIdx.y * nx;
    // index bits at or above n are ignored, so every read stays inside the half-states
    const uint64_t xj = x[j] & ((n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1));
    const int64_t ia = (int64_t)(xj >> nb);
    const int64_t ib = (int64_t)(xj & ((uint64_t(1) << nb) - 1));
    double re = 0.0, im = 0.0;
    for (int64_t p = lane; p < K; p += 64) {
        const double2 a = widen(A[p * ldA + ia]);
        const double2 b = widen(B[p * ldB + ib]);
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        re += __shfl_xor(re, s, 64);
        im += __shfl_xor(im, s, 64);
    }
    if (lane == 0) {
        if (accumulate) {
            re += out[j].x;
            im += out[j].y;
        }
        out[j] = make_double2(re, im);
    }
}

// ------------------------------------------------------------------ norms ----
constexpr int NORM_BLOCKS = 4096;

// Rows of the empty sum (no paths): `rows` rows of `cols` 8-byte words, row
// stride `ld` words, set to zero.
__global__ __launch_bounds__(256) void zero_rows(uint2* __restrict__ out, int64_t ld, int64_t rows, int64_t cols) {
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / cols;
        out[r * ld + (i - r * cols)] = make_uint2(0u, 0u);
    }
}

template <typename VA, typename VB, bool HAS_B>
__global__ __launch_bounds__(256) void norm_partial(const VA* __restrict__ a, const VB* __restrict__ b, int64_t n,
                                                    double* __restrict__ part) {
    double s1 = 0.0, s2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 av = widen(a[i]);
        s1 += av.x * av.x + av.y * av.y;
        if constexpr (HAS_B) {
            const double2 bv = widen(b[i]);
            const double dx = av.x - bv.x, dy = av.y - bv.y;
            s2 += dx * dx + dy * dy;
        }
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r1[0];
        part[2 * blockIdx.x + 1] = r2[0];
    }
}

__global__ __launch_bounds__(256) void norm_final(const double* __restrict__ part, int nblocks, double* __restrict__ out) {
    __shared__ double r1[256], r2[256];
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) {
        s1 += part[2 * i];
        s2 += part[2 * i + 1];
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r1[0];
        out[1] = r2[0];
    }
}

template <typename VA, typename VB, bool HAS_B>
hsf_status launch_norm(const void* a, const void* b, int64_t n, double* out, double* ws, hipStream_t st) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(NORM_BLOCKS, (n + 1023) / 1024));
    hipLaunchKernelGGL((norm_partial<VA, VB, HAS_B>), dim3(blocks), dim3(256), 0, st, (const VA*)a,
                       (const VB*)b, n, ws);
    hipLaunchKernelGGL(norm_final, dim3(1), dim3(256), 0, st, (const double*)ws, blocks, out);
    return hip_check(hipGetLastError(), "norm launch");
}

}  // namespace

int persistent_grid(const void* kernel, int threads, size_t shmem, int64_t tiles) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, shmem) != hipSuccess || per < 1) per = 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cus * per));
}

hsf_status launch_f32_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st) {
    const int grid = persistent_grid((const void*)pathsum_f32_batch, 256, 0, tiles);
    hipLaunchKernelGGL(pathsum_f32_batch, dim3(grid), dim3(256), 0, st, (const GemmDesc*)descs, n, base, tiles);
    return hip_check(hipGetLastError(), "pathsum_f32_batch launch");
}

size_t bf16x3_workspace(int na, int nb, int64_t n_paths) {
    // hi and lo BF16 planes of the real and imaginary parts of both operands,
    // paths padded to a multiple of 32 (the streaming kernel pads to 16, the
    // LDS-staged one to 32)
    const size_t kp = (size_t)std::max<int64_t>(32, (n_paths + 31) / 32 * 32);
    return kp * ((size_t(1) << na) + (size_t(1) << nb)) * 4 * sizeof(uint16_t) + 256;
}

hsf_status path_sum_bf16x3(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                           int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st);

// The planes of A (MA rows) start at the 256-byte aligned workspace and B's
// follow; the layout is the one the path sum of K paths takes.
hsf_status split_operands(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N,
                          int64_t K, void* ws, hipStream_t st) {
    unsigned short* PA = reinterpret_cast<unsigned short*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    if (path_sum_lds_fits(HSF_SUM_BF16X3, A, ldA, B, ldB, K, MA, N))
        return split_lds(A, ldA, MA, B, ldB, N, K, PA, PA + bf16x3_lds_planes(MA, K) / sizeof(uint16_t), st);
    return split_stream(A, ldA, MA, B, ldB, N, K, PA, PA + bf16x3_stream_planes(MA, K) / sizeof(uint16_t), st);
}

hsf_status path_sum_presplit(int64_t K, int64_t MA, int64_t row0, int64_t M, int64_t N, void* ws, float2* out,
                             int64_t ldo, int accumulate, hipStream_t st) {
    const unsigned short* PA = reinterpret_cast<const unsigned short*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    if (path_sum_lds_fits(HSF_SUM_BF16X3, nullptr, 0, nullptr, 0, K, MA, N))
        return sum_lds(PA, MA, row0, M, PA + bf16x3_lds_planes(MA, K) / sizeof(uint16_t), N, K, out, ldo, accumulate,
                       st);
    return sum_stream(PA, MA, row0, M, PA + bf16x3_stream_planes(MA, K) / sizeof(uint16_t), N, K, out, ldo, accumulate,
                      st);
}

hsf_status path_sum(int dtype, int mode, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K,
                    int64_t row0, int64_t M, int64_t N, void* out, int64_t ldo, int accumulate, void* ws,
                    hipStream_t st) {
    if (K == 0) {
        // the sum over no paths: zero rows, nothing to add when accumulating;
        // the operands are not read
        if (accumulate) return HSF_OK;
        const int64_t words = (mode == HSF_SUM_F64 || mode == HSF_SUM_C128) ? 2 : 1;
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (M * N * words + 255) / 256));
        hipLaunchKernelGGL(zero_rows, dim3((uint32_t)blocks), dim3(256), 0, st, (uint2*)out, ldo * words, M, N * words);
        return hip_check(hipGetLastError(), "zero_rows launch");
    }
    if (dtype == HSF_C64 && (mode == HSF_SUM_F32 || mode == HSF_SUM_BF16X3) && M <= 32) {
        // a row panel: FP32 products straight from the half-states (no split)
        const int64_t grid = (N + R_COLS - 1) / R_COLS;
        if (grid > 0x7fffffff) return fail(HSF_E_ARG, "too many output columns in one call");
        if (M <= 16)
            hipLaunchKernelGGL(pathsum_f32_rows16, dim3((uint32_t)grid), dim3(256), 0, st, (const float2*)A + row0,
                               ldA, (const float2*)B, ldB, K, M, N, (float2*)out, ldo, accumulate);
        else
            hipLaunchKernelGGL(pathsum_f32_rows, dim3((uint32_t)grid), dim3(256), 0, st, (const float2*)A + row0,
                               ldA, (const float2*)B, ldB, K, M, N, (float2*)out, ldo, accumulate);
        return hip_check(hipGetLastError(), "pathsum_f32_rows launch");
    }
    if (dtype == HSF_C64 && (mode == HSF_SUM_F32 || mode == HSF_SUM_BF16X3) &&
        path_sum_lds_fits(mode, (const float2*)A + row0, ldA, B, ldB, K, M, N)) {
        if (mode == HSF_SUM_F32)
            return path_sum_f32_lds((const float2*)A + row0, ldA, (const float2*)B, ldB, K, M, N, (float2*)out, ldo,
                                    accumulate, st);
        return path_sum_bf16x3_lds((const float2*)A + row0, ldA, (const float2*)B, ldB, K, M, N, (float2*)out, ldo,
                                   accumulate, ws, st);
    }
    if (dtype == HSF_C64 && mode == HSF_SUM_F32) {
        const int64_t tn = (N + F32_TILE - 1) / F32_TILE, tiles = tn * ((M + F32_TILE - 1) / F32_TILE);
        const int grid = persistent_grid((const void*)pathsum_f32, 256, 0, tiles);
        hipLaunchKernelGGL(pathsum_f32, dim3(grid), dim3(256), 0, st, (const float2*)A + row0, ldA, (const float2*)B,
                           ldB, K, M, N, (float2*)out, ldo, accumulate, tn, tiles);
        return hip_check(hipGetLastError(), "pathsum_f32 launch");
    }
    if (dtype == HSF_C64 && mode == HSF_SUM_BF16X3)
        return path_sum_bf16x3((const float2*)A + row0, ldA, (const float2*)B, ldB, K, M, N, (float2*)out, ldo,
                               accumulate, ws, st);
    if (path_sum_lds_fits(mode, A, ldA, B, ldB, K, M, N)) {
        const size_t esz = dtype == HSF_C64 ? sizeof(float2) : sizeof(double2);
        return path_sum_f64_lds(dtype != HSF_C64, (const unsigned char*)A + row0 * esz, ldA, B, ldB, K, M, N,
                                (double2*)out, ldo, accumulate, st);
    }
    const dim3 grid((uint32_t)((N + F64_TILE - 1) / F64_TILE), (uint32_t)((M + F64_TILE - 1) / F64_TILE));
    if (grid.y > 65535u) return fail(HSF_E_ARG, "too many output rows in one call (split the row range)");
    if (dtype == HSF_C64)
        hipLaunchKernelGGL(pathsum_f64<float2>, grid, dim3(256), 0, st, (const float2*)A + row0, ldA, (const float2*)B,
                           ldB, K, M, N, (double2*)out, ldo, accumulate);
    else
        hipLaunchKernelGGL(pathsum_f64<double2>, grid, dim3(256), 0, st, (const double2*)A + row0, ldA,
                           (const double2*)B, ldB, K, M, N, (double2*)out, ldo, accumulate);
    return hip_check(hipGetLastError(), "pathsum_f64 launch");
}

hsf_status gather_dot(int dtype, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K, int nb, int n,
                      const uint64_t* x, int64_t nx, void* out, int accumulate, hipStream_t st, int copies,
                      int64_t rsA, int64_t rsB) {
    const int waves = 4;
    if (copies < 1 || copies > 65535) return fail(HSF_E_ARG, "internal: replica count out of range");
    const dim3 grid((uint32_t)((nx + waves - 1) / waves), (uint32_t)copies);
    if (dtype == HSF_C64)
        hipLaunchKernelGGL(gather_dot_kernel<float2>, grid, dim3(64 * waves), 0, st, (const float2*)A, ldA,
                           (const float2*)B, ldB, K, nb, n, x, nx, (double2*)out, accumulate, rsA, rsB);
    else
        hipLaunchKernelGGL(gather_dot_kernel<double2>, grid, dim3(64 * waves), 0, st, (const double2*)A, ldA,
                           (const double2*)B, ldB, K, nb, n, x, nx, (double2*)out, accumulate, rsA, rsB);
    return hip_check(hipGetLastError(), "gather_dot launch");
}

hsf_status norm2(const void* a, int adt, const void* b, int bdt, int64_t n, double* out, double* ws,
                 hipStream_t st) {
    if (!b) {
        return adt == HSF_C64 ? launch_norm<float2, float2, false>(a, b, n, out, ws, st)
                              : launch_norm<double2, double2, false>(a, b, n, out, ws, st);
    }
    if (adt == HSF_C64 && bdt == HSF_C64) return launch_norm<float2, float2, true>(a, b, n, out, ws, st);
    if (adt == HSF_C64 && bdt == HSF_C128) return launch_norm<float2, double2, true>(a, b, n, out, ws, st);
    if (adt == HSF_C128 && bdt == HSF_C64) return launch_norm<double2, float2, true>(a, b, n, out, ws, st);
    return launch_norm<double2, double2, true>(a, b, n, out, ws, st);
}

}  // namespace hsf
