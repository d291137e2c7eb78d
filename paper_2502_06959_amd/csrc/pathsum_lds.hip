// Path sum for many paths (large contraction depth K).  The streaming
// kernels in pathsum.hip and bf16x3.hip read their operands straight from
// global memory, which suits a few dozen paths (the sum is then bound by the
// output write).  With thousands of paths the sum is bound by MFMA
// throughput, and operand reuse decides: here each 128 x 128 output tile
// stages a chunk of paths of its 128 A rows and 128 B columns in LDS (double
// buffered: the next chunk is fetched into registers while the current one
// feeds the MFMAs), so each operand byte fetched from L2 serves 128 outputs.
// The MFMA sequence per output block is the same as the streaming kernels',
// so both give bit-identical results.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "epilogue.h"

namespace hsf {

namespace {

using f32x16 = f32x16_t;
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using u16x8 = unsigned short __attribute__((ext_vector_type(8)));

// Output tile of a persistent workgroup's t-th work item.  Workgroups are
// dealt to the eight XCDs round-robin (t mod 8 names the XCD when the grid is
// a multiple of 8), so when the tile rows split evenly each XCD gets its own
// band of tile rows and walks it column by column: the tiles in flight on one
// XCD share their A rows and B columns in that XCD's L2.  Otherwise tiles go
// in groups of up to eight tile rows, column by column.
__device__ __forceinline__ void tile_coords(int64_t t, int64_t tiles_m, int64_t tiles_n, bool xcd_bands,
                                            int64_t& tm, int64_t& tn) {
    if (xcd_bands) {
        const int64_t band = tiles_m >> 3, x = t & 7, u = t >> 3;
        tm = x * band + u % band;
        tn = u / band;
        return;
    }
    const int64_t group = 8 * tiles_n, g = t / group, first = g * 8;
    const int64_t gm = tiles_m - first < 8 ? tiles_m - first : 8;
    const int64_t r = t - g * group;
    tm = first + r % gm;
    tn = r / gm;
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

// ---------------------------------------------------------------- FP32 ----
constexpr int F_KC = 16;                          // paths per stage
constexpr int F_STAGE = 2 * F_KC * 128;           // float2 entries of A and B per stage
constexpr size_t F_LDS = 2 * F_STAGE * sizeof(float2);

// One 128 x 128 output tile at (m0, n0).  A, B 16-byte aligned; ldA, ldB,
// M and N even (checked by the launchers).  Ends with a barrier, so the
// caller may start the next tile at once.
__device__ __forceinline__ void f32_lds_tile(const float2* __restrict__ A, int64_t ldA,
                                             const float2* __restrict__ B, int64_t ldB, int64_t K, int64_t M,
                                             int64_t N, float2* __restrict__ out, int64_t ldo, int accumulate,
                                             int64_t m0, int64_t n0, float2* fl) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int li = lane & 31, lk = lane >> 5, wm = w >> 1, wn = w & 1;
    const int64_t chunks = (K + F_KC - 1) / F_KC;
    {
        // staging: thread t moves entries 2q, 2q+1 of path row q / 64 for
        // q = t + 256 i, i < 4, of both operands
        float4 ra[4], rb[4];
        auto fetch = [&](int64_t c) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = t + 256 * i, k = q >> 6, e = (q & 63) * 2;
                const int64_t kk = c * F_KC + k;
                const bool kok = kk < K;
                ra[i] = (kok && m0 + e < M) ? *reinterpret_cast<const float4*>(A + kk * ldA + m0 + e)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
                rb[i] = (kok && n0 + e < N) ? *reinterpret_cast<const float4*>(B + kk * ldB + n0 + e)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        auto stash = [&](int buf) {
            float2* sa = fl + buf * F_STAGE;
            float2* sb = sa + F_KC * 128;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = t + 256 * i, k = q >> 6, e = (q & 63) * 2;
                *reinterpret_cast<float4*>(sa + k * 128 + e) = ra[i];
                *reinterpret_cast<float4*>(sb + k * 128 + e) = rb[i];
            }
        };
        f32x16 cr[2][2], ci[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = (f32x16)0.0f;
                ci[a][b] = (f32x16)0.0f;
            }
        fetch(0);
        stash(0);
        __syncthreads();
        for (int64_t c = 0; c < chunks; ++c) {
            const int buf = (int)(c & 1);
            if (c + 1 < chunks) fetch(c + 1);
            const float2* sa = fl + buf * F_STAGE;
            const float2* sb = sa + F_KC * 128;
#pragma unroll
            for (int j = 0; j < F_KC / 2; ++j) {
                const int kk = 2 * j + lk;
                float2 av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    av[a] = sa[kk * 128 + wm * 64 + a * 32 + li];
                    bv[a] = sb[kk * 128 + wn * 64 + a * 32 + li];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                        cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, -bv[b].y, cr[a][b], 0, 0, 0);
                        ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                        ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
                    }
            }
            if (c + 1 < chunks) stash(buf ^ 1);
            __syncthreads();
        }
        store_tile_128(cr, ci, m0, n0, M, N, out, ldo, accumulate);
    }
}

__global__ __launch_bounds__(256, 2) void pathsum_f32_lds(const float2* __restrict__ A, int64_t ldA,
                                                       const float2* __restrict__ B, int64_t ldB, int64_t K,
                                                       int64_t M, int64_t N, float2* __restrict__ out, int64_t ldo,
                                                       int accumulate, int64_t tiles_m, int64_t tiles_n,
                                                       int xcd_bands) {
    extern __shared__ __align__(16) float2 fl[];
    const int64_t tiles = tiles_m * tiles_n;
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        int64_t tm, tn;
        tile_coords(item, tiles_m, tiles_n, xcd_bands != 0, tm, tn);
        f32_lds_tile(A, ldA, B, ldB, K, M, N, out, ldo, accumulate, tm * 128, tn * 128, fl);
    }
}

// Persistent over the union of the output tiles of several circuits (a
// sorted table of descriptors, offsets from `base`).
__device__ __forceinline__ const GemmDesc& find_desc(const GemmDesc* __restrict__ d, int n, int64_t tile) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_start <= tile) lo = mid;
        else hi = mid - 1;
    }
    return d[lo];
}

__global__ __launch_bounds__(256, 2) void pathsum_f32_lds_batch(const GemmDesc* __restrict__ d, int n,
                                                             unsigned char* base, int64_t tiles) {
    extern __shared__ __align__(16) float2 fl[];
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        const GemmDesc& g = find_desc(d, n, item);
        int64_t tm, tn;
        tile_coords(item - g.tile_start, (g.M + 127) / 128, g.tiles_n, false, tm, tn);
        f32_lds_tile(reinterpret_cast<const float2*>(base + g.a_off), g.ldA,
                     reinterpret_cast<const float2*>(base + g.b_off), g.ldB, g.K, g.M, g.N, (float2*)g.out, g.ldo,
                     0, tm * 128, tn * 128, fl);
    }
}

// ------------------------------------------------------- split-BF16 x3 ----
// Chunked planes: for path chunk c (B_KC paths) and row r, B_RB contiguous
// bytes [re hi | re lo | im hi | im lo] x B_KC paths, so one tile's rows of
// one chunk are one contiguous run of 128 x B_RB bytes.  With 16-path chunks
// the double-buffered stages take 72 KiB of LDS: two workgroups per CU, so
// one's barrier and LDS waits are covered by the other's MFMAs.
constexpr int B_KC = kBf16Chunk;                 // paths per chunk (a multiple of 16)
constexpr int B_RB = 8 * B_KC;                    // bytes of one row of one chunk (4 planes x B_KC x 2 B)
constexpr int B_TPR = B_RB / 16;                  // threads per row when staging (16 bytes each)
constexpr int B_RPI = 256 / B_TPR;                // rows per staging instruction
constexpr int B_NF = 128 / B_RPI;                 // staging loads per operand per chunk
constexpr int B_ROW = B_RB + 16;                  // staged row bytes (16-byte pad: conflict-free b128 reads)
constexpr int B_STAGE = 2 * 128 * B_ROW;          // bytes of A and B rows per stage
constexpr size_t B_LDS = 2 * (size_t)B_STAGE;

// Thread: row r, eight consecutive paths 8y .. 8y+7 (zero at or beyond K).
__global__ __launch_bounds__(256) void split_chunked(const float2* __restrict__ X, int64_t ldx, int64_t K,
                                                     int64_t R, unsigned short* __restrict__ planes) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.y * 8;
    if (r >= R) return;
    u16x8 rh, rl, ih, il;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + e;
        const float2 v = k < K ? X[k * ldx + r] : make_float2(0.f, 0.f);
        const unsigned short a = bf16_rne(v.x), b = bf16_rne(v.y);
        rh[e] = a;
        rl[e] = bf16_rne(v.x - bf16_to_f32(a));
        ih[e] = b;
        il[e] = bf16_rne(v.y - bf16_to_f32(b));
    }
    const int64_t c = k0 / B_KC, off = k0 % B_KC;
    unsigned short* row = planes + (c * R + r) * (4 * B_KC) + off;
    *reinterpret_cast<u16x8*>(row) = rh;
    *reinterpret_cast<u16x8*>(row + B_KC) = rl;
    *reinterpret_cast<u16x8*>(row + 2 * B_KC) = ih;
    *reinterpret_cast<u16x8*>(row + 3 * B_KC) = il;
}

// Rows row0 + t / B_TPR + B_RPI i (i < B_NF) of path chunk c, bytes
// 16 (t % B_TPR) .. +15, of planes whose chunks hold R rows each; rows at or
// beyond lim read as zero (lim <= R).
__device__ __forceinline__ void fetch_rows(const unsigned short* __restrict__ P, int64_t R, int64_t lim, int64_t row0,
                                           int64_t c, int srow, int scol, uint4 (&r)[B_NF]) {
    const uint4* g = reinterpret_cast<const uint4*>(P + (c * R + row0) * (4 * B_KC));
#pragma unroll
    for (int i = 0; i < B_NF; ++i) {
        const int row = srow + B_RPI * i;
        const bool ok = row0 + row < lim;
        const uint4 v = g[(ok ? row : lim - 1 - row0) * B_TPR + scol];
        r[i] = ok ? v : make_uint4(0u, 0u, 0u, 0u);
    }
}

__device__ __forceinline__ void stash_rows(unsigned char* stage, int srow, int scol, const uint4 (&ra)[B_NF],
                                           const uint4 (&rb)[B_NF]) {
#pragma unroll
    for (int i = 0; i < B_NF; ++i) {
        const int off = (srow + B_RPI * i) * B_ROW + scol * 16;
        *reinterpret_cast<uint4*>(stage + off) = ra[i];
        *reinterpret_cast<uint4*>(stage + 128 * B_ROW + off) = rb[i];
    }
}

// One 128 x 128 output tile at (m0, n0) from chunked planes (A's chunks of
// RA >= M rows, PA at the product's first row); ends with a barrier.
__device__ __forceinline__ void bf16x3_lds_tile(const unsigned short* __restrict__ PA, int64_t M, int64_t RA,
                                                const unsigned short* __restrict__ PB, int64_t N, int64_t chunks,
                                                float2* __restrict__ out, int64_t ldo, int accumulate, int64_t m0,
                                                int64_t n0, unsigned char* bl) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int li = lane & 31, lk = lane >> 5, wm = w >> 1, wn = w & 1;
    {
        // staging: B_TPR threads move one row of a chunk; thread t takes rows
        // t / B_TPR + B_RPI i, i < B_NF, bytes 16 (t % B_TPR) .. +15, of both operands
        uint4 ra[B_NF], rb[B_NF];
        const int srow = t / B_TPR, scol = t % B_TPR;
        f32x16 cr[2][2], ci[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = (f32x16)0.0f;
                ci[a][b] = (f32x16)0.0f;
            }
        fetch_rows(PA, RA, M, m0, 0, srow, scol, ra);
        fetch_rows(PB, N, N, n0, 0, srow, scol, rb);
        stash_rows(bl, srow, scol, ra, rb);
        __syncthreads();
        for (int64_t c = 0; c < chunks; ++c) {
            const int buf = (int)(c & 1);
            if (c + 1 < chunks) {
                fetch_rows(PA, RA, M, m0, c + 1, srow, scol, ra);
                fetch_rows(PB, N, N, n0, c + 1, srow, scol, rb);
            }
            const unsigned char* sa = bl + buf * B_STAGE;
            const unsigned char* sb = sa + 128 * B_ROW;
#pragma unroll
            for (int s = 0; s < B_KC / 16; ++s) {
                // plane p of row r, paths 16 s + 8 lk .. +7: byte r * B_ROW + 2 B_KC p + 32 s + 16 lk
                u16x8 x[2][4], y[2][4];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const unsigned char* pa = sa + (wm * 64 + a * 32 + li) * B_ROW + 32 * s + 16 * lk;
                    const unsigned char* pb = sb + (wn * 64 + a * 32 + li) * B_ROW + 32 * s + 16 * lk;
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        x[a][p] = *reinterpret_cast<const u16x8*>(pa + 2 * B_KC * p);
                        y[a][p] = *reinterpret_cast<const u16x8*>(pb + 2 * B_KC * p);
                    }
                }
                // term-major order over the 2 x 2 blocks: consecutive MFMAs
                // write different accumulators; each accumulator sees its
                // six terms in the fixed order listed below
                bf16x8 xs[2][6], ys[2][6];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bf16x8 xrh = as_bf(x[a][0]), xrl = as_bf(x[a][1]), xih = as_bf(x[a][2]),
                                 xil = as_bf(x[a][3]);
                    const bf16x8 nih = as_bf(x[a][2] ^ (u16x8)0x8000), nil = as_bf(x[a][3] ^ (u16x8)0x8000);
                    // real part: xrh yrh, xrh yrl, xrl yrh, -xih yih, -xih yil, -xil yih
                    xs[a][0] = xrh; xs[a][1] = xrh; xs[a][2] = xrl; xs[a][3] = nih; xs[a][4] = nih; xs[a][5] = nil;
                    // imaginary part: xrh yih, xrh yil, xrl yih, xih yrh, xih yrl, xil yrh
                    ys[a][0] = xrh; ys[a][1] = xrh; ys[a][2] = xrl; ys[a][3] = xih; ys[a][4] = xih; ys[a][5] = xil;
                }
                bf16x8 yr[2][6], yi[2][6];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const bf16x8 yrh = as_bf(y[b][0]), yrl = as_bf(y[b][1]), yih = as_bf(y[b][2]),
                                 yil = as_bf(y[b][3]);
                    yr[b][0] = yrh; yr[b][1] = yrl; yr[b][2] = yrh; yr[b][3] = yih; yr[b][4] = yil; yr[b][5] = yih;
                    yi[b][0] = yih; yi[b][1] = yil; yi[b][2] = yih; yi[b][3] = yrh; yi[b][4] = yrl; yi[b][5] = yrh;
                }
#pragma unroll
                for (int term = 0; term < 6; ++term)
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) {
                            cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xs[a][term], yr[b][term], cr[a][b], 0, 0, 0);
                            ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ys[a][term], yi[b][term], ci[a][b], 0, 0, 0);
                        }
            }
            if (c + 1 < chunks) stash_rows(bl + (buf ^ 1) * B_STAGE, srow, scol, ra, rb);
            __syncthreads();
        }
        store_tile_128(cr, ci, m0, n0, M, N, out, ldo, accumulate);
    }
}

__global__ __launch_bounds__(256, 2) void pathsum_bf16x3_lds(const unsigned short* __restrict__ PA, int64_t M,
                                                          int64_t RA, const unsigned short* __restrict__ PB, int64_t N,
                                                          int64_t chunks, float2* __restrict__ out, int64_t ldo,
                                                          int accumulate, int64_t tiles_m, int64_t tiles_n,
                                                          int xcd_bands) {
    extern __shared__ __align__(16) unsigned char bl[];
    const int64_t tiles = tiles_m * tiles_n;
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        int64_t tm, tn;
        tile_coords(item, tiles_m, tiles_n, xcd_bands != 0, tm, tn);
        bf16x3_lds_tile(PA, M, RA, PB, N, chunks, out, ldo, accumulate, tm * 128, tn * 128, bl);
    }
}

// Batched: descriptors hold chunked planes (a_off, b_off) and the padded path
// count K (a multiple of 32).
__global__ __launch_bounds__(256, 2) void pathsum_bf16x3_lds_batch(const GemmDesc* __restrict__ d, int n,
                                                                unsigned char* base, int64_t tiles) {
    extern __shared__ __align__(16) unsigned char bl[];
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        const GemmDesc& g = find_desc(d, n, item);
        int64_t tm, tn;
        tile_coords(item - g.tile_start, (g.M + 127) / 128, g.tiles_n, false, tm, tn);
        bf16x3_lds_tile(reinterpret_cast<const unsigned short*>(base + g.a_off), g.M, g.M,
                        reinterpret_cast<const unsigned short*>(base + g.b_off), g.N, g.K / B_KC, (float2*)g.out,
                        g.ldo, 0, tm * 128, tn * 128, bl);
    }
}

// ---------------------------------------------------------------- FP64 ----
// 64 x 64 tiles of 4 waves (2 x 2, each 32 x 32 = 2 x 2 blocks of the
// 16x16x4 FP64 MFMA), chunks of 16 paths of the tile's 64 A rows and 64 B
// columns staged in LDS as complex128 (c64 inputs widened on the way in),
// double-buffered; the MFMA sequence per block is the streaming FP64
// kernel's.
constexpr int D_KC = 16;
constexpr int D_STAGE = 2 * D_KC * 64;            // double2 entries of A and B per stage
constexpr size_t D_LDS = 2 * D_STAGE * sizeof(double2);

using f64x4 = double __attribute__((ext_vector_type(4)));

template <typename VIN>
__device__ __forceinline__ double2 widen2(VIN v) {
    return make_double2((double)v.x, (double)v.y);
}

template <typename VIN>
__device__ __forceinline__ void f64_lds_tile(const VIN* __restrict__ A, int64_t ldA, const VIN* __restrict__ B,
                                             int64_t ldB, int64_t K, int64_t M, int64_t N,
                                             double2* __restrict__ out, int64_t ldo, int accumulate, int64_t m0,
                                             int64_t n0, double2* dl) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int li = lane & 15, lk = lane >> 4, wm = w >> 1, wn = w & 1;
    const int64_t chunks = (K + D_KC - 1) / D_KC;
    // staging: thread t moves entry q % 64 of path row q / 64, q = t + 256 i, i < 4
    double2 ra[4], rb[4];
    auto fetch = [&](int64_t c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = t + 256 * i, k = q >> 6, e = q & 63;
            const int64_t kk = c * D_KC + k;
            const bool kok = kk < K;
            ra[i] = (kok && m0 + e < M) ? widen2(A[kk * ldA + m0 + e]) : make_double2(0.0, 0.0);
            rb[i] = (kok && n0 + e < N) ? widen2(B[kk * ldB + n0 + e]) : make_double2(0.0, 0.0);
        }
    };
    auto stash = [&](int buf) {
        double2* sa = dl + buf * D_STAGE;
        double2* sb = sa + D_KC * 64;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = t + 256 * i;
            sa[q] = ra[i];
            sb[q] = rb[i];
        }
    };
    f64x4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = (f64x4)0.0;
            ci[a][b] = (f64x4)0.0;
        }
    fetch(0);
    stash(0);
    __syncthreads();
    for (int64_t c = 0; c < chunks; ++c) {
        const int buf = (int)(c & 1);
        if (c + 1 < chunks) fetch(c + 1);
        const double2* sa = dl + buf * D_STAGE;
        const double2* sb = sa + D_KC * 64;
#pragma unroll
        for (int j = 0; j < D_KC / 4; ++j) {
            const int kk = 4 * j + lk;
            double2 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                av[a] = sa[kk * 64 + wm * 32 + a * 16 + li];
                bv[a] = sb[kk * 64 + wn * 32 + a * 16 + li];
            }
            // term-major order: consecutive MFMAs write different
            // accumulators; each accumulator still sees its terms in the
            // streaming kernel's order
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, -bv[b].y, cr[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
                }
        }
        if (c + 1 < chunks) stash(buf ^ 1);
        __syncthreads();
    }
    // accumulator r of a 16x16 FP64 block: row lane/16 + 4 r, column lane%16
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t col = n0 + wn * 32 + b * 16 + li;
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * 32 + a * 16 + lk + 4 * r;
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

template <typename VIN>
__global__ __launch_bounds__(256) void pathsum_f64_lds(const VIN* __restrict__ A, int64_t ldA,
                                                       const VIN* __restrict__ B, int64_t ldB, int64_t K, int64_t M,
                                                       int64_t N, double2* __restrict__ out, int64_t ldo,
                                                       int accumulate, int64_t tiles_m, int64_t tiles_n) {
    extern __shared__ __align__(16) double2 dl[];
    const int64_t tiles = tiles_m * tiles_n;
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        int64_t tm, tn;
        tile_coords(item, tiles_m, tiles_n, false, tm, tn);
        f64_lds_tile<VIN>(A, ldA, B, ldB, K, M, N, out, ldo, accumulate, tm * 64, tn * 64, dl);
    }
}

// (cheap host calls, repeated per launch so that every device gets them)
hsf_status set_lds_attrs() {
    hsf_status s = hip_check(hipFuncSetAttribute((const void*)pathsum_bf16x3_lds,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)B_LDS),
                             "hipFuncSetAttribute");
    if (s != HSF_OK) return s;
    s = hip_check(hipFuncSetAttribute((const void*)pathsum_f32_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)F_LDS),
                  "hipFuncSetAttribute");
    if (s != HSF_OK) return s;
    s = hip_check(hipFuncSetAttribute((const void*)pathsum_bf16x3_lds_batch,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)B_LDS),
                  "hipFuncSetAttribute");
    if (s != HSF_OK) return s;
    s = hip_check(hipFuncSetAttribute((const void*)pathsum_f32_lds_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)F_LDS),
                  "hipFuncSetAttribute");
    if (s != HSF_OK) return s;
    s = hip_check(hipFuncSetAttribute((const void*)pathsum_f64_lds<float2>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)D_LDS),
                  "hipFuncSetAttribute");
    if (s != HSF_OK) return s;
    return hip_check(hipFuncSetAttribute((const void*)pathsum_f64_lds<double2>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)D_LDS),
                     "hipFuncSetAttribute");
}

void grid_shape(const void* kernel, size_t shmem, int64_t M, int64_t N, int64_t& tiles_m, int64_t& tiles_n,
                int& grid, int& bands) {
    tiles_m = (M + 127) / 128;
    tiles_n = (N + 127) / 128;
    grid = persistent_grid(kernel, 256, shmem, tiles_m * tiles_n);
    bands = (tiles_m % 8 == 0 && grid % 8 == 0) ? 1 : 0;
}

}  // namespace

bool path_sum_lds_fits(int mode, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K, int64_t M,
                       int64_t N) {
    if (K < kLdsMinPaths) return false;
    if (mode == HSF_SUM_F64 || mode == HSF_SUM_C128) return true;
    if (mode == HSF_SUM_BF16X3) return (K + B_KC - 1) / B_KC * (B_KC / 8) <= 65535;
    return ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && ldA % 2 == 0 && ldB % 2 == 0 && M % 2 == 0 &&
           N % 2 == 0;
}

hsf_status path_sum_f32_lds(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                            int64_t N, float2* out, int64_t ldo, int accumulate, hipStream_t st) {
    hsf_status s = set_lds_attrs();
    if (s != HSF_OK) return s;
    int64_t tm, tn;
    int grid, bands;
    grid_shape((const void*)pathsum_f32_lds, F_LDS, M, N, tm, tn, grid, bands);
    hipLaunchKernelGGL(pathsum_f32_lds, dim3(grid), dim3(256), F_LDS, st, A, ldA, B, ldB, K, M, N, out, ldo,
                       accumulate, tm, tn, bands);
    return hip_check(hipGetLastError(), "pathsum_f32_lds launch");
}

size_t bf16x3_lds_planes(int64_t rows, int64_t K) {
    const int64_t kp = (K + B_KC - 1) / B_KC * B_KC;
    return (size_t)(4 * rows * kp) * sizeof(uint16_t);
}

hsf_status split_lds(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N, int64_t K,
                     unsigned short* PA, unsigned short* PB, hipStream_t st) {
    const int64_t chunks = (K + B_KC - 1) / B_KC;
    const uint32_t gy = (uint32_t)(chunks * (B_KC / 8));
    hipLaunchKernelGGL(split_chunked, dim3((uint32_t)((MA + 255) / 256), gy), dim3(256), 0, st, A, ldA, K, MA, PA);
    hipLaunchKernelGGL(split_chunked, dim3((uint32_t)((N + 255) / 256), gy), dim3(256), 0, st, B, ldB, K, N, PB);
    return hip_check(hipGetLastError(), "split_chunked launch");
}

hsf_status sum_lds(const unsigned short* PA, int64_t RA, int64_t row0, int64_t M, const unsigned short* PB, int64_t N,
                   int64_t K, float2* out, int64_t ldo, int accumulate, hipStream_t st) {
    hsf_status s = set_lds_attrs();
    if (s != HSF_OK) return s;
    const int64_t chunks = (K + B_KC - 1) / B_KC;
    int64_t tm, tn;
    int grid, bands;
    grid_shape((const void*)pathsum_bf16x3_lds, B_LDS, M, N, tm, tn, grid, bands);
    hipLaunchKernelGGL(pathsum_bf16x3_lds, dim3(grid), dim3(256), B_LDS, st, PA + row0 * (4 * B_KC), M, RA, PB, N,
                       chunks, out, ldo, accumulate, tm, tn, bands);
    return hip_check(hipGetLastError(), "pathsum_bf16x3_lds launch");
}

hsf_status path_sum_bf16x3_lds(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                               int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st) {
    unsigned short* PA = reinterpret_cast<unsigned short*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    unsigned short* PB = PA + bf16x3_lds_planes(M, K) / sizeof(uint16_t);
    hsf_status s = split_lds(A, ldA, M, B, ldB, N, K, PA, PB, st);
    if (s != HSF_OK) return s;
    return sum_lds(PA, M, 0, M, PB, N, K, out, ldo, accumulate, st);
}

hsf_status launch_f32_lds_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st) {
    hsf_status s = set_lds_attrs();
    if (s != HSF_OK) return s;
    const int grid = persistent_grid((const void*)pathsum_f32_lds_batch, 256, F_LDS, tiles);
    hipLaunchKernelGGL(pathsum_f32_lds_batch, dim3(grid), dim3(256), F_LDS, st, (const GemmDesc*)descs, n, base,
                       tiles);
    return hip_check(hipGetLastError(), "pathsum_f32_lds_batch launch");
}

hsf_status launch_bf16x3_lds_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st) {
    hsf_status s = set_lds_attrs();
    if (s != HSF_OK) return s;
    const int grid = persistent_grid((const void*)pathsum_bf16x3_lds_batch, 256, B_LDS, tiles);
    hipLaunchKernelGGL(pathsum_bf16x3_lds_batch, dim3(grid), dim3(256), B_LDS, st, (const GemmDesc*)descs, n, base,
                       tiles);
    return hip_check(hipGetLastError(), "pathsum_bf16x3_lds_batch launch");
}

hsf_status path_sum_f64_lds(bool c128_in, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K, int64_t M,
                            int64_t N, double2* out, int64_t ldo, int accumulate, hipStream_t st) {
    hsf_status s = set_lds_attrs();
    if (s != HSF_OK) return s;
    const int64_t tm = (M + 63) / 64, tn = (N + 63) / 64;
    if (c128_in) {
        const int grid = persistent_grid((const void*)pathsum_f64_lds<double2>, 256, D_LDS, tm * tn);
        hipLaunchKernelGGL(pathsum_f64_lds<double2>, dim3(grid), dim3(256), D_LDS, st, (const double2*)A, ldA,
                           (const double2*)B, ldB, K, M, N, out, ldo, accumulate, tm, tn);
    } else {
        const int grid = persistent_grid((const void*)pathsum_f64_lds<float2>, 256, D_LDS, tm * tn);
        hipLaunchKernelGGL(pathsum_f64_lds<float2>, dim3(grid), dim3(256), D_LDS, st, (const float2*)A, ldA,
                           (const float2*)B, ldB, K, M, N, out, ldo, accumulate, tm, tn);
    }
    return hip_check(hipGetLastError(), "pathsum_f64_lds launch");
}

}  // namespace hsf
