// Path sum for many paths (large contraction depth K).  The streaming
// kernels in pathsum.hip and bf16x3.hip read their operands straight from
// global memory, which suits a few dozen paths (the sum is then bound by the
// output write).  With thousands of paths the sum is bound by MFMA
// throughput, and operand reuse decides: here each output tile stages a
// chunk of paths of its A rows and B columns in LDS, so each operand byte
// fetched from L2 serves 128 or more outputs.  FP32 and FP64: 128 x 128 (64 x
// 64) tiles, double buffered through registers (the next chunk is fetched
// while the current one feeds the MFMAs).  Split-BF16 x3: 256 x 128 tiles,
// chunks copied straight into three LDS stages by DMA loads.  The FP32
// kernel runs the streaming FP32 kernel's MFMA sequence per output block, so
// both give bit-identical results.
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
// Chunked planes: for path chunk c (B_KC paths) and row r, B_RB = 128
// contiguous bytes [re hi | re lo | im hi | im lo] x 16 paths, so one tile's
// rows of one chunk are one contiguous run.
//
// Sum kernel: output tiles of 256 A rows x 128 B rows, 8 waves in 4 x 2
// (each 64 x 64 outputs as 2 x 2 blocks of 32 x 32), one workgroup per CU.
// Chunks are copied global -> LDS by the DMA form of the vector load
// (global_load_lds_dwordx4: each lane's 16 bytes land at M0 + 16 lane), so no
// registers stage them, into three LDS stages of 48 KiB: while chunk c feeds
// the MFMAs, chunks c + 1 and c + 2 are in flight.  Each wave copies six 1 KiB
// pieces of a chunk; a barrier per chunk makes every piece visible.  LDS rows
// of 128 bytes hold eight 16-byte units XOR-swizzled by the row
// (unit u of row r at u ^ swz(r)): the lane order of a DMA fixes where each
// unit lands, so the swizzle is applied to the global addresses, and the
// 16-byte operand reads of 32 consecutive rows are then conflict-free.
constexpr int B_KC = kBf16Chunk;                 // paths per chunk
constexpr int B_RB = 8 * B_KC;                    // bytes of one row of one chunk
constexpr int B_TM = kBf16LdsTileRows, B_TN = 128, B_WAVES = 8;
constexpr int B_STAGE = (B_TM + B_TN) * B_RB;     // 48 KiB
constexpr int B_NST = 3;
constexpr size_t B_LDS = (size_t)B_NST * B_STAGE; // 144 KiB
constexpr int B_DMA = B_STAGE / 1024 / B_WAVES;   // 1 KiB DMA pieces per wave per chunk
constexpr int B_A_DMA = B_TM * B_RB / 1024;       // pieces of a chunk that hold A rows
static_assert(B_KC == 16 && B_RB == 128, "eight 16-byte units per staged row");
static_assert(B_DMA == 6, "the barrier's vmcnt below counts six DMA pieces per chunk");
static_assert(B_TM == 64 * (B_WAVES / 2), "waves in TM / 64 x 2");

__device__ __forceinline__ int b_swz(int r) { return ((r >> 1) ^ (r << 2)) & 7; }

// 16 bytes per lane from base + off into LDS at lds + 16 lane.  M0 is set
// for the copy and restored; it is read when the load issues.
__device__ __forceinline__ void lds_dma16(uint32_t lds, const void* base, uint32_t off) {
    uint32_t saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %2, %3\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds), "v"(off), "s"(base)
        : "memory");
}
// Every wave's copies of a chunk are in LDS and every wave's reads of the
// stage about to be refilled are done: this wave's own copies of all but the
// newest chunk (B_DMA pieces) and its LDS reads, then the barrier.  No
// release fence: it would wait for the copies still in flight.
__device__ __forceinline__ void dma_barrier_keep_one() {
    asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
__device__ __forceinline__ void dma_barrier_all() {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const void*)(((uint64_t)hi << 32) | lo);
}

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

// This wave's six pieces of chunk c of the tile at (m0, n0) into stage s:
// piece g = 6 w + j holds staged rows 8 g .. 8 g + 7 (A rows first, then B
// rows); rows at or beyond M (N) repeat the last row, whose products land
// only in outputs that are not stored.
__device__ __forceinline__ void bf16x3_issue(const unsigned char* PA, int64_t RA, int64_t M, int64_t m0,
                                             const unsigned char* PB, int64_t N, int64_t n0, int64_t c, int s,
                                             uint32_t lds0, int w, int lane) {
    const unsigned char* ba = (const unsigned char*)uniform_ptr(PA + c * RA * B_RB);
    const unsigned char* bb = (const unsigned char*)uniform_ptr(PB + c * N * B_RB);
#pragma unroll
    for (int j = 0; j < B_DMA; ++j) {
        const int g = w * B_DMA + j;
        const int rowl = g * 8 + (lane >> 3);
        const int unit = (lane & 7) ^ b_swz(rowl);
        const uint32_t dst = __builtin_amdgcn_readfirstlane(lds0 + (uint32_t)(s * B_STAGE + g * 1024));
        if (g < B_A_DMA) {
            const int64_t r = m0 + rowl < M ? m0 + rowl : M - 1;
            lds_dma16(dst, ba, (uint32_t)(r * B_RB + unit * 16));
        } else {
            const int64_t r = n0 + (rowl - B_TM) < N ? n0 + (rowl - B_TM) : N - 1;
            lds_dma16(dst, bb, (uint32_t)(r * B_RB + unit * 16));
        }
    }
}

// The six split terms of one 16-path chunk, terms [T0, T1), on the 2 x 2
// blocks of a wave; consecutive MFMAs write different accumulators and each
// accumulator sees its terms in the fixed order listed.
template <int T0, int T1>
__device__ __forceinline__ void bf16x3_terms(const u16x8 (&x)[2][4], const u16x8 (&y)[2][4], f32x16 (&cr)[2][2],
                                             f32x16 (&ci)[2][2]) {
    bf16x8 xs[2][6], ys[2][6];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const bf16x8 xrh = as_bf(x[a][0]), xrl = as_bf(x[a][1]), xih = as_bf(x[a][2]), xil = as_bf(x[a][3]);
        const bf16x8 nih = as_bf(x[a][2] ^ (u16x8)0x8000), nil = as_bf(x[a][3] ^ (u16x8)0x8000);
        // real part: xrh yrh, xrh yrl, xrl yrh, -xih yih, -xih yil, -xil yih
        xs[a][0] = xrh; xs[a][1] = xrh; xs[a][2] = xrl; xs[a][3] = nih; xs[a][4] = nih; xs[a][5] = nil;
        // imaginary part: xrh yih, xrh yil, xrl yih, xih yrh, xih yrl, xil yrh
        ys[a][0] = xrh; ys[a][1] = xrh; ys[a][2] = xrl; ys[a][3] = xih; ys[a][4] = xih; ys[a][5] = xil;
    }
    bf16x8 yr[2][6], yi[2][6];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const bf16x8 yrh = as_bf(y[b][0]), yrl = as_bf(y[b][1]), yih = as_bf(y[b][2]), yil = as_bf(y[b][3]);
        yr[b][0] = yrh; yr[b][1] = yrl; yr[b][2] = yrh; yr[b][3] = yih; yr[b][4] = yil; yr[b][5] = yih;
        yi[b][0] = yih; yi[b][1] = yil; yi[b][2] = yih; yi[b][3] = yrh; yi[b][4] = yrl; yi[b][5] = yrh;
    }
#pragma unroll
    for (int term = T0; term < T1; ++term)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xs[a][term], yr[b][term], cr[a][b], 0, 0, 0);
                ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ys[a][term], yi[b][term], ci[a][b], 0, 0, 0);
            }
}

// One 256 x 128 output tile at (m0, n0) from chunked planes (A's chunks of
// RA >= M rows, PA at the product's first row).  Starts with a barrier after
// every earlier store and LDS read of the workgroup, so tiles follow each
// other directly.
__device__ __forceinline__ void bf16x3_lds_tile(const unsigned char* PA, int64_t M, int64_t RA,
                                                const unsigned char* PB, int64_t N, int64_t chunks,
                                                float2* __restrict__ out, int64_t ldo, int accumulate, int64_t m0,
                                                int64_t n0, unsigned char* bl) {
    const uint32_t lds0 = (uint32_t)(uintptr_t)((__attribute__((address_space(3))) unsigned char*)bl);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int li = lane & 31, lk = lane >> 5, wm = w >> 1, wn = w & 1;
    dma_barrier_all();
    bf16x3_issue(PA, RA, M, m0, PB, N, n0, 0, 0, lds0, w, lane);
    if (chunks > 1) bf16x3_issue(PA, RA, M, m0, PB, N, n0, 1, 1, lds0, w, lane);
    f32x16 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = (f32x16)0.0f;
            ci[a][b] = (f32x16)0.0f;
        }
    int s = 0;
    for (int64_t c = 0; c < chunks; ++c) {
        // chunk c is in the LDS (only chunk c + 1 may still be in flight)
        if (c + 1 < chunks) dma_barrier_keep_one();
        else dma_barrier_all();
        const unsigned char* st = bl + s * B_STAGE;
        // plane p of staged row r, paths 8 lk .. 8 lk + 7: unit 2 p + lk
        u16x8 x[2][4], y[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int ra = wm * 64 + a * 32 + li;
            const int rb = B_TM + wn * 64 + a * 32 + li;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                x[a][p] = *reinterpret_cast<const u16x8*>(st + ra * B_RB + (((2 * p + lk) ^ b_swz(ra)) << 4));
                y[a][p] = *reinterpret_cast<const u16x8*>(st + rb * B_RB + (((2 * p + lk) ^ b_swz(rb)) << 4));
            }
        }
        // the copy of chunk c + 2 goes out after the first two terms: right
        // after the barrier the MFMAs start first (measured: 1.05x over
        // issuing the copy before the reads)
        bf16x3_terms<0, 2>(x, y, cr, ci);
        if (c + 2 < chunks)
            bf16x3_issue(PA, RA, M, m0, PB, N, n0, c + 2, s == 0 ? B_NST - 1 : s - 1, lds0, w, lane);
        bf16x3_terms<2, 6>(x, y, cr, ci);
        s = s == B_NST - 1 ? 0 : s + 1;
    }
    store_tile_128(cr, ci, m0, n0, M, N, out, ldo, accumulate);
}

__global__ __launch_bounds__(64 * B_WAVES, 1) void pathsum_bf16x3_lds(const unsigned short* __restrict__ PA, int64_t M,
                                                                    int64_t RA, const unsigned short* __restrict__ PB,
                                                                    int64_t N, int64_t chunks,
                                                                    float2* __restrict__ out, int64_t ldo,
                                                                    int accumulate, int64_t tiles_m, int64_t tiles_n,
                                                                    int xcd_bands) {
    extern __shared__ __align__(16) unsigned char bl[];
    const int64_t tiles = tiles_m * tiles_n;
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        int64_t tm, tn;
        tile_coords(item, tiles_m, tiles_n, xcd_bands != 0, tm, tn);
        bf16x3_lds_tile((const unsigned char*)PA, M, RA, (const unsigned char*)PB, N, chunks, out, ldo, accumulate,
                        tm * B_TM, tn * B_TN, bl);
    }
}

// Batched: descriptors hold chunked planes (a_off, b_off), the padded path
// count K (a multiple of 32) and tiles of B_TM x B_TN.
__global__ __launch_bounds__(64 * B_WAVES, 1) void pathsum_bf16x3_lds_batch(const GemmDesc* __restrict__ d, int n,
                                                                          unsigned char* base, int64_t tiles) {
    extern __shared__ __align__(16) unsigned char bl[];
    for (int64_t item = blockIdx.x; item < tiles; item += gridDim.x) {
        const GemmDesc& g = find_desc(d, n, item);
        int64_t tm, tn;
        tile_coords(item - g.tile_start, (g.M + B_TM - 1) / B_TM, g.tiles_n, false, tm, tn);
        bf16x3_lds_tile(base + g.a_off, g.M, g.M, base + g.b_off, g.N, g.K / B_KC, (float2*)g.out, g.ldo, 0,
                        tm * B_TM, tn * B_TN, bl);
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

// Persistent grid over tiles of tile_rows x 128 outputs; XCD bands when the
// tile rows and the grid split evenly over the eight XCDs.
void grid_shape(const void* kernel, int threads, size_t shmem, int64_t tile_rows, int64_t M, int64_t N,
                int64_t& tiles_m, int64_t& tiles_n, int& grid, int& bands) {
    tiles_m = (M + tile_rows - 1) / tile_rows;
    tiles_n = (N + 127) / 128;
    grid = persistent_grid(kernel, threads, shmem, tiles_m * tiles_n);
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
    grid_shape((const void*)pathsum_f32_lds, 256, F_LDS, 128, M, N, tm, tn, grid, bands);
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
    grid_shape((const void*)pathsum_bf16x3_lds, 64 * B_WAVES, B_LDS, B_TM, M, N, tm, tn, grid, bands);
    hipLaunchKernelGGL(pathsum_bf16x3_lds, dim3(grid), dim3(64 * B_WAVES), B_LDS, st, PA + row0 * (4 * B_KC), M, RA,
                       PB, N, chunks, out, ldo, accumulate, tm, tn, bands);
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
    const int grid = persistent_grid((const void*)pathsum_bf16x3_lds_batch, 64 * B_WAVES, B_LDS, tiles);
    hipLaunchKernelGGL(pathsum_bf16x3_lds_batch, dim3(grid), dim3(64 * B_WAVES), B_LDS, st, (const GemmDesc*)descs,
                       n, base, tiles);
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
