// Split-BF16 x3 path sum.  Every FP32 operand x is written as
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and each real product
// is taken as hi*hi + hi*lo + lo*hi on the BF16 MFMA with FP32
// accumulation (the lo*lo term, ~2^-16 relative, is dropped).  The complex
// product C = PsiA^T PsiB then needs 12 BF16 MFMAs per 32x32 block and
// 16-path chunk: Cr = Ar Br - Ai Bi, Ci = Ar Bi + Ai Br.
//
// A split pass first rewrites the half-states (rows = paths, interleaved
// complex) into four BF16 planes (re hi, re lo, im hi, im lo) laid out
// [row][path], paths padded to a multiple of 16, so that the eight path
// values one MFMA lane needs are one 16-byte load.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "epilogue.h"

namespace hsf {

namespace {

using f32x16 = f32x16_t;
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using u16x8 = unsigned short __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    // round to nearest even on the upper 16 bits (finite inputs)
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

// planes[p][r][k] for p in {re hi, re lo, im hi, im lo}, r < R, k < Kp.
// Thread: one row r, eight consecutive paths k0..k0+7 (zero beyond K).
__global__ __launch_bounds__(256) void split_planes(const float2* __restrict__ X, int64_t ldx, int64_t K,
                                                    int64_t R, int64_t Kp, unsigned short* __restrict__ planes) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.y * 8;
    if (r >= R || k0 >= Kp) return;
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
    const int64_t plane = R * Kp;
    u16x8* base = reinterpret_cast<u16x8*>(planes + r * Kp + k0);
    base[0] = rh;
    *reinterpret_cast<u16x8*>(planes + plane + r * Kp + k0) = rl;
    *reinterpret_cast<u16x8*>(planes + 2 * plane + r * Kp + k0) = ih;
    *reinterpret_cast<u16x8*>(planes + 3 * plane + r * Kp + k0) = il;
}

__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

// Workgroup: 4 waves in 2 x 2, each wave 64 x 64 complex outputs (2 x 2
// blocks of the 32x32x16 BF16 MFMA).  Lane l of a block supplies row
// (l % 32) and paths k0 + 8 (l / 32) .. +7.
constexpr int BF_TILE = 128;

__device__ __forceinline__ void bf16x3_tile(const unsigned short* __restrict__ PA, int64_t M,
                                            const unsigned short* __restrict__ PB, int64_t N, int64_t Kp,
                                            float2* __restrict__ out, int64_t ldo, int accumulate, int64_t row0,
                                            int64_t col0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int64_t m0 = row0 + (w >> 1) * 64;
    const int64_t n0 = col0 + (w & 1) * 64;
    const int64_t pa = M * Kp, pb = N * Kp;
    f32x16 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = (f32x16)0.0f;
            ci[a][b] = (f32x16)0.0f;
        }
    int64_t ra[2], rb[2];
    bool mok[2], nok[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t m = m0 + a * 32 + li, n = n0 + a * 32 + li;
        mok[a] = m < M;
        nok[a] = n < N;
        ra[a] = (mok[a] ? m : 0) * Kp;
        rb[a] = (nok[a] ? n : 0) * Kp;
    }
    const u16x8 zero = (u16x8)0;
    for (int64_t k0 = 0; k0 < Kp; k0 += 16) {
        const int64_t kk = k0 + lk * 8;
        u16x8 arh[2], arl[2], aih[2], ail[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const unsigned short* p = PA + ra[a] + kk;
            arh[a] = mok[a] ? *reinterpret_cast<const u16x8*>(p) : zero;
            arl[a] = mok[a] ? *reinterpret_cast<const u16x8*>(p + pa) : zero;
            aih[a] = mok[a] ? *reinterpret_cast<const u16x8*>(p + 2 * pa) : zero;
            ail[a] = mok[a] ? *reinterpret_cast<const u16x8*>(p + 3 * pa) : zero;
            const unsigned short* q = PB + rb[a] + kk;
            brh[a] = nok[a] ? *reinterpret_cast<const u16x8*>(q) : zero;
            brl[a] = nok[a] ? *reinterpret_cast<const u16x8*>(q + pb) : zero;
            bih[a] = nok[a] ? *reinterpret_cast<const u16x8*>(q + 2 * pb) : zero;
            bil[a] = nok[a] ? *reinterpret_cast<const u16x8*>(q + 3 * pb) : zero;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const bf16x8 xrh = as_bf(arh[a]), xrl = as_bf(arl[a]), xih = as_bf(aih[a]), xil = as_bf(ail[a]);
            const bf16x8 nih = as_bf(aih[a] ^ (u16x8)0x8000), nil = as_bf(ail[a] ^ (u16x8)0x8000);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const bf16x8 yrh = as_bf(brh[b]), yrl = as_bf(brl[b]), yih = as_bf(bih[b]), yil = as_bf(bil[b]);
                f32x16 r = cr[a][b], i = ci[a][b];
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yrh, r, 0, 0, 0);
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yrl, r, 0, 0, 0);
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrl, yrh, r, 0, 0, 0);
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, yih, r, 0, 0, 0);
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, yil, r, 0, 0, 0);
                r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nil, yih, r, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yih, i, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yil, i, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrl, yih, i, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, yrh, i, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, yrl, i, 0, 0, 0);
                i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xil, yrh, i, 0, 0, 0);
                cr[a][b] = r;
                ci[a][b] = i;
            }
        }
    }
    store_tile_128(cr, ci, row0, col0, M, N, out, ldo, accumulate);
}

// Persistent streaming kernel: 8 waves per 128 x 128 tile, wave (wm, wn) =
// (w / 4, w % 4) owns rows 64 wm .. +63 and columns 32 wn .. +31 (two 32x32
// blocks).  Half the accumulators and operands of a 64 x 64 wave tile leave
// room for two waves per SIMD, so one wave's stores drain while another
// multiplies.  The operands of the next tile's first two 16-path steps are
// loaded before this tile's results are stored: loads and stores share one
// completion counter, so loads issued after the stores would wait for them.
// Per output block the MFMA sequence is that of bf16x3_tile.
struct Bf16Step {
    u16x8 a[2][4], b[4];
};

__device__ __forceinline__ void load_step(const unsigned short* __restrict__ PA, int64_t M,
                                          const unsigned short* __restrict__ PB, int64_t N, int64_t Kp,
                                          int64_t m0, int64_t n0, int64_t k0, Bf16Step& st) {
    const int lane = threadIdx.x & 63, li = lane & 31, lk = lane >> 5;
    const int64_t pa = M * Kp, pb = N * Kp, kk = k0 + lk * 8;
    const u16x8 zero = (u16x8)0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t m = m0 + a * 32 + li;
        const bool mok = m < M;
        const unsigned short* p = PA + (mok ? m : 0) * Kp + kk;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) st.a[a][pl] = mok ? *reinterpret_cast<const u16x8*>(p + pl * pa) : zero;
    }
    const int64_t n = n0 + li;
    const bool nok = n < N;
    const unsigned short* q = PB + (nok ? n : 0) * Kp + kk;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) st.b[pl] = nok ? *reinterpret_cast<const u16x8*>(q + pl * pb) : zero;
}

__device__ __forceinline__ void mma_step(const Bf16Step& st, f32x16 (&cr)[2], f32x16 (&ci)[2]) {
    const bf16x8 yrh = as_bf(st.b[0]), yrl = as_bf(st.b[1]), yih = as_bf(st.b[2]), yil = as_bf(st.b[3]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const bf16x8 xrh = as_bf(st.a[a][0]), xrl = as_bf(st.a[a][1]), xih = as_bf(st.a[a][2]),
                     xil = as_bf(st.a[a][3]);
        const bf16x8 nih = as_bf(st.a[a][2] ^ (u16x8)0x8000), nil = as_bf(st.a[a][3] ^ (u16x8)0x8000);
        f32x16 r = cr[a], i = ci[a];
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yrh, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yrl, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrl, yrh, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, yih, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nih, yil, r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nil, yih, r, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yih, i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yil, i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrl, yih, i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, yrh, i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, yrl, i, 0, 0, 0);
        i = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xil, yrh, i, 0, 0, 0);
        cr[a] = r;
        ci[a] = i;
    }
}

// Stores a wave's 64 x 32 block pair (accumulator r of a 32x32 block at row
// (r/4)*8 + (lane/32)*4 + r%4, column lane%32).
__device__ __forceinline__ void store_64x32(const f32x16 (&cr)[2], const f32x16 (&ci)[2], int64_t m0, int64_t n0,
                                            int64_t M, int64_t N, float2* __restrict__ out, int64_t ldo,
                                            int accumulate) {
    const int lane = threadIdx.x & 63, li = lane & 31, lk = lane >> 5;
    const int64_t col = n0 + li;
    if (col >= N) return;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = m0 + a * 32 + (r >> 2) * 8 + lk * 4 + (r & 3);
            if (row >= M) continue;
            float2 v = make_float2(cr[a][r], ci[a][r]);
            float2* o = out + row * ldo + col;
            if (accumulate) {
                const float2 old = *o;
                v.x += old.x;
                v.y += old.y;
            }
            *o = v;
        }
}

__global__ __launch_bounds__(512) void pathsum_bf16x3_kernel(const unsigned short* __restrict__ PA, int64_t M,
                                                             const unsigned short* __restrict__ PB, int64_t N,
                                                             int64_t Kp, float2* __restrict__ out, int64_t ldo,
                                                             int accumulate, int64_t tiles_n, int64_t tiles) {
    const int w = threadIdx.x >> 6;
    const int64_t wr = (w >> 2) * 64, wc = (w & 3) * 32;
    int64_t tile = blockIdx.x;
    if (tile >= tiles) return;
    auto origin = [&](int64_t t, int64_t& r0, int64_t& c0) {
        const int64_t tm = t / tiles_n, tn = t - tm * tiles_n;
        r0 = tm * BF_TILE + wr;
        c0 = tn * BF_TILE + wc;
    };
    int64_t m0, n0;
    origin(tile, m0, n0);
    Bf16Step s0, s1;
    load_step(PA, M, PB, N, Kp, m0, n0, 0, s0);
    if (Kp > 16) load_step(PA, M, PB, N, Kp, m0, n0, 16, s1);
    for (;;) {
        f32x16 cr[2], ci[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            cr[a] = (f32x16)0.0f;
            ci[a] = (f32x16)0.0f;
        }
        mma_step(s0, cr, ci);
        if (Kp > 16) mma_step(s1, cr, ci);
        for (int64_t k0 = 32; k0 < Kp; k0 += 16) {
            load_step(PA, M, PB, N, Kp, m0, n0, k0, s1);
            mma_step(s1, cr, ci);
        }
        const int64_t next = tile + gridDim.x;
        int64_t nm0 = 0, nn0 = 0;
        if (next < tiles) {
            origin(next, nm0, nn0);
            load_step(PA, M, PB, N, Kp, nm0, nn0, 0, s0);
            if (Kp > 16) load_step(PA, M, PB, N, Kp, nm0, nn0, 16, s1);
        }
        store_64x32(cr, ci, m0, n0, M, N, out, ldo, accumulate);
        if (next >= tiles) break;
        tile = next;
        m0 = nm0;
        n0 = nn0;
    }
}

__global__ __launch_bounds__(256) void split_batch(const SplitDesc* __restrict__ d, int n, unsigned char* base) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block_start <= blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const SplitDesc& s = d[lo];
    const uint32_t local = blockIdx.x - s.block_start;
    const uint32_t by = local / s.blocks_x, bx = local - by * s.blocks_x;
    const int64_t r = (int64_t)bx * 256 + threadIdx.x;
    const int64_t k0 = (int64_t)by * 8;
    if (r >= s.R || k0 >= s.Kp) return;
    const float2* X = reinterpret_cast<const float2*>(base + s.x_off);
    unsigned short* planes = reinterpret_cast<unsigned short*>(base + s.planes_off);
    u16x8 rh, rl, ih, il;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + e;
        const float2 v = k < s.K ? X[k * s.ldx + r] : make_float2(0.f, 0.f);
        const unsigned short a = bf16_rne(v.x), b = bf16_rne(v.y);
        rh[e] = a;
        rl[e] = bf16_rne(v.x - bf16_to_f32(a));
        ih[e] = b;
        il[e] = bf16_rne(v.y - bf16_to_f32(b));
    }
    if (s.chunked) {
        // chunks of kBf16Chunk paths: row r of chunk c holds 4 planes x kBf16Chunk paths
        unsigned short* row = planes + ((k0 / kBf16Chunk) * s.R + r) * (4 * kBf16Chunk) + (k0 % kBf16Chunk);
        *reinterpret_cast<u16x8*>(row) = rh;
        *reinterpret_cast<u16x8*>(row + kBf16Chunk) = rl;
        *reinterpret_cast<u16x8*>(row + 2 * kBf16Chunk) = ih;
        *reinterpret_cast<u16x8*>(row + 3 * kBf16Chunk) = il;
        return;
    }
    const int64_t plane = s.R * s.Kp;
    *reinterpret_cast<u16x8*>(planes + r * s.Kp + k0) = rh;
    *reinterpret_cast<u16x8*>(planes + plane + r * s.Kp + k0) = rl;
    *reinterpret_cast<u16x8*>(planes + 2 * plane + r * s.Kp + k0) = ih;
    *reinterpret_cast<u16x8*>(planes + 3 * plane + r * s.Kp + k0) = il;
}

// Persistent over the union of all circuits' output tiles.
__global__ __launch_bounds__(256) void pathsum_bf16x3_batch(const GemmDesc* __restrict__ d, int n,
                                                            unsigned char* base, int64_t tiles) {
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
        bf16x3_tile(reinterpret_cast<const unsigned short*>(base + g.a_off), g.M,
                    reinterpret_cast<const unsigned short*>(base + g.b_off), g.N, g.K, (float2*)g.out, g.ldo, 0,
                    tm * BF_TILE, tn * BF_TILE);
    }
}

}  // namespace

hsf_status launch_split_batch(const void* descs, int n, uint32_t total_blocks, unsigned char* base, hipStream_t st) {
    hipLaunchKernelGGL(split_batch, dim3(total_blocks), dim3(256), 0, st, (const SplitDesc*)descs, n, base);
    return hip_check(hipGetLastError(), "split_batch launch");
}

hsf_status launch_bf16x3_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st) {
    const int grid = persistent_grid((const void*)pathsum_bf16x3_batch, 256, 0, tiles);
    hipLaunchKernelGGL(pathsum_bf16x3_batch, dim3(grid), dim3(256), 0, st, (const GemmDesc*)descs, n, base, tiles);
    return hip_check(hipGetLastError(), "pathsum_bf16x3_batch launch");
}

hsf_status path_sum_bf16x3(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                           int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st) {
    const int64_t Kp = std::max<int64_t>(16, (K + 15) / 16 * 16);
    unsigned short* PA = reinterpret_cast<unsigned short*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    unsigned short* PB = PA + 4 * M * Kp;
    {
        const dim3 ga((uint32_t)((M + 255) / 256), (uint32_t)(Kp / 8));
        const dim3 gb((uint32_t)((N + 255) / 256), (uint32_t)(Kp / 8));
        if (ga.y > 65535u) return fail(HSF_E_ARG, "too many paths in one HSF_SUM_BF16X3 call (split the path range)");
        hipLaunchKernelGGL(split_planes, ga, dim3(256), 0, st, A, ldA, K, M, Kp, PA);
        hipLaunchKernelGGL(split_planes, gb, dim3(256), 0, st, B, ldB, K, N, Kp, PB);
        hsf_status s = hip_check(hipGetLastError(), "split_planes launch");
        if (s != HSF_OK) return s;
    }
    const int64_t tn = (N + BF_TILE - 1) / BF_TILE, tiles = tn * ((M + BF_TILE - 1) / BF_TILE);
    const int grid = persistent_grid((const void*)pathsum_bf16x3_kernel, 512, 0, tiles);
    hipLaunchKernelGGL(pathsum_bf16x3_kernel, dim3(grid), dim3(512), 0, st, PA, M, PB, N, Kp, out, ldo, accumulate,
                       tn, tiles);
    return hip_check(hipGetLastError(), "pathsum_bf16x3 launch");
}

}  // namespace hsf
