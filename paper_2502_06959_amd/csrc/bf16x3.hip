// Split-BF16 x3 path sum.  Every FP32 operand x is written as
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and each real product
// is taken as hi*hi + hi*lo + lo*hi on the BF16 MFMA with FP32
// accumulation (the lo*lo term, ~2^-16 relative, is dropped).  The complex
// product C = PsiA^T PsiB (Cr = Ar Br - Ai Bi, Ci = Ar Bi + Ai Br) then
// costs 12 BF16 MFMAs per 32x32 complex outputs and 16 paths.
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

// One operand of the split: R rows of X (row k of path k at X + k ldx) into
// `planes`.
struct SplitOperand {
    const float2* X;
    int64_t ldx, R;
    unsigned short* planes;
};

// planes[p][r][k] for p in {re hi, re lo, im hi, im lo}, r < R, k < Kp.
// Thread: one row r, eight consecutive paths k0..k0+7 (zero beyond K).  Both
// operands in one launch: blockIdx.z 0 splits a, 1 splits b.
__global__ __launch_bounds__(256) void split_planes(SplitOperand a, SplitOperand b, int64_t K, int64_t Kp) {
    const bool second = blockIdx.z != 0;
    const float2* __restrict__ X = second ? b.X : a.X;
    const int64_t ldx = second ? b.ldx : a.ldx, R = second ? b.R : a.R;
    unsigned short* __restrict__ planes = second ? b.planes : a.planes;
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

// Persistent streaming kernel.  The complex product is taken as one real
// product with the real and imaginary parts of the output interleaved,
// exactly as the output is laid out in memory:
//   C2[m][2n]   = sum_k Ar[k][m] Br[k][n] + Ai[k][m] (-Bi[k][n])
//   C2[m][2n+1] = sum_k Ar[k][m] Bi[k][n] + Ai[k][m]   Br[k][n]
// i.e. A2 = [Ar | Ai] along a doubled path axis and real column 2n + p of
// B2 = [Br Bi ; -Bi Br] (column pairs).  An MFMA lane then holds single
// floats of consecutive output columns, stored as they are (no register
// pairing).  Per 16 paths a block takes the real-plane half of the axis with
// lane 2q holding Br and lane 2q+1 Bi of column n = q (one load each), then
// the imaginary-plane half with the two lanes' operands swapped (a DPP
// exchange) and the even lane's negated: each B value is loaded once.
//
// Workgroup tile: 256 rows x 128 complex columns; wave w owns rows
// 32 w .. +31 and all 256 real columns as eight 32x32 blocks side by side,
// so each wave writes whole 1 KiB row segments, which the HBM write path
// drains faster than narrower per-wave strips.  Each block's B2 operand for
// the next step (or the next tile's first step) is loaded right after the
// block's MFMAs, and A2's at the start of the chunk, so the loads of a
// tile's successor are issued before the tile's stores (loads and stores
// share one completion counter: loads issued after the stores would wait
// for them).  Per block and half: hi*hi + hi*lo + lo*hi.
constexpr int BW_ROWS = (int)kBf16StreamRows, BW_COLS = (int)kBf16StreamCols;
constexpr int BW_THREADS = 2 * BW_ROWS;    // one wave per 32 rows

// a value the caller knows to be equal in all lanes, kept in scalar registers
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A2 operands of the 16 paths from k0: row r0 + lane % 32, paths
// k0 + 8 (lane / 32) .. +7 of the four planes (re hi, re lo, im hi, im lo).
// lane = (lane % 32) Kp + 8 (lane / 32), the lane's fixed element offset.
// The planes hold pa_rows rows each (M <= pa_rows: a product may cover a
// row range of operands split over more rows).
template <bool FULL>
__device__ __forceinline__ void load_a2(const unsigned short* __restrict__ P, int64_t M, int64_t pa_rows, int64_t Kp,
                                        int64_t r0, int64_t k0, uint32_t lane_off, u16x8 (&v)[4]) {
    const int64_t plane = pa_rows * Kp;
    if (FULL) {
        // wave-uniform base in scalar registers + the 32-bit lane offset
        const unsigned short* base = P + uniform_i64(r0 * Kp + k0);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) v[pl] = *reinterpret_cast<const u16x8*>(base + pl * plane + lane_off);
        return;
    }
    const int lane = threadIdx.x & 63, li = lane & 31, lk = lane >> 5;
    const int64_t r = r0 + li;
    const bool ok = r < M;
    const unsigned short* p = P + (ok ? r : 0) * Kp + k0 + lk * 8;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) v[pl] = ok ? *reinterpret_cast<const u16x8*>(p + pl * plane) : (u16x8)0;
}

// B2 operand of the real-plane half for the 32 real columns c0 .. c0+31
// (c0 even): lane column c0 + lane % 32 is part lane % 2 of complex column
// c0/2 + (lane % 32)/2.  lane_off = ((lane % 32)/2) Kp + 8 (lane / 32) +
// (lane % 2) 2 N Kp, the lane's fixed element offset.
template <bool FULL>
__device__ __forceinline__ void load_b2(const unsigned short* __restrict__ P, int64_t N, int64_t Kp, int64_t c0,
                                        int64_t k0, uint32_t lane_off, u16x8& hi, u16x8& lo) {
    const int64_t plane = N * Kp;
    if (FULL) {
        const unsigned short* base = P + uniform_i64((c0 >> 1) * Kp + k0);
        hi = *reinterpret_cast<const u16x8*>(base + lane_off);
        lo = *reinterpret_cast<const u16x8*>(base + plane + lane_off);
        return;
    }
    const int lane = threadIdx.x & 63, li = lane & 31, lk = lane >> 5, par = li & 1;
    const int64_t n = (c0 >> 1) + (li >> 1);
    const bool ok = n < N;
    const unsigned short* p = P + (par ? 2 * plane : 0) + (ok ? n : 0) * Kp + k0 + lk * 8;
    hi = ok ? *reinterpret_cast<const u16x8*>(p) : (u16x8)0;
    lo = ok ? *reinterpret_cast<const u16x8*>(p + plane) : (u16x8)0;
}

// The imaginary-plane half's B2 operand: lanes 2q and 2q+1 exchange their
// values (Br <-> Bi) and the even lane negates (-Bi).
__device__ __forceinline__ u16x8 swap_pair(u16x8 v, uint32_t neg) {
    const auto d = __builtin_bit_cast(uint32_t __attribute__((ext_vector_type(4))), v);
    uint32_t __attribute__((ext_vector_type(4))) o;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        o[e] = (uint32_t)__builtin_amdgcn_mov_dpp((int)d[e], 0xB1, 0xF, 0xF, false) ^ neg;   // quad_perm [1,0,3,2]
    return __builtin_bit_cast(u16x8, o);
}

// One tile of work: the operand planes and output of one product, and the
// wave's origin in it (row m0, real column c0).  All fields are
// wave-uniform.
struct StreamJob {
    const unsigned short* PA;
    const unsigned short* PB;
    float* out;
    int64_t M, N, Kp, ldo, m0, c0, pa_rows;
};

// Persistent loop over `tiles` tiles handed out by loc(t) (t = this
// workgroup's tiles, blockIdx.x + i gridDim.x).
// FULL: every product has M a multiple of 256, N of 128, 32 output rows
// spanning less than 2^31 bytes and operand planes under 2^31 elements, and
// nothing is accumulated: no bounds tests anywhere, and every load and store
// takes a wave-uniform base plus a fixed 32-bit lane offset.
template <bool FULL, typename Loc>
__device__ __forceinline__ void stream_tiles(const Loc& loc, int64_t tiles, int accumulate) {
    const int lane = threadIdx.x & 63, li = lane & 31, lk = lane >> 5;
    const uint32_t neg = (li & 1) ? 0u : 0x80008000u;
    auto offsets = [&](const StreamJob& j, uint32_t& ao, uint32_t& bo) {
        ao = (uint32_t)li * (uint32_t)j.Kp + lk * 8;
        bo = (uint32_t)(li >> 1) * (uint32_t)j.Kp + lk * 8 + ((li & 1) ? (uint32_t)(2 * j.N * j.Kp) : 0u);
    };
    int64_t tile = blockIdx.x;
    if (tile >= tiles) return;
    StreamJob cur = loc(tile);
    uint32_t a_off, b_off;
    offsets(cur, a_off, b_off);
    u16x8 a[4], bh[8], bl[8];
    load_a2<FULL>(cur.PA, cur.M, cur.pa_rows, cur.Kp, cur.m0, 0, a_off, a);
#pragma unroll
    for (int blk = 0; blk < 8; ++blk)
        load_b2<FULL>(cur.PB, cur.N, cur.Kp, cur.c0 + blk * 32, 0, b_off, bh[blk], bl[blk]);
    for (;;) {
        const int64_t next = tile + gridDim.x;
        const StreamJob nxt = next < tiles ? loc(next) : cur;
        uint32_t na_off, nb_off;
        offsets(nxt, na_off, nb_off);
        f32x16 acc[8];
#pragma unroll
        for (int blk = 0; blk < 8; ++blk) acc[blk] = (f32x16)0.0f;
        for (int64_t k0 = 0; k0 < cur.Kp; k0 += 16) {
            // operands of the following 16 paths: this tile's, else the next tile's first
            const bool last = k0 + 16 >= cur.Kp, more = !last || next < tiles;
            const StreamJob& lj = last ? nxt : cur;
            const int64_t lk0 = last ? 0 : k0 + 16;
            const uint32_t la = last ? na_off : a_off, lb = last ? nb_off : b_off;
            const bf16x8 xrh = as_bf(a[0]), xrl = as_bf(a[1]), xih = as_bf(a[2]), xil = as_bf(a[3]);
            if (more) load_a2<FULL>(lj.PA, lj.M, lj.pa_rows, lj.Kp, lj.m0, lk0, la, a);
#pragma unroll
            for (int blk = 0; blk < 8; ++blk) {
                const bf16x8 yh = as_bf(bh[blk]), yl = as_bf(bl[blk]);
                const bf16x8 zh = as_bf(swap_pair(bh[blk], neg)), zl = as_bf(swap_pair(bl[blk], neg));
                f32x16 c = acc[blk];
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrh, yl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xrl, yh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, zh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xih, zl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xil, zh, c, 0, 0, 0);
                acc[blk] = c;
                if (more) load_b2<FULL>(lj.PB, lj.N, lj.Kp, lj.c0 + blk * 32, lk0, lb, bh[blk], bl[blk]);
            }
        }
        // accumulator r of block blk: row m0 + (r/4)*8 + (lane/32)*4 + r%4,
        // real column c0 + 32 blk + lane%32
        if (FULL) {
            const int64_t ldf = 2 * cur.ldo;
            const int64_t wofs = uniform_i64(cur.m0 * ldf + cur.c0);
            const uint32_t voff = (uint32_t)(lk * 4) * (uint32_t)ldf + (uint32_t)li;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t rofs =
                    wofs + (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)((r >> 2) * 8 + (r & 3)) * (uint32_t)ldf);
                float* __restrict__ pl = cur.out + rofs + voff;
#pragma unroll
                for (int blk = 0; blk < 8; ++blk) pl[blk * 32] = acc[blk][r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = cur.m0 + (r >> 2) * 8 + lk * 4 + (r & 3);
                if (row >= cur.M) continue;
#pragma unroll
                for (int blk = 0; blk < 8; ++blk) {
                    const int64_t col = cur.c0 + blk * 32 + li;
                    if ((col >> 1) >= cur.N) continue;
                    float* o = cur.out + row * 2 * cur.ldo + col;
                    *o = accumulate ? *o + acc[blk][r] : acc[blk][r];
                }
            }
        }
        if (next >= tiles) break;
        tile = next;
        cur = nxt;
        a_off = na_off;
        b_off = nb_off;
    }
}

// one product: tiles in row-major order
struct SingleLoc {
    const unsigned short* PA;
    const unsigned short* PB;
    float* out;
    int64_t M, N, Kp, ldo, tiles_n, pa_rows;
    int w;
    __device__ __forceinline__ StreamJob operator()(int64_t t) const {
        const int64_t tm = t / tiles_n, tn = t - tm * tiles_n;
        return {PA, PB, out, M, N, Kp, ldo, tm * BW_ROWS + w * 32, tn * (2 * BW_COLS), pa_rows};
    }
};

// PA: the planes' first row of this product (rows of the planes pa_rows
// apart per plane).
template <bool FULL>
__global__ __launch_bounds__(BW_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void pathsum_bf16x3_kernel(const unsigned short* __restrict__ PA, int64_t M,
                                                             int64_t pa_rows, const unsigned short* __restrict__ PB,
                                                             int64_t N, int64_t Kp, float2* __restrict__ out,
                                                             int64_t ldo, int accumulate, int64_t tiles_n,
                                                             int64_t tiles) {
    const SingleLoc loc{PA, PB, reinterpret_cast<float*>(out), M, N, Kp, ldo, tiles_n, pa_rows,
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)};
    stream_tiles<FULL>(loc, tiles, accumulate);
}

// several products (a batch of circuits): a sorted descriptor table read as
// uniform data, tiles numbered consecutively over the products
#if defined(__HIP_DEVICE_COMPILE__)
using cdesc = const __attribute__((address_space(4))) GemmDesc*;
#else
using cdesc = const GemmDesc*;
#endif

struct BatchLoc {
    cdesc d;
    int n;
    unsigned char* base;
    int w;
    __device__ __forceinline__ StreamJob operator()(int64_t t) const {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].tile_start <= t) lo = mid;
            else hi = mid - 1;
        }
        const int64_t local = t - d[lo].tile_start, tiles_n = d[lo].tiles_n;
        const int64_t tm = local / tiles_n, tn = local - tm * tiles_n;
        return {reinterpret_cast<const unsigned short*>(base + d[lo].a_off),
                reinterpret_cast<const unsigned short*>(base + d[lo].b_off),
                reinterpret_cast<float*>(d[lo].out),
                d[lo].M,
                d[lo].N,
                d[lo].K,
                d[lo].ldo,
                tm * BW_ROWS + w * 32,
                tn * (2 * BW_COLS),
                d[lo].M};
    }
};

template <bool FULL>
__global__ __launch_bounds__(BW_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void pathsum_bf16x3_batch(const GemmDesc* __restrict__ d, int n,
                                                            unsigned char* base, int64_t tiles) {
#if defined(__HIP_DEVICE_COMPILE__)
    const cdesc cd = (cdesc)d;
#else
    const cdesc cd = d;
#endif
    const BatchLoc loc{cd, n, base, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)};
    stream_tiles<FULL>(loc, tiles, 0);
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

}  // namespace

hsf_status launch_split_batch(const void* descs, int n, uint32_t total_blocks, unsigned char* base, hipStream_t st) {
    hipLaunchKernelGGL(split_batch, dim3(total_blocks), dim3(256), 0, st, (const SplitDesc*)descs, n, base);
    return hip_check(hipGetLastError(), "split_batch launch");
}

hsf_status launch_bf16x3_batch(const void* descs, int n, int64_t tiles, bool full, unsigned char* base,
                               hipStream_t st) {
    const void* kern = full ? (const void*)pathsum_bf16x3_batch<true> : (const void*)pathsum_bf16x3_batch<false>;
    const int grid = persistent_grid(kern, BW_THREADS, 0, tiles);
    if (full)
        hipLaunchKernelGGL(pathsum_bf16x3_batch<true>, dim3(grid), dim3(BW_THREADS), 0, st, (const GemmDesc*)descs, n, base,
                           tiles);
    else
        hipLaunchKernelGGL(pathsum_bf16x3_batch<false>, dim3(grid), dim3(BW_THREADS), 0, st, (const GemmDesc*)descs, n, base,
                           tiles);
    return hip_check(hipGetLastError(), "pathsum_bf16x3_batch launch");
}

size_t bf16x3_stream_planes(int64_t rows, int64_t K) {
    const int64_t Kp = std::max<int64_t>(16, (K + 15) / 16 * 16);
    return (size_t)(4 * rows * Kp) * sizeof(uint16_t);
}

hsf_status split_stream(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N, int64_t K,
                        unsigned short* PA, unsigned short* PB, hipStream_t st) {
    const int64_t Kp = std::max<int64_t>(16, (K + 15) / 16 * 16);
    const dim3 g((uint32_t)((std::max(MA, N) + 255) / 256), (uint32_t)(Kp / 8), 2);
    if (g.y > 65535u) return fail(HSF_E_ARG, "too many paths in one HSF_SUM_BF16X3 call (split the path range)");
    const SplitOperand a{A, ldA, MA, PA}, b{B, ldB, N, PB};
    hipLaunchKernelGGL(split_planes, g, dim3(256), 0, st, a, b, K, Kp);
    return hip_check(hipGetLastError(), "split_planes launch");
}

hsf_status sum_stream(const unsigned short* PA, int64_t pa_rows, int64_t row0, int64_t M, const unsigned short* PB,
                      int64_t N, int64_t K, float2* out, int64_t ldo, int accumulate, hipStream_t st) {
    const int64_t Kp = std::max<int64_t>(16, (K + 15) / 16 * 16);
    PA += row0 * Kp;
    const int64_t tn = (N + BW_COLS - 1) / BW_COLS, tiles = tn * ((M + BW_ROWS - 1) / BW_ROWS);
    const bool full = bf16x3_stream_full(M, N, Kp, ldo, accumulate) && 4 * pa_rows * Kp <= (int64_t)INT32_MAX;
    const void* kern = full ? (const void*)pathsum_bf16x3_kernel<true> : (const void*)pathsum_bf16x3_kernel<false>;
    const int grid = persistent_grid(kern, BW_THREADS, 0, tiles);
    if (full)
        hipLaunchKernelGGL(pathsum_bf16x3_kernel<true>, dim3(grid), dim3(BW_THREADS), 0, st, PA, M, pa_rows, PB, N, Kp,
                           out, ldo, 0, tn, tiles);
    else
        hipLaunchKernelGGL(pathsum_bf16x3_kernel<false>, dim3(grid), dim3(BW_THREADS), 0, st, PA, M, pa_rows, PB, N,
                           Kp, out, ldo, accumulate, tn, tiles);
    return hip_check(hipGetLastError(), "pathsum_bf16x3 launch");
}

hsf_status path_sum_bf16x3(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                           int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st) {
    unsigned short* PA = reinterpret_cast<unsigned short*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    unsigned short* PB = PA + bf16x3_stream_planes(M, K) / sizeof(uint16_t);
    hsf_status s = split_stream(A, ldA, M, B, ldB, N, K, PA, PB, st);
    if (s != HSF_OK) return s;
    return sum_stream(PA, M, 0, M, PB, N, K, out, ldo, accumulate, st);
}

}  // namespace hsf
