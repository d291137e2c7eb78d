// Half-state gate sweeps (Sec. II-A applied to each path's subcircuit,
// Sec. II-B).  One launch covers every path of a chunk on both sides.  A
// workgroup owns one tile of one path's half-state in LDS -- 2^L amplitudes
// spanning L of the side's qubits, the low qubits among them so that tile
// rows are contiguous in HBM -- and applies every op of the pass before
// writing the tile back.  When the whole half-state fits (L = n_side) there
// is a single pass that starts from |0...0> in LDS and writes HBM once.
//
// Inside a pass, runs of one-qubit gates and diagonal gates are grouped: a
// thread loads the 8 or 16 amplitudes that differ in three or four tile bits
// (group_bits of the tile size) into registers, applies the run there
// (one-qubit gates as 2x2 butterflies, diagonal gates as sign masks or phase
// rows), and stores them back, so LDS is touched once per group instead of
// once per gate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "device.h"

namespace hsf {

namespace {

template <typename T> struct Cx;
template <> struct Cx<float> { using v = float2; };
template <> struct Cx<double> { using v = double2; };

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename V>
__device__ __forceinline__ V cfma(V a, V b, V c) {  // c + a*b
    V r;
    r.x = c.x + a.x * b.x - a.y * b.y;
    r.y = c.y + a.x * b.y + a.y * b.x;
    return r;
}

// Device form of a group sub-op, with the 2x2 matrix (or the sign masks) in
// the arithmetic type so a record is 64 bytes (c64) or 96 bytes (c128).
template <typename T>
struct DSub {
    int32_t type;
    int32_t g;
    int32_t nc;
    int32_t mat;
    int32_t qb[4];
    union {
        T m[8];
        uint32_t mask[8];
    };
};

// Read-only plan tables (passes, ops, sub-op records, batch segments) are
// read through the constant address space: their loads are uniform, and the
// compiler may then use scalar loads, which it otherwise avoids because the
// kernels also store to global memory.
// (The host pass of this file never runs these device functions; it sees
// plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using ctab = const __attribute__((address_space(4))) T*;
#else
template <typename T>
using ctab = const T*;
#endif
template <typename T>
__device__ __forceinline__ ctab<T> as_table(const T* p) {
    return (ctab<T>)p;
}

struct SideArgs {
    const Pass* pass;        // device copy of the pass record
    void* psi;
    int64_t ld;
    const DevOp* ops;
    const void* subs;        // DSub<T>[]
    const void* pool;
    uint32_t n_tiles;
    uint32_t n_blocks;       // rows x tiles
    // Rows.  A launch row is a level row i = i_lo + j, the state of the S
    // paths [i S, (i + 1) S) (S = 1: one path); it is written to row
    // i - dst_lo of psi and takes its digits from the first of its paths at
    // or after p0, max(i S, p0).
    int64_t p0, S, i_lo, dst_lo;
    // Input: ROW_INPLACE its own row; ROW_SHARED the single state `src`;
    // ROW_PARENT row i S / S_par - src_lo of `src` (ld src_ld), the state of
    // the S_par paths it belongs to at the previous level.
    const void* src;
    int64_t src_ld, src_lo, S_par;
    int32_t mode;
    // Replicas of one run that differ only in their factor pools and buffers
    // (0: n_blocks, one run): workgroup b belongs to copy r = b / rep_blocks,
    // which reads pool + r pool_rs, writes psi + r dst_rs and (ROW_PARENT)
    // reads src + r src_rs (strides in complex elements).
    uint32_t rep_blocks;
    int64_t pool_rs, dst_rs, src_rs;
    // the launch covers tiles [tile0, tile0 + n_tiles) of each row, or with
    // tile_free != 0 the n_tiles = 2^popcount(tile_free) tiles tile0 | s, s
    // a subset of tile_free's bits
    uint32_t tile0;
    uint32_t tile_free;
};

// LDS position of tile element e: the low four index bits are XORed with the
// next four, so that the 16 lanes that vary the lowest free bits of a
// register group land on 16 distinct 8-byte bank pairs whatever the group's
// bits are (a bijection on [0, 2^L) for every L).  It is linear over XOR:
// swz(a ^ b) = swz(a) ^ swz(b).
__device__ __forceinline__ uint32_t swz(uint32_t e) { return e ^ ((e >> 4) & 15u); }

// Inserts a zero bit at position b of i.
__device__ __forceinline__ uint32_t ins0(uint32_t i, int b) {
    const uint32_t lo = i & ((1u << b) - 1u);
    return ((i >> b) << (b + 1)) | lo;
}

template <int K>
__device__ __forceinline__ void sort_bits(const int32_t* bit, int (&sb)[K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) sb[i] = bit[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i + 1; j < K; ++j)
            if (sb[j] < sb[i]) {
                const int t = sb[i];
                sb[i] = sb[j];
                sb[j] = t;
            }
}

// Dense 2^K x 2^K matrix on tile bits bit[0..K) (bit[0] most significant).
template <int K, typename V>
__device__ __forceinline__ void apply_dense(V* tile, uint32_t E, const int32_t* bit, const V* m,
                                            int tid, int nt) {
    constexpr int D = 1 << K;
    int sb[K];
    sort_bits<K>(bit, sb);
    uint32_t soff[D];                // swz(offset of element j); see apply_group
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((j >> (K - 1 - i)) & 1) o |= 1u << bit[i];
        soff[j] = swz(o);
    }
    const uint32_t groups = E >> K;
    for (uint32_t g = tid; g < groups; g += nt) {
        uint32_t base = g;
#pragma unroll
        for (int i = 0; i < K; ++i) base = ins0(base, sb[i]);
        const uint32_t sbase = swz(base);
        V v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = tile[sbase ^ soff[j]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc = cmul(m[r * D], v[0]);
#pragma unroll
            for (int j = 1; j < D; ++j) acc = cfma(m[r * D + j], v[j], acc);
            tile[sbase ^ soff[r]] = acc;
        }
    }
}

// 2x2 butterfly on register position G of a 2^K register group.
template <int K, int G, typename V>
__device__ __forceinline__ void d1g(V (&v)[1 << K], V m00, V m01, V m10, V m11) {
    if constexpr (G < K) {
#pragma unroll
        for (int j = 0; j < (1 << K); ++j) {
            if (j & (1 << G)) continue;
            const V x0 = v[j], x1 = v[j | (1 << G)];
            v[j] = cfma(m01, x1, cmul(m00, x0));
            v[j | (1 << G)] = cfma(m11, x1, cmul(m10, x0));
        }
    }
}

// Diagonal 2x2 (f00, f11) on register position G: one product per amplitude.
template <int K, int G, typename V>
__device__ __forceinline__ void d1diag(V (&v)[1 << K], V f00, V f11) {
    if constexpr (G < K) {
#pragma unroll
        for (int j = 0; j < (1 << K); ++j) v[j] = cmul((j & (1 << G)) ? f11 : f00, v[j]);
    }
}

// S1: the group may hold one-qubit factor pieces (SUB_SLOT1); instantiated
// separately so the kernels of passes without them keep their code.
// DIRECT: the pass is this one group (Pass::direct): amplitudes come from
// src and go to st at their row indices (gmap maps tile bits to side
// qubits), no LDS tile; init: the first pass, from |0...0>.
template <int K, typename T, bool S1, bool DIRECT = false>
__device__ __forceinline__ void apply_group(typename Cx<T>::v* tile, uint32_t E, const DevOp& op,
                                            ctab<DSub<T>> subs, const typename Cx<T>::v* __restrict__ pool,
                                            uint64_t gbase, int64_t path, int tid, int nt,
                                            ctab<Pass> ps = nullptr, typename Cx<T>::v* st = nullptr,
                                            const typename Cx<T>::v* src = nullptr, int init = 0) {
    const ctab<T> pool_s = as_table(reinterpret_cast<const T*>(pool));   // uniform reads of factor pieces
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    int sb[K];
    sort_bits<K>(op.bit, sb);
    // the swizzle is linear over XOR and a group's base and register bits
    // are disjoint: slot(base | off_j) = swz(base) ^ swz(off_j)
    uint32_t soff[D];
    uint64_t goff[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint32_t o = 0;
        uint64_t go = 0;
#pragma unroll
        for (int g = 0; g < K; ++g)
            if ((j >> g) & 1) {
                o |= 1u << op.bit[g];
                if constexpr (DIRECT) go |= uint64_t(1) << ps->local_q[op.bit[g]];
            }
        soff[j] = swz(o);
        goff[j] = go;
    }
    int nc = 0;
    if constexpr (DIRECT)
        while (nc < ps->n_local && ps->local_q[nc] == nc) ++nc;
    const int s0 = op.mat, ns = op.rank;
    const uint32_t groups = E >> K;
    for (uint32_t gi = tid; gi < groups; gi += nt) {
        uint32_t base = gi;
#pragma unroll
        for (int i = 0; i < K; ++i) base = ins0(base, sb[i]);
        const uint32_t sbase = swz(base);
        V v[D];
        uint64_t gb = 0;
        if constexpr (DIRECT) {
            // the group's row index: the tile's non-local bits, then its local bits
            gb = gbase | (base & ((1u << nc) - 1u));
            for (int i = nc; i < ps->n_local; ++i) gb |= (uint64_t)((base >> i) & 1u) << ps->local_q[i];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if (init) {
                    v[j].x = (gb | goff[j]) == 0 ? T(1) : T(0);
                    v[j].y = T(0);
                } else {
                    v[j] = src[gb | goff[j]];
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j) v[j] = tile[sbase ^ soff[j]];
        }
        // Records alternate between two register sets (unrolled by two, the
        // next index clamped so the loads are unconditional): the next
        // record's scalar loads are issued before the current one is applied,
        // with no register-to-register copies of the 64-byte records.
#define HSF_APPLY_SUB(so)                                                                                \
    {                                                                                                    \
        const int ty = (so).type;                                                                        \
        if (ty == SUB_D1) {                                                                              \
            V m00, m01, m10, m11;                                                                        \
            m00.x = (so).m[0]; m00.y = (so).m[1];                                                        \
            m01.x = (so).m[2]; m01.y = (so).m[3];                                                        \
            m10.x = (so).m[4]; m10.y = (so).m[5];                                                        \
            m11.x = (so).m[6]; m11.y = (so).m[7];                                                        \
            switch ((so).g) {                                                                            \
                case 0: d1g<K, 0>(v, m00, m01, m10, m11); break;                                         \
                case 1: d1g<K, 1>(v, m00, m01, m10, m11); break;                                         \
                case 2: d1g<K, 2>(v, m00, m01, m10, m11); break;                                         \
                default: d1g<K, 3>(v, m00, m01, m10, m11); break;                                        \
            }                                                                                            \
        } else if (S1 && ty == SUB_SLOT1) {                                                              \
            /* this path's factor: digit (path / stride) % rank (uniform) */                             \
            const int64_t dig = (so).mask[1]                                                             \
                ? ((path >> (so).mask[2]) & (int64_t)(so).mask[3])                                       \
                : (path / (int64_t)(((uint64_t)(so).mask[3] << 32) | (so).mask[2])) % (int64_t)(so).mask[0]; \
            const int64_t e0 = 2 * ((int64_t)(so).mat + 4 * dig);                                        \
            V f00, f01, f10, f11;                                                                        \
            f00.x = pool_s[e0]; f00.y = pool_s[e0 + 1];                                                  \
            f01.x = pool_s[e0 + 2]; f01.y = pool_s[e0 + 3];                                              \
            f10.x = pool_s[e0 + 4]; f10.y = pool_s[e0 + 5];                                              \
            f11.x = pool_s[e0 + 6]; f11.y = pool_s[e0 + 7];                                              \
            const int fl = (so).qb[0];                                                                   \
            if (fl & 2) {                                                                                \
                /* diagonal piece followed by another on this bit: multiply into the chain */           \
                ch0 = cmul(f00, ch0);                                                                    \
                ch1 = cmul(f11, ch1);                                                                    \
            } else if (fl & 1) {                                                                         \
                /* last diagonal piece of a chain: apply the product, one product per amplitude */      \
                f00 = cmul(f00, ch0);                                                                    \
                f11 = cmul(f11, ch1);                                                                    \
                ch0.x = T(1); ch0.y = T(0); ch1 = ch0;                                                   \
                if ((so).g < 0) {                                                                        \
                    /* a piece off the register bits: its qubit's bit is the group's own */             \
                    const int b = (so).qb[1];                                                            \
                    const uint32_t bit = b >= 0 ? (base >> b) & 1u : (uint32_t)((gbase >> (-1 - b)) & 1u); \
                    const V f = bit ? f11 : f00;                                                         \
                    _Pragma("unroll") for (int j = 0; j < D; ++j) v[j] = cmul(f, v[j]);                  \
                } else {                                                                                 \
                    switch ((so).g) {                                                                    \
                        case 0: d1diag<K, 0>(v, f00, f11); break;                                        \
                        case 1: d1diag<K, 1>(v, f00, f11); break;                                        \
                        case 2: d1diag<K, 2>(v, f00, f11); break;                                        \
                        default: d1diag<K, 3>(v, f00, f11); break;                                       \
                    }                                                                                    \
                }                                                                                        \
            } else {                                                                                     \
                if (fl & 4) {                                                                            \
                    /* a piece with folded gates ends a chain: the chain's diagonal comes first */        \
                    f00 = cmul(f00, ch0);                                                                \
                    f10 = cmul(f10, ch0);                                                                \
                    f01 = cmul(f01, ch1);                                                                \
                    f11 = cmul(f11, ch1);                                                                \
                    ch0.x = T(1); ch0.y = T(0); ch1 = ch0;                                               \
                }                                                                                        \
                switch ((so).g) {                                                                        \
                    case 0: d1g<K, 0>(v, f00, f01, f10, f11); break;                                     \
                    case 1: d1g<K, 1>(v, f00, f01, f10, f11); break;                                     \
                    case 2: d1g<K, 2>(v, f00, f01, f10, f11); break;                                     \
                    default: d1g<K, 3>(v, f00, f01, f10, f11); break;                                    \
                }                                                                                        \
            }                                                                                            \
        } else {                                                                                         \
            uint32_t c = 0;                                                                              \
            _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                              \
                if (i >= (so).nc) break;                                                                 \
                const int b = (so).qb[i];                                                                \
                const uint32_t bit = b >= 0 ? (base >> b) & 1u : (uint32_t)((gbase >> (-1 - b)) & 1u);   \
                c |= bit << i;                                                                           \
            }                                                                                            \
            if (ty == SUB_SIGN) {                                                                        \
                /* the 16 combos' masks are uniform; pick this group's by c */                          \
                uint32_t w = (so).mask[0];                                                               \
                _Pragma("unroll") for (int q = 1; q < 8; ++q) w = ((c >> 1) == (uint32_t)q) ? (so).mask[q] : w; \
                const uint32_t mask = (w >> ((c & 1u) * 16u)) & 0xffffu;                                 \
                _Pragma("unroll") for (int j = 0; j < D; ++j) if ((mask >> j) & 1u) {                    \
                    v[j].x = -v[j].x;                                                                    \
                    v[j].y = -v[j].y;                                                                    \
                }                                                                                        \
            } else {                                                                                     \
                const V* row = pool + (so).mat + (c << K);                                               \
                _Pragma("unroll") for (int j = 0; j < D; ++j) v[j] = cmul(row[j], v[j]);                 \
            }                                                                                            \
        }                                                                                                \
    }
        const int s_end = s0 + ns;
        // product of the chained diagonal factor pieces not yet applied
        V ch0, ch1;
        ch0.x = T(1); ch0.y = T(0); ch1 = ch0;
        DSub<T> ra = subs[s0];
        for (int s = s0; s < s_end; s += 2) {
            const DSub<T> rb = subs[s + 1 < s_end ? s + 1 : s_end - 1];
            HSF_APPLY_SUB(ra);
            if (s + 1 >= s_end) break;
            ra = subs[s + 2 < s_end ? s + 2 : s_end - 1];
            HSF_APPLY_SUB(rb);
        }
#undef HSF_APPLY_SUB
        if constexpr (DIRECT) {
#pragma unroll
            for (int j = 0; j < D; ++j) st[gb | goff[j]] = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j) tile[sbase ^ soff[j]] = v[j];
        }
    }
}

template <typename T> struct Threads;
template <> struct Threads<float> { static constexpr int max = 512; };
template <> struct Threads<double> { static constexpr int max = 512; };

// KG: register-group width, group_bits(L) of the pass's tile.
// One tile of one path's half-state through one LDS pass: load (or set
// |0...0>), apply the pass's ops, store.  `st` is the path's row.
template <typename T, int KG, bool S1>
__device__ __forceinline__ void sweep_tile(ctab<Pass> ps, ctab<DevOp> ops, ctab<DSub<T>> subs,
                                           const typename Cx<T>::v* __restrict__ pool,
                                           typename Cx<T>::v* st, const typename Cx<T>::v* src, uint32_t t,
                                           int64_t path, typename Cx<T>::v* tile) {
    using V = typename Cx<T>::v;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = ps->n_local;
    const uint32_t E = 1u << L;
    V* mstage = tile + E;       // 256-entry matrix staging area after the tile
    uint64_t base = 0;
    const int nnl = ps->n_nonlocal;
    for (int i = 0; i < nnl; ++i) base |= (uint64_t)((t >> i) & 1u) << ps->nonlocal_q[i];
    int nc = 0;
    while (nc < L && ps->local_q[nc] == nc) ++nc;
    const uint32_t cmask = (1u << nc) - 1u;
    auto gidx = [&](uint32_t e) -> uint64_t {
        uint64_t g = base | (e & cmask);
        for (int i = nc; i < L; ++i) g |= (uint64_t)((e >> i) & 1u) << ps->local_q[i];
        return g;
    };

    if (ps->direct) {
        // the pass is one register group: row to row, no LDS tile
        const DevOp op = ops[ps->op_begin];
        apply_group<KG, T, S1, true>(tile, E, op, subs, pool, base, path, tid, nt, ps, st, src, ps->init_zero);
        return;
    }

    if (ps->init_zero) {
        for (uint32_t e = tid; e < E; e += nt) {
            V z;
            z.x = (e == 0 && base == 0) ? T(1) : T(0);
            z.y = T(0);
            tile[swz(e)] = z;
        }
    } else {
        for (uint32_t e = tid; e < E; e += nt) tile[swz(e)] = src[gidx(e)];
    }
    __syncthreads();

    const int o1 = ps->op_end;
    for (int o = ps->op_begin; o < o1; ++o) {
        const DevOp op = ops[o];
        const int type = op.type;
        if (type == DOP_GROUP) {
            apply_group<KG, T, S1>(tile, E, op, subs, pool, base, path, tid, nt);
        } else {
            // dense factor or wide gate: its matrix goes through LDS so the
            // 4^k uniform entries are read as broadcasts, not held in registers
            int32_t mat = op.mat;
            if (type == DOP_SLOT) mat += (int32_t)((path / op.stride) % op.rank) << (2 * op.k);
            const int dd = 1 << (2 * op.k);
            for (int i = tid; i < dd; i += nt) mstage[i] = pool[mat + i];
            __syncthreads();
            switch (op.k) {
                case 1: apply_dense<1>(tile, E, op.bit, mstage, tid, nt); break;
                case 2: apply_dense<2>(tile, E, op.bit, mstage, tid, nt); break;
                case 3: apply_dense<3>(tile, E, op.bit, mstage, tid, nt); break;
                default: apply_dense<4>(tile, E, op.bit, mstage, tid, nt); break;
            }
        }
        // between two wave-private groups each wave reads only what it wrote
        // itself, and a wave's LDS accesses complete in issue order: the
        // compiler fence alone keeps them in that order
        if (op.barrier) __syncthreads();
        else asm volatile("" ::: "memory");
    }

    for (uint32_t e = tid; e < E; e += nt) st[gidx(e)] = tile[swz(e)];
}

template <typename T, int KG, bool S1>
__global__ __launch_bounds__(Threads<T>::max) void sweep_pass(SideArgs s0, SideArgs s1) {
    using V = typename Cx<T>::v;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // fields picked one by one (selects of kernel arguments, no copy of a whole record)
    const bool sd = blockIdx.x >= s0.n_blocks;
#define HSF_SEL(f) (sd ? s1.f : s0.f)
    const uint32_t n_tiles = HSF_SEL(n_tiles);
    uint32_t blk = sd ? blockIdx.x - s0.n_blocks : blockIdx.x;
    const uint32_t rb = HSF_SEL(rep_blocks);
    const uint32_t r = rb ? blk / rb : 0u;
    blk -= r * rb;
    const uint32_t pl = blk / n_tiles;
    const uint32_t ti = blk - pl * n_tiles;
    uint32_t t = HSF_SEL(tile0);
    const uint32_t tfree = HSF_SEL(tile_free);
    if (tfree) {
        // the ti-th subset of tile_free's bits, in order
        uint32_t i = ti;
        for (uint32_t m = tfree; m; m &= m - 1, i >>= 1)
            if (i & 1u) t |= m & (~m + 1u);
    } else {
        t += ti;
    }
    const int64_t i = HSF_SEL(i_lo) + (int64_t)pl;
    const int64_t S = HSF_SEL(S);
    const int64_t path = max(i * S, HSF_SEL(p0));
    V* st = reinterpret_cast<V*>(HSF_SEL(psi)) + (int64_t)r * HSF_SEL(dst_rs) + (i - HSF_SEL(dst_lo)) * HSF_SEL(ld);
    const V* src = st;
    const int32_t mode = HSF_SEL(mode);
    if (mode == ROW_SHARED)
        src = reinterpret_cast<const V*>(HSF_SEL(src));
    else if (mode == ROW_PARENT)
        src = reinterpret_cast<const V*>(HSF_SEL(src)) + (int64_t)r * HSF_SEL(src_rs) +
              ((i * S) / HSF_SEL(S_par) - HSF_SEL(src_lo)) * HSF_SEL(src_ld);
    sweep_tile<T, KG, S1>(as_table(HSF_SEL(pass)), as_table(HSF_SEL(ops)),
                          as_table(reinterpret_cast<const DSub<T>*>(HSF_SEL(subs))),
                          reinterpret_cast<const V*>(HSF_SEL(pool)) + (int64_t)r * HSF_SEL(pool_rs), st, src, t,
                          path, reinterpret_cast<V*>(smem_raw));
#undef HSF_SEL
}

// Many circuits' pass k in one launch: segment i covers workgroups
// [segs[i].block_start, segs[i+1].block_start); its half-states start at
// base + psi_off.
template <typename T, int KG, bool S1>
__global__ __launch_bounds__(Threads<T>::max) void sweep_batch(const BatchSeg* __restrict__ segs_in, int nseg,
                                                               unsigned char* base) {
    using V = typename Cx<T>::v;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ctab<BatchSeg> segs = as_table(segs_in);
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].block_start <= blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const BatchSeg sg = segs[lo];
    const uint32_t blk = blockIdx.x - sg.block_start;
    const uint32_t pl = blk / sg.n_tiles;
    const uint32_t t = blk - pl * sg.n_tiles;
    // a circuit's rows hold all its paths (p0 = 0)
    const int64_t i = sg.i_lo + (int64_t)pl;
    V* st = reinterpret_cast<V*>(base + sg.psi_off) + (int64_t)pl * sg.ld;
    const V* src = st;
    if (sg.mode == ROW_SHARED)
        src = reinterpret_cast<const V*>(sg.shared);
    else if (sg.mode == ROW_PARENT)
        src = reinterpret_cast<const V*>(base + sg.src_off) + ((i * sg.S) / sg.S_par - sg.src_lo) * sg.src_ld;
    sweep_tile<T, KG, S1>(as_table(sg.pass), as_table(sg.ops), as_table(reinterpret_cast<const DSub<T>*>(sg.subs)),
                      reinterpret_cast<const V*>(sg.pool), st, src, t, i * sg.S, reinterpret_cast<V*>(smem_raw));
}

std::mutex g_dev_mutex;

hsf_status upload(const void* src, size_t bytes, void** dst) {
    hsf_status s = hip_check(hipMalloc(dst, std::max<size_t>(bytes, 64)), "hipMalloc(plan tables)");
    if (s != HSF_OK || bytes == 0) return s;
    return hip_check(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(plan tables)");
}

template <typename T>
hsf_status upload_schedule(const Schedule& sc, DeviceSchedule& d) {
    using V = typename Cx<T>::v;
    hsf_status s;
    if ((s = upload(sc.passes.data(), sc.passes.size() * sizeof(Pass), &d.passes)) != HSF_OK) return s;
    if ((s = upload(sc.devops.data(), sc.devops.size() * sizeof(DevOp), &d.ops)) != HSF_OK) return s;
    std::vector<DSub<T>> hs(sc.subs.size());
    for (size_t i = 0; i < sc.subs.size(); ++i) {
        const SubOp& so = sc.subs[i];
        DSub<T>& o = hs[i];
        std::memset(&o, 0, sizeof(o));
        o.type = so.type;
        o.g = so.g;
        o.nc = so.nc;
        o.mat = so.mat;
        for (int j = 0; j < 4; ++j) o.qb[j] = so.qb[j];
        if (so.type == SUB_SIGN) {
            for (int j = 0; j < 8; ++j) o.mask[j] = so.mask[j];
        } else if (so.type == SUB_SLOT1) {
            // digit (path / stride) % rank: a shift and a mask when both are powers of two
            const bool pow2 = so.stride > 0 && (so.stride & (so.stride - 1)) == 0 && (so.rank & (so.rank - 1)) == 0;
            int lg = 0;
            while (pow2 && (int64_t(1) << lg) < so.stride) ++lg;
            o.mask[0] = (uint32_t)so.rank;
            o.mask[1] = pow2 ? 1u : 0u;
            o.mask[2] = pow2 ? (uint32_t)lg : (uint32_t)(uint64_t)so.stride;
            o.mask[3] = pow2 ? (uint32_t)(so.rank - 1) : (uint32_t)((uint64_t)so.stride >> 32);
        }
        else
            for (int j = 0; j < 8; ++j) o.m[j] = (T)so.m[j];
    }
    if ((s = upload(hs.data(), hs.size() * sizeof(DSub<T>), &d.subs)) != HSF_OK) return s;
    std::vector<V> h(sc.pool.size());
    for (size_t i = 0; i < sc.pool.size(); ++i) {
        h[i].x = (T)sc.pool[i].real();
        h[i].y = (T)sc.pool[i].imag();
    }
    return upload(h.data(), h.size() * sizeof(V), &d.pool);
}

bool g_attr_done[2] = {false, false};

// Tile bits per register group; must match the planner's group width.

}  // namespace

int max_tile_bits(int dtype) { return dtype == HSF_C128 ? 13 : 14; }

namespace {
hsf_status launch_pass(bool dbl, int kg, bool s1, uint32_t total, int threads, size_t shmem, hipStream_t stream,
                       const SideArgs& a, const SideArgs& b);
}  // namespace

// Runs a schedule's prefix passes for a single path into a new buffer (the
// side's state after its path-independent ops); every path's first
// remaining pass then reads that buffer.
hsf_status compute_prefix(const Plan& p, DeviceSchedule& ds, const Schedule& sc, int nq) {
    if (sc.n_prefix_passes == 0) return HSF_OK;
    const bool dbl = p.dtype == HSF_C128;
    const size_t esz = dbl ? 16 : 8;
    hsf_status s = hip_check(hipMalloc(&ds.prefix, esz << std::max(nq, 0)), "hipMalloc(prefix state)");
    if (s != HSF_OK) {
        ds.prefix = nullptr;
        return s;
    }
    for (int k = 0; k < sc.n_prefix_passes; ++k) {
        const Pass& ps = sc.passes[k];
        SideArgs a, b;
        std::memset(&a, 0, sizeof(a));
        std::memset(&b, 0, sizeof(b));
        a.pass = reinterpret_cast<const Pass*>(ds.passes) + k;
        a.psi = ds.prefix;
        a.ld = int64_t(1) << std::max(nq, 0);
        a.ops = (const DevOp*)ds.ops;
        a.subs = ds.subs;
        a.pool = ds.pool;
        a.n_tiles = 1u << ps.n_nonlocal;
        a.n_blocks = a.n_tiles;
        a.S = 1;              // one row (path 0), in place
        a.mode = ROW_INPLACE;
        const uint32_t E = 1u << ps.n_local;
        const int kg = group_bits(ps.n_local);
        const int threads = (int)std::min<uint32_t>(512u, std::max<uint32_t>(64u, E >> kg));
        s = launch_pass(dbl, kg, ps.has_slot1 != 0, a.n_blocks, threads, ((size_t)E + 256) * esz, nullptr, a, b);
        if (s != HSF_OK) return s;
    }
    return HSF_OK;
}



hsf_status ensure_device(Plan& p, DeviceCopy** out) {
    int dev = 0;
    hsf_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (s != HSF_OK) return s;
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    for (DeviceCopy& d : p.dev)
        if (d.device == dev) {
            *out = &d;
            return HSF_OK;
        }
    p.dev.emplace_back();
    DeviceCopy& d = p.dev.back();
    d.device = dev;
    for (int side = 0; side < 2; ++side)
        for (int tr = 0; tr < 4; ++tr)
            for (const Schedule& sc : tr == 3   ? p.side[side].post
                                      : tr == 2 ? p.side[side].seg
                                      : tr      ? p.side[side].tree
                                                : p.side[side].sched) {
                std::vector<DeviceSchedule>& v = tr == 3 ? d.post[side] : tr == 2 ? d.seg[side] : tr ? d.tree[side] : d.side[side];
                v.emplace_back();
                s = p.dtype == HSF_C128 ? upload_schedule<double>(sc, v.back()) : upload_schedule<float>(sc, v.back());
                if (s != HSF_OK) {
                    release_device(p);
                    return s;
                }
            }
    const int di = p.dtype == HSF_C128 ? 1 : 0;
    if (!g_attr_done[di]) {
        const size_t bytes = ((size_t(1) << max_tile_bits(p.dtype)) + 256) * (p.dtype == HSF_C128 ? 16 : 8);
        const bool c128 = p.dtype == HSF_C128;
        const void* ks[4] = {c128 ? (const void*)sweep_pass<double, 3, false> : (const void*)sweep_pass<float, 3, false>,
                             c128 ? (const void*)sweep_pass<double, 4, false> : (const void*)sweep_pass<float, 4, false>,
                             c128 ? (const void*)sweep_pass<double, 3, true> : (const void*)sweep_pass<float, 3, true>,
                             c128 ? (const void*)sweep_pass<double, 4, true> : (const void*)sweep_pass<float, 4, true>};
        for (const void* kf : ks) {
            s = hip_check(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                          "hipFuncSetAttribute");
            if (s != HSF_OK) return s;
        }
        g_attr_done[di] = true;
    }
    // the shared prefix states, once per schedule (passes without factor
    // slots, one path), before any caller's work
    for (int side = 0; side < 2; ++side)
        for (int tr = 0; tr < 2; ++tr) {
            const std::vector<Schedule>& v = tr ? p.side[side].tree : p.side[side].sched;
            for (size_t q = 0; q < v.size(); ++q) {
                s = compute_prefix(p, (tr ? d.tree[side] : d.side[side])[q], v[q], p.side[side].nq);
                if (s != HSF_OK) {
                    release_device(p);
                    return s;
                }
            }
        }
    s = hip_check(hipStreamSynchronize(nullptr), "prefix states");
    if (s != HSF_OK) {
        release_device(p);
        return s;
    }
    *out = &d;
    return HSF_OK;
}

void release_device(Plan& p) {
    int cur = 0;
    if (p.dev.empty() || hipGetDevice(&cur) != hipSuccess) return;
    for (DeviceCopy& d : p.dev) {
        (void)hipSetDevice(d.device);
        for (int side = 0; side < 2; ++side)
            for (int tr = 0; tr < 4; ++tr)
                for (DeviceSchedule& ds : tr == 3 ? d.post[side] : tr == 2 ? d.seg[side] : tr ? d.tree[side] : d.side[side])
                    for (void* q : {ds.passes, ds.ops, ds.subs, ds.pool, ds.prefix})
                        if (q) (void)hipFree(q);
    }
    (void)hipSetDevice(cur);
    p.dev.clear();
}

namespace {

template <typename T, bool S1>
hsf_status launch_pass_ts(int kg, uint32_t total, int threads, size_t shmem, hipStream_t stream, const SideArgs& a,
                          const SideArgs& b) {
    switch (kg) {
        case 4: hipLaunchKernelGGL((sweep_pass<T, 4, S1>), dim3(total), dim3(threads), shmem, stream, a, b); break;
        case 3: hipLaunchKernelGGL((sweep_pass<T, 3, S1>), dim3(total), dim3(threads), shmem, stream, a, b); break;
        case 2: hipLaunchKernelGGL((sweep_pass<T, 2, S1>), dim3(total), dim3(threads), shmem, stream, a, b); break;
        default: hipLaunchKernelGGL((sweep_pass<T, 1, S1>), dim3(total), dim3(threads), shmem, stream, a, b); break;
    }
    return hip_check(hipGetLastError(), "sweep_pass launch");
}

hsf_status launch_pass(bool dbl, int kg, bool s1, uint32_t total, int threads, size_t shmem, hipStream_t stream,
                       const SideArgs& a, const SideArgs& b) {
    if (dbl)
        return s1 ? launch_pass_ts<double, true>(kg, total, threads, shmem, stream, a, b)
                  : launch_pass_ts<double, false>(kg, total, threads, shmem, stream, a, b);
    return s1 ? launch_pass_ts<float, true>(kg, total, threads, shmem, stream, a, b)
              : launch_pass_ts<float, false>(kg, total, threads, shmem, stream, a, b);
}

}  // namespace

hsf_status launch_sweep_batch(int kg, bool s1, const void* segs, int nseg, uint32_t total_blocks, int threads,
                              size_t shmem, unsigned char* base, hipStream_t stream) {
    const BatchSeg* sg = (const BatchSeg*)segs;
    if (kg == 4 && s1)
        hipLaunchKernelGGL((sweep_batch<float, 4, true>), dim3(total_blocks), dim3(threads), shmem, stream, sg, nseg, base);
    else if (kg == 4)
        hipLaunchKernelGGL((sweep_batch<float, 4, false>), dim3(total_blocks), dim3(threads), shmem, stream, sg, nseg, base);
    else if (kg == 3 && s1)
        hipLaunchKernelGGL((sweep_batch<float, 3, true>), dim3(total_blocks), dim3(threads), shmem, stream, sg, nseg, base);
    else if (kg == 3)
        hipLaunchKernelGGL((sweep_batch<float, 3, false>), dim3(total_blocks), dim3(threads), shmem, stream, sg, nseg, base);
    else
        return fail(HSF_E_UNSUPPORTED, "batched sweeps need groups of 3 or 4 tile bits");
    return hip_check(hipGetLastError(), "sweep_batch launch");
}

void batch_sweep_prepare() {
    static bool done = false;
    if (done) return;
    const size_t bytes = ((size_t(1) << max_tile_bits(HSF_C64)) + 256) * 8;
    for (const void* kf : {(const void*)sweep_batch<float, 3, false>, (const void*)sweep_batch<float, 4, false>,
                           (const void*)sweep_batch<float, 3, true>, (const void*)sweep_batch<float, 4, true>})
        (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done = true;
}

hsf_status run_segment(const Plan& p, const DeviceSchedule& ds, const Schedule& sc, void* psi, int64_t ld, int64_t rows,
                       hipStream_t stream) {
    const bool dbl = p.dtype == HSF_C128;
    const size_t esz = dbl ? 16 : 8;
    for (size_t k = 0; k < sc.passes.size(); ++k) {
        const Pass& ps = sc.passes[k];
        SideArgs a, b;
        std::memset(&a, 0, sizeof(a));
        std::memset(&b, 0, sizeof(b));
        a.pass = reinterpret_cast<const Pass*>(ds.passes) + k;
        a.psi = psi;
        a.ld = ld;
        a.ops = (const DevOp*)ds.ops;
        a.subs = ds.subs;
        a.pool = ds.pool;
        a.n_tiles = 1u << ps.n_nonlocal;
        a.S = 1;             // rows 0 .. rows-1 in place (no factor slots: digits unused)
        a.mode = ROW_INPLACE;
        const uint32_t E = 1u << ps.n_local;
        const int kg = group_bits(ps.n_local);
        const int threads = (int)std::min<uint32_t>(512u, std::max<uint32_t>(64u, E >> kg));
        const int64_t max_rows = std::max<int64_t>(1, (int64_t(1) << 29) / a.n_tiles);
        for (int64_t r0 = 0; r0 < rows; r0 += max_rows) {
            SideArgs c = a;
            c.psi = (unsigned char*)psi + (size_t)(r0 * ld) * esz;
            c.n_blocks = (uint32_t)(std::min(max_rows, rows - r0) * a.n_tiles);
            hsf_status s = launch_pass(dbl, kg, ps.has_slot1 != 0, c.n_blocks, threads, ((size_t)E + 256) * esz, stream,
                                       c, b);
            if (s != HSF_OK) return s;
        }
    }
    return HSF_OK;
}

namespace {

// Level rows of a chunk of n paths from p_begin: [p_begin / S, (p_begin + n - 1) / S].
int64_t level_rows(int64_t p_begin, int64_t n, int64_t S) { return (p_begin + n - 1) / S - p_begin / S + 1; }
// A bound on level_rows over every p_begin.
int64_t level_rows_max(int64_t n, int64_t S) { return (n - 1) / S + 2; }

}  // namespace

TreeScratch tree_scratch(const Plan& p, int64_t n_paths) {
    TreeScratch t;
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    size_t o = 0;
    for (int s = 0; s < 2; ++s) {
        if (p.side[s].tree.empty()) continue;
        const std::vector<TreeLevel>& lv = p.side[s].tree[0].levels;
        int64_t rows[2] = {0, 0};
        for (size_t l = 0; l + 1 < lv.size(); ++l)
            rows[l % 2] = std::max(rows[l % 2], level_rows_max(n_paths, lv[l].S));
        for (int b = 0; b < 2; ++b) {
            t.off[s][b] = o;
            o += ((size_t)rows[b] * ((size_t)1 << p.side[s].nq) * esz + 255) & ~size_t(255);
        }
    }
    t.total = o == 0 ? 0 : o + 256;
    return t;
}

// Flat: every per-path pass over every path of the chunk (the first reads
// the prefix state when there is one).  Tree: level by level, each level's
// rows written to its scratch buffer (the last level to psi), its first pass
// reading the prefix state or the previous level.
std::vector<SweepItem> side_items(const Schedule& sc, bool tree, const void* prefix, int64_t p_begin, int64_t n_paths,
                             void* psi, int64_t ld, unsigned char* buf0, unsigned char* buf1, int64_t dim,
                             const unsigned char* const* keep, int start, const unsigned char* parent) {
    std::vector<SweepItem> v;
    const size_t first = prefix ? (size_t)sc.n_prefix_passes : 0;
    if (!tree) {
        for (size_t k = first; k < sc.passes.size(); ++k) {
            const bool sh = k == first && prefix;
            SweepItem it{k, sh ? ROW_SHARED : ROW_INPLACE, 1, p_begin, n_paths, psi, ld, sh ? prefix : nullptr, 0, 0, 1};
            it.src_shared = sh ? 1 : 0;
            v.push_back(it);
        }
        return v;
    }
    unsigned char* buf[2] = {buf0, buf1};
    const size_t nl = sc.levels.size();
    // level l's rows below the last: its own kept buffer, else one of two
    auto level_buf = [&](size_t l) -> unsigned char* { return keep ? (unsigned char*)keep[l] : buf[l % 2]; };
    for (size_t l = (size_t)std::max(start, 0); l < nl; ++l) {
        const TreeLevel& tl = sc.levels[l];
        const int64_t lo = p_begin / tl.S, rows = level_rows(p_begin, n_paths, tl.S);
        void* dst = l + 1 == nl ? psi : (void*)level_buf(l);
        const int64_t dld = l + 1 == nl ? ld : dim;
        for (size_t k = (size_t)tl.pass_begin; k < (size_t)tl.pass_end; ++k) {
            SweepItem it{k, ROW_INPLACE, tl.S, lo, rows, dst, dld, nullptr, 0, 0, 1};
            if (k == (size_t)tl.pass_begin && l == 0 && prefix) {
                it.mode = ROW_SHARED;
                it.src = prefix;
                it.src_shared = 1;
            } else if (k == (size_t)tl.pass_begin && l > 0) {
                it.mode = ROW_PARENT;
                // a resumed run's first level reads the given parent level
                const bool resumed = (int)l == start && parent;
                it.src = resumed ? (const void*)parent : (const void*)level_buf(l - 1);
                it.src_shared = resumed ? 1 : 0;
                it.src_ld = dim;
                it.S_par = sc.levels[l - 1].S;
                it.src_lo = p_begin / it.S_par;
            }
            v.push_back(it);
        }
    }
    return v;
}

size_t level_keep_offset(const Plan& p, int64_t n_paths, int side, int l) {
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    if (p.side[side].tree.empty()) return 0;
    const std::vector<TreeLevel>& lv = p.side[side].tree[0].levels;
    size_t o = 0;
    for (int i = 0; i < l && i + 1 < (int)lv.size(); ++i)
        o += ((size_t)level_rows_max(n_paths, lv[(size_t)i].S) * ((size_t)1 << p.side[side].nq) * esz + 255) &
             ~size_t(255);
    return o;
}

size_t tree_workspace(const Plan& p, int64_t n_paths) {
    if (n_paths <= 0 || !choose_sweep(p, n_paths).tree) return 0;
    return tree_scratch(p, n_paths).total;
}

hsf_status run_sides(Plan& p, DeviceCopy& d, int64_t p_begin, int64_t n_paths, void* psiA, int64_t ldA,
                     void* psiB, int64_t ldB, void* ws, size_t ws_bytes, hipStream_t stream,
                     const SweepReplicas* reps, int64_t a_row_begin, int64_t a_row_end, const SweepLevels* levels) {
    const bool dbl = p.dtype == HSF_C128;
    const size_t esz = dbl ? 16 : 8;
    const int64_t R = reps ? std::max(1, reps->R) : 1;
    if (R > 1 && (reps->ws_rs % esz != 0 || reps->ws_rs % 256 != 0))
        return fail(HSF_E_ARG, "internal: replica workspace stride not a multiple of 256 bytes");
    // the path tree when it pays and the caller's workspace holds its levels
    SweepChoice ch = choose_sweep(p, n_paths);
    TreeScratch tsc;
    unsigned char* base = reinterpret_cast<unsigned char*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    if (ch.tree) {
        tsc = tree_scratch(p, n_paths);
        if (ws == nullptr || ws_bytes < tsc.total) ch = choose_sweep(p, n_paths, false);
    }
    const bool tree = ch.tree;
    const int pick = ch.sched;
    void* psi[2] = {psiA, psiB};
    const int64_t ld[2] = {ldA, ldB};
    const Schedule* sc[2];
    const DeviceSchedule* dsc[2];
    std::vector<SweepItem> items[2];
    size_t rounds = 0;
    for (int s = 0; s < 2; ++s) {
        const std::vector<Schedule>& hv = tree ? p.side[s].tree : p.side[s].sched;
        const std::vector<DeviceSchedule>& dv = tree ? d.tree[s] : d.side[s];
        const size_t si = std::min<size_t>((size_t)pick, hv.size() - 1);
        sc[s] = &hv[si];
        dsc[s] = &dv[si];
        if (!psi[s]) continue;
        // a side with a shared prefix state starts after its prefix passes
        std::vector<unsigned char*> keep;
        if (tree && levels && levels->keep[s]) {
            const size_t nlv = sc[s]->levels.size();
            for (size_t l = 0; l + 1 < nlv; ++l)
                keep.push_back(levels->keep[s] + level_keep_offset(p, n_paths, s, (int)l));
        }
        items[s] = side_items(*sc[s], tree, dsc[s]->prefix, p_begin, n_paths, psi[s], ld[s],
                              tree ? base + tsc.off[s][0] : nullptr, tree ? base + tsc.off[s][1] : nullptr,
                              int64_t(1) << p.side[s].nq, keep.empty() ? nullptr : keep.data(),
                              tree && levels ? levels->start[s] : 0, tree && levels ? levels->parent[s] : nullptr);
        rounds = std::max(rounds, items[s].size());
    }
    // Rows [a_row_begin, a_row_end) of side a only: walking side a's passes
    // from the last, the side-a indices still needed form a cube (free bits
    // F, the others fixed to V; first the rows, then widened by each pass's
    // tile bits, since a tile's outputs read its whole input tile).  A pass
    // need only run the tiles whose non-local bits agree with the cube (the
    // fixed ones from V, the free ones in every combination); the walk stops
    // at the first pass that needs all of its tiles.
    std::vector<uint32_t> a_tile0(items[0].size(), 0), a_ntiles(items[0].size(), 0), a_free(items[0].size(), 0);
    if (a_row_end > a_row_begin && a_row_begin >= 0 && !items[0].empty()) {
        const uint64_t diff = (uint64_t)a_row_begin ^ (uint64_t)(a_row_end - 1);
        uint64_t F = 0;
        while ((F & diff) != diff) F = (F << 1) | 1u;
        const uint64_t V = (uint64_t)a_row_begin & ~F;
        for (size_t j = items[0].size(); j-- > 0;) {
            const Pass& ps = sc[0]->passes[items[0][j].k];
            const uint64_t fixed = V & ~F;    // bits freed by later passes are no longer fixed
            uint32_t t0 = 0, tf = 0;
            for (int b = 0; b < ps.n_nonlocal; ++b) {
                t0 |= (uint32_t)((fixed >> ps.nonlocal_q[b]) & 1u) << b;
                tf |= (uint32_t)((F >> ps.nonlocal_q[b]) & 1u) << b;
            }
            const int nf = __builtin_popcount(tf);
            if (nf >= ps.n_nonlocal) break;
            a_tile0[j] = t0;
            a_ntiles[j] = 1u << nf;
            a_free[j] = tf;
            for (int i = 0; i < ps.n_local; ++i) F |= uint64_t(1) << ps.local_q[i];
        }
    }
    // rows per launch bounded so the grid stays below 2^31 workgroups
    int64_t tiles_max = 1;
    for (int s = 0; s < 2; ++s)
        for (const SweepItem& it : items[s]) tiles_max = std::max<int64_t>(tiles_max, int64_t(1) << sc[s]->passes[it.k].n_nonlocal);
    const int64_t max_rows = std::max<int64_t>(1, (int64_t(1) << 29) / (tiles_max * R));
    for (size_t j = 0; j < rounds; ++j) {
        SideArgs a[2];
        std::memset(a, 0, sizeof(a));
        const SweepItem* it[2] = {nullptr, nullptr};
        uint32_t emax = 1;
        int64_t rows_max = 0;
        for (int s = 0; s < 2; ++s) {
            if (j >= items[s].size()) continue;
            it[s] = &items[s][j];
            const SweepItem& m = *it[s];
            const Pass& ps = sc[s]->passes[m.k];
            const DeviceSchedule& ds = *dsc[s];
            a[s].pass = reinterpret_cast<const Pass*>(ds.passes) + m.k;
            a[s].psi = m.dst;
            a[s].ld = m.dst_ld;
            a[s].ops = (const DevOp*)ds.ops;
            a[s].subs = ds.subs;
            a[s].pool = ds.pool;
            a[s].n_tiles = 1u << ps.n_nonlocal;
            a[s].p0 = p_begin;
            a[s].S = m.S;
            a[s].dst_lo = m.i_lo;
            a[s].src = m.src;
            a[s].src_ld = m.src_ld;
            a[s].src_lo = m.src_lo;
            a[s].S_par = m.S_par;
            a[s].mode = m.mode;
            if (s == 0 && a_ntiles[j] > 0) {
                // only the tiles the wanted rows depend on (the cube above)
                a[s].tile0 = a_tile0[j];
                a[s].n_tiles = a_ntiles[j];
                a[s].tile_free = a_free[j];
            }
            if (R > 1) {
                // the last level writes the caller's rows, the others a copy's tree levels
                const int64_t lvl_rs = (int64_t)(reps->ws_rs / esz);
                a[s].pool_rs = reps->pool_rs;
                a[s].dst_rs = m.dst == psi[s] ? reps->psi_rs[s] : lvl_rs;
                a[s].src_rs = m.mode == ROW_PARENT && !m.src_shared ? lvl_rs : 0;
            }
            emax = std::max(emax, 1u << ps.n_local);
            rows_max = std::max(rows_max, m.rows);
        }
        // group width: every group of a pass uses group_bits(L) bits (L = that side's tile)
        int kg = 4;
        for (int s = 0; s < 2; ++s)
            if (a[s].pass) kg = std::min(kg, group_bits(sc[s]->passes[it[s]->k].n_local));
        bool kg_mixed = false;
        for (int s = 0; s < 2; ++s)
            if (a[s].pass && group_bits(sc[s]->passes[it[s]->k].n_local) != kg) kg_mixed = true;
        const int threads = (int)std::min<uint32_t>(512u, std::max<uint32_t>(64u, emax >> kg));
        const size_t shmem = ((size_t)emax + 256) * esz;
        for (int64_t r0 = 0; r0 < rows_max; r0 += max_rows) {
            SideArgs b[2] = {a[0], a[1]};
            for (int s = 0; s < 2; ++s) {
                if (!b[s].pass) continue;
                const int64_t nr = std::max<int64_t>(0, std::min(max_rows, it[s]->rows - r0));
                b[s].i_lo = it[s]->i_lo + r0;
                b[s].rep_blocks = (uint32_t)(nr * b[s].n_tiles);
                b[s].n_blocks = (uint32_t)(nr * b[s].n_tiles * R);
                if (nr == 0) b[s].pass = nullptr;
            }
            // a side with no pass this round contributes no workgroups
            const uint32_t total = b[0].n_blocks + b[1].n_blocks;
            if (total == 0) continue;
            // sides with different group widths (a side narrower than four qubits) go in separate launches
            for (int part = 0; part < (kg_mixed ? 2 : 1); ++part) {
                SideArgs c[2] = {b[0], b[1]};
                int kgp = kg;
                if (kg_mixed) {
                    c[1 - part].n_blocks = 0;
                    c[1 - part].pass = nullptr;
                    if (!c[part].pass) continue;
                    kgp = group_bits(sc[part]->passes[it[part]->k].n_local);
                }
                const uint32_t tot = c[0].n_blocks + c[1].n_blocks;
                if (tot == 0) continue;
                bool s1 = false;
                for (int q = 0; q < 2; ++q)
                    if (c[q].pass && c[q].n_blocks) s1 |= sc[q]->passes[it[q]->k].has_slot1 != 0;
                hsf_status s = launch_pass(dbl, kgp, s1, tot, threads, shmem, stream, c[0], c[1]);
                if (s != HSF_OK) return s;
            }
        }
    }
    return HSF_OK;
}

}  // namespace hsf
