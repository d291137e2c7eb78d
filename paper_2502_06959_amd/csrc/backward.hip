// Gradient with respect to rotation angles of a real loss of the amplitudes
// psi(x_j) of chosen basis states: by default L = sum_j |psi(x_j)|^2, or any
// loss whose cotangents g_j = dL/dRe psi(x_j) + i dL/dIm psi(x_j) the caller
// passes; with c_j = g_j / 2 (c_j = psi(x_j) for the default),
// dL/dt = 2 Re sum_j conj(c_j) dpsi(x_j)/dt.
//
// psi(x) = sum_p a_p[x_a] b_p[x_b] (Sec. II-B), so for an angle t of a gate
// outside every block, on side a,
//   dL/dt = 2 Re sum_p ( w_p , da_p/dt ),  w_p[y] = sum_{j: x_j,a = y} conj(psi(x_j)) b_p[x_j,b]
// with the bilinear pairing (u, v) = sum_y u[y] v[y] (side b symmetric).  With
// a_p = V U(t) V' |0>, da_p/dt = V D U V' |0> for dU/dt = D U, and
// (w, V D s) = (V^T w, D s): the adjoint lambda = V^T w is carried backwards
// through the side program (lambda <- M^T lambda), the state s backwards by
// the inverse of each gate (s <- M^dagger s).  Schmidt factors are not
// invertible, so the forward pass keeps a checkpoint of the state in front of
// every factor slot and the backward pass restores it there.
//
// Angles inside a block's hull change the block operator and with it the SVD;
// they use the shift rule on the amplitudes: every gate here is
// U(t) = exp(-i t P / 2) with P^2 = 1, so dU/dt = U(t + pi) / 2 and
// dpsi/dt = psi(t + pi) / 2 exactly, psi(t + pi) being a full forward with
// that block re-factored at t + pi: dL/dt = Re sum_j conj(c_j) psi_j(t + pi),
// one shifted forward per occurrence of the angle.
//
// Every reduction runs in a fixed order (no atomics), so results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <thread>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

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

// Fused multiply-adds in a fixed chain (the compiler contracts a*b - c*d + e
// into a multiply, an FMA and an add).
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += m x
template <typename V>
__device__ __forceinline__ void cfma(V& acc, V m, V x) {
    acc.x = fmad(m.x, x.x, acc.x);
    acc.x = fmad(-m.y, x.y, acc.x);
    acc.y = fmad(m.x, x.y, acc.y);
    acc.y = fmad(m.y, x.x, acc.y);
}

// m x, as two FMAs on top of two products
template <typename V>
__device__ __forceinline__ V cmulf(V m, V x) {
    V r;
    r.x = fmad(m.x, x.x, -(m.y * x.y));
    r.y = fmad(m.x, x.y, m.y * x.x);
    return r;
}

// m x and acc += m x for a real coefficient m.x (m.y = 0)
template <typename V>
__device__ __forceinline__ V rmul(V m, V x) {
    V r;
    r.x = m.x * x.x;
    r.y = m.x * x.y;
    return r;
}
template <typename V>
__device__ __forceinline__ void rfma(V& acc, V m, V x) {
    acc.x = fmad(m.x, x.x, acc.x);
    acc.y = fmad(m.x, x.y, acc.y);
}

// (ar, ai) += l t (no conjugate)
template <typename V, typename A>
__device__ __forceinline__ void cdot(A& ar, A& ai, V l, V t) {
    ar = fmad(l.x, t.x, ar);
    ar = fmad(-l.y, t.y, ar);
    ai = fmad(l.x, t.y, ai);
    ai = fmad(l.y, t.x, ai);
}

__device__ __forceinline__ uint64_t ins0(uint64_t i, int b) {
    const uint64_t lo = i & ((uint64_t(1) << b) - 1);
    return ((i >> b) << (b + 1)) | lo;
}

struct Bits {
    int32_t b[4];
};

template <int K>
__device__ __forceinline__ void group_offsets(const Bits& bits, uint64_t g, uint64_t (&idx)[1 << K]) {
    int sb[K];
    for (int i = 0; i < K; ++i) sb[i] = bits.b[i];
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j)
            if (sb[j] < sb[i]) {
                const int t = sb[i];
                sb[i] = sb[j];
                sb[j] = t;
            }
    uint64_t base = g;
    for (int i = 0; i < K; ++i) base = ins0(base, sb[i]);
#pragma unroll
    for (int j = 0; j < (1 << K); ++j) {
        uint64_t o = base;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((j >> (K - 1 - i)) & 1) o |= uint64_t(1) << bits.b[i];
        idx[j] = o;
    }
}

// x <- M x on every row, M = mats + ((p_begin + row) / stride % rank) * D^2.
// Grid: rows x blocks_per_row; a block works inside one row.
template <int K, typename T>
__global__ __launch_bounds__(256) void bw_apply(typename Cx<T>::v* __restrict__ x, int64_t ld, int nq, Bits bits,
                                                const typename Cx<T>::v* __restrict__ mats, int rank, int64_t stride,
                                                int64_t p_begin, uint32_t blocks_per_row) {
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    __shared__ V m[D * D];
    const uint32_t row = blockIdx.x / blocks_per_row;
    const uint32_t blk = blockIdx.x - row * blocks_per_row;
    const int sel = rank > 1 ? (int)(((p_begin + row) / stride) % rank) : 0;
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) m[i] = mats[sel * D * D + i];
    __syncthreads();
    const uint64_t groups = uint64_t(1) << (nq - K);
    const uint64_t g = (uint64_t)blk * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    V* r = x + (int64_t)row * ld;
    uint64_t idx[D];
    group_offsets<K>(bits, g, idx);
    V v[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = r[idx[j]];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        V acc;
        acc.x = 0;
        acc.y = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const V t = cmul(m[i * D + j], v[j]);
            acc.x += t.x;
            acc.y += t.y;
        }
        r[idx[i]] = acc;
    }
}

// s <- Ms s and l <- Ml l on every row (one unitary gate undone; adjoint moved back).
template <int K, typename T>
__global__ __launch_bounds__(256) void bw_apply2(typename Cx<T>::v* __restrict__ s, typename Cx<T>::v* __restrict__ l,
                                                 int64_t ld, int nq, Bits bits, const typename Cx<T>::v* __restrict__ ms,
                                                 const typename Cx<T>::v* __restrict__ ml, uint32_t blocks_per_row) {
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    __shared__ V m1[D * D], m2[D * D];
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
        m1[i] = ms[i];
        m2[i] = ml[i];
    }
    __syncthreads();
    const uint32_t row = blockIdx.x / blocks_per_row;
    const uint32_t blk = blockIdx.x - row * blocks_per_row;
    const uint64_t groups = uint64_t(1) << (nq - K);
    const uint64_t g = (uint64_t)blk * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    uint64_t idx[D];
    group_offsets<K>(bits, g, idx);
    for (int w = 0; w < 2; ++w) {
        V* r = (w ? l : s) + (int64_t)row * ld;
        const V* m = w ? m2 : m1;
        V v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = r[idx[j]];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const V t = cmul(m[i * D + j], v[j]);
                acc.x += t.x;
                acc.y += t.y;
            }
            r[idx[i]] = acc;
        }
    }
}

// bw_apply2 for an op with an angle, and first, from the same loads,
// partial[row * blocks_per_row + blk] = sum over the block's groups of
// sum_y l[y] (Dg s)[y] (FP64, fixed-order reduction in the block): the
// gradient term of the op's angle before the op is undone.
template <int K, typename T>
__global__ __launch_bounds__(256) void bw_apply2_grad(typename Cx<T>::v* __restrict__ s,
                                                      typename Cx<T>::v* __restrict__ l, int64_t ld, int nq, Bits bits,
                                                      const typename Cx<T>::v* __restrict__ ms,
                                                      const typename Cx<T>::v* __restrict__ ml,
                                                      const typename Cx<T>::v* __restrict__ dg,
                                                      double2* __restrict__ partial, uint32_t blocks_per_row) {
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    __shared__ V m1[D * D], m2[D * D], m3[D * D];
    __shared__ double rr[256], ri[256];
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
        m1[i] = ms[i];
        m2[i] = ml[i];
        m3[i] = dg[i];
    }
    __syncthreads();
    const uint32_t row = blockIdx.x / blocks_per_row;
    const uint32_t blk = blockIdx.x - row * blocks_per_row;
    const uint64_t groups = uint64_t(1) << (nq - K);
    const uint64_t g = (uint64_t)blk * blockDim.x + threadIdx.x;
    double accr = 0.0, acci = 0.0;
    if (g < groups) {
        // 32-bit element offsets (the host sends rows of under 2^31 amplitudes)
        uint32_t idx[D];
        {
            uint64_t i64[D];
            group_offsets<K>(bits, g, i64);
#pragma unroll
            for (int j = 0; j < D; ++j) idx[j] = (uint32_t)i64[j];
        }
        V* sr = s + (int64_t)row * ld;
        V* lr = l + (int64_t)row * ld;
        V vs[D], vl[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            vs[j] = sr[idx[j]];
            vl[j] = lr[idx[j]];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double tr = 0.0, ti = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const V t = cmul(m3[i * D + j], vs[j]);
                tr += (double)t.x;
                ti += (double)t.y;
            }
            accr += (double)vl[i].x * tr - (double)vl[i].y * ti;
            acci += (double)vl[i].x * ti + (double)vl[i].y * tr;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            V as, al;
            as.x = as.y = al.x = al.y = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const V t1 = cmul(m1[i * D + j], vs[j]);
                const V t2 = cmul(m2[i * D + j], vl[j]);
                as.x += t1.x;
                as.y += t1.y;
                al.x += t2.x;
                al.y += t2.y;
            }
            sr[idx[i]] = as;
            lr[idx[i]] = al;
        }
    }
    rr[threadIdx.x] = accr;
    ri[threadIdx.x] = acci;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rr[threadIdx.x] += rr[threadIdx.x + w];
            ri[threadIdx.x] += ri[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(rr[0], ri[0]);
}

// Runs of gates on at most three qubits together, at most kAdjMaxOps of them,
// are undone in registers inside the adjoint tile passes below.
constexpr int kAdjMaxOps = 16;
constexpr int kAdjMaxBits = 3;

template <typename V>
__device__ __forceinline__ void cacc(V& acc, V m, V x) {
    acc.x += m.x * x.x - m.y * x.y;
    acc.y += m.x * x.y + m.y * x.x;
}

// ---------------------------------------------------------- adjoint tiles ----
// The run units of one tile pass (their qubits all lie in the tile's qubit
// set; the host's scheduler picks them) are undone in one pass over LDS tiles of 2^L amplitudes of both the state and
// the adjoint of one path row (the tile holds the row's five lowest qubits, so
// its loads and stores are whole 256-byte runs): each run as register groups
// of its 2^K amplitudes, a barrier between runs.  Each angle's term is summed
// per thread over its groups, per wave by a butterfly of lane exchanges and
// per tile over the waves in order: one partial per (row, tile), no atomics.

// Read-only tables through the constant address space (uniform scalar loads).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using ctab = const __attribute__((address_space(4))) T*;
#else
template <typename T>
using ctab = const T*;
#endif

constexpr int kTileMaxAngles = 64;
constexpr int kTileThreads = 256;
constexpr int kTileWaves = kTileThreads / 64;
// a pass's gate matrices (M^dagger, M^T, D) are staged in LDS; at most this
// many bytes of them per pass (tile + partial slots + matrices fit twice per CU)
constexpr size_t kTileMatBytes = 12 << 10;

struct AdjTileOp {
    int32_t k, rb0, rb1, ang;      // register bits of the op's qubits (q[0] first); pass-local angle or -1
    int32_t inv, tr, dg;           // element offsets of M^dagger, M^T, D in the pass's matrix block (dg: ang >= 0)
    int32_t form;                  // FORM_*: which entries of M^dagger, M^T and D are read
};
struct AdjTileUnit {
    int32_t K, op_begin, op_end;
    int32_t bit[3];                // tile bit of register bit K - 1 - i
};
struct AdjTilePass {
    int32_t L, nc, n_nonlocal, unit_begin, unit_end, n_ang;
    int32_t local_q[16];           // ascending; local_q[i] = i for i < nc
    int32_t nonlocal_q[32];
    int64_t occ_begin;             // occurrence of angle a: occ[occ_begin + a]
    int64_t mat_begin;             // the pass's matrix block: elements [mat_begin, mat_begin + n_mat) of the table
    int32_t n_mat, pad;
};

__device__ __forceinline__ uint32_t tswz(uint32_t e) { return e ^ ((e >> 4) & 15u); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Gate helpers of the tile passes: the state takes M^dagger, the adjoint M^T,
// and an angle's term (l, D s) is accumulated first in A (FP32 for complex64
// rows: each thread sums a few dozen terms, the waves and tiles then in FP64).
// DG: M and D diagonal (RZ, RZZ, PHASE, CP), only their diagonal entries read.
// Matrix forms of a tile op (AdjTileOp::form).  One-qubit forms: REAL1, M
// real (RY), D zero on its diagonal and real (with an angle); ANTI1, D zero
// on its diagonal (RX).
enum : int32_t { FORM_DENSE = 0, FORM_DIAG = 1, FORM_REAL1 = 2, FORM_ANTI1 = 3 };

template <int K, int RB, typename V, typename A, int F>
__device__ __forceinline__ void tadj1(V (&vs)[1 << K], V (&vl)[1 << K], const V* mi, const V* mt, const V* md,
                                      A& ar, A& ai) {
    constexpr bool DG = F == FORM_DIAG;
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) {
        if (b & (1 << RB)) continue;
        const int i0 = b, i1 = b | (1 << RB);
        const V s0 = vs[i0], s1 = vs[i1], l0 = vl[i0], l1 = vl[i1];
        if constexpr (F == FORM_REAL1) {
            if (md) {
                cdot(ar, ai, l0, rmul(md[1], s1));
                cdot(ar, ai, l1, rmul(md[2], s0));
            }
            V a0 = rmul(mi[0], s0), a1 = rmul(mi[2], s0), c0 = rmul(mt[0], l0), c1 = rmul(mt[2], l0);
            rfma(a0, mi[1], s1);
            rfma(a1, mi[3], s1);
            rfma(c0, mt[1], l1);
            rfma(c1, mt[3], l1);
            vs[i0] = a0; vs[i1] = a1; vl[i0] = c0; vl[i1] = c1;
        } else if constexpr (DG) {
            if (md) {
                cdot(ar, ai, l0, cmulf(md[0], s0));
                cdot(ar, ai, l1, cmulf(md[3], s1));
            }
            vs[i0] = cmulf(mi[0], s0);
            vs[i1] = cmulf(mi[3], s1);
            vl[i0] = cmulf(mt[0], l0);
            vl[i1] = cmulf(mt[3], l1);
        } else {
            if (md) {
                if constexpr (F == FORM_ANTI1) {
                    cdot(ar, ai, l0, cmulf(md[1], s1));
                    cdot(ar, ai, l1, cmulf(md[2], s0));
                } else {
                    V t0 = cmulf(md[0], s0), t1 = cmulf(md[2], s0);
                    cfma(t0, md[1], s1);
                    cfma(t1, md[3], s1);
                    cdot(ar, ai, l0, t0);
                    cdot(ar, ai, l1, t1);
                }
            }
            V a0 = cmulf(mi[0], s0), a1 = cmulf(mi[2], s0), c0 = cmulf(mt[0], l0), c1 = cmulf(mt[2], l0);
            cfma(a0, mi[1], s1);
            cfma(a1, mi[3], s1);
            cfma(c0, mt[1], l1);
            cfma(c1, mt[3], l1);
            vs[i0] = a0; vs[i1] = a1; vl[i0] = c0; vl[i1] = c1;
        }
    }
}

// Two-qubit gate on register bits R0 (its q[0], the matrix index's high bit)
// and R1.
template <int K, int R0, int R1, typename V, typename A, bool DG>
__device__ __forceinline__ void tadj2(V (&vs)[1 << K], V (&vl)[1 << K], const V* mi, const V* mt, const V* md,
                                      A& ar, A& ai) {
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) {
        if (b & ((1 << R0) | (1 << R1))) continue;
        const int ix[4] = {b, b | (1 << R1), b | (1 << R0), b | (1 << R0) | (1 << R1)};
        V x[4], y[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            x[m] = vs[ix[m]];
            y[m] = vl[ix[m]];
        }
        if constexpr (DG) {
            if (md) {
#pragma unroll
                for (int r = 0; r < 4; ++r) cdot(ar, ai, y[r], cmulf(md[r * 5], x[r]));
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                vs[ix[r]] = cmulf(mi[r * 5], x[r]);
                vl[ix[r]] = cmulf(mt[r * 5], y[r]);
            }
        } else {
            if (md) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    V t = cmulf(md[r * 4], x[0]);
#pragma unroll
                    for (int c = 1; c < 4; ++c) cfma(t, md[r * 4 + c], x[c]);
                    cdot(ar, ai, y[r], t);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                V a = cmulf(mi[r * 4], x[0]), c2 = cmulf(mt[r * 4], y[0]);
#pragma unroll
                for (int c = 1; c < 4; ++c) {
                    cfma(a, mi[r * 4 + c], x[c]);
                    cfma(c2, mt[r * 4 + c], y[c]);
                }
                vs[ix[r]] = a;
                vl[ix[r]] = c2;
            }
        }
    }
}

template <int K, typename V, typename A, int F>
__device__ __forceinline__ void tadj_op(V (&vs)[1 << K], V (&vl)[1 << K], int k, int r0, int r1, const V* mi,
                                        const V* mt, const V* md, A& ar, A& ai) {
    constexpr bool DG = F == FORM_DIAG;
    if (k == 1) {
        switch (r0) {
            case 0: tadj1<K, 0, V, A, F>(vs, vl, mi, mt, md, ar, ai); break;
            case 1: if constexpr (K > 1) tadj1<K, 1, V, A, F>(vs, vl, mi, mt, md, ar, ai); break;
            default: if constexpr (K > 2) tadj1<K, 2, V, A, F>(vs, vl, mi, mt, md, ar, ai); break;
        }
        return;
    }
    if constexpr (K >= 2 && F <= FORM_DIAG) {
#define HSF_TADJ2(A0, B0) \
    if (r0 == A0 && r1 == B0) { if constexpr (A0 < K && B0 < K) tadj2<K, A0, B0, V, A, DG>(vs, vl, mi, mt, md, ar, ai); return; }
        HSF_TADJ2(0, 1) HSF_TADJ2(1, 0) HSF_TADJ2(0, 2) HSF_TADJ2(2, 0) HSF_TADJ2(1, 2) HSF_TADJ2(2, 1)
#undef HSF_TADJ2
    }
}

template <int K, typename T>
__device__ __forceinline__ void adj_tile_unit(typename Cx<T>::v* ts, typename Cx<T>::v* tl, uint32_t E,
                                              const AdjTileUnit& u, ctab<AdjTileOp> ops,
                                              const typename Cx<T>::v* mats, double2* wsum) {
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int sb[K];
#pragma unroll
    for (int i = 0; i < K; ++i) sb[i] = u.bit[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i + 1; j < K; ++j)
            if (sb[j] < sb[i]) {
                const int t = sb[i];
                sb[i] = sb[j];
                sb[j] = t;
            }
    uint32_t soff[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((j >> (K - 1 - i)) & 1) o |= 1u << u.bit[i];
        soff[j] = tswz(o);
    }
    const int n_ops = u.op_end - u.op_begin;
    T ar[kAdjMaxOps], ai[kAdjMaxOps];
#pragma unroll
    for (int j = 0; j < kAdjMaxOps; ++j) ar[j] = ai[j] = T(0);
    const uint32_t groups = E >> K;
    for (uint32_t g = tid; g < groups; g += kTileThreads) {
        uint32_t base = g;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint32_t lo = base & ((1u << sb[i]) - 1u);
            base = ((base >> sb[i]) << (sb[i] + 1)) | lo;
        }
        const uint32_t sbase = tswz(base);
        V vs[D], vl[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            vs[j] = ts[sbase ^ soff[j]];
            vl[j] = tl[sbase ^ soff[j]];
        }
#pragma unroll
        for (int j = 0; j < kAdjMaxOps; ++j) {
            if (j >= n_ops) break;
            const AdjTileOp op = ops[u.op_begin + j];
            const V* md = op.ang >= 0 ? mats + op.dg : nullptr;
            switch (op.form) {
                case FORM_DIAG:
                    tadj_op<K, V, T, FORM_DIAG>(vs, vl, op.k, op.rb0, op.rb1, mats + op.inv, mats + op.tr, md, ar[j],
                                                ai[j]);
                    break;
                case FORM_REAL1:
                    tadj_op<K, V, T, FORM_REAL1>(vs, vl, op.k, op.rb0, op.rb1, mats + op.inv, mats + op.tr, md, ar[j],
                                                 ai[j]);
                    break;
                case FORM_ANTI1:
                    tadj_op<K, V, T, FORM_ANTI1>(vs, vl, op.k, op.rb0, op.rb1, mats + op.inv, mats + op.tr, md, ar[j],
                                                 ai[j]);
                    break;
                default:
                    tadj_op<K, V, T, FORM_DENSE>(vs, vl, op.k, op.rb0, op.rb1, mats + op.inv, mats + op.tr, md, ar[j],
                                                 ai[j]);
                    break;
            }
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            ts[sbase ^ soff[j]] = vs[j];
            tl[sbase ^ soff[j]] = vl[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kAdjMaxOps; ++j) {
        if (j >= n_ops) break;
        const int a = ops[u.op_begin + j].ang;
        if (a < 0) continue;
        const double r = wave_sum((double)ar[j]), i = wave_sum((double)ai[j]);
        if (lane == 0) wsum[a * kTileWaves + wave] = make_double2(r, i);
    }
}

// Grid: rows x tiles per row.  partial[occ * pstride + row * n_tiles + tile].
template <typename T>
__global__ __launch_bounds__(kTileThreads) void bw_adj_tile(typename Cx<T>::v* __restrict__ s,
                                                            typename Cx<T>::v* __restrict__ l, int64_t ld,
                                                            AdjTilePass ps, const AdjTileUnit* __restrict__ units_in,
                                                            const AdjTileOp* __restrict__ ops_in,
                                                            const typename Cx<T>::v* __restrict__ mats_in,
                                                            const int64_t* __restrict__ occ, double2* partial,
                                                            int64_t pstride, uint32_t n_tiles) {
    using V = typename Cx<T>::v;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t E = 1u << ps.L;
    V* ts = reinterpret_cast<V*>(smem);
    V* tl = ts + E;
    double2* wsum = reinterpret_cast<double2*>(tl + E);
    V* sm = reinterpret_cast<V*>(wsum + kTileMaxAngles * kTileWaves);
    const ctab<AdjTileUnit> units = (ctab<AdjTileUnit>)units_in;
    const ctab<AdjTileOp> ops = (ctab<AdjTileOp>)ops_in;
    for (int i = threadIdx.x; i < ps.n_mat; i += kTileThreads) sm[i] = mats_in[ps.mat_begin + i];
    const uint32_t row = blockIdx.x / n_tiles, tile = blockIdx.x - row * n_tiles;
    uint64_t base = 0;
    for (int i = 0; i < ps.n_nonlocal; ++i) base |= (uint64_t)((tile >> i) & 1u) << ps.nonlocal_q[i];
    const uint32_t cmask = (1u << ps.nc) - 1u;
    auto gidx = [&](uint32_t e) -> uint64_t {
        uint64_t g = base | (e & cmask);
        for (int i = ps.nc; i < ps.L; ++i) g |= (uint64_t)((e >> i) & 1u) << ps.local_q[i];
        return g;
    };
    V* sr = s + (int64_t)row * ld;
    V* lr = l + (int64_t)row * ld;
    for (uint32_t e = threadIdx.x; e < E; e += kTileThreads) {
        const uint64_t g = gidx(e);
        ts[tswz(e)] = sr[g];
        tl[tswz(e)] = lr[g];
    }
    __syncthreads();
    for (int ui = ps.unit_begin; ui < ps.unit_end; ++ui) {
        const AdjTileUnit u = units[ui];
        switch (u.K) {
            case 1: adj_tile_unit<1, T>(ts, tl, E, u, ops, sm, wsum); break;
            case 2: adj_tile_unit<2, T>(ts, tl, E, u, ops, sm, wsum); break;
            default: adj_tile_unit<3, T>(ts, tl, E, u, ops, sm, wsum); break;
        }
        __syncthreads();
    }
    for (uint32_t e = threadIdx.x; e < E; e += kTileThreads) {
        const uint64_t g = gidx(e);
        sr[g] = ts[tswz(e)];
        lr[g] = tl[tswz(e)];
    }
    if ((int)threadIdx.x < ps.n_ang) {
        double2 acc = wsum[threadIdx.x * kTileWaves];
        for (int w = 1; w < kTileWaves; ++w) {
            acc.x += wsum[threadIdx.x * kTileWaves + w].x;
            acc.y += wsum[threadIdx.x * kTileWaves + w].y;
        }
        partial[occ[ps.occ_begin + threadIdx.x] * pstride + (int64_t)row * n_tiles + tile] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bw_fill(typename Cx<T>::v* __restrict__ x, int64_t ld, int64_t dim, int64_t rows,
                                               int one_at_zero) {
    const int64_t n = rows * dim;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dim, c = i - r * dim;
        typename Cx<T>::v z;
        z.x = (one_at_zero && c == 0) ? T(1) : T(0);
        z.y = T(0);
        x[r * ld + c] = z;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bw_copy_rows(const typename Cx<T>::v* __restrict__ src, int64_t lds,
                                                    typename Cx<T>::v* __restrict__ dst, int64_t ldd, int64_t dim,
                                                    int64_t rows) {
    const int64_t n = rows * dim;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dim, c = i - r * dim;
        dst[r * ldd + c] = src[r * lds + c];
    }
}

// lam[row][gidx[g]] = sum_{t in [off[g], off[g+1])} conj(psi_x[jj[t]]) other[row][oidx[jj[t]]]
template <typename T>
__global__ __launch_bounds__(256) void bw_cotangent(const typename Cx<T>::v* __restrict__ other, int64_t ldo,
                                                    typename Cx<T>::v* __restrict__ lam, int64_t ldl,
                                                    const int64_t* __restrict__ off, const int64_t* __restrict__ jj,
                                                    const int64_t* __restrict__ gidx, const int64_t* __restrict__ oidx,
                                                    const double2* __restrict__ psi_x, int64_t ngroups,
                                                    uint32_t blocks_per_row) {
    const uint32_t row = blockIdx.x / blocks_per_row;
    const int64_t g = (int64_t)(blockIdx.x - row * blocks_per_row) * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    double sr = 0.0, si = 0.0;
    for (int64_t t = off[g]; t < off[g + 1]; ++t) {
        const int64_t j = jj[t];
        const double2 c = psi_x[j];
        const auto o = other[(int64_t)row * ldo + oidx[j]];
        // conj(c) * o
        sr += c.x * (double)o.x + c.y * (double)o.y;
        si += c.x * (double)o.y - c.y * (double)o.x;
    }
    typename Cx<T>::v v;
    v.x = (T)sr;
    v.y = (T)si;
    lam[(int64_t)row * ldl + gidx[g]] = v;
}

// grad[t] += sum over occurrences o of t, over the rows x per_row[o] block
// partials of o, of 2 Re partial[o][.]: one workgroup per angle, each
// thread a strided share, then a fixed-order tree (bitwise reproducible)
__global__ __launch_bounds__(256) void bw_reduce(const double2* __restrict__ partial, int64_t stride, int64_t rows,
                                                 const int64_t* __restrict__ occ_off, const int64_t* __restrict__ occ,
                                                 const int64_t* __restrict__ per_row, double* __restrict__ grad) {
    __shared__ double r[256];
    const int64_t t = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = occ_off[t]; i < occ_off[t + 1]; ++i) {
        const double2* p = partial + occ[i] * stride;
        const int64_t n = rows * per_row[occ[i]];
        for (int64_t e = threadIdx.x; e < n; e += 256) acc += p[e].x;
    }
    r[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[t] += 2.0 * r[0];
}

__global__ void bw_zero_doubles(double* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

// out = sum_j |amp_j|^2 in a fixed order (one block)
__global__ __launch_bounds__(256) void bw_loss(const double2* __restrict__ amp, int64_t n, double* __restrict__ out) {
    __shared__ double r[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += amp[i].x * amp[i].x + amp[i].y * amp[i].y;
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = r[0];
}

// out = Re sum_j conj(c_j) amp_j in a fixed order (one workgroup per copy)
__global__ __launch_bounds__(256) void bw_shift_dot(const double2* __restrict__ c, const double2* __restrict__ amp,
                                                    int64_t n, double* __restrict__ out) {
    // workgroup r: copy r of the shifted amplitudes (amp + r n) into out[r]
    amp += (int64_t)blockIdx.x * n;
    out += blockIdx.x;
    __shared__ double r[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += c[i].x * amp[i].x + c[i].y * amp[i].y;
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = r[0];
}

// grad[t[i]] += v[i] for i = 0, 1, ..., n - 1 in that order (one thread)
__global__ void bw_shift_add(const double* __restrict__ v, const int64_t* __restrict__ t, int64_t n,
                             double* __restrict__ grad) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int64_t i = 0; i < n; ++i) grad[t[i]] += v[i];
}

// c_j = g_j / 2: the caller's cotangents as the coefficients of the adjoint
__global__ void bw_half(const double2* __restrict__ g, double2* __restrict__ c, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c[i] = make_double2(0.5 * g[i].x, 0.5 * g[i].y);
}

// ---------------------------------------------------------------- host ----

struct Layout {
    size_t adj_tiles, adj_tiles_bytes;   // tile-pass tables of the adjoint (units, ops, occurrences)
    size_t shift_t;                      // parameter id of each shifted run
    size_t vA, vB, lA, lB, ckA, ckB, psi_x, loss, partial, tables, mats, pools, tree, tree_bytes, total;
    size_t repA, repB, rep_psi, rep_tree, rep_tree_bytes;   // copies of the shifted forward run
    size_t keep, keep_off[2];            // the unshifted forward's path-tree levels below the last
    int64_t reps;          // copies per batch of shifted forward runs
    int64_t dimA, dimB;
    int ka, kb;            // checkpoints per side
    int64_t n_occ;         // parametrised ops outside blocks, both sides
    int64_t per_row_max;   // block partials per path row, largest over those ops
    int64_t n_shift;       // shifted forward runs for angles inside blocks
    size_t table_elems, mat_elems, pool_elems;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device memory of the shifted forward runs' copies (half-states, bitstring
// amplitudes and tree levels of each): one run's early path-tree levels hold
// too few states to fill the chip, so up to this much goes to running many
// shifted runs as copies of one in the same launches.
constexpr size_t kShiftCopyBytes = size_t(4) << 30;

// Workgroups per path row of the per-op adjoint kernels (one group of 2^k
// amplitudes per thread, 256 threads).
int64_t adj_blocks_per_row(int nq, int k) {
    return std::max<int64_t>(1, ((int64_t(1) << (nq - k)) + 255) / 256);
}

size_t side_mat_elems(const SideProgram& sp) {
    size_t e = 0;
    for (const SideOp& o : sp.raw) {
        const size_t d2 = (size_t)1 << (2 * o.k);
        if (o.kind == SideOp::SLOT) e += 2 * o.rank * d2;      // factors and their transposes
        else e += 3 * d2 + (o.param_id >= 0 ? d2 : 0);         // M, M^dagger, M^T (+ D)
    }
    return e;
}

// The schedules the forward runs over chunks of `chunk` paths take (tree
// levels in tree_workspace(p, chunk) bytes): used[2 side + tree][index].
// Only these get patched factor pools for the shifted runs.
std::vector<std::vector<char>> forward_schedules(const Plan& p, int64_t chunk) {
    std::vector<std::vector<char>> used(4);
    for (int s = 0; s < 2; ++s)
        for (int tr = 0; tr < 2; ++tr) used[2 * s + tr].assign((tr ? p.side[s].tree : p.side[s].sched).size(), 0);
    if (p.P <= 0) return used;
    const size_t tb = tree_workspace(p, std::min(chunk, p.P));
    std::vector<int64_t> sizes{std::min(chunk, p.P)};
    if (p.P > chunk && p.P % chunk) sizes.push_back(p.P % chunk);
    for (int64_t n : sizes) {
        SweepChoice ch = choose_sweep(p, n);
        if (ch.tree && tree_scratch(p, n).total > tb) ch = choose_sweep(p, n, false);
        for (int s = 0; s < 2; ++s) {
            std::vector<char>& u = used[2 * s + (ch.tree ? 1 : 0)];
            if (!u.empty()) u[std::min<size_t>((size_t)ch.sched, u.size() - 1)] = 1;
        }
    }
    return used;
}

// reps_cap > 0: at most that many copies per batch of shifted runs.
Layout layout(const Plan& p, int64_t chunk, int64_t nx, int64_t reps_cap = 0) {
    Layout L{};
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    L.dimA = int64_t(1) << p.na;
    L.dimB = int64_t(1) << p.nb;
    // one checkpoint per factor op of each side (a product-form block has one per qubit)
    L.ka = L.kb = 0;
    for (const SideOp& o : p.side[0].raw) L.ka += o.kind == SideOp::SLOT;
    for (const SideOp& o : p.side[1].raw) L.kb += o.kind == SideOp::SLOT;
    L.n_occ = 0;
    for (int s = 0; s < 2; ++s)
        for (const SideOp& o : p.side[s].raw) L.n_occ += o.param_id >= 0;
    // block partials per path row of the fused adjoint kernel, the most of any op with an angle
    L.per_row_max = 1;
    for (int s = 0; s < 2; ++s)
        for (const SideOp& o : p.side[s].raw)
            if (o.param_id >= 0) L.per_row_max = std::max(L.per_row_max, adj_blocks_per_row(s == 0 ? p.na : p.nb, o.k));
    L.table_elems = 2 * (size_t)(4 * nx + 1) + (size_t)(p.n_params + 1) + 2 * (size_t)L.n_occ;
    L.mat_elems = side_mat_elems(p.side[0]) + side_mat_elems(p.side[1]);
    L.pool_elems = 0;
    const std::vector<std::vector<char>> used = forward_schedules(p, chunk);
    for (int s = 0; s < 2; ++s)
        for (int tr = 0; tr < 2; ++tr) {
            const std::vector<Schedule>& v = tr ? p.side[s].tree : p.side[s].sched;
            for (size_t q = 0; q < v.size(); ++q)
                if (used[2 * s + tr][q]) L.pool_elems += std::max<size_t>(v[q].pool.size(), 1);
        }
    // shifts of angles inside blocks: one forward run per occurrence, each
    // with its own copy of the pools
    L.n_shift = 0;
    for (const Block& b : p.blocks) L.n_shift += (int64_t)b.params.size();
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.vA = take((size_t)chunk * L.dimA * esz);
    L.vB = take((size_t)chunk * L.dimB * esz);
    L.lA = take((size_t)chunk * L.dimA * esz);
    L.lB = take((size_t)chunk * L.dimB * esz);
    L.ckA = take((size_t)L.ka * chunk * L.dimA * esz);
    L.ckB = take((size_t)L.kb * chunk * L.dimB * esz);
    L.psi_x = take((size_t)nx * 16);
    L.loss = take((size_t)std::max<int64_t>(4, L.n_shift) * sizeof(double));
    L.shift_t = take((size_t)std::max<int64_t>(1, L.n_shift) * sizeof(int64_t));
    L.partial = take((size_t)std::max<int64_t>(L.n_occ, 1) * chunk * L.per_row_max * 16);
    L.tables = take(L.table_elems * sizeof(int64_t));
    L.mats = take(L.mat_elems * esz);
    L.pools = take(L.pool_elems * (size_t)std::max<int64_t>(1, L.n_shift) * esz);
    L.tree_bytes = tree_workspace(p, chunk);     // path-tree levels of the forward runs
    L.tree = take(L.tree_bytes);
    // the shifted forward runs in balanced batches of `reps` copies, within
    // kShiftCopyBytes (at least one copy)
    L.rep_tree_bytes = align256(L.tree_bytes);
    {
        const size_t per = (size_t)chunk * (L.dimA + L.dimB) * esz + (size_t)nx * 16 + L.rep_tree_bytes;
        const int64_t ns = std::max<int64_t>(1, L.n_shift);
        int64_t rmax = std::max<int64_t>(1, std::min<int64_t>(ns, (int64_t)(kShiftCopyBytes / std::max<size_t>(per, 1))));
        if (reps_cap > 0) rmax = std::min(rmax, reps_cap);
        const int64_t batches = (ns + rmax - 1) / rmax;
        L.reps = L.n_shift > 0 ? (ns + batches - 1) / batches : 0;
    }
    L.repA = take((size_t)L.reps * chunk * L.dimA * esz);
    L.repB = take((size_t)L.reps * chunk * L.dimB * esz);
    L.rep_psi = take((size_t)std::max<int64_t>(1, L.n_shift) * nx * 16);
    L.rep_tree = take((size_t)L.reps * L.rep_tree_bytes);
    // every level below the last of the unshifted forward, kept for the
    // shifted runs to start from (path trees only)
    {
        size_t kb = 0;
        for (int s = 0; s < 2; ++s) {
            L.keep_off[s] = kb;
            if (L.n_shift > 0) kb += level_keep_offset(p, chunk, s, 1 << 30);
        }
        L.keep = take(kb);
    }
    const size_t n_raw = p.side[0].raw.size() + p.side[1].raw.size();
    size_t tile_mats = 0;
    for (int s = 0; s < 2; ++s)
        for (const SideOp& o : p.side[s].raw) tile_mats += (size_t)3 << (2 * o.k);
    L.adj_tiles_bytes = n_raw * (sizeof(AdjTileUnit) + sizeof(AdjTileOp) + sizeof(int64_t)) + tile_mats * esz + 4 * 256;
    L.adj_tiles = take(L.adj_tiles_bytes);
    L.total = o + 256;
    return L;
}

template <typename T>
void to_dev(const std::vector<cd>& h, std::vector<typename Cx<T>::v>& out) {
    out.resize(h.size());
    for (size_t i = 0; i < h.size(); ++i) {
        out[i].x = (T)h[i].real();
        out[i].y = (T)h[i].imag();
    }
}

std::vector<cd> dense_of(const SideOp& o) {
    const int d = 1 << o.k;
    if (o.kind != SideOp::DIAG) return std::vector<cd>(o.m.begin(), o.m.begin() + (size_t)d * d);
    std::vector<cd> m((size_t)d * d, cd(0));
    for (int i = 0; i < d; ++i) m[(size_t)i * d + i] = o.m[i];
    return m;
}

std::vector<cd> adjoint_of(const std::vector<cd>& m, int d) {
    std::vector<cd> r((size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) r[(size_t)i * d + j] = std::conj(m[(size_t)j * d + i]);
    return r;
}

std::vector<cd> transpose_of(const std::vector<cd>& m, int d) {
    std::vector<cd> r((size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) r[(size_t)i * d + j] = m[(size_t)j * d + i];
    return r;
}

// Whether an op's matrix (and, with an angle, its D) is diagonal: two such
// ops commute even where their qubits overlap.
bool adj_diagonal(const SideOp& o) {
    if (o.kind != SideOp::DIAG) return false;
    if (o.param_id < 0) return true;
    const int d = 1 << o.k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && o.dgen[(size_t)r * d + c] != cd(0)) return false;
    return true;
}

// Which entries of a raw op's matrices the tile pass reads (FORM_*): M is
// `fwd` (2^k x 2^k); with an angle, D is the op's dgen.
int32_t adj_form(const SideOp& o, const cd* fwd) {
    if (adj_diagonal(o)) return FORM_DIAG;
    if (o.k != 1) return FORM_DENSE;
    const bool anti = o.param_id < 0 || (o.dgen[0] == cd(0) && o.dgen[3] == cd(0));
    bool real = true;
    for (int e = 0; e < 4; ++e) real = real && fwd[e].imag() == 0.0;
    if (o.param_id >= 0)
        for (int e = 0; e < 4; ++e) real = real && o.dgen[(size_t)e].imag() == 0.0;
    if (real && anti) return FORM_REAL1;
    if (anti && o.param_id >= 0) return FORM_ANTI1;
    return FORM_DENSE;
}

// The adjoint pass's units of one side, in the order it takes them: a factor
// slot alone, a gate on more than two qubits alone (and every gate of a side
// of 31 qubits or more), or a run of gates on at most kAdjMaxBits qubits
// together (at most kAdjMaxOps of them).
struct AdjUnit {
    int kind;              // 0 run, 1 slot, 2 single wide gate
    int K;
    int q[4];              // run: its qubits; register bit K - 1 - i holds q[i]
    std::vector<int> ops;  // raw indices, in the order the pass undoes them
};

// Consecutive run units undone in one pass over LDS tiles of the qubits
// local_q (ascending; the side's five lowest among them).
struct TileGroup {
    int u_begin, u_end;              // units[u_begin, u_end)
    std::vector<int> local_q;
};

int adj_tile_bits(int nq, bool c128) { return std::min(nq, c128 ? 11 : 12); }

// matrix elements an op stages in a tile pass: M^dagger, M^T (and D)
size_t tile_op_mats(const SideOp& o) { return (size_t)(o.param_id >= 0 ? 3 : 2) << (2 * o.k); }

// The adjoint pass of one side as units and tile passes.  Gates are undone in
// reverse program order up to commutation: two gates commute when their
// qubits are disjoint or both are diagonal, and then either order leaves the
// same state and adjoint, and each angle's term 2 Re <lambda, D s> (its D
// commutes with the same gates) is the same at either place.  Factor slots and
// wide gates keep their places.  Between two of them, a tile pass takes the
// side's five lowest qubits and those of the next gates up to L qubits, then
// units are built greedily: scanning the gates left in order, a gate joins
// the unit if its qubits lie in the tile, the unit stays within kAdjMaxBits
// qubits and kAdjMaxOps gates (and the pass within its angle and matrix
// slots), and no gate passed over before it fails to commute with it (a
// passed-over gate blocks its qubits for the rest of the scan).
hsf_status adj_schedule(const SideProgram& sp, int L, size_t mat_cap, std::vector<AdjUnit>& units,
                        std::vector<TileGroup>& groups) {
    const auto& raw = sp.raw;
    const int nq = sp.nq, n = (int)raw.size();
    std::vector<char> diag((size_t)n), done((size_t)n, 0);
    for (int i = 0; i < n; ++i) diag[(size_t)i] = adj_diagonal(raw[(size_t)i]);
    auto barrier = [&](int i) { return raw[(size_t)i].kind == SideOp::SLOT || raw[(size_t)i].k > 2 || nq >= 31; };
    int pos = n - 1;   // the latest op in program order not yet undone
    while (pos >= 0) {
        if (done[(size_t)pos]) {
            --pos;
            continue;
        }
        if (barrier(pos)) {
            AdjUnit a{};
            a.kind = raw[(size_t)pos].kind == SideOp::SLOT ? 1 : 2;
            a.K = raw[(size_t)pos].k;
            a.ops.push_back(pos);
            units.push_back(std::move(a));
            done[(size_t)pos] = 1;
            --pos;
            continue;
        }
        int lo = pos;     // the segment is (lo, pos]: lo is a barrier or -1
        while (lo >= 0 && !barrier(lo)) --lo;
        std::vector<char> in((size_t)nq, 0);
        int count = 0;
        for (int q = 0; q < std::min(5, L); ++q) in[(size_t)q] = 1, ++count;
        for (int i = pos; i > lo; --i) {
            if (done[(size_t)i]) continue;
            const SideOp& o = raw[(size_t)i];
            int add = 0;
            for (int e = 0; e < o.k; ++e) add += in[(size_t)o.q[e]] ? 0 : 1;
            if (count + add > L) break;
            for (int e = 0; e < o.k; ++e)
                if (!in[(size_t)o.q[e]]) in[(size_t)o.q[e]] = 1, ++count;
        }
        for (int q = 0; q < nq && count < L; ++q)
            if (!in[(size_t)q]) in[(size_t)q] = 1, ++count;
        TileGroup g;
        g.u_begin = (int)units.size();
        int angles = 0;
        size_t mats = 0;
        for (;;) {
            std::vector<char> b_dense((size_t)nq, 0), b_diag((size_t)nq, 0);   // blocked by a passed-over gate
            AdjUnit a{};
            a.kind = 0;
            int uang = 0;
            size_t umat = 0;
            for (int i = pos; i > lo; --i) {
                if (done[(size_t)i]) continue;
                const SideOp& o = raw[(size_t)i];
                bool ok = (int)a.ops.size() < kAdjMaxOps;
                int add[2], n_add = 0;
                for (int e = 0; e < o.k; ++e) {
                    const int q = o.q[e];
                    if (b_dense[(size_t)q] || (!diag[(size_t)i] && b_diag[(size_t)q]) || !in[(size_t)q]) ok = false;
                    bool have = false;
                    for (int t = 0; t < a.K; ++t) have |= a.q[t] == q;
                    if (!have) add[n_add++] = q;
                }
                if (ok && a.K + n_add > kAdjMaxBits) ok = false;
                const int ga = o.param_id >= 0 ? 1 : 0;
                const size_t gm = tile_op_mats(o);
                if (ok && (angles + uang + ga > kTileMaxAngles || mats + umat + gm > mat_cap)) ok = false;
                if (ok) {
                    for (int t = 0; t < n_add; ++t) a.q[a.K++] = add[t];
                    a.ops.push_back(i);
                    uang += ga;
                    umat += gm;
                } else {
                    for (int e = 0; e < o.k; ++e) (diag[(size_t)i] ? b_diag : b_dense)[(size_t)o.q[e]] = 1;
                }
            }
            if (a.ops.empty()) break;
            for (int i : a.ops) done[(size_t)i] = 1;
            angles += uang;
            mats += umat;
            units.push_back(std::move(a));
        }
        g.u_end = (int)units.size();
        if (g.u_end == g.u_begin) return fail(HSF_E_ARG, "internal: an adjoint tile pass took no gate");
        for (int q = 0; q < nq; ++q)
            if (in[(size_t)q]) g.local_q.push_back(q);
        groups.push_back(std::move(g));
    }
    return HSF_OK;
}

// Offsets (in complex elements, inside the backward matrix area) of each raw op's matrices.
struct OpMats {
    size_t fwd, inv, tr, dg;
};

template <typename T>
struct Runner {
    using V = typename Cx<T>::v;
    const Plan& p;
    hipStream_t st;

    template <typename F>
    hsf_status dispatch_k(int k, F f) {
        switch (k) {
            case 1: return f(std::integral_constant<int, 1>());
            case 2: return f(std::integral_constant<int, 2>());
            case 3: return f(std::integral_constant<int, 3>());
            default: return f(std::integral_constant<int, 4>());
        }
    }

    static Bits bits_of(const SideOp& o) {
        Bits b{};
        for (int i = 0; i < o.k; ++i) b.b[i] = o.q[i];
        return b;
    }

    hsf_status apply(V* x, int64_t ld, int64_t rows, int nq, const SideOp& o, const V* mats, int rank,
                     int64_t stride, int64_t p_begin) {
        const uint64_t groups = uint64_t(1) << (nq - o.k);
        const uint32_t bpr = (uint32_t)((groups + 255) / 256);
        return dispatch_k(o.k, [&](auto kk) {
            constexpr int K = decltype(kk)::value;
            hipLaunchKernelGGL((bw_apply<K, T>), dim3((uint32_t)(rows * bpr)), dim3(256), 0, st, x, ld, nq, bits_of(o),
                               mats, rank, stride, p_begin, bpr);
            return hip_check(hipGetLastError(), "bw_apply launch");
        });
    }

    hsf_status apply2(V* s, V* l, int64_t ld, int64_t rows, int nq, const SideOp& o, const V* ms, const V* ml) {
        const uint64_t groups = uint64_t(1) << (nq - o.k);
        const uint32_t bpr = (uint32_t)((groups + 255) / 256);
        return dispatch_k(o.k, [&](auto kk) {
            constexpr int K = decltype(kk)::value;
            hipLaunchKernelGGL((bw_apply2<K, T>), dim3((uint32_t)(rows * bpr)), dim3(256), 0, st, s, l, ld, nq,
                               bits_of(o), ms, ml, bpr);
            return hip_check(hipGetLastError(), "bw_apply2 launch");
        });
    }

    hsf_status apply2_grad(V* s, V* l, int64_t ld, int64_t rows, int nq, const SideOp& o, const V* ms, const V* ml,
                           const V* dg, double2* partial) {
        const uint32_t bpr = (uint32_t)adj_blocks_per_row(nq, o.k);
        return dispatch_k(o.k, [&](auto kk) {
            constexpr int K = decltype(kk)::value;
            hipLaunchKernelGGL((bw_apply2_grad<K, T>), dim3((uint32_t)(rows * bpr)), dim3(256), 0, st, s, l, ld, nq,
                               bits_of(o), ms, ml, dg, partial, bpr);
            return hip_check(hipGetLastError(), "bw_apply2_grad launch");
        });
    }


    hsf_status fill(V* x, int64_t ld, int64_t dim, int64_t rows, int one) {
        const int64_t n = rows * dim;
        const uint32_t g = (uint32_t)std::min<int64_t>(65536, (n + 255) / 256);
        hipLaunchKernelGGL(bw_fill<T>, dim3(std::max(g, 1u)), dim3(256), 0, st, x, ld, dim, rows, one);
        return hip_check(hipGetLastError(), "bw_fill launch");
    }

    hsf_status copy_rows(const V* src, int64_t lds, V* dst, int64_t ldd, int64_t dim, int64_t rows) {
        const int64_t n = rows * dim;
        const uint32_t g = (uint32_t)std::min<int64_t>(65536, (n + 255) / 256);
        hipLaunchKernelGGL(bw_copy_rows<T>, dim3(std::max(g, 1u)), dim3(256), 0, st, src, lds, dst, ldd, dim, rows);
        return hip_check(hipGetLastError(), "bw_copy_rows launch");
    }
};

template <typename T>
hsf_status backward_t(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, const double2* dl_dpsi, double* grad,
                      int64_t n_params, int64_t chunk, void* ws, size_t ws_bytes, hipStream_t st) {
    using V = typename Cx<T>::v;
    // as many copies of the shifted run per batch as the workspace holds
    Layout Lo = layout(p, chunk, nx);
    if (ws_bytes < Lo.total) {
        int64_t lo = 1, hi = std::max<int64_t>(1, Lo.reps - 1);
        if (ws_bytes < layout(p, chunk, nx, 1).total) return fail(HSF_E_ARG, "workspace too small for hsf_backward");
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (layout(p, chunk, nx, mid).total <= ws_bytes) lo = mid;
            else hi = mid - 1;
        }
        Lo = layout(p, chunk, nx, lo);
    }
    if (nx == 0 || p.n_params == 0) {
        // no bitstrings (L = 0 for every angle) or no angles: the gradient is zero
        hipLaunchKernelGGL(bw_zero_doubles, dim3(std::max<uint32_t>(1, (uint32_t)((n_params + 255) / 256))), dim3(256),
                           0, st, grad, n_params);
        return hip_check(hipGetLastError(), "zero grad");
    }
    unsigned char* base = reinterpret_cast<unsigned char*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    V* vS[2] = {(V*)(base + Lo.vA), (V*)(base + Lo.vB)};
    V* lS[2] = {(V*)(base + Lo.lA), (V*)(base + Lo.lB)};
    V* ck[2] = {(V*)(base + Lo.ckA), (V*)(base + Lo.ckB)};
    double2* psi_x = (double2*)(base + Lo.psi_x);
    double* lossb = (double*)(base + Lo.loss);
    double2* partial = (double2*)(base + Lo.partial);
    int64_t* tables = (int64_t*)(base + Lo.tables);
    V* mats = (V*)(base + Lo.mats);
    V* pools = (V*)(base + Lo.pools);
    const int64_t dim[2] = {Lo.dimA, Lo.dimB};
    const int nq[2] = {p.na, p.nb};
    hsf_status s;

    // ---- angles inside blocks (amplitude shift rule): every shifted block is
    // re-factored on host threads, started here so that they run while the
    // tables are built and the forward and adjoint passes are enqueued and run
    bool any = false;
    for (const Block& b : p.blocks) any |= !b.params.empty();
    int64_t* shift_t_d = reinterpret_cast<int64_t*>(base + Lo.shift_t);
    const std::vector<std::vector<char>> used_sched = forward_schedules(p, chunk);
    std::vector<std::vector<size_t>> pool_at(4);     // offset of a used schedule's pool in a shift's block
    struct Shift {
        size_t k;
        int64_t gid;
        int t;
    };
    std::vector<Shift> shifts;
    std::vector<int64_t> shift_ids;
    if (any) {
        // device pools of the schedules the forward runs use (flat, then
        // path-tree), to be patched per shifted block
        size_t o = 0;
        for (int side = 0; side < 2; ++side)
            for (int tr = 0; tr < 2; ++tr) {
                const std::vector<Schedule>& v = tr ? p.side[side].tree : p.side[side].sched;
                pool_at[2 * side + tr].assign(v.size(), 0);
                for (size_t q = 0; q < v.size(); ++q)
                    if (used_sched[2 * side + tr][q]) {
                        pool_at[2 * side + tr][q] = o;
                        o += std::max<size_t>(v[q].pool.size(), 1);
                    }
            }
        for (size_t k = 0; k < p.blocks.size(); ++k)
            for (const auto& gp : p.blocks[k].params)
                if (gp.second < n_params) shifts.push_back({k, gp.first, gp.second});
        for (const Shift& sh : shifts) shift_ids.push_back(sh.t);
    }
    const size_t ns = shifts.size();
    std::vector<V> staged(ns * Lo.pool_elems);     // host copy of the shifted pools; must outlive the upload
    std::vector<hsf_status> hst(ns, HSF_OK);
    std::vector<std::string> herr(ns);
    auto refactor = [&](size_t i) {
        const Shift& sh = shifts[i];
        const Block& b = p.blocks[sh.k];
        Factors fs;
        const double ang = p.gates[sh.gid].param + 2.0 * std::acos(0.0);   // theta + pi
        hsf_status e = factor_block_rank(p, b, sh.gid, ang, b.rank, fs);
        if (e != HSF_OK) {
            hst[i] = e;
            herr[i] = hsf::g_last_error_copy();
            return;
        }
        const int r = fs.rank;
        if (r > b.rank) {
            hst[i] = HSF_E_UNSUPPORTED;
            herr[i] = "a shifted block has a larger Schmidt rank than the plan's";
            return;
        }
        if (fs.product != b.product || fs.pa.size() != b.pa.size() || fs.pb.size() != b.pb.size()) {
            hst[i] = HSF_E_UNSUPPORTED;
            herr[i] = "a shifted block changes its decomposition form";
            return;
        }
        // patched pools: factors of block k replaced (missing ranks zero)
        std::vector<cd> all;
        all.reserve(Lo.pool_elems);
        for (int side = 0; side < 2; ++side) {
            const std::vector<FactorPiece>& pcs = side == 0 ? fs.pa : fs.pb;
            for (int tr = 0; tr < 2; ++tr)
            for (size_t q = 0; q < (tr ? p.side[side].tree : p.side[side].sched).size(); ++q) {
                if (!used_sched[2 * side + tr][q]) continue;
                const Schedule& sc = (tr ? p.side[side].tree : p.side[side].sched)[q];
                std::vector<cd> pl = sc.pool;
                // rank m's matrix of a patched piece, with the gates the
                // plan folded into that piece (post * f_m)
                auto patched = [&](const std::vector<cd>& f, int m, size_t d2, const std::vector<cd>& post) {
                    std::vector<cd> fm(f.begin() + (size_t)m * d2, f.begin() + (size_t)(m + 1) * d2);
                    if (post.empty()) return fm;
                    std::vector<cd> out(4, cd(0));
                    for (int i = 0; i < 2; ++i)
                        for (int j = 0; j < 2; ++j)
                            for (int l = 0; l < 2; ++l) out[(size_t)i * 2 + j] += post[(size_t)i * 2 + l] * fm[(size_t)l * 2 + j];
                    return out;
                };
                for (const DevOp& op : sc.devops)
                    if (op.type == DOP_SLOT && op.block == (int)sh.k) {
                        const std::vector<cd>& f = pcs[op.piece].m;
                        const size_t d2 = (size_t)1 << (2 * op.k);
                        static const std::vector<cd> none;
                        const std::vector<cd>* post = &none;
                        for (const SideOp& so : p.side[side].ops)
                            if (so.kind == SideOp::SLOT && so.block == op.block && so.piece == op.piece) post = &so.post;
                        for (int m = 0; m < b.rank; ++m) {
                            const std::vector<cd> fm = m < r ? patched(f, m, d2, *post) : std::vector<cd>(d2, cd(0));
                            for (size_t e2 = 0; e2 < d2; ++e2) pl[op.mat + m * d2 + e2] = fm[e2];
                        }
                    }
                // one-qubit factor pieces applied inside register groups
                for (const SubOp& so : sc.subs)
                    if (so.type == SUB_SLOT1 && so.block == (int)sh.k) {
                        const std::vector<cd>& f = pcs[so.piece].m;
                        for (int m = 0; m < b.rank; ++m) {
                            const std::vector<cd> fm = m < r ? patched(f, m, 4, so.post) : std::vector<cd>(4, cd(0));
                            for (size_t e2 = 0; e2 < 4; ++e2) pl[so.mat + m * 4 + e2] = fm[e2];
                        }
                    }
                if (pl.empty()) pl.push_back(cd(0));
                all.insert(all.end(), pl.begin(), pl.end());
            }
        }
        std::vector<V> av;
        to_dev<T>(all, av);
        std::copy(av.begin(), av.end(), staged.begin() + i * Lo.pool_elems);
    };
    // joined before the pools are uploaded, and on every exit
    std::atomic<size_t> next_shift(0);
    struct Workers {
        std::vector<std::thread> t;
        void join() {
            for (std::thread& th : t)
                if (th.joinable()) th.join();
        }
        ~Workers() { join(); }
    } workers;
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        // a few cores stay free for this thread's enqueueing and the runtime's
        const size_t nthr = std::min<size_t>(ns, std::min(12u, hw));
        for (size_t w = 0; w < nthr; ++w)
            workers.t.emplace_back([&]() {
                for (size_t i = next_shift++; i < ns; i = next_shift++) refactor(i);
            });
    }

    const int tbits[2] = {adj_tile_bits(p.na, p.dtype == HSF_C128), adj_tile_bits(p.nb, p.dtype == HSF_C128)};
    const size_t mat_cap = kTileMatBytes / sizeof(V);
    std::vector<AdjUnit> units[2];
    std::vector<TileGroup> tgroups[2];
    for (int side = 0; side < 2; ++side)
        if ((s = adj_schedule(p.side[side], tbits[side], mat_cap, units[side], tgroups[side])) != HSF_OK) return s;

    // ---- host tables: bitstring groups per side, parameter occurrences
    std::vector<uint64_t> hx((size_t)std::max<int64_t>(nx, 1));
    if (nx > 0) {
        if ((s = hip_check(hipMemcpyAsync(hx.data(), x, nx * sizeof(uint64_t), hipMemcpyDeviceToHost, st), "copy x")) != HSF_OK)
            return s;
        if ((s = hip_check(hipStreamSynchronize(st), "sync")) != HSF_OK) return s;
    }
    const uint64_t maskn = p.n >= 64 ? ~uint64_t(0) : ((uint64_t(1) << p.n) - 1);
    const uint64_t maskb = (uint64_t(1) << p.nb) - 1;
    std::vector<int64_t> ht(Lo.table_elems, 0);
    int64_t ngroups[2] = {0, 0};
    size_t toff[2][4];   // off, jj, gidx, oidx
    {
        size_t o = 0;
        for (int side = 0; side < 2; ++side) {
            std::vector<std::pair<int64_t, int64_t>> key(nx);   // (own index, j)
            for (int64_t j = 0; j < nx; ++j) {
                const uint64_t xj = hx[j] & maskn;
                const int64_t own = side == 0 ? (int64_t)(xj >> p.nb) : (int64_t)(xj & maskb);
                key[j] = {own, j};
            }
            std::sort(key.begin(), key.end());
            toff[side][0] = o;
            toff[side][1] = o + nx + 1;
            toff[side][2] = o + 2 * nx + 1;
            toff[side][3] = o + 3 * nx + 1;
            int64_t ng = 0;
            for (int64_t t = 0; t < nx; ++t) {
                if (t == 0 || key[t].first != key[t - 1].first) {
                    ht[toff[side][0] + ng] = t;
                    ht[toff[side][2] + ng] = key[t].first;
                    ++ng;
                }
                ht[toff[side][1] + t] = key[t].second;
            }
            ht[toff[side][0] + ng] = nx;
            ngroups[side] = ng;
            for (int64_t j = 0; j < nx; ++j) {
                const uint64_t xj = hx[j] & maskn;
                ht[toff[side][3] + j] = side == 0 ? (int64_t)(xj & maskb) : (int64_t)(xj >> p.nb);
            }
            o += 4 * (size_t)nx + 1;
        }
        // occurrences: param id -> raw-op occurrence numbers (side a first, program order)
        const size_t occ_off = o, occ_list = o + (size_t)p.n_params + 1;
        std::vector<std::vector<int64_t>> per(p.n_params);
        int64_t occ = 0;
        for (int side = 0; side < 2; ++side)
            for (const SideOp& op : p.side[side].raw)
                if (op.param_id >= 0) per[op.param_id].push_back(occ++);
        int64_t w = 0;
        for (int64_t t = 0; t < p.n_params; ++t) {
            ht[occ_off + t] = w;
            for (int64_t q : per[t]) ht[occ_list + w++] = q;
        }
        ht[occ_off + p.n_params] = w;
        // block partials per row of each occurrence: those of the adjoint
        // unit that holds its gate
        const size_t occ_rows = occ_list + (size_t)Lo.n_occ;
        int64_t q = 0;
        for (int side = 0; side < 2; ++side) {
            // angles of run units: one partial per (row, tile) of their tile
            // pass; wider gates: one per workgroup of their own kernel
            std::vector<int> width(p.side[side].raw.size(), 1);
            std::vector<char> in_run(p.side[side].raw.size(), 0);
            for (const AdjUnit& a : units[side])
                for (int i : a.ops) {
                    width[(size_t)i] = a.K;
                    in_run[(size_t)i] = a.kind == 0;
                }
            const int64_t n_tiles = int64_t(1) << (nq[side] - tbits[side]);
            for (size_t i = 0; i < p.side[side].raw.size(); ++i)
                if (p.side[side].raw[i].param_id >= 0)
                    ht[occ_rows + q++] = in_run[i] ? n_tiles : adj_blocks_per_row(nq[side], width[i]);
        }
        if ((s = hip_check(hipMemcpyAsync(tables, ht.data(), ht.size() * sizeof(int64_t), hipMemcpyHostToDevice, st),
                           "upload tables")) != HSF_OK)
            return s;
    }
    const int64_t* occ_off_d = tables + 2 * (4 * nx + 1);
    const int64_t* occ_d = occ_off_d + p.n_params + 1;
    const int64_t* occ_rows_d = occ_d + Lo.n_occ;
    const int64_t pstride = chunk * Lo.per_row_max;

    // ---- matrices of the raw side programs
    std::vector<std::vector<OpMats>> om(2);
    std::vector<cd> hm;
    hm.reserve(Lo.mat_elems);
    for (int side = 0; side < 2; ++side)
        for (const SideOp& o : p.side[side].raw) {
            const int dd = 1 << o.k;
            OpMats m{};
            if (o.kind == SideOp::SLOT) {
                m.fwd = hm.size();
                hm.insert(hm.end(), o.m.begin(), o.m.end());
                m.tr = hm.size();
                for (int r = 0; r < o.rank; ++r) {
                    std::vector<cd> f(o.m.begin() + (size_t)r * dd * dd, o.m.begin() + (size_t)(r + 1) * dd * dd);
                    const std::vector<cd> t = transpose_of(f, dd);
                    hm.insert(hm.end(), t.begin(), t.end());
                }
            } else {
                const std::vector<cd> M = dense_of(o);
                m.fwd = hm.size();
                hm.insert(hm.end(), M.begin(), M.end());
                m.inv = hm.size();
                const std::vector<cd> a = adjoint_of(M, dd);
                hm.insert(hm.end(), a.begin(), a.end());
                m.tr = hm.size();
                const std::vector<cd> t = transpose_of(M, dd);
                hm.insert(hm.end(), t.begin(), t.end());
                if (o.param_id >= 0) {
                    m.dg = hm.size();
                    hm.insert(hm.end(), o.dgen.begin(), o.dgen.end());
                }
            }
            om[side].push_back(m);
        }
    std::vector<V> hmv;
    to_dev<T>(hm, hmv);
    if (!hmv.empty() &&
        (s = hip_check(hipMemcpyAsync(mats, hmv.data(), hmv.size() * sizeof(V), hipMemcpyHostToDevice, st), "upload mats")) != HSF_OK)
        return s;

    // occurrence of each raw op with an angle (numbered in program order, side
    // a first), -1 for the others
    std::vector<int64_t> occ_of[2];
    {
        int64_t q = 0;
        for (int side = 0; side < 2; ++side) {
            occ_of[side].assign(p.side[side].raw.size(), -1);
            for (size_t i = 0; i < p.side[side].raw.size(); ++i)
                if (p.side[side].raw[i].param_id >= 0) occ_of[side][i] = q++;
        }
    }

    // ---- tile-pass tables of the adjoint: units, ops, angle occurrences
    std::vector<AdjTileUnit> tu;
    std::vector<AdjTileOp> to;
    std::vector<int64_t> tocc;
    std::vector<cd> tmats;             // each pass's matrices, contiguous
    std::vector<AdjTilePass> tpass[2];
    {
        for (int side = 0; side < 2; ++side) {
            const auto& raw = p.side[side].raw;
            for (const TileGroup& g : tgroups[side]) {
                AdjTilePass ps{};
                ps.L = (int)g.local_q.size();
                std::vector<int> tbit(nq[side], -1);
                for (int i = 0; i < ps.L; ++i) {
                    ps.local_q[i] = g.local_q[i];
                    tbit[g.local_q[i]] = i;
                }
                ps.nc = 0;
                while (ps.nc < ps.L && ps.local_q[ps.nc] == ps.nc) ++ps.nc;
                for (int qq = 0; qq < nq[side]; ++qq)
                    if (tbit[qq] < 0) ps.nonlocal_q[ps.n_nonlocal++] = qq;
                ps.unit_begin = (int)tu.size();
                ps.occ_begin = (int64_t)tocc.size();
                ps.mat_begin = (int64_t)tmats.size();
                auto stage = [&](size_t at, int k) {
                    const int32_t off = (int32_t)(tmats.size() - (size_t)ps.mat_begin);
                    tmats.insert(tmats.end(), hm.begin() + (int64_t)at, hm.begin() + (int64_t)(at + ((size_t)1 << (2 * k))));
                    return off;
                };
                for (int ui = g.u_begin; ui < g.u_end; ++ui) {
                    const AdjUnit& u = units[side][(size_t)ui];
                    AdjTileUnit r{};
                    r.K = u.K;
                    for (int t = 0; t < u.K; ++t) r.bit[t] = tbit[u.q[t]];
                    r.op_begin = (int)to.size();
                    for (int ri_ : u.ops) {
                        const size_t ri = (size_t)ri_;
                        const SideOp& gop = raw[ri];
                        AdjTileOp op{};
                        op.k = gop.k;
                        for (int e = 0; e < gop.k; ++e) {
                            int pos = 0;
                            while (u.q[pos] != gop.q[e]) ++pos;
                            (e == 0 ? op.rb0 : op.rb1) = u.K - 1 - pos;
                        }
                        op.inv = stage(om[side][ri].inv, gop.k);
                        op.tr = stage(om[side][ri].tr, gop.k);
                        op.form = adj_form(gop, hm.data() + om[side][ri].fwd);
                        op.ang = -1;
                        if (gop.param_id >= 0) {
                            op.dg = stage(om[side][ri].dg, gop.k);
                            op.ang = ps.n_ang++;
                            tocc.push_back(occ_of[side][ri]);
                        }
                        to.push_back(op);
                    }
                    r.op_end = (int)to.size();
                    tu.push_back(r);
                }
                ps.unit_end = (int)tu.size();
                ps.n_mat = (int32_t)(tmats.size() - (size_t)ps.mat_begin);
                tpass[side].push_back(ps);
            }
        }
    }
    AdjTileUnit* tu_d = reinterpret_cast<AdjTileUnit*>(base + Lo.adj_tiles);
    AdjTileOp* to_d = reinterpret_cast<AdjTileOp*>(base + Lo.adj_tiles + align256(tu.size() * sizeof(AdjTileUnit)));
    int64_t* tocc_d = reinterpret_cast<int64_t*>(reinterpret_cast<unsigned char*>(to_d) +
                                                 align256(to.size() * sizeof(AdjTileOp)));
    V* tmats_d = reinterpret_cast<V*>(reinterpret_cast<unsigned char*>(tocc_d) + align256(tocc.size() * sizeof(int64_t)));
    std::vector<V> tmats_v;
    to_dev<T>(tmats, tmats_v);
    if (!tu.empty()) {
        if (align256(tu.size() * sizeof(AdjTileUnit)) + align256(to.size() * sizeof(AdjTileOp)) +
                align256(tocc.size() * sizeof(int64_t)) + tmats_v.size() * sizeof(V) > Lo.adj_tiles_bytes)
            return fail(HSF_E_ARG, "internal: adjoint tile tables exceed their workspace");
        if ((s = hip_check(hipMemcpyAsync(tmats_d, tmats_v.data(), tmats_v.size() * sizeof(V), hipMemcpyHostToDevice,
                                          st),
                           "upload tile matrices")) != HSF_OK)
            return s;
        if ((s = hip_check(hipMemcpyAsync(tu_d, tu.data(), tu.size() * sizeof(AdjTileUnit), hipMemcpyHostToDevice, st),
                           "upload tile units")) != HSF_OK ||
            (s = hip_check(hipMemcpyAsync(to_d, to.data(), to.size() * sizeof(AdjTileOp), hipMemcpyHostToDevice, st),
                           "upload tile ops")) != HSF_OK)
            return s;
        if (!tocc.empty() &&
            (s = hip_check(hipMemcpyAsync(tocc_d, tocc.data(), tocc.size() * sizeof(int64_t), hipMemcpyHostToDevice, st),
                           "upload tile occurrences")) != HSF_OK)
            return s;
        for (int side = 0; side < 2; ++side)
            if (!tpass[side].empty()) {
                const size_t shm = 2 * ((size_t)1 << tbits[side]) * sizeof(V) +
                                   (size_t)kTileMaxAngles * kTileWaves * sizeof(double2) + kTileMatBytes;
                if ((s = hip_check(hipFuncSetAttribute((const void*)bw_adj_tile<T>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm),
                                   "hipFuncSetAttribute")) != HSF_OK)
                    return s;
            }
    }

    Runner<T> R{p, st};
    hipLaunchKernelGGL(bw_zero_doubles, dim3(std::max<uint32_t>(1, (uint32_t)((n_params + 255) / 256))), dim3(256), 0, st,
                       grad, n_params);
    if ((s = hip_check(hipGetLastError(), "zero grad")) != HSF_OK) return s;

    // ---- coefficients c_j: psi(x_j) for every bitstring (tiled forward over
    // all paths), or half the caller's cotangents
    if (dl_dpsi) {
        hipLaunchKernelGGL(bw_half, dim3((uint32_t)std::min<int64_t>(1024, (nx + 255) / 256)), dim3(256), 0, st,
                           dl_dpsi, psi_x, nx);
        if ((s = hip_check(hipGetLastError(), "bw_half launch")) != HSF_OK) return s;
    } else {
        for (int64_t p0 = 0; p0 < p.P; p0 += chunk) {
            const int64_t np = std::min(chunk, p.P - p0);
            if ((s = run_sides(p, d, p0, np, vS[0], dim[0], vS[1], dim[1], base + Lo.tree, Lo.tree_bytes, st)) !=
                HSF_OK)
                return s;
            if ((s = gather_dot(p.dtype, vS[0], dim[0], vS[1], dim[1], np, p.nb, p.n, x, nx, psi_x, p0 > 0 ? 1 : 0,
                                st)) != HSF_OK)
                return s;
        }
    }

    // ---- angles inside blocks: amplitude shift rule on the re-factored block.
    // The shifted forwards need only the coefficients c_j and the re-factored
    // blocks.  They run in batches of Lo.reps copies of one forward run (the
    // same launches, each copy with its own block's factors at the shifted
    // angle) on a stream of their own (default priority), which starts once
    // the coefficients are on the device, beside the adjoint pass on the
    // caller's stream.  The guard drains that stream and the caller's (host
    // staging buffers declared above may still be read) and destroys it on
    // every exit.
    struct ShiftStream {
        hipStream_t st = nullptr, caller = nullptr;
        std::vector<hipEvent_t> evs;
        hsf_status record(hipStream_t on, hipEvent_t* out) {
            hipEvent_t e = nullptr;
            hsf_status r = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
            if (r != HSF_OK) return r;
            evs.push_back(e);
            *out = e;
            return hip_check(hipEventRecord(e, on), "hipEventRecord");
        }
        ~ShiftStream() {
            if (caller) (void)hipStreamSynchronize(caller);
            if (st) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
            }
            for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        }
    } ss;
    ss.caller = st;
    if (ns > 0) {
        if ((s = hip_check(hipMemcpyAsync(shift_t_d, shift_ids.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, st),
                           "upload shift ids")) != HSF_OK)
            return s;
        hipEvent_t start = nullptr;
        if ((s = ss.record(st, &start)) != HSF_OK ||
            (s = hip_check(hipStreamCreateWithFlags(&ss.st, hipStreamNonBlocking), "hipStreamCreate")) != HSF_OK ||
            (s = hip_check(hipStreamWaitEvent(ss.st, start, 0), "hipStreamWaitEvent")) != HSF_OK)
            return s;
    }
    // ---- adjoint over angles outside blocks
    const int64_t* gt[2][4];
    for (int side = 0; side < 2; ++side)
        for (int i = 0; i < 4; ++i) gt[side][i] = tables + toff[side][i];
    for (int64_t p0 = 0; p0 < p.P; p0 += chunk) {
        const int64_t np = std::min(chunk, p.P - p0);
        // forward replay with a checkpoint in front of every factor slot: the
        // runs of ops between slots as LDS passes (their segment schedules),
        // each slot as one launch
        for (int side = 0; side < 2; ++side) {
            if ((s = R.fill(vS[side], dim[side], dim[side], np, 1)) != HSF_OK) return s;
            int kc = 0;
            size_t sg = 0;
            const SideProgram& sp = p.side[side];
            const auto& raw = sp.raw;
            for (size_t i = 0; i < raw.size(); ++i) {
                const SideOp& o = raw[i];
                if (o.kind == SideOp::SLOT) {
                    if (kc >= (side == 0 ? Lo.ka : Lo.kb))
                        return fail(HSF_E_ARG, "internal: more factor slots than checkpoints");
                    V* c = ck[side] + (size_t)kc * chunk * dim[side];
                    if ((s = R.copy_rows(vS[side], dim[side], c, dim[side], dim[side], np)) != HSF_OK) return s;
                    ++kc;
                    s = R.apply(vS[side], dim[side], np, nq[side], o, mats + om[side][i].fwd, o.rank, o.stride, p0);
                } else if (sg < sp.seg.size() && (size_t)sp.seg_lo[sg] == i) {
                    s = run_segment(p, d.seg[side][sg], sp.seg[sg], vS[side], dim[side], np, st);
                    i = (size_t)sp.seg_hi[sg] - 1;
                    ++sg;
                } else {
                    s = R.apply(vS[side], dim[side], np, nq[side], o, mats + om[side][i].fwd, 1, 1, p0);
                }
                if (s != HSF_OK) return s;
            }
        }
        // cotangents: lambda_a from psi_x and side b, lambda_b from psi_x and side a
        for (int side = 0; side < 2; ++side) {
            if ((s = R.fill(lS[side], dim[side], dim[side], np, 0)) != HSF_OK) return s;
            const int other = 1 - side;
            const uint32_t bpr = (uint32_t)std::max<int64_t>(1, (ngroups[side] + 255) / 256);
            if (ngroups[side] > 0) {
                hipLaunchKernelGGL(bw_cotangent<T>, dim3((uint32_t)(np * bpr)), dim3(256), 0, st, vS[other], dim[other],
                                   lS[side], dim[side], gt[side][0], gt[side][1], gt[side][2], gt[side][3],
                                   (const double2*)psi_x, ngroups[side], bpr);
                if ((s = hip_check(hipGetLastError(), "bw_cotangent launch")) != HSF_OK) return s;
            }
        }
        // backward sweep
        for (int side = 0; side < 2; ++side) {
            const auto& raw = p.side[side].raw;
            int kc = 0;
            for (const SideOp& o : raw) kc += o.kind == SideOp::SLOT;
            size_t tg = 0;                    // next tile pass of this side
            for (size_t ui = 0; ui < units[side].size(); ++ui) {
                const AdjUnit& u = units[side][ui];
                const int ii = u.ops[0];
                if (tg < tgroups[side].size() && (size_t)tgroups[side][tg].u_begin == ui) {
                    // a tile pass over this and the following run units
                    const AdjTilePass& ps = tpass[side][tg];
                    const uint32_t n_tiles = 1u << (nq[side] - ps.L);
                    if (ps.n_ang > 0 && (int64_t)n_tiles > Lo.per_row_max)
                        return fail(HSF_E_ARG, "internal: more adjoint tiles per row than partial slots");
                    const size_t shm = 2 * ((size_t)1 << ps.L) * sizeof(V) +
                                       (size_t)kTileMaxAngles * kTileWaves * sizeof(double2) + kTileMatBytes;
                    hipLaunchKernelGGL(bw_adj_tile<T>, dim3((uint32_t)(np * n_tiles)), dim3(kTileThreads), shm, st,
                                       vS[side], lS[side], dim[side], ps, tu_d, to_d, tmats_d, tocc_d, partial,
                                       pstride, n_tiles);
                    if ((s = hip_check(hipGetLastError(), "bw_adj_tile launch")) != HSF_OK) return s;
                    ui = (size_t)tgroups[side][tg].u_end - 1;
                    ++tg;
                    continue;
                }
                const SideOp& o = raw[(size_t)ii];
                if (u.kind == 1) {
                    if (o.param_id >= 0) return fail(HSF_E_ARG, "internal: an angle on a factor slot");
                    --kc;
                    V* c = ck[side] + (size_t)kc * chunk * dim[side];
                    if ((s = R.copy_rows(c, dim[side], vS[side], dim[side], dim[side], np)) != HSF_OK) return s;
                    if ((s = R.apply(lS[side], dim[side], np, nq[side], o, mats + om[side][ii].tr, o.rank, o.stride, p0)) != HSF_OK)
                        return s;
                    continue;
                }
                if (u.kind == 2) {
                    if (o.param_id >= 0) {
                        // the angle's term from the state and adjoint after the gate, then the gate undone
                        s = R.apply2_grad(vS[side], lS[side], dim[side], np, nq[side], o, mats + om[side][ii].inv,
                                          mats + om[side][ii].tr, mats + om[side][ii].dg,
                                          partial + occ_of[side][(size_t)ii] * pstride);
                    } else {
                        s = R.apply2(vS[side], lS[side], dim[side], np, nq[side], o, mats + om[side][ii].inv,
                                     mats + om[side][ii].tr);
                    }
                    if (s != HSF_OK) return s;
                    continue;
                }
                return fail(HSF_E_ARG, "internal: a register run outside every adjoint tile pass");
            }
        }
        if (p.n_params > 0) {
            hipLaunchKernelGGL(bw_reduce, dim3((uint32_t)p.n_params), dim3(256), 0, st, (const double2*)partial, pstride,
                               np, occ_off_d, occ_d, occ_rows_d, grad);
            if ((s = hip_check(hipGetLastError(), "bw_reduce launch")) != HSF_OK) return s;
        }
    }

    if (ns > 0) {
        workers.join();
        for (size_t i = 0; i < ns; ++i)
            if (hst[i] != HSF_OK) return fail(hst[i], herr[i]);
        // one upload for all shifted pools (the host copy lives until the final sync)
        if ((s = hip_check(hipMemcpyAsync(pools, staged.data(), staged.size() * sizeof(V), hipMemcpyHostToDevice,
                                          ss.st),
                           "upload shifted factors")) != HSF_OK)
            return s;
        V* repS[2] = {(V*)(base + Lo.repA), (V*)(base + Lo.repB)};
        double2* rpsi = (double2*)(base + Lo.rep_psi);
        unsigned char* keep[2] = {base + Lo.keep + Lo.keep_off[0], base + Lo.keep + Lo.keep_off[1]};
        DeviceCopy dd = d;
        // batches: runs of shifts of one block, at most Lo.reps each
        std::vector<std::pair<size_t, int>> batches;
        for (size_t i0 = 0; i0 < ns;) {
            size_t i1 = i0 + 1;
            while (i1 < ns && i1 - i0 < (size_t)Lo.reps && shifts[i1].k == shifts[i0].k) ++i1;
            batches.push_back({i0, (int)(i1 - i0)});
            i0 = i1;
        }
        for (int64_t p0 = 0; p0 < p.P; p0 += chunk) {
            const int64_t np = std::min(chunk, p.P - p0);
            // the unshifted forward of this chunk, its levels below the last kept
            SweepLevels kl;
            kl.keep[0] = keep[0];
            kl.keep[1] = keep[1];
            if ((s = run_sides(p, d, p0, np, repS[0], dim[0], repS[1], dim[1], base + Lo.rep_tree, Lo.tree_bytes,
                               ss.st, nullptr, 0, -1, &kl)) != HSF_OK)
                return s;
            for (const auto& bt : batches) {
                // shifts i0 .. i0 + R - 1 of block k: copy r reads the pools of shift i0 + r
                const size_t i0 = bt.first;
                const int R = bt.second;
                for (int side = 0; side < 2; ++side)
                    for (int tr = 0; tr < 2; ++tr) {
                        std::vector<DeviceSchedule>& dv = tr ? dd.tree[side] : dd.side[side];
                        for (size_t q = 0; q < dv.size(); ++q)
                            if (used_sched[2 * side + tr][q])
                                dv[q].pool = pools + i0 * Lo.pool_elems + pool_at[2 * side + tr][q];
                    }
                // the copies start at each side's first level whose states
                // depend on block k's digit (S <= its stride), from the kept
                // level before it: the earlier levels do not see the shift
                SweepLevels rl;
                const int64_t stride = p.blocks[shifts[i0].k].stride;
                for (int side = 0; side < 2; ++side) {
                    if (p.side[side].tree.empty()) continue;
                    const std::vector<TreeLevel>& lv = p.side[side].tree[0].levels;
                    int st0 = 0;
                    while (st0 + 1 < (int)lv.size() && lv[(size_t)st0].S > stride) ++st0;
                    rl.start[side] = st0;
                    rl.parent[side] = st0 > 0 ? keep[side] + level_keep_offset(p, np, side, st0 - 1) : nullptr;
                }
                const SweepReplicas rp{R, (int64_t)Lo.pool_elems, {chunk * dim[0], chunk * dim[1]},
                                       Lo.rep_tree_bytes};
                if ((s = run_sides(p, dd, p0, np, repS[0], dim[0], repS[1], dim[1], base + Lo.rep_tree,
                                   Lo.tree_bytes, ss.st, &rp, 0, -1, &rl)) != HSF_OK ||
                    (s = gather_dot(p.dtype, repS[0], dim[0], repS[1], dim[1], np, p.nb, p.n, x, nx,
                                    rpsi + i0 * (size_t)nx, p0 > 0 ? 1 : 0, ss.st, R, chunk * dim[0],
                                    chunk * dim[1])) != HSF_OK)
                    return s;
            }
        }
        hipLaunchKernelGGL(bw_shift_dot, dim3((uint32_t)ns), dim3(256), 0, ss.st, (const double2*)psi_x,
                           (const double2*)rpsi, nx, lossb);
        if ((s = hip_check(hipGetLastError(), "bw_shift_dot launch")) != HSF_OK) return s;
        // the caller's stream waits for the shifted runs, then dL/dt +=
        // Re sum_j conj(c_j) psi_j(t + pi) per occurrence, in plan order
        hipEvent_t done = nullptr;
        if ((s = ss.record(ss.st, &done)) != HSF_OK ||
            (s = hip_check(hipStreamWaitEvent(st, done, 0), "hipStreamWaitEvent")) != HSF_OK)
            return s;
        hipLaunchKernelGGL(bw_shift_add, dim3(1), dim3(1), 0, st, lossb, shift_t_d, (int64_t)ns, grad);
        if ((s = hip_check(hipGetLastError(), "bw_shift_add launch")) != HSF_OK) return s;
    }
    // host staging buffers above must outlive their async uploads
    return hip_check(hipStreamSynchronize(st), "sync");
}

}  // namespace

size_t backward_workspace(const Plan& p, int64_t chunk, int64_t nx, bool minimal) {
    return layout(p, chunk, nx, minimal ? 1 : 0).total;
}

// hsf_loss: half-states of both sides per path chunk, then psi(x_j)
// accumulated over the chunks (FP64), then L = sum_j |psi(x_j)|^2.
size_t loss_workspace(const Plan& p, int64_t chunk, int64_t nx) {
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    return align256((size_t)chunk * ((size_t)1 << p.na) * esz) + align256((size_t)chunk * ((size_t)1 << p.nb) * esz) +
           align256((size_t)nx * 16) + align256(tree_workspace(p, chunk)) + 256;
}

hsf_status prob_mass(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, double* loss, void* amps, int64_t chunk,
                     void* ws, size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < loss_workspace(p, chunk, nx)) return fail(HSF_E_ARG, "workspace too small for hsf_loss");
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    const int64_t dA = int64_t(1) << p.na, dB = int64_t(1) << p.nb;
    unsigned char* b = reinterpret_cast<unsigned char*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    void* vA = b;
    b += align256((size_t)chunk * dA * esz);
    void* vB = b;
    b += align256((size_t)chunk * dB * esz);
    double2* amp = amps ? (double2*)amps : (double2*)b;
    b += align256((size_t)nx * 16);
    unsigned char* tree = b;
    const size_t tree_bytes = tree_workspace(p, chunk);
    hsf_status s = HSF_OK;
    if (nx > 0) {
        if (p.P == 0) {
            hipLaunchKernelGGL(bw_zero_doubles, dim3((uint32_t)std::min<int64_t>(1024, (2 * nx + 255) / 256)),
                               dim3(256), 0, st, (double*)amp, 2 * nx);
            if ((s = hip_check(hipGetLastError(), "zero amplitudes")) != HSF_OK) return s;
        }
        for (int64_t p0 = 0; p0 < p.P; p0 += chunk) {
            const int64_t np = std::min(chunk, p.P - p0);
            if ((s = run_sides(p, d, p0, np, vA, dA, vB, dB, tree, tree_bytes, st)) != HSF_OK) return s;
            if ((s = gather_dot(p.dtype, vA, dA, vB, dB, np, p.nb, p.n, x, nx, amp, p0 > 0 ? 1 : 0, st)) != HSF_OK)
                return s;
        }
    }
    hipLaunchKernelGGL(bw_loss, dim3(1), dim3(256), 0, st, (const double2*)amp, nx, loss);
    return hip_check(hipGetLastError(), "bw_loss launch");
}

hsf_status backward(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, const void* dl_dpsi, double* grad,
                    int64_t n_params, int64_t chunk, void* ws, size_t ws_bytes, hipStream_t stream) {
    const double2* g = (const double2*)dl_dpsi;
    if (p.dtype == HSF_C128) return backward_t<double>(p, d, x, nx, g, grad, n_params, chunk, ws, ws_bytes, stream);
    return backward_t<float>(p, d, x, nx, g, grad, n_params, chunk, ws, ws_bytes, stream);
}

}  // namespace hsf
