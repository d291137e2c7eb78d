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

// A run of consecutive gates (program order reversed) on at most three
// qubits (four need more registers than the kernel's occupancy allows),
// undone in registers in one pass over the rows: each thread holds the
// 2^K amplitudes of the state and of the adjoint that differ in those qubits.
constexpr int kAdjMaxOps = 8;
constexpr int kAdjMaxBits = 3;
struct AdjRun {
    int32_t n_ops;
    int32_t k[kAdjMaxOps];             // 1 or 2
    int32_t rb[kAdjMaxOps][2];         // register bits of the op's qubits (q[0] first)
    const void* inv[kAdjMaxOps];       // M^dagger, M^T and (angle ops) D, 2^k x 2^k
    const void* tr[kAdjMaxOps];
    const void* dg[kAdjMaxOps];        // null: no angle
    double2* partial[kAdjMaxOps];      // block partials of the angle's term
};

template <typename V>
__device__ __forceinline__ void cacc(V& acc, V m, V x) {
    acc.x += m.x * x.x - m.y * x.y;
    acc.y += m.x * x.y + m.y * x.x;
}

// One-qubit gate on register bit RB of both register sets, with the angle's
// term first when md is set.
template <int K, int RB, typename V>
__device__ __forceinline__ void adj1(V (&vs)[1 << K], V (&vl)[1 << K], const V* mi, const V* mt, const V* md,
                                     double& ar, double& ai) {
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) {
        if (b & (1 << RB)) continue;
        // matrices are re-read from LDS per pair (broadcasts) rather than held
        asm volatile("" ::: "memory");
        const int i0 = b, i1 = b | (1 << RB);
        const V s0 = vs[i0], s1 = vs[i1], l0 = vl[i0], l1 = vl[i1];
        if (md) {
            V t0, t1;
            t0.x = t0.y = t1.x = t1.y = 0;
            cacc(t0, md[0], s0); cacc(t0, md[1], s1);
            cacc(t1, md[2], s0); cacc(t1, md[3], s1);
            ar += (double)l0.x * t0.x - (double)l0.y * t0.y + (double)l1.x * t1.x - (double)l1.y * t1.y;
            ai += (double)l0.x * t0.y + (double)l0.y * t0.x + (double)l1.x * t1.y + (double)l1.y * t1.x;
        }
        V a0, a1, c0, c1;
        a0.x = a0.y = a1.x = a1.y = c0.x = c0.y = c1.x = c1.y = 0;
        cacc(a0, mi[0], s0); cacc(a0, mi[1], s1);
        cacc(a1, mi[2], s0); cacc(a1, mi[3], s1);
        cacc(c0, mt[0], l0); cacc(c0, mt[1], l1);
        cacc(c1, mt[2], l0); cacc(c1, mt[3], l1);
        vs[i0] = a0; vs[i1] = a1; vl[i0] = c0; vl[i1] = c1;
    }
}

// Two-qubit gate on register bits R0 (its q[0], the matrix index's high bit)
// and R1.
template <int K, int R0, int R1, typename V>
__device__ __forceinline__ void adj2(V (&vs)[1 << K], V (&vl)[1 << K], const V* mi, const V* mt, const V* md,
                                     double& ar, double& ai) {
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) {
        if (b & ((1 << R0) | (1 << R1))) continue;
        asm volatile("" ::: "memory");
        const int ix[4] = {b, b | (1 << R1), b | (1 << R0), b | (1 << R0) | (1 << R1)};
        V x[4], y[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            x[m] = vs[ix[m]];
            y[m] = vl[ix[m]];
        }
        // one matrix at a time (fences keep the compiler from loading all
        // three 4x4 matrices at once)
        if (md) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                V t;
                t.x = t.y = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) cacc(t, md[r * 4 + c], x[c]);
                ar += (double)y[r].x * t.x - (double)y[r].y * t.y;
                ai += (double)y[r].x * t.y + (double)y[r].y * t.x;
            }
            asm volatile("" ::: "memory");
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            V a;
            a.x = a.y = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) cacc(a, mi[r * 4 + c], x[c]);
            vs[ix[r]] = a;
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            V c2;
            c2.x = c2.y = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) cacc(c2, mt[r * 4 + c], y[c]);
            vl[ix[r]] = c2;
        }
    }
}

template <int K, typename V>
__device__ __forceinline__ void adj_op(V (&vs)[1 << K], V (&vl)[1 << K], int k, int r0, int r1, const V* mi,
                                       const V* mt, const V* md, double& ar, double& ai) {
    if (k == 1) {
        switch (r0) {
            case 0: adj1<K, 0>(vs, vl, mi, mt, md, ar, ai); break;
            case 1: if constexpr (K > 1) adj1<K, 1>(vs, vl, mi, mt, md, ar, ai); break;
            case 2: if constexpr (K > 2) adj1<K, 2>(vs, vl, mi, mt, md, ar, ai); break;
            default: if constexpr (K > 3) adj1<K, 3>(vs, vl, mi, mt, md, ar, ai); break;
        }
        return;
    }
    if constexpr (K >= 2) {
#define HSF_ADJ2(A, B) \
    if (r0 == A && r1 == B) { if constexpr (A < K && B < K) adj2<K, A, B>(vs, vl, mi, mt, md, ar, ai); return; }
        HSF_ADJ2(0, 1) HSF_ADJ2(1, 0) HSF_ADJ2(0, 2) HSF_ADJ2(2, 0) HSF_ADJ2(0, 3) HSF_ADJ2(3, 0)
        HSF_ADJ2(1, 2) HSF_ADJ2(2, 1) HSF_ADJ2(1, 3) HSF_ADJ2(3, 1) HSF_ADJ2(2, 3) HSF_ADJ2(3, 2)
#undef HSF_ADJ2
    }
}

// The run's gates in order on every row (grid: rows x blocks_per_row, one
// group of 2^K amplitudes per thread), each angle's term from the state and
// adjoint just after its gate, reduced per workgroup in a fixed order.
template <int K, typename T>
__global__ __launch_bounds__(256) void bw_adj_run(typename Cx<T>::v* __restrict__ s, typename Cx<T>::v* __restrict__ l,
                                                  int64_t ld, int nq, Bits bits, AdjRun a, uint32_t blocks_per_row) {
    using V = typename Cx<T>::v;
    constexpr int D = 1 << K;
    __shared__ V mm[kAdjMaxOps][3][16];
    __shared__ double rr[kAdjMaxOps][256], ri[kAdjMaxOps][256];
#pragma unroll
    for (int j = 0; j < kAdjMaxOps; ++j) {
        if (j >= a.n_ops) break;
        const int d2 = 1 << (2 * a.k[j]);
        for (int i = threadIdx.x; i < d2; i += blockDim.x) {
            mm[j][0][i] = reinterpret_cast<const V*>(a.inv[j])[i];
            mm[j][1][i] = reinterpret_cast<const V*>(a.tr[j])[i];
            if (a.dg[j]) mm[j][2][i] = reinterpret_cast<const V*>(a.dg[j])[i];
        }
    }
    __syncthreads();
    const uint32_t row = blockIdx.x / blocks_per_row;
    const uint32_t blk = blockIdx.x - row * blocks_per_row;
    const uint64_t groups = uint64_t(1) << (nq - K);
    const uint64_t g = (uint64_t)blk * blockDim.x + threadIdx.x;
    // each thread's share of every angle's term, parked in LDS right after
    // its gate (threads past the last group contribute zero)
#pragma unroll
    for (int j = 0; j < kAdjMaxOps; ++j) {
        if (j >= a.n_ops) break;
        rr[j][threadIdx.x] = 0.0;
        ri[j][threadIdx.x] = 0.0;
    }
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
        // one copy of each gate form's code: the run's table is read by index
#pragma unroll 1
        for (int j = 0; j < a.n_ops; ++j) {
            double ar = 0.0, ai = 0.0;
            adj_op<K>(vs, vl, a.k[j], a.rb[j][0], a.rb[j][1], mm[j][0], mm[j][1], a.dg[j] ? mm[j][2] : nullptr, ar, ai);
            rr[j][threadIdx.x] = ar;
            ri[j][threadIdx.x] = ai;
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sr[idx[j]] = vs[j];
            lr[idx[j]] = vl[j];
        }
    }
    __syncthreads();
    // fixed-order tree over the workgroup for every angle at once
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < kAdjMaxOps; ++j) {
                if (j >= a.n_ops) break;
                rr[j][threadIdx.x] += rr[j][threadIdx.x + w];
                ri[j][threadIdx.x] += ri[j][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kAdjMaxOps; ++j) {
            if (j >= a.n_ops) break;
            if (a.dg[j]) a.partial[j][blockIdx.x] = make_double2(rr[j][0], ri[j][0]);
        }
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

// out = Re sum_j conj(c_j) amp_j in a fixed order (one block)
__global__ __launch_bounds__(256) void bw_shift_dot(const double2* __restrict__ c, const double2* __restrict__ amp,
                                                    int64_t n, double* __restrict__ out) {
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

__global__ void bw_shift_add(const double* __restrict__ v, double* __restrict__ grad, int64_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) grad[t] += *v;
}

// c_j = g_j / 2: the caller's cotangents as the coefficients of the adjoint
__global__ void bw_half(const double2* __restrict__ g, double2* __restrict__ c, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c[i] = make_double2(0.5 * g[i].x, 0.5 * g[i].y);
}

// ---------------------------------------------------------------- host ----

struct Layout {
    size_t vA, vB, lA, lB, ckA, ckB, psi_x, psi_s, loss, partial, tables, mats, pools, tree, tree_bytes, lane,
        lane_bytes, total;
    int lanes;             // concurrent shifted forward runs
    int64_t dimA, dimB;
    int ka, kb;            // checkpoints per side
    int64_t n_occ;         // parametrised ops outside blocks, both sides
    int64_t per_row_max;   // block partials per path row, largest over those ops
    int64_t n_shift;       // shifted forward runs for angles inside blocks
    size_t table_elems, mat_elems, pool_elems;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Streams the parameter-shift forward runs share: the early path-tree levels
// of one run hold too few states to fill the chip, so several runs go at
// once (at most the hardware queues a process gets by default).
constexpr int kShiftLanes = 4;

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

Layout layout(const Plan& p, int64_t chunk, int64_t nx) {
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
    for (int s = 0; s < 2; ++s)
        for (int tr = 0; tr < 2; ++tr)
            for (const Schedule& sc : tr ? p.side[s].tree : p.side[s].sched)
                L.pool_elems += std::max<size_t>(sc.pool.size(), 1);
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
    L.psi_s = take((size_t)nx * 16);
    L.loss = take((size_t)std::max<int64_t>(4, L.n_shift) * sizeof(double));
    L.partial = take((size_t)std::max<int64_t>(L.n_occ, 1) * chunk * L.per_row_max * 16);
    L.tables = take(L.table_elems * sizeof(int64_t));
    L.mats = take(L.mat_elems * esz);
    L.pools = take(L.pool_elems * (size_t)std::max<int64_t>(1, L.n_shift) * esz);
    L.tree_bytes = tree_workspace(p, chunk);     // path-tree levels of the forward runs
    L.tree = take(L.tree_bytes);
    // the shifted forward runs go round kShiftLanes streams; lanes past the
    // first bring their own half-states, bitstring amplitudes and tree levels
    L.lanes = (int)std::min<int64_t>(kShiftLanes, std::max<int64_t>(1, L.n_shift));
    L.lane_bytes = align256((size_t)chunk * L.dimA * esz) + align256((size_t)chunk * L.dimB * esz) +
                   align256((size_t)nx * 16) + align256(L.tree_bytes);
    L.lane = take(L.lane_bytes * (size_t)(L.lanes - 1));
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

// The adjoint pass's units of one side, in the order it takes them (program
// order reversed): a factor slot alone, a gate on more than two qubits alone
// (and every gate of a side of 31 qubits or more), or a run of consecutive
// gates on at most kAdjMaxBits qubits together (at most kAdjMaxOps of them),
// raw indices hi, hi - 1, ..., hi - n + 1.
struct AdjUnit {
    int kind;             // 0 run, 1 slot, 2 single wide gate
    int hi, n, K;
    int q[4];             // run: its qubits; register bit K - 1 - i holds q[i]
};

std::vector<AdjUnit> adj_units(const SideProgram& sp) {
    std::vector<AdjUnit> u;
    const auto& raw = sp.raw;
    for (int ii = (int)raw.size() - 1; ii >= 0;) {
        AdjUnit a{};
        a.hi = ii;
        a.n = 1;
        const SideOp& o = raw[ii];
        if (o.kind == SideOp::SLOT || o.k > 2 || sp.nq >= 31) {
            a.kind = o.kind == SideOp::SLOT ? 1 : 2;
            a.K = o.k;
            u.push_back(a);
            --ii;
            continue;
        }
        a.kind = 0;
        for (int j = 0; j < o.k; ++j) a.q[a.K++] = o.q[j];
        int j = ii - 1;
        while (j >= 0 && a.n < kAdjMaxOps && raw[j].kind != SideOp::SLOT && raw[j].k <= 2 && sp.nq < 31) {
            int qq[4], nq = a.K;
            for (int t = 0; t < a.K; ++t) qq[t] = a.q[t];
            bool fits = true;
            for (int t = 0; t < raw[j].k && fits; ++t) {
                bool have = false;
                for (int r = 0; r < nq; ++r) have |= qq[r] == raw[j].q[t];
                if (!have) {
                    if (nq == kAdjMaxBits) fits = false;
                    else qq[nq++] = raw[j].q[t];
                }
            }
            if (!fits) break;
            a.K = nq;
            for (int t = 0; t < nq; ++t) a.q[t] = qq[t];
            ++a.n;
            --j;
        }
        u.push_back(a);
        ii = j;
    }
    return u;
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

    hsf_status adj_run(V* s, V* l, int64_t ld, int64_t rows, int nq, const Bits& bits, int K, const AdjRun& a) {
        const uint32_t bpr = (uint32_t)adj_blocks_per_row(nq, K);
        auto go = [&](auto kk) {
            constexpr int KK = decltype(kk)::value;
            hipLaunchKernelGGL((bw_adj_run<KK, T>), dim3((uint32_t)(rows * bpr)), dim3(256), 0, st, s, l, ld, nq, bits,
                               a, bpr);
            return hip_check(hipGetLastError(), "bw_adj_run launch");
        };
        switch (K) {
            case 1: return go(std::integral_constant<int, 1>());
            case 2: return go(std::integral_constant<int, 2>());
            case 3: return go(std::integral_constant<int, 3>());
            default: return fail(HSF_E_ARG, "internal: an adjoint run wider than three qubits");
        }
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
    const Layout Lo = layout(p, chunk, nx);
    if (ws_bytes < Lo.total) return fail(HSF_E_ARG, "workspace too small for hsf_backward");
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
    double2* psi_s = (double2*)(base + Lo.psi_s);
    double* lossb = (double*)(base + Lo.loss);
    double2* partial = (double2*)(base + Lo.partial);
    int64_t* tables = (int64_t*)(base + Lo.tables);
    V* mats = (V*)(base + Lo.mats);
    V* pools = (V*)(base + Lo.pools);
    const int64_t dim[2] = {Lo.dimA, Lo.dimB};
    const int nq[2] = {p.na, p.nb};
    hsf_status s;

    const std::vector<AdjUnit> units[2] = {adj_units(p.side[0]), adj_units(p.side[1])};

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
            std::vector<int> width(p.side[side].raw.size(), 1);
            for (const AdjUnit& a : units[side])
                for (int t = 0; t < a.n; ++t) width[(size_t)(a.hi - t)] = a.K;
            for (size_t i = 0; i < p.side[side].raw.size(); ++i)
                if (p.side[side].raw[i].param_id >= 0) ht[occ_rows + q++] = adj_blocks_per_row(nq[side], width[i]);
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
        int64_t occ = 0;
        for (int side = 0; side < 2; ++side) {
            const auto& raw = p.side[side].raw;
            int64_t occ_side = occ;
            for (const SideOp& o : raw) occ += o.param_id >= 0;
            int64_t oc = occ;                 // occurrences are numbered in program order
            int kc = 0;
            for (const SideOp& o : raw) kc += o.kind == SideOp::SLOT;
            for (const AdjUnit& u : units[side]) {
                const int ii = u.hi;
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
                        --oc;
                        s = R.apply2_grad(vS[side], lS[side], dim[side], np, nq[side], o, mats + om[side][ii].inv,
                                          mats + om[side][ii].tr, mats + om[side][ii].dg, partial + oc * pstride);
                    } else {
                        s = R.apply2(vS[side], lS[side], dim[side], np, nq[side], o, mats + om[side][ii].inv,
                                     mats + om[side][ii].tr);
                    }
                    if (s != HSF_OK) return s;
                    continue;
                }
                // a run of gates in registers, each angle's term at its gate
                AdjRun a{};
                a.n_ops = u.n;
                Bits bits{};
                for (int t = 0; t < u.K; ++t) bits.b[t] = u.q[t];
                for (int t = 0; t < u.n; ++t) {
                    const SideOp& g = raw[(size_t)(ii - t)];
                    a.k[t] = g.k;
                    for (int e = 0; e < g.k; ++e) {
                        int pos = 0;
                        while (u.q[pos] != g.q[e]) ++pos;
                        a.rb[t][e] = u.K - 1 - pos;
                    }
                    a.inv[t] = mats + om[side][(size_t)(ii - t)].inv;
                    a.tr[t] = mats + om[side][(size_t)(ii - t)].tr;
                    a.dg[t] = nullptr;
                    a.partial[t] = nullptr;
                    if (g.param_id >= 0) {
                        --oc;
                        a.dg[t] = mats + om[side][(size_t)(ii - t)].dg;
                        a.partial[t] = partial + oc * pstride;
                    }
                }
                if ((s = R.adj_run(vS[side], lS[side], dim[side], np, nq[side], bits, u.K, a)) != HSF_OK) return s;
            }
            (void)occ_side;
        }
        if (p.n_params > 0) {
            hipLaunchKernelGGL(bw_reduce, dim3((uint32_t)p.n_params), dim3(256), 0, st, (const double2*)partial, pstride,
                               np, occ_off_d, occ_d, occ_rows_d, grad);
            if ((s = hip_check(hipGetLastError(), "bw_reduce launch")) != HSF_OK) return s;
        }
    }

    // ---- angles inside blocks: amplitude shift rule on the re-factored block
    bool any = false;
    for (const Block& b : p.blocks) any |= !b.params.empty();
    std::vector<V> staged;    // host copy of the shifted pools; must outlive the upload (final sync)
    if (any) {
        // device pools of every schedule (flat, then path-tree), to be
        // patched per shifted block
        std::vector<std::vector<size_t>> pool_at(4);
        size_t o = 0;
        for (int side = 0; side < 2; ++side)
            for (int tr = 0; tr < 2; ++tr)
                for (const Schedule& sc : tr ? p.side[side].tree : p.side[side].sched) {
                    pool_at[2 * side + tr].push_back(o);
                    o += std::max<size_t>(sc.pool.size(), 1);
                }
        const double pi = 2.0 * std::acos(0.0);
        struct Shift {
            size_t k;
            int64_t gid;
            int t;
        };
        std::vector<Shift> shifts;
        for (size_t k = 0; k < p.blocks.size(); ++k)
            for (const auto& gp : p.blocks[k].params)
                if (gp.second < n_params) shifts.push_back({k, gp.first, gp.second});
        const size_t ns = shifts.size();
        // every shifted block re-factored on the host, in parallel (they are
        // independent), into its own patched copy of the pools
        staged.assign(ns * Lo.pool_elems, V{});
        std::vector<hsf_status> hst(ns, HSF_OK);
        std::vector<std::string> herr(ns);
        auto refactor = [&](size_t i) {
            const Shift& sh = shifts[i];
            const Block& b = p.blocks[sh.k];
            Factors fs;
            const double ang = p.gates[sh.gid].param + pi;
            hsf_status e = factor_block(p, b, sh.gid, ang, fs);
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
                for (const Schedule& sc : tr ? p.side[side].tree : p.side[side].sched) {
                    std::vector<cd> pl = sc.pool;
                    for (const DevOp& op : sc.devops)
                        if (op.type == DOP_SLOT && op.block == (int)sh.k) {
                            const std::vector<cd>& f = pcs[op.piece].m;
                            const size_t d2 = (size_t)1 << (2 * op.k);
                            for (int m = 0; m < b.rank; ++m)
                                for (size_t e2 = 0; e2 < d2; ++e2)
                                    pl[op.mat + m * d2 + e2] = m < r ? f[m * d2 + e2] : cd(0);
                        }
                    // one-qubit factor pieces applied inside register groups
                    for (const SubOp& so : sc.subs)
                        if (so.type == SUB_SLOT1 && so.block == (int)sh.k) {
                            const std::vector<cd>& f = pcs[so.piece].m;
                            for (int m = 0; m < b.rank; ++m)
                                for (size_t e2 = 0; e2 < 4; ++e2)
                                    pl[so.mat + m * 4 + e2] = m < r ? f[m * 4 + e2] : cd(0);
                        }
                    if (pl.empty()) pl.push_back(cd(0));
                    all.insert(all.end(), pl.begin(), pl.end());
                }
            }
            std::vector<V> av;
            to_dev<T>(all, av);
            std::copy(av.begin(), av.end(), staged.begin() + i * Lo.pool_elems);
        };
        {
            const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
            const size_t nthr = std::min<size_t>(ns, std::min(16u, hw));
            std::atomic<size_t> next(0);
            std::vector<std::thread> pool_threads;
            for (size_t w = 0; w < nthr; ++w)
                pool_threads.emplace_back([&]() {
                    for (size_t i = next++; i < ns; i = next++) refactor(i);
                });
            for (std::thread& th : pool_threads) th.join();
        }
        for (size_t i = 0; i < ns; ++i)
            if (hst[i] != HSF_OK) return fail(hst[i], herr[i]);
        // one upload for all shifted pools (the host copy lives until the final sync)
        if ((s = hip_check(hipMemcpyAsync(pools, staged.data(), staged.size() * sizeof(V), hipMemcpyHostToDevice, st),
                           "upload shifted factors")) != HSF_OK)
            return s;
        // shift i runs on lane i mod lanes: lane 0 on the caller's stream with
        // the buffers above, the others on streams of their own (default
        // priority) that start after everything queued so far
        const int nl = (int)std::max<size_t>(1, std::min<size_t>((size_t)Lo.lanes, ns));
        struct Lane {
            hipStream_t st;
            V* v[2];
            double2* psi;
            unsigned char* tree;
        };
        std::vector<Lane> lanes((size_t)nl);
        std::vector<hipEvent_t> evs;
        auto cleanup = [&]() {
            for (size_t l = 1; l < lanes.size(); ++l)
                if (lanes[l].st) (void)hipStreamDestroy(lanes[l].st);
            for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        };
        lanes[0] = {st, {vS[0], vS[1]}, psi_s, base + Lo.tree};
        hipEvent_t start = nullptr;
        if (nl > 1) {
            if ((s = hip_check(hipEventCreateWithFlags(&start, hipEventDisableTiming), "hipEventCreate")) != HSF_OK)
                return s;
            evs.push_back(start);
            if ((s = hip_check(hipEventRecord(start, st), "hipEventRecord")) != HSF_OK) {
                cleanup();
                return s;
            }
        }
        for (int l = 1; l < nl; ++l) {
            unsigned char* lb = base + Lo.lane + (size_t)(l - 1) * Lo.lane_bytes;
            Lane& ln = lanes[(size_t)l];
            ln.st = nullptr;
            ln.v[0] = (V*)lb;
            lb += align256((size_t)chunk * dim[0] * sizeof(V));
            ln.v[1] = (V*)lb;
            lb += align256((size_t)chunk * dim[1] * sizeof(V));
            ln.psi = (double2*)lb;
            lb += align256((size_t)nx * 16);
            ln.tree = lb;
            if ((s = hip_check(hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking), "hipStreamCreate")) != HSF_OK ||
                (s = hip_check(hipStreamWaitEvent(ln.st, start, 0), "hipStreamWaitEvent")) != HSF_OK) {
                cleanup();
                return s;
            }
        }
        DeviceCopy dd = d;
        for (size_t i = 0; i < ns && s == HSF_OK; ++i) {
            const Lane& ln = lanes[i % (size_t)nl];
            for (int side = 0; side < 2; ++side)
                for (int tr = 0; tr < 2; ++tr) {
                    std::vector<DeviceSchedule>& dv = tr ? dd.tree[side] : dd.side[side];
                    for (size_t q = 0; q < dv.size(); ++q) dv[q].pool = pools + i * Lo.pool_elems + pool_at[2 * side + tr][q];
                }
            for (int64_t p0 = 0; p0 < p.P && s == HSF_OK; p0 += chunk) {
                const int64_t np = std::min(chunk, p.P - p0);
                s = run_sides(p, dd, p0, np, ln.v[0], dim[0], ln.v[1], dim[1], ln.tree, Lo.tree_bytes, ln.st);
                if (s == HSF_OK)
                    s = gather_dot(p.dtype, ln.v[0], dim[0], ln.v[1], dim[1], np, p.nb, p.n, x, nx, ln.psi,
                                   p0 > 0 ? 1 : 0, ln.st);
            }
            if (s != HSF_OK) break;
            hipLaunchKernelGGL(bw_shift_dot, dim3(1), dim3(256), 0, ln.st, (const double2*)psi_x,
                               (const double2*)ln.psi, nx, lossb + i);
            s = hip_check(hipGetLastError(), "bw_shift_dot launch");
        }
        // the caller's stream waits for every lane before combining
        for (int l = 1; l < nl && s == HSF_OK; ++l) {
            hipEvent_t e = nullptr;
            if ((s = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")) != HSF_OK) break;
            evs.push_back(e);
            if ((s = hip_check(hipEventRecord(e, lanes[(size_t)l].st), "hipEventRecord")) != HSF_OK ||
                (s = hip_check(hipStreamWaitEvent(st, e, 0), "hipStreamWaitEvent")) != HSF_OK)
                break;
        }
        if (s != HSF_OK) {
            for (int l = 1; l < nl; ++l)
                if (lanes[(size_t)l].st) (void)hipStreamSynchronize(lanes[(size_t)l].st);
            cleanup();
            return s;
        }
        // dL/dt += Re sum_j conj(c_j) psi_j(t + pi) per occurrence, in plan order
        for (size_t i = 0; i < ns && s == HSF_OK; ++i) {
            hipLaunchKernelGGL(bw_shift_add, dim3(1), dim3(1), 0, st, lossb + i, grad, (int64_t)shifts[i].t);
            s = hip_check(hipGetLastError(), "bw_shift_add launch");
        }
        // the lanes' streams go once the caller's stream has drained them
        const hsf_status sync = hip_check(hipStreamSynchronize(st), "sync");
        cleanup();
        if (s != HSF_OK) return s;
        return sync;
    }
    // host staging buffers above must outlive their async uploads
    return hip_check(hipStreamSynchronize(st), "sync");
}

}  // namespace

size_t backward_workspace(const Plan& p, int64_t chunk, int64_t nx) { return layout(p, chunk, nx).total; }

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
