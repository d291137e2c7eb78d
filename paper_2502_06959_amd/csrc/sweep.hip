// Half-state gate sweeps (Sec. II-A applied to each path's subcircuit,
// Sec. II-B): every launch covers all paths of a chunk.  A workgroup owns one
// tile of one path's half-state in LDS -- 2^L amplitudes spanning L of the
// side's qubits, the low qubits always among them so that tile rows are
// contiguous in HBM -- and applies every op of the pass to it before writing
// it back.  When the whole half-state fits (L = n_side) there is a single
// pass that starts from |0...0> in LDS and only writes HBM once.
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

struct PassArgs {
    int32_t n_local;
    int32_t init_zero;
    int32_t op_begin, op_end;
    int32_t n_nonlocal;
    int32_t n_contig;            // local_q[i] == i for i < n_contig
    int32_t local_q[kMaxTileBits];
    int32_t nonlocal_q[kMaxTileBits];
};

// Inserts a zero bit at position b of i.
__device__ __forceinline__ uint32_t ins0(uint32_t i, int b) {
    const uint32_t lo = i & ((1u << b) - 1u);
    return ((i >> b) << (b + 1)) | lo;
}

template <int K, typename V>
__device__ __forceinline__ void apply_dense(V* tile, uint32_t E, const int32_t* bit, const V* __restrict__ m,
                                            int tid, int nt) {
    constexpr int D = 1 << K;
    int sb[K];
    for (int i = 0; i < K; ++i) sb[i] = bit[i];
    // ascending order for zero insertion
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j)
            if (sb[j] < sb[i]) { int t = sb[i]; sb[i] = sb[j]; sb[j] = t; }
    uint32_t off[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((j >> (K - 1 - i)) & 1) o |= 1u << bit[i];
        off[j] = o;
    }
    // K <= 2: matrix in registers; wider ops read it through the scalar cache
    constexpr int DM = K <= 2 ? D * D : 1;
    V mm[DM];
    if constexpr (K <= 2) {
#pragma unroll
        for (int j = 0; j < D * D; ++j) mm[j] = m[j];
    }
    auto M_ = [&](int idx) -> V {
        if constexpr (K <= 2) return mm[idx];
        else return m[idx];
    };
    const uint32_t groups = E >> K;
    for (uint32_t g = tid; g < groups; g += nt) {
        uint32_t base = g;
#pragma unroll
        for (int i = 0; i < K; ++i) base = ins0(base, sb[i]);
        V v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = tile[base | off[j]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc = cmul(M_(r * D), v[0]);
#pragma unroll
            for (int j = 1; j < D; ++j) acc = cfma(M_(r * D + j), v[j], acc);
            tile[base | off[r]] = acc;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void sweep_pass(PassArgs a, typename Cx<T>::v* __restrict__ psi, int64_t ld,
                                                   int64_t p_begin, uint32_t n_tiles,
                                                   const DevOp* __restrict__ ops,
                                                   const typename Cx<T>::v* __restrict__ pool) {
    using V = typename Cx<T>::v;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* tile = reinterpret_cast<V*>(smem_raw);
    const int L = a.n_local;
    const uint32_t E = 1u << L;
    const uint32_t pl = blockIdx.x / n_tiles;
    const uint32_t t = blockIdx.x - pl * n_tiles;
    const int64_t path = p_begin + pl;
    V* st = psi + (int64_t)pl * ld;
    const int tid = threadIdx.x, nt = blockDim.x;

    uint64_t base = 0;
    for (int i = 0; i < a.n_nonlocal; ++i) base |= (uint64_t)((t >> i) & 1u) << a.nonlocal_q[i];
    const uint32_t cmask = (1u << a.n_contig) - 1u;
    auto gidx = [&](uint32_t e) -> uint64_t {
        uint64_t g = base | (e & cmask);
        for (int i = a.n_contig; i < L; ++i) g |= (uint64_t)((e >> i) & 1u) << a.local_q[i];
        return g;
    };

    if (a.init_zero) {
        for (uint32_t e = tid; e < E; e += nt) {
            V z;
            z.x = (e == 0 && base == 0) ? T(1) : T(0);
            z.y = T(0);
            tile[e] = z;
        }
    } else {
        for (uint32_t e = tid; e < E; e += nt) tile[e] = st[gidx(e)];
    }
    __syncthreads();

    for (int o = a.op_begin; o < a.op_end; ++o) {
        const DevOp& op = ops[o];
        const int type = op.type;
        if (type == DOP_DENSE1) {
            const int b = op.bit[0];
            const V m00 = pool[op.mat], m01 = pool[op.mat + 1], m10 = pool[op.mat + 2], m11 = pool[op.mat + 3];
            const uint32_t half = E >> 1;
            for (uint32_t i = tid; i < half; i += nt) {
                const uint32_t i0 = ins0(i, b), i1 = i0 | (1u << b);
                const V x0 = tile[i0], x1 = tile[i1];
                tile[i0] = cfma(m01, x1, cmul(m00, x0));
                tile[i1] = cfma(m11, x1, cmul(m10, x0));
            }
        } else if (type == DOP_DENSE2) {
            apply_dense<2>(tile, E, op.bit, pool + op.mat, tid, nt);
        } else if (type == DOP_DENSEK || type == DOP_SLOT) {
            int32_t mat = op.mat;
            const int D2 = 1 << (2 * op.k);
            if (type == DOP_SLOT) mat += (int32_t)((path / op.stride) % op.rank) * D2;
            switch (op.k) {
                case 1: apply_dense<1>(tile, E, op.bit, pool + mat, tid, nt); break;
                case 2: apply_dense<2>(tile, E, op.bit, pool + mat, tid, nt); break;
                case 3: apply_dense<3>(tile, E, op.bit, pool + mat, tid, nt); break;
                default: apply_dense<4>(tile, E, op.bit, pool + mat, tid, nt); break;
            }
        } else {  // DOP_DIAG
            const int k = op.k;
            uint32_t c0 = 0;
            int lb[4], ls[4], nl = 0;
            for (int i = 0; i < k; ++i) {
                const int b = op.bit[i];
                if (b >= 0) {
                    lb[nl] = b;
                    ls[nl] = k - 1 - i;
                    ++nl;
                } else {
                    c0 |= (uint32_t)((base >> (-1 - b)) & 1u) << (k - 1 - i);
                }
            }
            const V* dg = pool + op.mat;
            for (uint32_t e = tid; e < E; e += nt) {
                uint32_t idx = c0;
                for (int i = 0; i < nl; ++i) idx |= ((e >> lb[i]) & 1u) << ls[i];
                tile[e] = cmul(dg[idx], tile[e]);
            }
        }
        __syncthreads();
    }

    for (uint32_t e = tid; e < E; e += nt) st[gidx(e)] = tile[e];
}

std::mutex g_dev_mutex;

template <typename T>
hsf_status upload_side(const SideProgram& sp, void** ops, void** pool) {
    using V = typename Cx<T>::v;
    hsf_status s;
    const size_t no = std::max<size_t>(sp.devops.size(), 1);
    if ((s = hip_check(hipMalloc(ops, no * sizeof(DevOp)), "hipMalloc(ops)")) != HSF_OK) return s;
    if (!sp.devops.empty() &&
        (s = hip_check(hipMemcpy(*ops, sp.devops.data(), sp.devops.size() * sizeof(DevOp), hipMemcpyHostToDevice), "hipMemcpy(ops)")) != HSF_OK)
        return s;
    std::vector<V> h(std::max<size_t>(sp.pool.size(), 1));
    for (size_t i = 0; i < sp.pool.size(); ++i) {
        h[i].x = (T)sp.pool[i].real();
        h[i].y = (T)sp.pool[i].imag();
    }
    if ((s = hip_check(hipMalloc(pool, h.size() * sizeof(V)), "hipMalloc(pool)")) != HSF_OK) return s;
    return hip_check(hipMemcpy(*pool, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice), "hipMemcpy(pool)");
}

bool g_attr_done[2] = {false, false};

}  // namespace

int max_tile_bits(int dtype) { return dtype == HSF_C128 ? 13 : 14; }

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
    DeviceCopy d;
    d.device = dev;
    for (int side = 0; side < 2; ++side) {
        s = p.dtype == HSF_C128 ? upload_side<double>(p.side[side], &d.ops[side], &d.pool[side])
                                : upload_side<float>(p.side[side], &d.ops[side], &d.pool[side]);
        if (s != HSF_OK) {
            for (int j = 0; j < 2; ++j) {
                if (d.ops[j]) (void)hipFree(d.ops[j]);
                if (d.pool[j]) (void)hipFree(d.pool[j]);
            }
            return s;
        }
    }
    const int di = p.dtype == HSF_C128 ? 1 : 0;
    if (!g_attr_done[di]) {
        const size_t bytes = (size_t(1) << max_tile_bits(p.dtype)) * (p.dtype == HSF_C128 ? 16 : 8);
        if (p.dtype == HSF_C128)
            s = hip_check(hipFuncSetAttribute((const void*)sweep_pass<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes), "hipFuncSetAttribute");
        else
            s = hip_check(hipFuncSetAttribute((const void*)sweep_pass<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes), "hipFuncSetAttribute");
        if (s != HSF_OK) return s;
        g_attr_done[di] = true;
    }
    p.dev.push_back(d);
    *out = &p.dev.back();
    return HSF_OK;
}

void release_device(Plan& p) {
    int cur = 0;
    if (p.dev.empty() || hipGetDevice(&cur) != hipSuccess) return;
    for (DeviceCopy& d : p.dev) {
        (void)hipSetDevice(d.device);
        for (int j = 0; j < 2; ++j) {
            if (d.ops[j]) (void)hipFree(d.ops[j]);
            if (d.pool[j]) (void)hipFree(d.pool[j]);
        }
    }
    (void)hipSetDevice(cur);
    p.dev.clear();
}

hsf_status run_side(Plan& p, DeviceCopy& d, int side, int64_t p_begin, int64_t n_paths, void* psi, int64_t ld,
                    hipStream_t stream) {
    const SideProgram& sp = p.side[side];
    const bool dbl = p.dtype == HSF_C128;
    const size_t esz = dbl ? 16 : 8;
    for (const Pass& ps : sp.passes) {
        PassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.n_local = ps.n_local;
        a.init_zero = ps.init_zero;
        a.op_begin = ps.op_begin;
        a.op_end = ps.op_end;
        a.n_nonlocal = ps.n_nonlocal;
        int c = 0;
        while (c < ps.n_local && ps.local_q[c] == c) ++c;
        a.n_contig = c;
        for (int i = 0; i < kMaxTileBits; ++i) {
            a.local_q[i] = ps.local_q[i];
            a.nonlocal_q[i] = ps.nonlocal_q[i];
        }
        const uint32_t n_tiles = 1u << ps.n_nonlocal;
        const uint32_t E = 1u << ps.n_local;
        const int threads = (int)std::min<uint32_t>(dbl ? 512u : 1024u, std::max<uint32_t>(64u, E / 2));
        const size_t shmem = (size_t)E * esz;
        const int64_t max_paths = std::max<int64_t>(1, (int64_t(1) << 30) / n_tiles);
        for (int64_t p0 = 0; p0 < n_paths; p0 += max_paths) {
            const int64_t np = std::min(max_paths, n_paths - p0);
            const dim3 grid((uint32_t)(np * n_tiles));
            if (dbl)
                hipLaunchKernelGGL(sweep_pass<double>, grid, dim3(threads), shmem, stream, a,
                                   (double2*)psi + p0 * ld, ld, p_begin + p0, n_tiles, (const DevOp*)d.ops[side],
                                   (const double2*)d.pool[side]);
            else
                hipLaunchKernelGGL(sweep_pass<float>, grid, dim3(threads), shmem, stream, a,
                                   (float2*)psi + p0 * ld, ld, p_begin + p0, n_tiles, (const DevOp*)d.ops[side],
                                   (const float2*)d.pool[side]);
            hsf_status s = hip_check(hipGetLastError(), "sweep_pass launch");
            if (s != HSF_OK) return s;
        }
    }
    return HSF_OK;
}

}  // namespace hsf
