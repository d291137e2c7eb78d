// Batches of independent circuits run together: every circuit's LDS pass k
// in one launch (a table of (circuit, side) segments), one split launch and
// one persistent path-sum launch over the union of all circuits' output
// tiles.  The launch sequence is captured once into a HIP graph and replayed;
// an autotuner picks the tile policy by timing the candidates on the device.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace hsf {

struct Batch {
    std::vector<Plan*> plans;
    // 0: largest tiles; 1: per-circuit fill rule; 2: one size smaller (all
    // flat sweeps); 3: each circuit's form and tile size from the planner's
    // estimate (path tree where it pays)
    int policy = 3;
    int device = -1;
    // workspace layout (bytes from the 256-aligned base)
    std::vector<int64_t> offA, offB, offPA, offPB, kp;
    std::vector<int64_t> offT;           // each circuit's path-tree scratch (tree_scratch offsets from here)
    size_t ws_f32 = 0, ws_bf16 = 0;
    // device tables
    void* segs = nullptr;
    void* splits = nullptr;
    void* gemms = nullptr;               // streaming path sums (fewer than kLdsMinPaths paths)
    void* gemms_lds = nullptr;           // LDS-staged path sums
    int n_gemm = 0, n_gemm_lds = 0;
    bool stream_full = false;            // every streaming product takes the bounds-free kernel
    int64_t tiles_lds = 0;
    std::vector<int> round_first, round_n, round_kg, round_s1;
    std::vector<uint32_t> round_blocks, round_emax;
    int n_split = 0;
    uint32_t split_blocks = 0;
    int64_t tiles = 0;
    // what the tables were built for
    int built_policy = -1, built_mode = -1;
    std::vector<void*> built_outs;
    // graph cache
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned char* graph_base = nullptr;
    bool graph_valid = false;
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

SweepChoice sweep_choice(const Batch& b, const Plan& p) {
    const int n = (int)std::max(p.side[0].sched.size(), p.side[1].sched.size());
    SweepChoice c;
    if (b.policy == 3) return choose_sweep(p, p.P);
    c.sched = b.policy == 0 ? 0 : b.policy == 1 ? pick_schedule(p, p.P) : std::min(1, n - 1);
    return c;
}

void free_tables(Batch& b) {
    for (void* q : {b.segs, b.splits, b.gemms, b.gemms_lds})
        if (q) (void)hipFree(q);
    b.segs = b.splits = b.gemms = b.gemms_lds = nullptr;
    b.built_policy = b.built_mode = -1;
    b.built_outs.clear();
}

void drop_graph(Batch& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.graph_valid = false;
}

template <typename T>
hsf_status upload_table(const std::vector<T>& v, void** dst) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    hsf_status s = hip_check(hipMalloc(dst, std::max<size_t>(v.size() * sizeof(T), 64)), "hipMalloc(batch table)");
    if (s != HSF_OK || v.empty()) return s;
    return hip_check(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy(batch table)");
}

hsf_status build_tables(Batch& b, void* const* outs, int mode) {
    const int n = (int)b.plans.size();
    for (int i = 0; i < n; ++i) {
        const Plan& p = *b.plans[i];
        for (int s = 0; s < 2; ++s)
            for (int tr = 0; tr < 2; ++tr)
                for (const Schedule& sc : tr ? p.side[s].tree : p.side[s].sched)
                    for (const Pass& ps : sc.passes)
                        if (ps.n_local < 3)
                            return fail(HSF_E_UNSUPPORTED, "batched sweeps need sides of at least 3 qubits");
    }
    std::vector<DeviceCopy*> dc(n);
    for (int i = 0; i < n; ++i) {
        hsf_status s = ensure_device(*b.plans[i], &dc[i]);
        if (s != HSF_OK) return s;
    }
    batch_sweep_prepare();
    // sweep segments, round by round
    std::vector<BatchSeg> segs;
    b.round_first.clear();
    b.round_n.clear();
    b.round_kg.clear();
    b.round_s1.clear();
    b.round_blocks.clear();
    b.round_emax.clear();
    // every (circuit, side)'s launches, as for a single plan over all its
    // paths: flat, or path-tree levels in the circuit's scratch
    std::vector<SweepChoice> ch(n);
    std::vector<std::vector<SweepItem>> items(2 * (size_t)n);
    std::vector<const Schedule*> hs(2 * (size_t)n);
    std::vector<const DeviceSchedule*> dsv(2 * (size_t)n);
    size_t rounds = 0;
    for (int i = 0; i < n; ++i) {
        const Plan& p = *b.plans[i];
        ch[i] = sweep_choice(b, p);
        const TreeScratch ts = tree_scratch(p, p.P);
        for (int s = 0; s < 2; ++s) {
            const std::vector<Schedule>& hv = ch[i].tree ? p.side[s].tree : p.side[s].sched;
            const std::vector<DeviceSchedule>& dv = ch[i].tree ? dc[i]->tree[s] : dc[i]->side[s];
            const size_t idx = std::min<size_t>((size_t)ch[i].sched, hv.size() - 1);
            const size_t q = 2 * (size_t)i + s;
            hs[q] = &hv[idx];
            dsv[q] = &dv[idx];
            // offsets from the workspace base stand in for the pointers
            auto off = [](int64_t o) { return reinterpret_cast<unsigned char*>((uintptr_t)o); };
            const int64_t dim = int64_t(1) << (s == 0 ? p.na : p.nb);
            items[q] = side_items(*hs[q], ch[i].tree, dsv[q]->prefix, 0, p.P, off(s == 0 ? b.offA[i] : b.offB[i]), dim,
                                  off(b.offT[i] + (int64_t)ts.off[s][0]), off(b.offT[i] + (int64_t)ts.off[s][1]), dim);
            rounds = std::max(rounds, items[q].size());
        }
    }
    // item j of every (circuit, side), split by group width: one launch each
    for (size_t j = 0; j < rounds; ++j)
        for (int kg = 3; kg <= 4; ++kg) {
            const int first = (int)segs.size();
            uint32_t start = 0, emax = 1;
            int s1 = 0;
            for (int i = 0; i < n; ++i) {
                for (int s = 0; s < 2; ++s) {
                    const size_t q = 2 * (size_t)i + s;
                    if (j >= items[q].size()) continue;
                    const SweepItem& it = items[q][j];
                    const Schedule& sc = *hs[q];
                    const size_t k = it.k;
                    if (group_bits(sc.passes[k].n_local) != kg) continue;
                    const DeviceSchedule& ds = *dsv[q];
                    BatchSeg g{};
                    g.pass = reinterpret_cast<const Pass*>(ds.passes) + k;
                    g.psi_off = (int64_t)(uintptr_t)it.dst;
                    g.ld = it.dst_ld;
                    g.ops = (const DevOp*)ds.ops;
                    g.subs = ds.subs;
                    g.pool = ds.pool;
                    g.n_tiles = 1u << sc.passes[k].n_nonlocal;
                    g.block_start = start;
                    g.mode = it.mode;
                    g.shared = it.mode == ROW_SHARED ? it.src : nullptr;
                    g.S = it.S;
                    g.i_lo = it.i_lo;
                    g.src_off = it.mode == ROW_PARENT ? (int64_t)(uintptr_t)it.src : 0;
                    g.src_ld = it.src_ld;
                    g.src_lo = it.src_lo;
                    g.S_par = it.S_par;
                    start += (uint32_t)(it.rows * g.n_tiles);
                    emax = std::max(emax, 1u << sc.passes[k].n_local);
                    s1 |= sc.passes[k].has_slot1;
                    segs.push_back(g);
                }
            }
            if ((int)segs.size() == first) continue;
            b.round_first.push_back(first);
            b.round_n.push_back((int)segs.size() - first);
            b.round_kg.push_back(kg);
            b.round_s1.push_back(s1);
            b.round_blocks.push_back(start);
            b.round_emax.push_back(emax);
        }
    hsf_status s = upload_table(segs, &b.segs);
    if (s != HSF_OK) return s;
    // split descriptors (BF16 planes) and path-sum descriptors
    std::vector<SplitDesc> sp;
    std::vector<GemmDesc> gm, gl;
    uint32_t sb = 0;
    int64_t tiles = 0, tiles_lds = 0;
    bool stream_full = true;
    for (int i = 0; i < n; ++i) {
        const Plan& p = *b.plans[i];
        const int64_t M = int64_t(1) << p.na, N = int64_t(1) << p.nb;
        const bool deep = p.P >= kLdsMinPaths;
        if (mode == HSF_SUM_BF16X3) {
            for (int side = 0; side < 2; ++side) {
                SplitDesc d{};
                d.x_off = side == 0 ? b.offA[i] : b.offB[i];
                d.ldx = side == 0 ? M : N;
                d.K = p.P;
                d.R = side == 0 ? M : N;
                d.Kp = b.kp[i];
                d.planes_off = side == 0 ? b.offPA[i] : b.offPB[i];
                d.blocks_x = (uint32_t)((d.R + 255) / 256);
                d.block_start = sb;
                d.chunked = deep ? 1u : 0u;
                sb += d.blocks_x * (uint32_t)(d.Kp / 8);
                sp.push_back(d);
            }
        }
        GemmDesc g{};
        if (mode == HSF_SUM_BF16X3) {
            g.a_off = b.offPA[i];
            g.b_off = b.offPB[i];
            g.K = b.kp[i];
        } else {
            g.a_off = b.offA[i];
            g.b_off = b.offB[i];
            g.K = p.P;
        }
        g.ldA = M;
        g.ldB = N;
        g.M = M;
        g.N = N;
        g.out = outs[i];
        g.ldo = N;
        int64_t& t = deep ? tiles_lds : tiles;
        g.tile_start = t;
        if (mode == HSF_SUM_BF16X3 && !deep) {
            // streaming split-BF16 tiles
            g.tiles_n = (N + kBf16StreamCols - 1) / kBf16StreamCols;
            t += g.tiles_n * ((M + kBf16StreamRows - 1) / kBf16StreamRows);
            stream_full = stream_full && bf16x3_stream_full(M, N, g.K, g.ldo, 0);
        } else {
            const int64_t tile_rows = mode == HSF_SUM_BF16X3 ? kBf16LdsTileRows : 128;
            g.tiles_n = (N + 127) / 128;
            t += g.tiles_n * ((M + tile_rows - 1) / tile_rows);
        }
        (deep ? gl : gm).push_back(g);
    }
    if ((s = upload_table(sp, &b.splits)) != HSF_OK) return s;
    if ((s = upload_table(gm, &b.gemms)) != HSF_OK) return s;
    if ((s = upload_table(gl, &b.gemms_lds)) != HSF_OK) return s;
    b.n_gemm = (int)gm.size();
    b.n_gemm_lds = (int)gl.size();
    b.tiles_lds = tiles_lds;
    b.n_split = (int)sp.size();
    b.split_blocks = sb;
    b.tiles = tiles;
    b.stream_full = stream_full;
    b.built_policy = b.policy;
    b.built_mode = mode;
    b.built_outs.assign(outs, outs + n);
    return HSF_OK;
}

hsf_status enqueue(Batch& b, int mode, unsigned char* base, hipStream_t st) {
    hsf_status s;
    for (size_t k = 0; k < b.round_first.size(); ++k) {
        const uint32_t emax = b.round_emax[k];
        const int threads = (int)std::min<uint32_t>(512u, std::max<uint32_t>(64u, emax >> b.round_kg[k]));
        const size_t shmem = ((size_t)emax + 256) * 8;
        if (b.round_blocks[k] == 0) continue;
        s = launch_sweep_batch(b.round_kg[k], b.round_s1[k] != 0, reinterpret_cast<const BatchSeg*>(b.segs) + b.round_first[k], b.round_n[k],
                               b.round_blocks[k], threads, shmem, base, st);
        if (s != HSF_OK) return s;
    }
    const bool bf = mode == HSF_SUM_BF16X3;
    if (bf && (s = launch_split_batch(b.splits, b.n_split, b.split_blocks, base, st)) != HSF_OK) return s;
    if (b.n_gemm_lds > 0) {
        s = bf ? launch_bf16x3_lds_batch(b.gemms_lds, b.n_gemm_lds, b.tiles_lds, base, st)
               : launch_f32_lds_batch(b.gemms_lds, b.n_gemm_lds, b.tiles_lds, base, st);
        if (s != HSF_OK) return s;
    }
    if (b.n_gemm == 0) return HSF_OK;
    return bf ? launch_bf16x3_batch(b.gemms, b.n_gemm, b.tiles, b.stream_full, base, st)
              : launch_f32_batch(b.gemms, b.n_gemm, b.tiles, base, st);
}

}  // namespace

hsf_status batch_create(Plan* const* plans, int n, Batch** out) {
    for (int i = 0; i < n; ++i)
        if (plans[i]->dtype != HSF_C64) return fail(HSF_E_UNSUPPORTED, "batches run complex64 plans");
    Batch* b = new Batch();
    b->plans.assign(plans, plans + n);
    size_t o = 0, ob = 0;
    for (int i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        const int64_t M = int64_t(1) << p.na, N = int64_t(1) << p.nb;
        b->offA.push_back((int64_t)o);
        o += a256((size_t)p.P * M * 8);
        b->offB.push_back((int64_t)o);
        o += a256((size_t)p.P * N * 8);
    }
    // path-tree scratch for every circuit that has tree schedules
    for (int i = 0; i < n; ++i) {
        b->offT.push_back((int64_t)o);
        o += a256(tree_scratch(*plans[i], plans[i]->P).total);
    }
    ob = o;
    for (int i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        const int64_t M = int64_t(1) << p.na, N = int64_t(1) << p.nb;
        // streaming kernel: paths padded to 16; LDS-staged kernel: chunks of 32
        const int64_t kp = p.P >= kLdsMinPaths ? (p.P + 31) / 32 * 32 : std::max<int64_t>(16, (p.P + 15) / 16 * 16);
        b->kp.push_back(kp);
        b->offPA.push_back((int64_t)ob);
        ob += a256((size_t)4 * M * kp * 2);
        b->offPB.push_back((int64_t)ob);
        ob += a256((size_t)4 * N * kp * 2);
    }
    b->ws_f32 = o + 256;
    b->ws_bf16 = ob + 256;
    *out = b;
    return HSF_OK;
}

void batch_destroy(Batch* b) {
    if (!b) return;
    drop_graph(*b);
    free_tables(*b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

size_t batch_workspace(const Batch& b, int mode) { return mode == HSF_SUM_BF16X3 ? b.ws_bf16 : b.ws_f32; }

hsf_status batch_run(Batch& b, void* const* outs, int mode, int use_graph, void* ws, hipStream_t st) {
    unsigned char* base = reinterpret_cast<unsigned char*>(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const int n = (int)b.plans.size();
    const bool same = b.built_policy == b.policy && b.built_mode == mode &&
                      b.built_outs.size() == (size_t)n && std::equal(b.built_outs.begin(), b.built_outs.end(), outs);
    hsf_status s;
    if (!same) {
        drop_graph(b);
        if ((s = build_tables(b, outs, mode)) != HSF_OK) return s;
    }
    if (!use_graph) return enqueue(b, mode, base, st);
    if (!b.graph_valid || b.graph_base != base) {
        drop_graph(b);
        if (!b.cap && (s = hip_check(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking), "hipStreamCreate")) != HSF_OK)
            return s;
        if ((s = hip_check(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")) != HSF_OK)
            return s;
        hsf_status se = enqueue(b, mode, base, b.cap);
        hipGraph_t g = nullptr;
        hsf_status sc = hip_check(hipStreamEndCapture(b.cap, &g), "hipStreamEndCapture");
        if (se != HSF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return se;
        }
        if (sc != HSF_OK) return sc;
        b.graph = g;
        if ((s = hip_check(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "hipGraphInstantiate")) != HSF_OK) {
            drop_graph(b);
            return s;
        }
        b.graph_base = base;
        b.graph_valid = true;
    }
    return hip_check(hipGraphLaunch(b.exec, st), "hipGraphLaunch");
}

namespace {

// Tuned policies by batch shape, shared by the process: the path-sum mode
// and, circuit by circuit in batch order, n_a, n_b, P and the fused op count
// of each side.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int> g_tune_cache;

std::vector<int64_t> tune_key(const Batch& b, int mode) {
    std::vector<int64_t> k{mode, (int64_t)b.plans.size()};
    for (const Plan* p : b.plans) {
        k.push_back(p->na);
        k.push_back(p->nb);
        k.push_back(p->P);
        k.push_back((int64_t)p->side[0].ops.size());
        k.push_back((int64_t)p->side[1].ops.size());
    }
    return k;
}

}  // namespace

int batch_tune_cached(Batch& b, int mode) {
    const std::vector<int64_t> k = tune_key(b, mode);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune_cache.find(k);
    if (it == g_tune_cache.end()) return -1;
    b.policy = it->second;
    return it->second;
}

hsf_status batch_tune(Batch& b, void* const* outs, int mode, void* ws, hipStream_t st, int* chosen) {
    hipEvent_t e0, e1;
    hsf_status s;
    if ((s = hip_check(hipEventCreate(&e0), "hipEventCreate")) != HSF_OK) return s;
    if ((s = hip_check(hipEventCreate(&e1), "hipEventCreate")) != HSF_OK) {
        (void)hipEventDestroy(e0);
        return s;
    }
    float best = 1e30f;
    int best_p = 0;
    for (int pol = 0; pol < 4; ++pol) {
        b.policy = pol;
        if ((s = batch_run(b, outs, mode, 0, ws, st)) != HSF_OK) break;     // warm-up, builds tables
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3; ++r)
            if ((s = batch_run(b, outs, mode, 0, ws, st)) != HSF_OK) break;
        (void)hipEventRecord(e1, st);
        if (s != HSF_OK) break;
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            best_p = pol;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b.policy = best_p;
    if (chosen) *chosen = best_p;
    if (s == HSF_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[tune_key(b, mode)] = best_p;
    }
    return s;
}

}  // namespace hsf
