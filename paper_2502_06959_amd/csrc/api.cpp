// extern "C" entry points of libhsf: argument checks, status codes and the
// thread-local error message.  The work itself is in plan.cpp (host) and in
// the HIP sources (device).
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace hsf {

thread_local std::string g_last_error;

hsf_status fail(hsf_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

std::string g_last_error_copy() { return g_last_error; }

}  // namespace hsf

using namespace hsf;

#define HSF_GUARD_BEGIN try {
#define HSF_GUARD_END                                                      \
    }                                                                      \
    catch (const std::bad_alloc&) {                                        \
        return fail(HSF_E_ARG, "host allocation failed");                  \
    }                                                                      \
    catch (const std::exception& e) {                                      \
        return fail(HSF_E_ARG, std::string("internal error: ") + e.what()); \
    }

namespace hsf {

// Argument checks and dispatch of hsf_amplitudes_full (also the body of its
// variant on the library's static scratch).
hsf_status amplitudes_full(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB, int64_t ldB,
                           int64_t n_paths, int64_t row_begin, int64_t row_end, void* out, int64_t ldo, int32_t mode,
                           int32_t accumulate, void* ws, size_t ws_bytes, hipStream_t stream) {
    const bool presplit = mode == HSF_SUM_BF16X3_SPLIT;
    if (!plan || (n_paths > 0 && !presplit && (!psiA || !psiB))) return fail(HSF_E_ARG, "null argument");
    const Plan* p = reinterpret_cast<const Plan*>(plan);
    const int64_t M = int64_t(1) << p->na, N = int64_t(1) << p->nb;
    if (n_paths < 0) return fail(HSF_E_ARG, "negative path count");
    if (row_begin < 0 || row_end > M || row_begin > row_end) return fail(HSF_E_ARG, "row range outside [0, 2^n_a)");
    if ((!presplit && (ldA < M || ldB < N)) || ldo < N) return fail(HSF_E_ARG, "leading dimension too small");
    if (mode < HSF_SUM_F32 || mode > HSF_SUM_BF16X3_SPLIT) return fail(HSF_E_ARG, "unknown path-sum mode");
    if (p->dtype == HSF_C128 && (mode == HSF_SUM_F32 || mode == HSF_SUM_BF16X3 || presplit))
        return fail(HSF_E_ARG, "c128 half-states need HSF_SUM_F64 or HSF_SUM_C128");
    if ((mode == HSF_SUM_BF16X3 || presplit) && ws_bytes < bf16x3_workspace(p->na, p->nb, n_paths))
        return fail(HSF_E_ARG, "workspace too small for HSF_SUM_BF16X3");
    if (presplit && n_paths > 0 && (!ws || ws != p->split_ws || n_paths != p->split_paths))
        return fail(HSF_E_ARG, "HSF_SUM_BF16X3_SPLIT needs the workspace and path count of the plan's last "
                               "hsf_split_operands call");
    if (row_begin == row_end) return HSF_OK;
    if (!out) return fail(HSF_E_ARG, "null argument");
    if (presplit && n_paths > 0)
        return path_sum_presplit(n_paths, M, row_begin, row_end - row_begin, N, ws, (float2*)out, ldo, accumulate,
                                 stream);
    return path_sum(p->dtype, mode, psiA, ldA, psiB, ldB, n_paths, row_begin, row_end - row_begin, N, out, ldo,
                    accumulate, ws, stream);
}

}  // namespace hsf

extern "C" {

const char* hsf_last_error(void) { return g_last_error.c_str(); }
const char* hsf_version(void) { return "libhsf 0.1 (gfx950)"; }

hsf_status hsf_plan(const hsf_circuit* circuit, int32_t cut, const int64_t* block_gate_ids,
                    const int64_t* block_offsets, int32_t n_blocks, const hsf_plan_options* opts,
                    hsf_plan_t* out) {
    HSF_GUARD_BEGIN
    if (!out) return fail(HSF_E_ARG, "null output pointer");
    *out = nullptr;
    Plan* p = nullptr;
    hsf_status s = build_plan(circuit, cut, block_gate_ids, block_offsets, n_blocks, opts, &p);
    if (s != HSF_OK) return s;
    *out = reinterpret_cast<hsf_plan_t>(p);
    return HSF_OK;
    HSF_GUARD_END
}

hsf_status hsf_find_blocks(const hsf_circuit* circuit, int32_t cut, int64_t* order, int64_t* block_gate_ids,
                           int64_t* block_offsets, int32_t* n_blocks) {
    HSF_GUARD_BEGIN
    return find_blocks(circuit, cut, order, block_gate_ids, block_offsets, n_blocks);
    HSF_GUARD_END
}

void hsf_plan_destroy(hsf_plan_t plan) {
    if (!plan) return;
    Plan* p = reinterpret_cast<Plan*>(plan);
    release_device(*p);
    delete p;
}

static Plan* P_(hsf_plan_t h) { return reinterpret_cast<Plan*>(h); }

hsf_status hsf_plan_dims(hsf_plan_t plan, int32_t* n, int32_t* cut, int32_t* n_a, int32_t* n_b,
                         int32_t* n_blocks, int64_t* n_paths) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    const Plan* p = P_(plan);
    if (n) *n = p->n;
    if (cut) *cut = p->cut;
    if (n_a) *n_a = p->na;
    if (n_b) *n_b = p->nb;
    if (n_blocks) *n_blocks = (int32_t)p->blocks.size();
    if (n_paths) *n_paths = p->P;
    return HSF_OK;
}

int64_t hsf_num_paths(hsf_plan_t plan) { return plan ? P_(plan)->P : -1; }

hsf_status hsf_block_info(hsf_plan_t plan, int32_t k, int32_t* rank, int64_t* stride, int32_t* n_sa,
                          int32_t* sa, int32_t* n_sb, int32_t* sb, int64_t* hull_len,
                          int32_t* caller_index) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    const Plan* p = P_(plan);
    if (k < 0 || k >= (int32_t)p->blocks.size()) return fail(HSF_E_ARG, "block index out of range");
    const Block& b = p->blocks[k];
    if (rank) *rank = b.rank;
    if (stride) *stride = b.stride;
    if (n_sa) *n_sa = (int32_t)b.sa.size();
    if (n_sb) *n_sb = (int32_t)b.sb.size();
    if (sa)
        for (size_t i = 0; i < b.sa.size(); ++i) sa[i] = b.sa[i];
    if (sb)
        for (size_t i = 0; i < b.sb.size(); ++i) sb[i] = b.sb[i];
    if (hull_len) *hull_len = (int64_t)b.hull.size();
    if (caller_index) *caller_index = b.caller_index;
    return HSF_OK;
}

hsf_status hsf_block_hull(hsf_plan_t plan, int32_t k, int64_t* ids) {
    if (!plan || !ids) return fail(HSF_E_ARG, "null argument");
    const Plan* p = P_(plan);
    if (k < 0 || k >= (int32_t)p->blocks.size()) return fail(HSF_E_ARG, "block index out of range");
    std::memcpy(ids, p->blocks[k].hull.data(), p->blocks[k].hull.size() * sizeof(int64_t));
    return HSF_OK;
}

hsf_status hsf_block_factors(hsf_plan_t plan, int32_t k, double* sigma, double* xa, double* yb) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    const Plan* p = P_(plan);
    if (k < 0 || k >= (int32_t)p->blocks.size()) return fail(HSF_E_ARG, "block index out of range");
    const Block& b = p->blocks[k];
    if ((xa && b.xa.empty() && !b.sa.empty()) || (yb && b.yb.empty() && !b.sb.empty()))
        return fail(HSF_E_UNSUPPORTED, "the block's factor on a side wider than 8 qubits is not expanded");
    if (sigma) std::memcpy(sigma, b.sigma.data(), b.sigma.size() * sizeof(double));
    if (xa) std::memcpy(xa, b.xa.data(), b.xa.size() * sizeof(cd));
    if (yb) std::memcpy(yb, b.yb.data(), b.yb.size() * sizeof(cd));
    return HSF_OK;
}

hsf_status hsf_path_digits(hsf_plan_t plan, int64_t path, int32_t* digits) {
    if (!plan || !digits) return fail(HSF_E_ARG, "null argument");
    const Plan* p = P_(plan);
    if (path < 0 || path >= p->P) return fail(HSF_E_ARG, "path index out of range");
    for (size_t k = 0; k < p->blocks.size(); ++k)
        digits[k] = (int32_t)((path / p->blocks[k].stride) % p->blocks[k].rank);
    return HSF_OK;
}

hsf_status hsf_side_stats(hsf_plan_t plan, int32_t side, int64_t* ops_logical, int64_t* ops_fused,
                          int32_t* passes, int32_t* tile_qubits, int64_t* ops_shared, int32_t* shared_passes) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    if (side != 0 && side != 1) return fail(HSF_E_ARG, "side must be 0 (a) or 1 (b)");
    const Plan* p = P_(plan);
    const SideProgram& s = p->side[side];
    const size_t i = std::min<size_t>((size_t)pick_schedule(*p, p->P), s.sched.size() - 1);
    if (ops_logical) *ops_logical = s.ops_logical;
    if (ops_fused) *ops_fused = (int64_t)s.ops.size();
    if (passes) *passes = (int32_t)(s.sched[i].passes.size() - (size_t)s.sched[i].n_prefix_passes);
    if (tile_qubits) *tile_qubits = s.sched[i].tile_bits;
    if (ops_shared) *ops_shared = s.n_prefix;
    if (shared_passes) *shared_passes = s.sched[i].n_prefix_passes;
    return HSF_OK;
}

hsf_status hsf_side_levels(hsf_plan_t plan, int32_t side, int32_t cap, int32_t* n_levels, int64_t* ops,
                           int64_t* states) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    if (side != 0 && side != 1) return fail(HSF_E_ARG, "side must be 0 (a) or 1 (b)");
    if (cap < 0) return fail(HSF_E_ARG, "cap must be non-negative");
    const Plan* p = P_(plan);
    const SideProgram& s = p->side[side];
    std::vector<int64_t> o(1, (int64_t)s.n_prefix), st(1, 1);
    if (!s.tree.empty())
        for (const TreeLevel& tl : s.tree[0].levels) {
            o.push_back(tl.ops);
            st.push_back(p->P / tl.S);
        }
    if (n_levels) *n_levels = (int32_t)o.size();
    for (size_t i = 0; i < o.size() && (int32_t)i < cap; ++i) {
        if (ops) ops[i] = o[i];
        if (states) states[i] = st[i];
    }
    return HSF_OK;
}

hsf_status hsf_sweep_form(hsf_plan_t plan, int64_t n_paths, int32_t* tree, int32_t* tile_qubits) {
    if (!plan) return fail(HSF_E_ARG, "null plan");
    if (n_paths <= 0) return fail(HSF_E_ARG, "n_paths must be positive");
    const Plan* p = P_(plan);
    const SweepChoice ch = choose_sweep(*p, n_paths);
    if (tree) *tree = ch.tree ? 1 : 0;
    if (tile_qubits)
        for (int s = 0; s < 2; ++s) {
            const std::vector<Schedule>& v = ch.tree ? p->side[s].tree : p->side[s].sched;
            tile_qubits[s] = v[std::min<size_t>((size_t)ch.sched, v.size() - 1)].tile_bits;
        }
    return HSF_OK;
}

size_t hsf_workspace_size(hsf_plan_t plan, int32_t op, int64_t n_paths, int32_t mode) {
    if (!plan || n_paths < 0) return 0;
    const Plan* p = P_(plan);
    if (op == 0) return tree_workspace(*p, n_paths);
    if (op == 1 && (mode == HSF_SUM_BF16X3 || mode == HSF_SUM_BF16X3_SPLIT))
        return bf16x3_workspace(p->na, p->nb, n_paths);
    if (op == 2) return backward_workspace(*p, n_paths, mode);
    if (op == 4) return backward_workspace(*p, n_paths, mode, true);
    if (op == 3) return loss_workspace(*p, std::max<int64_t>(n_paths, 1), mode);
    return 0;
}

hsf_status hsf_run_paths(hsf_plan_t plan, int64_t p_begin, int64_t p_end, void* psiA, int64_t ldA,
                         void* psiB, int64_t ldB, void* ws, size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan) return fail(HSF_E_ARG, "null plan");
    Plan* p = P_(plan);
    if (p_begin < 0 || p_end > p->P || p_begin > p_end) return fail(HSF_E_ARG, "path range outside [0, P)");
    if (psiA && ldA < (int64_t(1) << p->na)) return fail(HSF_E_ARG, "ldA smaller than 2^n_a");
    if (psiB && ldB < (int64_t(1) << p->nb)) return fail(HSF_E_ARG, "ldB smaller than 2^n_b");
    if (p_begin == p_end) return HSF_OK;
    DeviceCopy* d = nullptr;
    hsf_status s = ensure_device(*p, &d);
    if (s != HSF_OK) return s;
    return run_sides(*p, *d, p_begin, p_end - p_begin, psiA, ldA, psiB, ldB, ws, ws_bytes, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_run_paths_rows(hsf_plan_t plan, int64_t p_begin, int64_t p_end, int64_t row_begin, int64_t row_end,
                              void* psiA, int64_t ldA, void* psiB, int64_t ldB, void* ws, size_t ws_bytes,
                              hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan || !psiA) return fail(HSF_E_ARG, "null argument");
    Plan* p = P_(plan);
    if (p_begin < 0 || p_end > p->P || p_begin > p_end) return fail(HSF_E_ARG, "path range outside [0, P)");
    if (row_begin < 0 || row_end > (int64_t(1) << p->na) || row_begin > row_end)
        return fail(HSF_E_ARG, "row range outside [0, 2^n_a)");
    if (row_end - row_begin > (int64_t(1) << 20)) return fail(HSF_E_ARG, "more than 2^20 rows: use hsf_run_paths");
    if (ldA < (int64_t(1) << p->na)) return fail(HSF_E_ARG, "ldA smaller than 2^n_a");
    if (psiB && ldB < (int64_t(1) << p->nb)) return fail(HSF_E_ARG, "ldB smaller than 2^n_b");
    if (p_begin == p_end) return HSF_OK;
    DeviceCopy* d = nullptr;
    hsf_status s = ensure_device(*p, &d);
    if (s != HSF_OK) return s;
    return run_sides(*p, *d, p_begin, p_end - p_begin, psiA, ldA, psiB, ldB, ws, ws_bytes, (hipStream_t)stream,
                     nullptr, row_begin, row_end);
    HSF_GUARD_END
}

hsf_status hsf_amplitudes_full(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB,
                               int64_t ldB, int64_t n_paths, int64_t row_begin, int64_t row_end,
                               void* out, int64_t ldo, int32_t mode, int32_t accumulate, void* ws,
                               size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    return amplitudes_full(plan, psiA, ldA, psiB, ldB, n_paths, row_begin, row_end, out, ldo, mode, accumulate, ws,
                           ws_bytes, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_split_operands(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB, int64_t ldB,
                              int64_t n_paths, void* ws, size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan) return fail(HSF_E_ARG, "null plan");
    Plan* p = P_(plan);
    const int64_t M = int64_t(1) << p->na, N = int64_t(1) << p->nb;
    if (p->dtype != HSF_C64) return fail(HSF_E_ARG, "split-BF16 planes are made from c64 half-states");
    if (n_paths < 0) return fail(HSF_E_ARG, "negative path count");
    if (n_paths > 0 && (!psiA || !psiB || !ws)) return fail(HSF_E_ARG, "null argument");
    if (ldA < M || ldB < N) return fail(HSF_E_ARG, "leading dimension too small");
    if (ws_bytes < bf16x3_workspace(p->na, p->nb, n_paths))
        return fail(HSF_E_ARG, "workspace too small for the split planes");
    if (n_paths > 0) {
        hsf_status s = split_operands((const float2*)psiA, ldA, M, (const float2*)psiB, ldB, N, n_paths, ws,
                                      (hipStream_t)stream);
        if (s != HSF_OK) return s;
    }
    p->split_ws = ws;
    p->split_paths = n_paths;
    return HSF_OK;
    HSF_GUARD_END
}

hsf_status hsf_amplitudes_bitstrings(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB,
                                     int64_t ldB, int64_t n_paths, const uint64_t* x, int64_t n_x,
                                     void* out, int32_t accumulate, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan || (n_x > 0 && (!x || !out)) || (n_x > 0 && n_paths > 0 && (!psiA || !psiB)))
        return fail(HSF_E_ARG, "null argument");
    const Plan* p = P_(plan);
    if (!p->side[1].post.empty())
        return fail(HSF_E_UNSUPPORTED, "the plan defers side b's suffix to output rows (hsf_apply_b_suffix)");
    if (n_paths < 0 || n_x < 0) return fail(HSF_E_ARG, "negative size");
    if (ldA < (int64_t(1) << p->na) || ldB < (int64_t(1) << p->nb)) return fail(HSF_E_ARG, "leading dimension too small");
    if (n_x == 0) return HSF_OK;
    return gather_dot(p->dtype, psiA, ldA, psiB, ldB, n_paths, p->nb, p->n, x, n_x, out, accumulate,
                      (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_norm2(const void* a, int32_t a_dtype, const void* b, int32_t b_dtype, int64_t n, double* out,
                     void* ws, size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if ((!a && n > 0) || !out || !ws) return fail(HSF_E_ARG, "null argument");
    if ((a_dtype != HSF_C64 && a_dtype != HSF_C128) || (b && b_dtype != HSF_C64 && b_dtype != HSF_C128))
        return fail(HSF_E_ARG, "dtype must be HSF_C64 or HSF_C128");
    if (n < 0) return fail(HSF_E_ARG, "negative size");
    if (ws_bytes < kNormWsDoubles * sizeof(double)) return fail(HSF_E_ARG, "workspace too small");
    return norm2(a, a_dtype, b, b_dtype, n, out, (double*)ws, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_backward(hsf_plan_t plan, const uint64_t* x, int64_t n_x, const void* dL_dpsi, double* grad,
                        int64_t n_params, int64_t chunk, void* ws, size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan || !grad || (n_x > 0 && !x)) return fail(HSF_E_ARG, "null argument");
    Plan* p = P_(plan);
    if (!p->side[1].post.empty())
        return fail(HSF_E_UNSUPPORTED, "the plan defers side b's suffix to output rows (hsf_apply_b_suffix)");
    if (n_params < p->n_params) return fail(HSF_E_ARG, "grad has fewer slots than the circuit's parameter ids");
    if (chunk <= 0) return fail(HSF_E_ARG, "chunk must be positive");
    if (n_x < 0) return fail(HSF_E_ARG, "negative bitstring count");
    if (ws_bytes < backward_workspace(*p, chunk, n_x, true)) return fail(HSF_E_ARG, "workspace too small");
    DeviceCopy* d = nullptr;
    hsf_status s = ensure_device(*p, &d);
    if (s != HSF_OK) return s;
    return backward(*p, *d, x, n_x, n_x > 0 ? dL_dpsi : nullptr, grad, n_params, chunk, ws, ws_bytes,
                    (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_loss(hsf_plan_t plan, const uint64_t* x, int64_t n_x, double* loss, void* amps, int64_t chunk,
                    void* ws, size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan || !loss || (n_x > 0 && !x) || !ws) return fail(HSF_E_ARG, "null argument");
    Plan* p = P_(plan);
    if (!p->side[1].post.empty())
        return fail(HSF_E_UNSUPPORTED, "the plan defers side b's suffix to output rows (hsf_apply_b_suffix)");
    if (chunk <= 0) return fail(HSF_E_ARG, "chunk must be positive");
    if (n_x < 0) return fail(HSF_E_ARG, "negative bitstring count");
    if (ws_bytes < loss_workspace(*p, chunk, n_x)) return fail(HSF_E_ARG, "workspace too small");
    DeviceCopy* d = nullptr;
    hsf_status s = ensure_device(*p, &d);
    if (s != HSF_OK) return s;
    return prob_mass(*p, *d, x, n_x, loss, amps, chunk, ws, ws_bytes, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_apply_b_suffix(hsf_plan_t plan, void* out, int64_t ldo, int64_t rows, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    if (!plan || (rows > 0 && !out)) return fail(HSF_E_ARG, "null argument");
    Plan* p = P_(plan);
    if (rows < 0) return fail(HSF_E_ARG, "negative row count");
    if (ldo < (int64_t(1) << p->nb)) return fail(HSF_E_ARG, "leading dimension too small");
    if (p->side[1].post.empty() || rows == 0) return HSF_OK;
    DeviceCopy* d = nullptr;
    hsf_status s = ensure_device(*p, &d);
    if (s != HSF_OK) return s;
    return run_segment(*p, d->post[1][0], p->side[1].post[0], out, ldo, rows, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_batch_create(const hsf_plan_t* plans, int32_t n_plans, hsf_batch_t* out) {
    HSF_GUARD_BEGIN
    if (!out || (n_plans > 0 && !plans) || n_plans <= 0) return fail(HSF_E_ARG, "need at least one plan");
    *out = nullptr;
    std::vector<Plan*> ps(n_plans);
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i]) return fail(HSF_E_ARG, "null plan in batch");
        ps[i] = P_(plans[i]);
        if (!ps[i]->side[1].post.empty())
            return fail(HSF_E_UNSUPPORTED, "a plan in the batch defers side b's suffix (hsf_apply_b_suffix)");
    }
    Batch* b = nullptr;
    hsf_status s = batch_create(ps.data(), n_plans, &b);
    if (s != HSF_OK) return s;
    *out = reinterpret_cast<hsf_batch_t>(b);
    return HSF_OK;
    HSF_GUARD_END
}

void hsf_batch_destroy(hsf_batch_t batch) { batch_destroy(reinterpret_cast<Batch*>(batch)); }

size_t hsf_batch_workspace_size(hsf_batch_t batch, int32_t mode) {
    return batch ? batch_workspace(*reinterpret_cast<Batch*>(batch), mode) : 0;
}

static hsf_status batch_args(hsf_batch_t batch, void* const* outs, int32_t mode, void* ws, size_t ws_bytes) {
    if (!batch || !outs || !ws) return fail(HSF_E_ARG, "null argument");
    if (mode != HSF_SUM_F32 && mode != HSF_SUM_BF16X3) return fail(HSF_E_ARG, "batches use HSF_SUM_F32 or HSF_SUM_BF16X3");
    Batch* b = reinterpret_cast<Batch*>(batch);
    if (ws_bytes < batch_workspace(*b, mode)) return fail(HSF_E_ARG, "workspace too small for the batch");
    return HSF_OK;
}

hsf_status hsf_batch_run(hsf_batch_t batch, void* const* outs, int32_t mode, int32_t use_graph, void* ws,
                         size_t ws_bytes, hsf_stream_t stream) {
    HSF_GUARD_BEGIN
    hsf_status s = batch_args(batch, outs, mode, ws, ws_bytes);
    if (s != HSF_OK) return s;
    return batch_run(*reinterpret_cast<Batch*>(batch), outs, mode, use_graph, ws, (hipStream_t)stream);
    HSF_GUARD_END
}

hsf_status hsf_batch_tune(hsf_batch_t batch, void* const* outs, int32_t mode, void* ws, size_t ws_bytes,
                          hsf_stream_t stream, int32_t* policy) {
    HSF_GUARD_BEGIN
    hsf_status s = batch_args(batch, outs, mode, ws, ws_bytes);
    if (s != HSF_OK) return s;
    int chosen = 0;
    s = batch_tune(*reinterpret_cast<Batch*>(batch), outs, mode, ws, (hipStream_t)stream, &chosen);
    if (policy) *policy = chosen;
    return s;
    HSF_GUARD_END
}

hsf_status hsf_batch_tune_cached(hsf_batch_t batch, int32_t mode, int32_t* policy) {
    HSF_GUARD_BEGIN
    if (!batch || !policy) return fail(HSF_E_ARG, "null batch or policy");
    if (mode != HSF_SUM_F32 && mode != HSF_SUM_BF16X3) return fail(HSF_E_ARG, "batches use HSF_SUM_F32 or HSF_SUM_BF16X3");
    *policy = batch_tune_cached(*reinterpret_cast<Batch*>(batch), mode);
    return HSF_OK;
    HSF_GUARD_END
}

}  // extern "C"
