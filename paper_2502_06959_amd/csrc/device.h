// Device-side launchers of libhsf (implemented in the .hip sources).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace hsf {

constexpr size_t kNormWsDoubles = 8192;

// Path-tree levels kept or resumed (hsf_backward's shifted forward runs):
// keep[s] non-null: side s's levels below the last each go to a buffer of
// their own, level l at keep[s] + level_keep_offset(p, n_paths, s, l); so a
// later run over the same paths can start at level start[s] > 0, its first
// pass reading level start[s] - 1 from parent[s] (laid out as kept; shared by
// every copy of a replicated run).
struct SweepLevels {
    unsigned char* keep[2] = {nullptr, nullptr};
    int start[2] = {0, 0};
    const unsigned char* parent[2] = {nullptr, nullptr};
};
// Bytes from the start of a side's kept levels to level l's rows for a chunk
// of n_paths paths (l = the number of levels below the last: the total).
size_t level_keep_offset(const Plan& p, int64_t n_paths, int side, int l);

// R copies of one forward run in the same launches, which differ only in
// their factor pools and buffers: copy r reads every schedule's pool at
// pool + r pool_rs, writes its half-states at psi + r psi_rs[side] (strides
// in complex elements) and keeps its path-tree levels at ws + r ws_rs bytes
// (a multiple of 256, each copy's share at least tree_workspace bytes).
struct SweepReplicas {
    int R;
    int64_t pool_rs;
    int64_t psi_rs[2];
    size_t ws_rs;
};

// Runs both sides' programs (a side with a null pointer is skipped) for
// paths [p_begin, p_begin + n_paths), one launch per LDS pass.
// Half-states of paths [p_begin, p_begin + n_paths) into psiA / psiB (either
// may be null).  ws: tree_workspace(p, n_paths) bytes for the path-tree
// levels; with less (or null) every path runs every per-path op.  reps: the
// run's copies (null: one).  a_row_end >= 0: only side a's amplitudes
// [a_row_begin, a_row_end) are wanted (at most 2^20 of them): side a's
// passes, from its last back, run only the tiles they depend on, so the rest
// of each side-a row (and of its tree levels) is left unspecified.
hsf_status run_sides(Plan& p, DeviceCopy& d, int64_t p_begin, int64_t n_paths, void* psiA, int64_t ldA,
                     void* psiB, int64_t ldB, void* ws, size_t ws_bytes, hipStream_t stream,
                     const SweepReplicas* reps = nullptr, int64_t a_row_begin = 0, int64_t a_row_end = -1,
                     const SweepLevels* levels = nullptr);
size_t tree_workspace(const Plan& p, int64_t n_paths);

// How a sweep launch row finds its input.  ROW_INPLACE: its own row.
// ROW_SHARED: one shared state (the prefix).  ROW_PARENT: its parent's row at
// the previous path-tree level.
enum RowMode : int32_t { ROW_INPLACE = 0, ROW_SHARED = 1, ROW_PARENT = 2 };

// One launch's worth of one side: pass k over the level rows [i_lo, i_lo +
// rows), row i written to dst + (i - i_lo) * dst_ld (elements), its input
// per `mode` (ROW_PARENT: src row i S / S_par - src_lo, ld src_ld).  dst and
// src may be offsets from a workspace base (batches) instead of pointers.
struct SweepItem {
    size_t k;
    int32_t mode;
    int64_t S, i_lo, rows;
    void* dst;
    int64_t dst_ld;
    const void* src;
    int64_t src_ld, src_lo, S_par;
    int32_t src_shared = 0;   // src is one buffer for every copy of a replicated run
};

// Scratch of the path-tree levels below the last for a chunk of n_paths
// paths: two buffers per side (byte offsets), level l in buffer l % 2.
struct TreeScratch {
    size_t off[2][2] = {{0, 0}, {0, 0}}, total = 0;
};
TreeScratch tree_scratch(const Plan& p, int64_t n_paths);

// The launches of one side's sweep over paths [p_begin, p_begin + n_paths):
// flat (every per-path pass on every path, the first reading `prefix` when
// it is non-null) or level by level (buf0 / buf1: the side's tree scratch).
std::vector<SweepItem> side_items(const Schedule& sc, bool tree, const void* prefix, int64_t p_begin,
                                  int64_t n_paths, void* psi, int64_t ld, unsigned char* buf0, unsigned char* buf1,
                                  int64_t dim, const unsigned char* const* keep = nullptr, int start = 0,
                                  const unsigned char* parent = nullptr);
// The passes of one flat schedule without factor slots over rows 0 .. rows-1
// of psi (ld elements apart), in place.
hsf_status run_segment(const Plan& p, const DeviceSchedule& ds, const Schedule& sc, void* psi, int64_t ld, int64_t rows,
                       hipStream_t stream);

size_t bf16x3_workspace(int na, int nb, int64_t n_paths);

// Path sums staged through LDS for K >= kLdsMinPaths (pathsum_lds.hip); their
// split-BF16 planes are chunked by kBf16Chunk paths (a multiple of 16).
constexpr int kBf16Chunk = 16;
// Output tiles of the LDS-staged split-BF16 path sum: kBf16LdsTileRows A rows
// x 128 B rows (batches count their tiles in this shape).
constexpr int64_t kBf16LdsTileRows = 256;
constexpr int64_t kLdsMinPaths = 64;
bool path_sum_lds_fits(int mode, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K, int64_t M,
                       int64_t N);
hsf_status path_sum_f32_lds(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                            int64_t N, float2* out, int64_t ldo, int accumulate, hipStream_t st);
hsf_status path_sum_f64_lds(bool c128_in, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K, int64_t M,
                            int64_t N, double2* out, int64_t ldo, int accumulate, hipStream_t st);
hsf_status path_sum_bf16x3_lds(const float2* A, int64_t ldA, const float2* B, int64_t ldB, int64_t K, int64_t M,
                               int64_t N, float2* out, int64_t ldo, int accumulate, void* ws, hipStream_t st);
// Split-BF16 planes, and the path sum over planes split beforehand: the
// chunked layout of the LDS-staged kernel (split_lds / sum_lds) and the
// [plane][row][path] layout of the streaming kernel (split_stream /
// sum_stream).  MA: rows of A split; the sums take rows row0 .. row0+M-1 of
// A's planes (RA / pa_rows rows per chunk or plane).
size_t bf16x3_lds_planes(int64_t rows, int64_t K);
size_t bf16x3_stream_planes(int64_t rows, int64_t K);
hsf_status split_lds(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N, int64_t K,
                     unsigned short* PA, unsigned short* PB, hipStream_t st);
hsf_status sum_lds(const unsigned short* PA, int64_t RA, int64_t row0, int64_t M, const unsigned short* PB, int64_t N,
                   int64_t K, float2* out, int64_t ldo, int accumulate, hipStream_t st);
hsf_status split_stream(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N, int64_t K,
                        unsigned short* PA, unsigned short* PB, hipStream_t st);
hsf_status sum_stream(const unsigned short* PA, int64_t pa_rows, int64_t row0, int64_t M, const unsigned short* PB,
                      int64_t N, int64_t K, float2* out, int64_t ldo, int accumulate, hipStream_t st);
// Whole-operand split for later row-range sums (hsf_split_operands), and the
// sum of rows [row0, row0 + M) from those planes.
hsf_status split_operands(const float2* A, int64_t ldA, int64_t MA, const float2* B, int64_t ldB, int64_t N,
                          int64_t K, void* ws, hipStream_t st);
hsf_status path_sum_presplit(int64_t K, int64_t MA, int64_t row0, int64_t M, int64_t N, void* ws, float2* out,
                             int64_t ldo, int accumulate, hipStream_t st);

// Batched launches (tables are device arrays; offsets are relative to `base`).
hsf_status launch_sweep_batch(int kg, bool s1, const void* segs, int nseg, uint32_t total_blocks, int threads,
                              size_t shmem, unsigned char* base, hipStream_t stream);
void batch_sweep_prepare();
hsf_status launch_split_batch(const void* descs, int n, uint32_t total_blocks, unsigned char* base, hipStream_t st);
// full: every product qualifies for the bounds-free streaming kernel (see
// bf16x3_stream_full)
hsf_status launch_bf16x3_batch(const void* descs, int n, int64_t tiles, bool full, unsigned char* base,
                               hipStream_t st);
// Tile shape of the streaming split-BF16 path sum (rows x complex columns)
// and whether a product of M x N outputs over Kp padded paths, leading
// dimension ldo, takes its bounds-free form.
constexpr int64_t kBf16StreamRows = 256, kBf16StreamCols = 128;
inline bool bf16x3_stream_full(int64_t M, int64_t N, int64_t Kp, int64_t ldo, int accumulate) {
    return !accumulate && M % kBf16StreamRows == 0 && N % kBf16StreamCols == 0 && ldo <= (int64_t)(INT32_MAX / 8 / 32) &&
           4 * (M > N ? M : N) * Kp <= (int64_t)INT32_MAX;
}
hsf_status launch_f32_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st);
hsf_status launch_f32_lds_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st);
hsf_status launch_bf16x3_lds_batch(const void* descs, int n, int64_t tiles, unsigned char* base, hipStream_t st);
int persistent_grid(const void* kernel, int threads, size_t shmem, int64_t tiles);

// out[r * ldo + c] (+)= sum_k A[k * ldA + row0 + r] * B[k * ldB + c], r < M, c < N.
hsf_status path_sum(int dtype, int mode, const void* A, int64_t ldA, const void* B, int64_t ldB,
                    int64_t K, int64_t row0, int64_t M, int64_t N, void* out, int64_t ldo,
                    int accumulate, void* ws, hipStream_t stream);

// hsf_amplitudes_full's checks and dispatch (api.cpp).
hsf_status amplitudes_full(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB, int64_t ldB,
                           int64_t n_paths, int64_t row_begin, int64_t row_end, void* out, int64_t ldo, int32_t mode,
                           int32_t accumulate, void* ws, size_t ws_bytes, hipStream_t stream);

// psi(x_j) = sum over the K paths of A[p][x_j >> nb] B[p][x_j mod 2^nb]
// (FP64 sums), into out[j] (added to it with accumulate).  copies > 1: the
// same for replicated half-states, copy r at A + r rsA, B + r rsB (elements)
// into out + r nx.
hsf_status gather_dot(int dtype, const void* A, int64_t ldA, const void* B, int64_t ldB, int64_t K,
                      int nb, int n, const uint64_t* x, int64_t nx, void* out, int accumulate,
                      hipStream_t stream, int copies = 1, int64_t rsA = 0, int64_t rsB = 0);

hsf_status norm2(const void* a, int adt, const void* b, int bdt, int64_t n, double* out, double* ws,
                 hipStream_t stream);

// Workspace of hsf_backward: the preferred size (shifted forward runs in
// batches of as many copies as fit a fixed budget), or the minimal one (one
// copy per batch).
size_t backward_workspace(const Plan& p, int64_t chunk, int64_t nx, bool minimal = false);
// dl_dpsi: n x complex128 cotangents on the device, or null for the
// probability mass
hsf_status backward(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, const void* dl_dpsi, double* grad,
                    int64_t n_params, int64_t chunk, void* ws, size_t ws_bytes, hipStream_t stream);
size_t loss_workspace(const Plan& p, int64_t chunk, int64_t nx);
hsf_status prob_mass(Plan& p, DeviceCopy& d, const uint64_t* x, int64_t nx, double* loss, void* amps, int64_t chunk,
                     void* ws, size_t ws_bytes, hipStream_t stream);

inline hsf_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return HSF_OK;
    return fail(HSF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace hsf
