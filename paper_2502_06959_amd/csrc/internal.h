// Internal data structures of libhsf (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "hsf.h"

namespace hsf {

using cd = std::complex<double>;

constexpr int kMaxSideQubits = 4;     // widest block support per side (SVD-factored blocks)
constexpr int kMaxProductSide = 16;   // widest side of a product-form block (must match HSF_MAX_BLOCK_SIDE)
constexpr int kMaxExpandSide = 8;     // product factors are expanded to dense matrices up to this width
constexpr int kMaxOpQubits = 4;       // widest dense op in a side program
constexpr int kMaxTileBits = 24;

hsf_status fail(hsf_status s, const std::string& msg);   // records the thread-local message
std::string g_last_error_copy();                        // the current thread-local message

struct Gate {
    int kind = 0;
    int nq = 0;
    int q[4] = {0, 0, 0, 0};
    double param = 0.0;
    int param_id = -1;
    std::vector<cd> m;     // 2^nq x 2^nq, row-major, q[0] most significant
    bool diag = false;     // matrix is exactly diagonal
};

// Builds the matrix of a gate from its definition; false if the kind is unknown.
bool gate_matrix(int kind, int nq, double param, const double* explicit_m, std::vector<cd>& out);

// Singular value decomposition A = W diag(s) Vh of a row-major m x n complex
// matrix by one-sided (Hestenes) Jacobi rotations in FP64.  W is m x r
// (column-major: W[j * m + i]), Vh is r x n row-major, r = min(m, n), s is
// descending.  Columns of W for zero singular values are left zero.
void jacobi_svd(int m, int n, const std::vector<cd>& A, std::vector<cd>& W,
                std::vector<double>& s, std::vector<cd>& Vh);

// Factor of one block applied on one side, on qubits q (ascending, global
// numbering): rank matrices of size 2^|q| x 2^|q| (q.back() = most
// significant bit of the matrix index).
struct FactorPiece {
    std::vector<int> q;
    std::vector<cd> m;
};

// The decomposition U_k = sum_m X_m (x) Y_m of one block.  SVD-factored
// blocks have one piece per side (X_m = sqrt(s_m) times the m-th right
// singular operator, Y_m likewise).  Product-form blocks (every gate
// diagonal and touching at most one qubit of the wide side) are decomposed
// in the computational basis of the narrow side: X_m (x) Y_m =
// |m><m| (x) prod_j phi_j(m), one 1-qubit piece per qubit.
struct Factors {
    std::vector<double> sigma;       // singular values of the block operator, descending
    int rank = 0;
    bool product = false;
    std::vector<FactorPiece> pa, pb; // pieces on side a / side b
};

struct Block {
    int caller_index = 0;
    std::vector<std::pair<int64_t, int>> params;   // (gate id, param id) of rotations in the hull
    std::vector<int64_t> hull;       // gate ids, ascending
    std::vector<int> sa, sb;         // supports, ascending qubits
    std::vector<double> sigma;       // all singular values, descending
    int rank = 0;
    int64_t stride = 1;              // R_k
    std::vector<cd> xa;              // rank x (dA x dA): the whole side-a factor (empty if too wide to expand)
    std::vector<cd> yb;              // rank x (dB x dB)
    bool product = false;            // product-form decomposition (see Factors)
    std::vector<FactorPiece> pa, pb; // what the side programs apply
};

// One op of a side program on side-local qubits (q[0] = most significant
// bit of the op's matrix index).
struct SideOp {
    enum Kind { DENSE = 0, DIAG = 1, SLOT = 2 };
    int kind = DENSE;
    int k = 0;
    int q[kMaxOpQubits] = {0, 0, 0, 0};
    std::vector<cd> m;       // DENSE: d x d; DIAG: d entries; SLOT: rank x d x d
    int block = -1;          // SLOT: plan block index
    int piece = 0;           // SLOT: which piece of the block's factor on this side
    bool product = false;    // SLOT: a product-form piece (diagonal for every angle of the block)
    int rank = 1;
    int64_t stride = 1;
    int64_t logical = 1;     // circuit gates represented by this op
    int param_id = -1;       // rotation angle of a single gate (before fusion), -1 if none
    std::vector<cd> dgen;    // D with dU/dparam = D U on the op's qubits (param_id >= 0)
    // SLOT on one qubit: the one-qubit gates that followed the piece on its
    // qubit, folded into it (2x2, applied after each rank's matrix); empty:
    // none
    std::vector<cd> post;
};

// Rank r's 2^k x 2^k matrix of a factor slot with its folded gates applied
// (post * m_r for a one-qubit piece).
std::vector<cd> slot_matrix(const SideOp& o, int r);

// Device op (plain data, read by the sweep kernels).
// A register group whose bits all lie below 6 + k ("wave-private") maps the
// 64 lanes and its k bits onto tile bits 0 .. 5+k, so wave w only touches the
// elements whose higher tile bits spell w (and the loop index): two
// consecutive wave-private groups need no workgroup barrier between them.
//   DOP_GROUP: every thread holds the 2^k amplitudes that differ in tile bits
//     bit[0..k) (register position g <-> tile bit bit[g]) and applies the
//     sub-ops subs[mat .. mat + rank) to them in order.
//   DOP_DENSEK / DOP_SLOT: a dense 2^k x 2^k matrix on tile bits bit[0..k)
//     (bit[0] = most significant); SLOT picks matrix (path / stride) % rank.
enum DevOpType : int32_t { DOP_GROUP = 0, DOP_DENSEK = 2, DOP_SLOT = 4 };
struct DevOp {
    int32_t type;
    int32_t k;
    int32_t bit[4];
    int32_t mat;         // DENSEK/SLOT: pool offset (complex); GROUP: first sub-op
    int32_t rank;        // SLOT: factor count; GROUP: sub-op count
    int64_t stride;      // SLOT: digit stride R_k
    int32_t block;       // SLOT: plan block index
    int32_t piece;       // SLOT: factor piece of that block on this side
    int32_t barrier;     // 1: workgroup barrier after this op (0: only this wave's own slice was touched)
    int32_t spare;
};

// Sub-op of a group.  D1: 2x2 matrix m on register position g.  SIGN/PHASE:
// a diagonal; its qubits outside the group (nc of them, tile bit qb[i] >= 0
// or -1 - q for a qubit outside the tile) form the combo index
// c = sum_i bit_i 2^i, uniform over a thread's group; SIGN negates register
// element j when bit j of the 16-bit mask (mask[c / 2] >> 16 (c % 2)) is set,
// PHASE multiplies element j by pool[mat + c 2^k + j].
enum SubOpType : int32_t { SUB_D1 = 0, SUB_SIGN = 1, SUB_PHASE = 2, SUB_SLOT1 = 3 };
struct SubOp {
    int32_t type;
    int32_t g;
    int32_t nc;
    int32_t mat;          // PHASE: table offset in the pool; SLOT1: first of the rank 2x2 factors
    int32_t qb[4];
    uint32_t mask[8];
    double m[8];
    // SLOT1 (a one-qubit factor piece on register position g; the path's
    // digit (path / stride) % rank picks the 2x2 matrix)
    int32_t rank = 1;
    int64_t stride = 1;
    int32_t block = -1, piece = 0;
    std::vector<cd> post;  // SLOT1: the slot's folded gates (empty: none)
};

struct Pass {
    int32_t n_local = 0;               // tile bits L
    int32_t init_zero = 0;             // start from |0...0> instead of reading
    int32_t op_begin = 0, op_end = 0;  // DevOp range
    int32_t local_q[kMaxTileBits] = {};   // side-local qubit of tile bit i (ascending)
    int32_t n_nonlocal = 0;
    int32_t nonlocal_q[kMaxTileBits] = {};
    int32_t has_slot1 = 0;             // some group applies a one-qubit factor piece (SUB_SLOT1)
    int32_t prefix = 0;                // applies ops of the path-independent prefix only
    // one register group is the whole pass: each thread takes its group's
    // amplitudes straight from the source row and stores them to the
    // destination (no LDS tile, no barriers); its filler bits are high tile bits
    int32_t direct = 0;
};

// One level of a path-tree schedule: passes [pass_begin, pass_end) apply
// the ops whose result depends on the digits m_0 .. m_{d-1} only (block 0
// most significant), so the level keeps one state per value of those
// digits, shared by the S = prod_{k >= d} r_k paths that agree on them.
struct TreeLevel {
    int pass_begin = 0, pass_end = 0;
    int64_t S = 1;
    int64_t ops = 0;                  // fused ops in the level
};

// LDS pass schedule of one side for one tile size.
struct Schedule {
    int tile_bits = 0;
    // passes [0, n_prefix_passes) apply the side's path-independent prefix
    // (every op before the first factor op); the pass after them reads the
    // state they leave, which is the same for every path
    int n_prefix_passes = 0;
    std::vector<Pass> passes;
    std::vector<DevOp> devops;
    std::vector<SubOp> subs;
    std::vector<cd> pool;             // matrices referenced by devops / subs
    // path-tree schedules only: the per-path passes level by level (the
    // first level reads the prefix state, each later one its parent level)
    std::vector<TreeLevel> levels;
};

struct SideProgram {
    int nq = 0;
    std::vector<SideOp> raw;          // before fusion (one op per gate or slot)
    std::vector<SideOp> ops;          // after fusion
    int n_prefix = 0;                 // leading ops of `ops` without factor slots
    int64_t ops_logical = 0;
    std::vector<Schedule> sched;      // one per candidate tile size, largest first
    // the same tile sizes as path-tree schedules (empty when the plan has
    // no blocks); ops reordered by level, see level_order
    std::vector<Schedule> tree;
    // the gradient's forward replay of `raw`: one flat schedule per run of
    // raw ops between factor slots, raw[seg_lo[i] .. seg_hi[i]) (plans with
    // angles only)
    std::vector<Schedule> seg;
    std::vector<int> seg_lo, seg_hi;
    // side b's ops after its last factor slot when the plan defers them to
    // the output rows (hsf_apply_b_suffix): their count before fusion and
    // one flat schedule (empty otherwise)
    int64_t post_ops = 0;
    std::vector<Schedule> post;
};

// One (circuit, side) segment of a batched sweep launch (device table).
struct BatchSeg {
    const Pass* pass;
    int64_t psi_off;         // bytes from the batch workspace base to the segment's output row 0
    int64_t ld;
    const DevOp* ops;
    const void* subs;
    const void* pool;
    uint32_t n_tiles;
    uint32_t block_start;    // first workgroup of the segment
    const void* shared;      // ROW_SHARED: the state every row starts from (the shared prefix)
    // rows as in a single plan's sweep: level rows i = i_lo + j, paths
    // [i S, (i + 1) S), written to output row i - i_lo; ROW_PARENT reads row
    // i S / S_par - src_lo of the buffer at base + src_off (ld src_ld)
    int64_t S, i_lo, src_off, src_ld, src_lo, S_par;
    int32_t mode;
    int32_t spare;
};

// Batched path sum: one circuit's operands and output (device tables).
struct SplitDesc {           // split of one operand into BF16 planes
    int64_t x_off;           // bytes from the workspace base to the half-states
    int64_t ldx, K, R, Kp;
    int64_t planes_off;      // bytes from the workspace base to the planes
    uint32_t blocks_x;       // workgroups along R
    uint32_t block_start;
    uint32_t chunked;        // 1: planes chunked by 32 paths (LDS-staged path sum); 0: [plane][row][Kp]
    uint32_t pad;
};
struct GemmDesc {
    int64_t a_off, b_off;    // bytes from the workspace base (planes or half-states)
    int64_t ldA, ldB, K, M, N;
    void* out;
    int64_t ldo;
    int64_t tiles_n;
    int64_t tile_start;      // first output tile of this circuit in the batch (tiles_n per tile row)
};

struct DeviceSchedule {
    void* passes = nullptr;           // Pass[]
    void* ops = nullptr;              // DevOp[]
    void* subs = nullptr;             // SubOp[]
    void* pool = nullptr;             // float2[] or double2[]
    void* prefix = nullptr;           // the side's state after the prefix passes (2^nq amplitudes), or null
};

struct DeviceCopy {
    int device = -1;
    std::vector<DeviceSchedule> side[2];
    std::vector<DeviceSchedule> tree[2];   // the sides' path-tree schedules
    std::vector<DeviceSchedule> seg[2];    // the gradient's replay segments
    std::vector<DeviceSchedule> post[2];   // a deferred side-b suffix
};

struct Plan {
    int n = 0, cut = 0, na = 0, nb = 0;
    int dtype = HSF_C64;
    double rank_tol = 1e-10;
    int max_side = kMaxSideQubits;
    int fuse = 1;
    int tile_req = 0;
    int tree_mode = 0;                // path-tree sweeps: 0 = by cost estimate, 1 = never, 2 = always
    int defer_b = 0;                  // side b's suffix deferred to the output rows (hsf_apply_b_suffix)
    std::vector<Gate> gates;
    std::vector<Block> blocks;
    int64_t P = 1;
    SideProgram side[2];              // 0 = side a (upper), 1 = side b (lower)
    std::vector<DeviceCopy> dev;
    int64_t n_params = 0;
    // the workspace and path count of the last hsf_split_operands call, which
    // HSF_SUM_BF16X3_SPLIT path sums must name again
    const void* split_ws = nullptr;
    int64_t split_paths = -1;
};

// Joint blocks of commuting crossing gates (blocks.cpp): a gate order and
// the blocks as positions in that order (hsf_find_blocks).
hsf_status find_blocks(const hsf_circuit* c, int32_t cut, int64_t* order, int64_t* ids, int64_t* offs,
                       int32_t* n_blocks);

// Register-group width (tile bits per thread group) for an L-bit LDS tile:
// 16 amplitudes per thread on tiles of 2^13 amplitudes or more, where LDS
// capacity already caps occupancy and the wider group halves the LDS round
// trips (measured: about 20% faster sweeps on 14-bit tiles); 8 otherwise,
// where more threads per tile matter more.  The planner and every launcher
// use this.
constexpr int kWideGroupTile = 13;
inline int group_bits(int L) { return L >= kWideGroupTile ? 4 : (L < 3 ? L : 3); }

// Validates gate i of an n-qubit circuit and builds its matrix.
hsf_status load_gate(const hsf_gate& in, int n, int64_t i, Gate& g);

hsf_status build_plan(const hsf_circuit* c, int32_t cut, const int64_t* ids, const int64_t* offs,
                      int32_t n_blocks, const hsf_plan_options* opts, Plan** out);

// Operator-Schmidt decomposition of block b with gate `gate_id` taking angle
// `param` instead of its own (gate_id < 0: unchanged), as factor pieces,
// with the rank under the plan's tolerance.  A block that qualifies for the
// product form gets it; others need at most kMaxSideQubits per side.
hsf_status factor_block(const Plan& p, const Block& b, int64_t gate_id, double param, Factors& f);
// factor_block for a block whose Schmidt rank is at most `rank` (a gate moved
// to another angle): range finder with `rank` probes and an r x cols SVD
// instead of the full decomposition, checked by reconstruction (falls back to
// factor_block when the check fails).
hsf_status factor_block_rank(const Plan& p, const Block& b, int64_t gate_id, double param, int rank, Factors& f);
// Dense side factors (rank x d x d) from the pieces; empty if the side has
// more than kMaxExpandSide qubits.
void expand_factors(const Block& b, const Factors& f, std::vector<cd>& xa, std::vector<cd>& yb);

// dU/dparam = D U for a rotation gate (RX, RY, RZ, RZZ, PHASE, CP); false otherwise.
bool gate_generator(int kind, int nq, std::vector<cd>& d);

// Side-program fusion and pass scheduling (plan.cpp).
void fuse_side(Plan& p, int side);
// The same fusion on an op list of an nq-qubit side (the deferred suffix).
void fuse_list(const Plan& p, std::vector<SideOp>& ops, int nq);
// Commutes diagonal gates ahead of diagonal factor pieces and sets n_prefix.
void order_prefix(SideProgram& sp);
// Fused ops of a side in path-tree order (stable by level) and the bounds
// of each level's range (cuts[0] = 0, ..., cuts.back() = ops) with the
// level of each range.
std::vector<SideOp> level_order(const Plan& p, int side, std::vector<int>& cuts, std::vector<int>& levels);
// Passes for ops[cuts[0] .. cuts[1]) (the shared prefix, may be empty) and
// then each range [cuts[i], cuts[i+1]); tree: record each later range as a
// TreeLevel with S from `levels`.
Schedule schedule_side(const Plan& p, int side, int tile_bits, const std::vector<SideOp>& ops,
                       const std::vector<int>& cuts, const std::vector<int>& levels, bool tree);
// The sweep form and tile schedule run_sides takes for a chunk of n_paths
// paths: the path tree or the flat sweep (as the plan's option allows) and
// the candidate tile size, whichever a timing estimate puts lowest.
struct SweepChoice {
    bool tree = false;
    int sched = 0;      // index into SideProgram::sched / tree (clamped per side)
};
SweepChoice choose_sweep(const Plan& p, int64_t n_paths, bool allow_tree = true);
// Index of the schedule used for a launch over n_paths paths.
int pick_schedule(const Plan& p, int64_t n_paths);

// Batches of circuits (batch.cpp).
struct Batch;
hsf_status batch_create(Plan* const* plans, int n, Batch** out);
void batch_destroy(Batch* b);
size_t batch_workspace(const Batch& b, int mode);
hsf_status batch_run(Batch& b, void* const* outs, int mode, int use_graph, void* ws, hipStream_t st);
hsf_status batch_tune(Batch& b, void* const* outs, int mode, void* ws, hipStream_t st, int* chosen);
// The policy an earlier batch_tune in this process chose for a batch of the
// same shapes and mode, applied to b; -1 (b unchanged) if there is none.
int batch_tune_cached(Batch& b, int mode);

// Device side (sweep.hip / pathsum.hip).
hsf_status ensure_device(Plan& p, DeviceCopy** out);
void release_device(Plan& p);
int max_tile_bits(int dtype);

}  // namespace hsf
