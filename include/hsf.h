/*
 * hsf.h -- C ABI of libhsf, joint-cut hybrid Schroedinger-Feynman (HSF)
 * simulation on AMD Instinct MI355X (gfx950).
 *
 * Method (Joint Cutting for Hybrid Schroedinger-Feynman Simulation of Quantum
 * Circuits, arXiv:2502.06959):
 *   - the qubits are split at a cut between qubit l and l+1: side b holds
 *     qubits 0..l, side a holds l+1..n-1 (Sec. IV-A);
 *   - gates that cross the cut are grouped by the caller into blocks, and
 *     every block is multiplied into one operator and split by an
 *     operator-Schmidt decomposition A = sum_m s_m X_m (x) Y_m (Sec. II-B,
 *     Sec. III-A, Sec. IV-A);
 *   - a path picks one term per block; there are prod_k r_k paths (Sec. III);
 *   - per path the two half-register states are simulated independently and
 *     the output is the sum over paths of their Kronecker products (Sec. II-B).
 *
 * Index conventions (Sec. II-A): amplitude index i = sum_q i_q 2^q.  A gate's
 * matrix is written with its first qubit q[0] as the most significant bit.
 * Half-state index of side a: i_a = i >> n_b; of side b: i_b = i & (2^n_b - 1),
 * so psi[i_a * 2^n_b + i_b] = sum_p psiA[p][i_a] * psiB[p][i_b], i.e. the
 * row-major matrix C = PsiA^T PsiB is the state.
 *
 * Ownership: a plan owns its host tables and the small device buffers it
 * uploads (gate matrices, Schmidt factors, pass programs; uploaded on first
 * use on each device).  The caller owns every large buffer: half-states,
 * outputs, bitstrings, gradients and workspaces, all device pointers.
 *
 * Errors: every call returns a status; on a non-OK status nothing was
 * launched, the outputs are untouched, and hsf_last_error() returns a
 * thread-local message.  Launch failures map to HSF_E_DEVICE; faults inside
 * a kernel surface when the caller synchronises the stream.  No C++
 * exception crosses this interface.  All work is enqueued on the caller's
 * stream; no call synchronises it except where stated.
 */
#ifndef HSF_H
#define HSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hsf_stream_t; /* a hipStream_t; NULL = default stream */
typedef struct hsf_plan_s* hsf_plan_t;

typedef enum {
    HSF_OK = 0,
    HSF_E_ARG = 1,              /* bad argument (null pointer, range, size)          */
    HSF_E_CUT = 2,              /* cut outside 0..n-2                                */
    HSF_E_BLOCK_UNCOVERED = 3,  /* a crossing gate lies in no block                  */
    HSF_E_BLOCK_OVERLAP = 4,    /* two block hulls share a gate                      */
    HSF_E_BLOCK_CYCLE = 5,      /* contracted circuit has a cycle                    */
    HSF_E_BLOCK_TOO_LARGE = 6,  /* block hull wider than max_side_qubits on a side   */
    HSF_E_RANK_AMBIGUOUS = 7,   /* a singular-value ratio lies in (1e-13, 1e-7]      */
    HSF_E_PATHS_OVERFLOW = 8,   /* more than 2^62 paths                              */
    HSF_E_DEVICE = 9,           /* HIP error (allocation, launch, copy)              */
    HSF_E_UNSUPPORTED = 10      /* valid request the library does not implement      */
} hsf_status;

typedef enum {
    HSF_GATE_U = 0,   /* explicit 2^nq x 2^nq matrix (nq = 1..3)                     */
    HSF_GATE_H, HSF_GATE_X, HSF_GATE_Y, HSF_GATE_Z, HSF_GATE_S, HSF_GATE_SDG,
    HSF_GATE_T, HSF_GATE_TDG,
    HSF_GATE_RX,      /* exp(-i t X / 2)                                             */
    HSF_GATE_RY,      /* exp(-i t Y / 2)                                             */
    HSF_GATE_RZ,      /* exp(-i t Z / 2)                                             */
    HSF_GATE_PHASE,   /* diag(1, e^{it})                                             */
    HSF_GATE_CX,      /* q[0] control, q[1] target                                   */
    HSF_GATE_CZ,
    HSF_GATE_CP,      /* diag(1, 1, 1, e^{it})                                       */
    HSF_GATE_RZZ,     /* exp(-i t Z(x)Z / 2)                                         */
    HSF_GATE_SWAP,
    HSF_GATE_ISWAP
} hsf_gate_kind;

typedef enum { HSF_C64 = 0, HSF_C128 = 1 } hsf_dtype;

/* Path-sum arithmetic for hsf_amplitudes_full / _bitstrings.                  */
typedef enum {
    HSF_SUM_F32 = 0,     /* c64 in, FP32 MFMA with FP32 accumulation, c64 out      */
    HSF_SUM_BF16X3 = 1,  /* c64 in, split-BF16 x3 MFMA, FP32 accumulation, c64 out */
    HSF_SUM_F64 = 2,     /* c64 or c128 in, FP64 MFMA, c128 out (reference mode)   */
    HSF_SUM_C128 = 3,    /* alias of HSF_SUM_F64 for c128 plans                    */
    HSF_SUM_BF16X3_SPLIT = 4 /* HSF_SUM_BF16X3 from the planes hsf_split_operands
                                left in the workspace (no split in the call)     */
} hsf_sum_mode;

typedef struct {
    int32_t kind;            /* hsf_gate_kind                                      */
    int32_t nq;              /* number of qubits (1..3)                            */
    int32_t q[4];            /* qubits; q[0] is the matrix's most significant bit  */
    double param;            /* angle for RX/RY/RZ/PHASE/CP/RZZ                    */
    int32_t param_id;        /* gradient slot of `param`, -1 if none               */
    int32_t reserved;
    const double* matrix;    /* HSF_GATE_U: 2^nq x 2^nq row-major complex128,
                                interleaved (re, im); copied by hsf_plan          */
} hsf_gate;

typedef struct {
    int32_t n_qubits;        /* 2..62                                              */
    int32_t reserved;
    int64_t n_gates;
    const hsf_gate* gates;   /* host array, list order = circuit order             */
} hsf_circuit;

typedef struct {
    double rank_tol;         /* s_m counted if s_m > rank_tol * s_0 (default 1e-10) */
    int32_t max_side_qubits; /* hull qubits per side of SVD-factored blocks (default
                                4, max 4); product-form blocks: see hsf_plan       */
    int32_t dtype;           /* hsf_dtype of the half-states (default HSF_C64)      */
    int32_t tile_qubits;     /* qubits per LDS tile (0 = largest that fits)         */
    int32_t fuse;            /* 1 = fuse gates on the host (default), 0 = off       */
    int32_t tree;            /* path-tree sweeps (hsf_side_levels): 0 = where the
                                planner's cost estimate favours them (default),
                                1 = never, 2 = always                               */
    int32_t defer_b_suffix;  /* 1 = side b's ops after its last factor slot are
                                left out of the half-states and applied to output
                                rows by hsf_apply_b_suffix (default 0)             */
} hsf_plan_options;

/* ---------------------------------------------------------------- plan ---- */

/* Build a plan (host only; no device call).  Sec. IV-A (partition, reshape,
 * SVD), Sec. III-A (joint cutting of blocks), Sec. III (path count).
 *   circuit         host circuit; copied.
 *   cut             last qubit of side b (Table II's "cut pos."), 0..n-2.
 *   block_gate_ids  gate ids of all blocks back to back; block k is
 *   block_offsets   ids[offsets[k] .. offsets[k+1]), offsets has n_blocks+1
 *                   entries.  Each block is closed to its hull (all gates
 *                   between two of its gates along shared qubits).  Every
 *                   crossing gate must be in some hull.
 *   opts            NULL for defaults.
 *   out             receives the plan; destroy with hsf_plan_destroy.
 * Blocks are renumbered in the order of a topological sort of the circuit
 * with blocks contracted (ready node with smallest gate id first), and path
 * p has digit m_k = (p / R_k) mod r_k, R_k = prod_{k'>k} r_k'.
 * Decomposition: a hull made of diagonal gates that each touch at most one
 * qubit of one side (a cascade, Sec. V, and the analytic decompositions of
 * Sec. IV's cascade example) is decomposed in the computational basis of its
 * other side s: U = sum_m c(m) |m><m| (x) prod_j diag(phi_j(m, 0),
 * phi_j(m, 1)), r_k = 2^|s|, |s| <= 4 and up to HSF_MAX_BLOCK_SIDE qubits on
 * the wide side; it is used only when 2^|s| equals the Schmidt rank (the
 * singular values of the operator's reshape).  Every other hull is reshaped
 * and SVD-factored (Sec. IV-A) and may have at most max_side_qubits per
 * side (HSF_E_BLOCK_TOO_LARGE otherwise).                                  */
hsf_status hsf_plan(const hsf_circuit* circuit, int32_t cut, const int64_t* block_gate_ids,
                    const int64_t* block_offsets, int32_t n_blocks,
                    const hsf_plan_options* opts, hsf_plan_t* out);
void hsf_plan_destroy(hsf_plan_t plan);

/* Deferred side-b suffix (Sec. II-B, by linearity of the path sum).  With
 * hsf_plan_options.defer_b_suffix = 1, side b's program stops at its last
 * factor slot: the gates after it act on every path's side-b state alike, so
 * for each output row (x >> n_b fixed) they can be applied once to the row's
 * 2^{n_b} amplitudes after the sum over paths instead of to every path's
 * half-state.  This pays when few rows are wanted (the first amplitudes of
 * Sec. V: a few rows of 2^{n_b} amplitudes against P half-states).  Such a
 * plan's half-states (hsf_run_paths) and path sums (hsf_amplitudes_full,
 * hsf_amplitudes_full_noalloc) lack those gates until hsf_apply_b_suffix
 * runs on the output rows; hsf_amplitudes_bitstrings, hsf_loss,
 * hsf_backward and hsf_batch_create reject the plan (HSF_E_UNSUPPORTED).
 *   out    device, `rows` rows of 2^{n_b} amplitudes (c64 or c128 as the
 *          plan), row r at out + r * ldo elements; updated in place.
 *   ldo    >= 2^{n_b}.
 * Call it once per row, after every path has been summed into it (the ops
 * are linear, so rows summed in several accumulating calls take it once at
 * the end).  A plan without a deferred suffix returns HSF_OK and leaves
 * `out` unchanged.  Asynchronous on `stream`; HSF_E_ARG for null arguments,
 * rows < 0 or ldo < 2^{n_b}.                                                 */
hsf_status hsf_apply_b_suffix(hsf_plan_t plan, void* out, int64_t ldo, int64_t rows, hsf_stream_t stream);

/* Joint blocks for a cut (host only), Sec. III-A and Sec. V: the gates of
 * every maximal run of consecutive diagonal gates commute, so the run's
 * crossing two-qubit gates are regrouped into the fewest stars (gates that
 * share one qubit; each star has Schmidt rank <= 2), a minimum vertex cover
 * of the bipartite graph of those gates (Koenig's theorem).  Other crossing
 * gates are blocks of their own.
 *   order           n_gates entries: a gate order with the same unitary
 *                   (order[i] = original index of the i-th gate); inside a
 *                   run the non-crossing gates come first (circuit order),
 *                   then each star's gates together.
 *   block_gate_ids  positions in `order` of every block's gates, back to back
 *                   (at most n_gates entries);
 *   block_offsets   n_blocks + 1 entries (room for n_gates + 1);
 *   n_blocks        receives the block count.
 * Pass the reordered circuit and these blocks to hsf_plan.                   */
hsf_status hsf_find_blocks(const hsf_circuit* circuit, int32_t cut, int64_t* order,
                           int64_t* block_gate_ids, int64_t* block_offsets, int32_t* n_blocks);

/* Dimensions: n, cut, n_a = n - cut - 1, n_b = cut + 1, K blocks, P paths.  */
hsf_status hsf_plan_dims(hsf_plan_t plan, int32_t* n, int32_t* cut, int32_t* n_a,
                         int32_t* n_b, int32_t* n_blocks, int64_t* n_paths);
int64_t hsf_num_paths(hsf_plan_t plan);

/* Block k (plan order): rank r_k, digit stride R_k, side-a and side-b
 * supports (ascending qubits; sa and sb need room for HSF_MAX_BLOCK_SIDE
 * entries each, or are NULL), hull size and the caller's index of the block. */
#define HSF_MAX_BLOCK_SIDE 16
hsf_status hsf_block_info(hsf_plan_t plan, int32_t k, int32_t* rank, int64_t* stride,
                          int32_t* n_sa, int32_t* sa, int32_t* n_sb, int32_t* sb,
                          int64_t* hull_len, int32_t* caller_index);
/* Hull gate ids of block k, ascending (hull_len entries).                    */
hsf_status hsf_block_hull(hsf_plan_t plan, int32_t k, int64_t* ids);
/* Schmidt data of block k (Sec. IV-A): all singular values (SVD-factored:
 * 4^min(|sa|,|sb|) entries; product form: 2^min(|sa|,|sb|); descending) and
 * the factors the half-states receive, X_m (side a) and Y_m (side b),
 * m < r_k, each row-major 2^|s| x 2^|s| complex128 interleaved, ascending
 * qubit = ascending significance (SVD-factored: sqrt(s_m) times the singular
 * operators; product form: the products of hsf_plan).  Any pointer may be
 * NULL.  HSF_E_UNSUPPORTED if a factor is requested for a side of more than
 * 8 qubits.                                                                   */
hsf_status hsf_block_factors(hsf_plan_t plan, int32_t k, double* sigma, double* xa, double* yb);
/* Digits m_k(p) of path p (K entries).                                       */
hsf_status hsf_path_digits(hsf_plan_t plan, int64_t p, int32_t* digits);
/* Gate-program statistics of side 0 = a, 1 = b: ops before fusion, ops after
 * fusion, LDS passes per path after the shared prefix, qubits per tile, and
 * the shared prefix itself: the fused ops that are not factor slots and
 * commute with every factor slot before them (disjoint qubits, or both
 * diagonal), applied once per plan and device to a single state that every
 * path then starts from (Sec. II-B: they act the same way on all paths), and
 * the LDS passes that apply them.  Any pointer may be NULL.                   */
hsf_status hsf_side_stats(hsf_plan_t plan, int32_t side, int64_t* ops_logical,
                          int64_t* ops_fused, int32_t* passes, int32_t* tile_qubits,
                          int64_t* ops_shared, int32_t* shared_passes);

/* Path-tree levels of side 0 = a, 1 = b.  A path's half-state depends on its
 * digits only through the factor slots applied so far (Sec. II-B), so the
 * paths that agree on the leading digits m_0 .. m_{d-1} (block 0 most
 * significant) share one state until the first op that needs a later digit.
 * The level of a fused op is the number of leading digits its result depends
 * on (a slot of block k needs k + 1, and an op follows every earlier op it
 * does not commute with); the ops, stably sorted by level, are swept level by
 * level, each level keeping P / S states (S = prod_{k >= d} r_k) for all P
 * paths.  Level 0 is the shared prefix (one state).
 *   cap        entries of ops and states;
 *   n_levels   receives the number of levels (at least 1);
 *   ops        fused ops of the first min(cap, n_levels) levels;
 *   states     their state counts for all P paths.
 * Any output pointer may be NULL.                                              */
hsf_status hsf_side_levels(hsf_plan_t plan, int32_t side, int32_t cap, int32_t* n_levels, int64_t* ops,
                           int64_t* states);
/* How hsf_run_paths sweeps a chunk of n_paths paths (given the workspace
 * hsf_workspace_size(plan, 0, n_paths, 0)): tree receives 1 for level by
 * level (path tree), 0 if every path runs every per-path op; tile_qubits
 * (2 entries, side a and b) the LDS tile sizes.  The planner takes the form
 * and tile size with the lowest timing estimate (or the form the plan's
 * option forces).  Either pointer may be NULL.                              */
hsf_status hsf_sweep_form(hsf_plan_t plan, int64_t n_paths, int32_t* tree, int32_t* tile_qubits);

/* --------------------------------------------------------------- paths ---- */

/* Device workspace in bytes for `op` over `n_paths` paths:
 *   op 0 = hsf_run_paths (the path-tree levels below the last, when the
 *   planner sweeps n_paths paths level by level; else 0), 1 =
 *   hsf_amplitudes_full with path-sum mode
 *   `mode`, 2 = hsf_backward with chunks of `n_paths` paths and `mode` =
 *   number of bitstrings n_x (the preferred size), 3 = hsf_loss with chunks
 *   of `n_paths` paths and `mode` = n_x, 4 = the least workspace
 *   hsf_backward accepts (same arguments as op 2).                             */
size_t hsf_workspace_size(hsf_plan_t plan, int32_t op, int64_t n_paths, int32_t mode);

/* Per-path half-states for paths [p_begin, p_end) (Sec. II-B): row j of
 * psiA (ld ldA elements) receives side a's state for path p_begin + j,
 * 2^n_a amplitudes; psiB likewise with 2^n_b.  Either side may be NULL to
 * skip it.  Element type is the plan's dtype (c64 = 2 x float, c128 =
 * 2 x double).  Rows are overwritten; nothing is read.  The first call on a
 * device uploads the plan's tables and simulates each side's shared prefix
 * once (device memory of 2^n_side amplitudes per side and tile schedule,
 * owned by the plan, freed by hsf_plan_destroy; this call synchronizes the
 * device once).  ws: hsf_workspace_size(plan, 0, p_end - p_begin, 0) bytes
 * (device) for the path-tree levels (hsf_side_levels); with a smaller or
 * NULL workspace every path runs every per-path op (same result).  Calls
 * that overlap on one workspace race.                                       */
hsf_status hsf_run_paths(hsf_plan_t plan, int64_t p_begin, int64_t p_end, void* psiA,
                         int64_t ldA, void* psiB, int64_t ldB, void* ws, size_t ws_bytes,
                         hsf_stream_t stream);

/* hsf_run_paths for callers that need only the amplitudes [row_begin,
 * row_end) of side a (at most 2^20), such as the first amplitudes of the
 * state (Sec. V computes the first 10^6): side a's passes, from its last
 * back, run only the tiles those rows depend on (a pass's tile reads the
 * same tile of its input, so the needed amplitudes widen by each pass's tile
 * qubits; the walk stops at the first pass that needs every tile), so the
 * rest of each psiA row is left unspecified (psiA is required and keeps its
 * full layout, ldA >= 2^n_a).
 * Side b (psiB, may be NULL) is computed in full.  The wanted rows equal
 * hsf_run_paths' bit for bit.  Other arguments, errors and ownership as in
 * hsf_run_paths.                                                            */
hsf_status hsf_run_paths_rows(hsf_plan_t plan, int64_t p_begin, int64_t p_end, int64_t row_begin,
                              int64_t row_end, void* psiA, int64_t ldA, void* psiB, int64_t ldB,
                              void* ws, size_t ws_bytes, hsf_stream_t stream);

/* Path sum (Sec. II-B), output rows [row_begin, row_end) of C = PsiA^T PsiB:
 * out[(r - row_begin) * ldo + c] = sum_{j < n_paths} psiA[j][r] psiB[j][c],
 * c < 2^n_b.  Input type: the plan's dtype.  Output type: c64 for HSF_SUM_F32
 * and HSF_SUM_BF16X3, c128 for HSF_SUM_F64 / HSF_SUM_C128.  accumulate = 1
 * adds into `out` (path chunks, resume).  ws: hsf_workspace_size(plan, 1,
 * n_paths, mode) bytes (HSF_SUM_BF16X3 uses it as scratch; with
 * HSF_SUM_BF16X3_SPLIT it holds the planes of hsf_split_operands, psiA and
 * psiB are not read and may be NULL).  A range of at most 32 rows (the
 * first amplitudes of a large state) is bound by reading psiB once: there
 * HSF_SUM_F32 and HSF_SUM_BF16X3 both run FP32 MFMA products straight from
 * the half-states (no split, the workspace is not touched).  n_paths = 0 is
 * the empty sum: the rows are set to zero (left as they are with
 * accumulate = 1) and psiA / psiB are not read (they may be NULL).  An empty
 * row range writes nothing and `out` may then be NULL.                      */
hsf_status hsf_amplitudes_full(hsf_plan_t plan, const void* psiA, int64_t ldA,
                               const void* psiB, int64_t ldB, int64_t n_paths,
                               int64_t row_begin, int64_t row_end, void* out, int64_t ldo,
                               int32_t mode, int32_t accumulate, void* ws, size_t ws_bytes,
                               hsf_stream_t stream);

/* Split-BF16 operand planes for the path sum of Sec. II-B taken in the
 * split-BF16 x3 arithmetic: every FP32 value x of the first n_paths rows of
 * psiA (all 2^n_a amplitudes) and psiB (all 2^n_b) becomes hi = bf16(x) and
 * lo = bf16(x - hi), written into ws (hsf_workspace_size(plan, 1, n_paths,
 * HSF_SUM_BF16X3) bytes, device) in the layout the path sum of n_paths paths
 * reads.  Later hsf_amplitudes_full calls with HSF_SUM_BF16X3_SPLIT, the
 * same ws and the same n_paths then sum any row range without splitting
 * again (row tiles of one large output split each operand once).  The plan
 * records ws and n_paths of its last split; a HSF_SUM_BF16X3_SPLIT call that
 * names others fails with HSF_E_ARG.  c64 plans only.  Overwriting psiA /
 * psiB afterwards does not change the planes; calls that overlap on one ws
 * race.                                                                      */
hsf_status hsf_split_operands(hsf_plan_t plan, const void* psiA, int64_t ldA, const void* psiB, int64_t ldB,
                              int64_t n_paths, void* ws, size_t ws_bytes, hsf_stream_t stream);

/* Amplitudes of chosen basis states (Sec. V computes a subset):
 * out[j] = sum_{p < n_paths} psiA[p][x_j >> n_b] psiB[p][x_j & (2^n_b - 1)],
 * accumulated in FP64; `out` is c128 (2 doubles per entry).  x: device
 * array of n_x indices < 2^n.  accumulate = 1 adds into `out`.  n_x = 0
 * writes nothing (x and out may then be NULL); n_paths = 0 gives zeros (psiA
 * and psiB may then be NULL).                                                */
hsf_status hsf_amplitudes_bitstrings(hsf_plan_t plan, const void* psiA, int64_t ldA,
                                     const void* psiB, int64_t ldB, int64_t n_paths,
                                     const uint64_t* x, int64_t n_x, void* out,
                                     int32_t accumulate, hsf_stream_t stream);

/* hsf_amplitudes_full without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * hsf_amplitudes_full, except: the scratch of HSF_SUM_BF16X3 (the split-BF16
 * planes) lives in a static device array of HSF_NOALLOC_SCRATCH_BYTES bytes
 * that the library holds on every device it runs on until the process ends;
 * a call whose planes, hsf_workspace_size(plan, 1, n_paths, HSF_SUM_BF16X3),
 * would exceed it fails with HSF_E_ARG before any launch (sum fewer paths per
 * call with accumulate = 1).  HSF_SUM_BF16X3_SPLIT is rejected (its planes
 * are the caller's).  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  All calls on one device share its array, so
 * calls that overlap on one device (other streams, other threads) race; a
 * call leaves the array holding its own planes.                              */
#define HSF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hsf_status hsf_amplitudes_full_noalloc(hsf_plan_t plan, const void* psiA, int64_t ldA,
                                       const void* psiB, int64_t ldB, int64_t n_paths,
                                       int64_t row_begin, int64_t row_end, void* out, int64_t ldo,
                                       int32_t mode, int32_t accumulate, hsf_stream_t stream);

/* ------------------------------------------------------------- checks ---- */

/* FP64-accumulated sums over n complex entries of type dtype: out[0] =
 * sum |a_i|^2 and, if b != NULL, out[1] = sum |a_i - b_i|^2 (b of the same
 * type; b may be c64 or c128 per b_dtype).  out: 2 device doubles.
 * Deterministic (fixed reduction order).  ws: at least 4096 doubles.  n = 0
 * gives zeros (a may then be NULL).                                          */
hsf_status hsf_norm2(const void* a, int32_t a_dtype, const void* b, int32_t b_dtype, int64_t n,
                     double* out, void* ws, size_t ws_bytes, hsf_stream_t stream);

/* ------------------------------------------------------------ gradient ---- */

/* Probability mass of chosen basis states (Sec. V computes a subset of the
 * amplitudes): L = sum_j |psi(x_j)|^2 over the n_x basis states x (device
 * array of indices < 2^n), psi the HSF state of Sec. II-B summed over all
 * paths.  The library runs the half-states of both sides `chunk` paths at a
 * time (the path tree where it pays), accumulates psi(x_j) in FP64 over the
 * chunks and reduces L in a fixed order (bitwise reproducible).  loss: one
 * device double, overwritten.  amps: NULL, or n_x complex128 device entries
 * that receive psi(x_j).  ws: hsf_workspace_size(plan, 3, chunk, n_x) bytes
 * (device).  n_x = 0 gives L = 0 (x may then be NULL).                      */
hsf_status hsf_loss(hsf_plan_t plan, const uint64_t* x, int64_t n_x, double* loss, void* amps,
                    int64_t chunk, void* ws, size_t ws_bytes, hsf_stream_t stream);

/* Gradient with respect to every parameter id (0..n_params-1) of the
 * circuit's rotation gates (RX, RY, RZ, RZZ; PHASE and CP outside blocks) of
 * a real loss L of the amplitudes psi(x_j) of n_x basis states x (device
 * array); psi is the HSF state of Sec. II-B and d psi/d t follows from the
 * chain rule through the per-path half-states.  dL_dpsi: NULL for the
 * probability mass L = sum_j |psi(x_j)|^2, else n_x complex128 device
 * cotangents g_j = dL/dRe psi(x_j) + i dL/dIm psi(x_j) (the convention of
 * torch's complex gradients), giving grad[t] = sum_j Re(conj(g_j)
 * d psi(x_j)/d t).  Angles outside blocks use an adjoint sweep per path
 * (state checkpointed in front of each Schmidt factor, which has no
 * inverse); an angle inside a block's hull uses the exact shift rule on the
 * amplitudes, d psi/d t = psi(t + pi) / 2 (every such gate is exp(-i t P/2)
 * with P^2 = 1), psi(t + pi) being one forward with the block re-factored
 * (Sec. IV-A) at the shifted angle.  grad: n_params device doubles,
 * overwritten.  Paths are processed `chunk` at a time; ws: at least
 * hsf_workspace_size(plan, 4, chunk, n_x) bytes, best
 * hsf_workspace_size(plan, 2, chunk, n_x): the shifted forward runs go as
 * copies of one run in the same launches, as many per batch as the
 * workspace holds (up to 4 GiB of copies; the result does not depend on
 * it).  Reductions run in a fixed order (bitwise reproducible).
 * Synchronises `stream` (host tables are staged through it), so it cannot
 * be captured in a graph; the shifted forward runs use one stream of its own
 * (default priority, created and destroyed within the call, joined to
 * `stream` before it returns).  Returns HSF_E_UNSUPPORTED if a shifted block
 * needs more Schmidt terms than the plan.  n_x = 0, or a circuit without
 * angles, gives a zero gradient.                                            */
hsf_status hsf_backward(hsf_plan_t plan, const uint64_t* x, int64_t n_x, const void* dL_dpsi, double* grad,
                        int64_t n_params, int64_t chunk, void* ws, size_t ws_bytes,
                        hsf_stream_t stream);

/* -------------------------------------------------------------- batches ---- */

/* Many independent circuits run together (paths of different circuits are as
 * independent as paths of one, Sec. II-B): every circuit's LDS pass k goes in
 * one launch, the path sums of all circuits in one persistent MFMA launch
 * over the union of their output tiles.  Plans must be complex64, with sides
 * of at least 3 qubits, and must outlive the batch.                           */
typedef struct hsf_batch_s* hsf_batch_t;
hsf_status hsf_batch_create(const hsf_plan_t* plans, int32_t n_plans, hsf_batch_t* out);
void hsf_batch_destroy(hsf_batch_t batch);
/* Workspace bytes for hsf_batch_run with path-sum `mode` (F32 or BF16X3):
 * every circuit's half-states (all paths) and path-tree levels, plus BF16
 * planes for BF16X3.                                                         */
size_t hsf_batch_workspace_size(hsf_batch_t batch, int32_t mode);
/* Full state of every circuit: outs[i] is a device array of 2^n_i complex64
 * amplitudes of circuit i (row-major, index i_a 2^n_b + i_b as for one plan).
 * use_graph = 1 records the launch sequence in a HIP graph on the first call
 * and replays it afterwards (the graph is rebuilt when `outs`, `mode`, the
 * workspace address or the tuned policy change); small device tables are
 * (re)built with synchronous copies when those change, outside any capture. */
hsf_status hsf_batch_run(hsf_batch_t batch, void* const* outs, int32_t mode, int32_t use_graph, void* ws,
                         size_t ws_bytes, hsf_stream_t stream);
/* Autotuner: times the sweep policies (0: largest tiles, fewest passes; 1:
 * per-circuit tiles that fill the device alone; 2: one size smaller -- all
 * flat sweeps; 3, the default before tuning: each circuit's sweep form and
 * tile size as hsf_sweep_form gives them, path trees where they pay) with 3
 * runs each on `stream`, keeps the fastest for later hsf_batch_run calls and
 * returns it in *policy.  Synchronises `stream`.                             */
hsf_status hsf_batch_tune(hsf_batch_t batch, void* const* outs, int32_t mode, void* ws, size_t ws_bytes,
                          hsf_stream_t stream, int32_t* policy);
/* Tuner cache: every successful hsf_batch_tune records its choice in a
 * process-wide table keyed by the path-sum mode and, circuit by circuit in
 * batch order, n_a, n_b, the path count and each side's fused op count.
 * hsf_batch_tune_cached looks `batch` up there: on a hit it applies the
 * recorded policy to the batch (as hsf_batch_tune would) and returns it in
 * *policy; otherwise *policy = -1 and the batch is unchanged.  Host only (no
 * device work, no timing); HSF_E_ARG for a null batch or policy or a mode
 * other than HSF_SUM_F32 / HSF_SUM_BF16X3.  Thread-safe.                     */
hsf_status hsf_batch_tune_cached(hsf_batch_t batch, int32_t mode, int32_t* policy);

/* Thread-local message for the last non-OK status on this thread.            */
const char* hsf_last_error(void);
/* Library version string.                                                    */
const char* hsf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HSF_H */
