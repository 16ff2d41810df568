/*
 * hodlr.h -- C ABI of the MI355X (gfx950) mixed-precision HODLR
 * matrix-(multi)vector product.
 *
 * Method: Carson, Chen, Liu, "Mixed Precision HODLR Matrices"
 * (arXiv 2407.21637).  The library holds an eps-HODLR operator given as
 * fp64 leaf blocks and truncated-SVD factors U_b V_b^T of every off-diagonal
 * block, stores each level's factors in the precision the adaptive rule
 * picks (Alg. "Adaptive-precision HODLR Format", eq. (3.3)) or that the
 * caller forces (Alg. "Mixed-precision HODLR Format"), and computes
 * Y = A_H X on the GPU (Alg. "HODLR_MATVEC").
 *
 * Conventions shared by every entry point:
 *  - All functions return hodlr_status; no exception or abort crosses the
 *    ABI.  On error nothing is enqueued on any stream and the handle is
 *    unchanged; hodlr_last_error_message() gives a detail string
 *    (thread-local).
 *  - Matrices are column-major.  X and Y are n x nrhs with leading
 *    dimension ldx, ldy >= n; Y is overwritten (the algorithm starts from
 *    b = 0).  X and Y are device pointers owned by the caller and must stay
 *    valid until the stream work completes.
 *  - Host input arrays passed to hodlr_create are deep-copied; the caller
 *    may free them when the call returns.  Device memory of an operator is
 *    owned by the library and released by hodlr_destroy.
 *  - Indices are 0-based.  Node j of level k (j = 0..2^k-1) is the paper's
 *    I_{j+1}^k (Def. 2.1).  The canonical order of the 2^(depth+1)-2
 *    off-diagonal blocks is: level k ascending, then row node j ascending;
 *    block (k, j) has rows node j and columns node j^1 (its sibling), so the
 *    upper block of each pair (rows I_{2i-1}, cols I_{2i}, eq. (2.1))
 *    precedes the lower one, and its index is (2^k - 2) + j.
 *  - Threading: after create/assign, a handle is read-only, and matvec
 *    calls on the same handle may run concurrently on different streams
 *    (each call uses its own workspace slot; see hodlr_matvec).  create,
 *    assign, set_level_precisions and destroy must not overlap other use of
 *    the same handle.
 */
#ifndef HODLR_H
#define HODLR_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>   /* hipStream_t */

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hodlr_op_s* hodlr_op;

typedef enum {
    HODLR_OK = 0,
    HODLR_E_ARG = 1,          /* invalid or inconsistent argument */
    HODLR_E_STATE = 2,        /* wrong state (e.g. host-only handle asked for a product) */
    HODLR_E_NOMEM = 3,        /* host or device allocation failed */
    HODLR_E_DEVICE = 4,       /* a HIP runtime call or a launch failed */
    HODLR_E_RANGE = 5,        /* a factor overflows its storage format (no column scaling) */
    HODLR_E_UNSUPPORTED = 6   /* valid request the library does not support */
} hodlr_status;

/* Storage / arithmetic formats.  u = 2^-t: fp64 2^-53, fp32 2^-24, bf16 2^-8,
 * fp16 2^-11, fp8 e4m3 (OCP E4M3FN, max 448) 2^-4, fp8 e5m2 (the paper's q52)
 * 2^-3 (Table 1.1). */
typedef enum {
    HODLR_FP64 = 0,
    HODLR_FP32 = 1,
    HODLR_BF16 = 2,
    HODLR_FP16 = 3,
    HODLR_FP8_E4M3 = 4,
    HODLR_FP8_E5M2 = 5
} hodlr_dtype;

/* Flags of hodlr_assign_precision / hodlr_set_level_precisions. */
#define HODLR_NO_COLUMN_SCALE 0x1u  /* store fp16/fp8 without per-column 2^e scales */
#define HODLR_ACC_FP32        0x2u  /* force fp32 accumulation of Y */
#define HODLR_ACC_FP64        0x4u  /* force fp64 accumulation of Y */
#define HODLR_PER_BLOCK       0x8u  /* hodlr_assign_precision: one format per block (see there) */

/* One off-diagonal block U V^T: U is r_b x rank (orthonormal columns,
 * eq. (3.1)), V is c_b x rank, both fp64 column-major on the host. */
typedef struct {
    int32_t rank;
    const double* U;
    int64_t ldu;
    const double* V;
    int64_t ldv;
} hodlr_lowrank;

typedef struct {
    int64_t n;
    int32_t depth;
    int32_t nblocks;          /* 2^(depth+1) - 2 */
    int32_t acc_dtype;        /* HODLR_FP32 or HODLR_FP64: accumulation of Y */
    int32_t max_rank;
    int32_t on_device;        /* 1 if the operator lives on a GPU */
    int32_t device;
    double eps;               /* eps of the last assign (0 after create / set_level) */
    int64_t leaf_bytes;       /* fp64 leaf blocks as stored (8 sum m_i^2) */
    int64_t factor_bytes;     /* sum_b (r_b + c_b) p_b s(f_b): codes of all U, V */
    int64_t scale_bytes;      /* one byte per scaled column */
    int64_t device_bytes;     /* size of the packed device image incl. padding */
} hodlr_info;

typedef struct {
    int32_t level;            /* k = 1..depth */
    int32_t rank;             /* p_b */
    int64_t row0, nrows;      /* rows of the block: node j of level k */
    int64_t col0, ncols;      /* columns: node j^1 */
    int32_t dtype;            /* storage format of the block's level */
    int32_t scaled;           /* 1 if per-column exponents are in use */
} hodlr_block_info;

/* ---- tree (Def. 2.1; left child = ceil(parent/2), Sect. 4) ------------ */

/* Smallest depth l >= 0 with leaf * 2^l >= n (leaves of the ceil split then
 * hold at most `leaf` indices).  Returns -1 if n < 1 or leaf < 1. */
int32_t hodlr_depth_for_leaf(int64_t n, int64_t leaf);

/* Node boundaries of every level.  leaf_bounds: NULL for the ceil split, or
 * 2^depth+1 non-decreasing values from 0 to n (empty nodes allowed).
 * bounds_out receives levels 0..depth one after another, level k holding
 * 2^k+1 values; total 2^(depth+1) + depth values.  E_ARG on bad input. */
hodlr_status hodlr_tree_bounds(int64_t n, int32_t depth, const int64_t* leaf_bounds,
                               int64_t* bounds_out);

/* Canonical off-diagonal blocks (eq. (2.1)): 5 int64 per block
 * (level, row0, nrows, col0, ncols), 2^(depth+1)-2 blocks. */
hodlr_status hodlr_tree_blocks(int64_t n, int32_t depth, const int64_t* leaf_bounds,
                               int64_t* desc_out);

/* ---- construction on the GPU from a kernel matrix ---------------------- */

/* Kernel matrices the library evaluates itself: A_ij = k(p_i, p_j) for
 * points p_i of dimension `dim` (r = |p_i - p_j|), plus diag_shift on the
 * diagonal; with diag_given the diagonal entries are diag_value (before
 * the shift) instead of k(p_i, p_i). */
#define HODLR_KERNEL_GAUSSIAN   0   /* exp(-r^2 / a), a > 0 */
#define HODLR_KERNEL_INV_DIST   1   /* 1 / (r + a) */
#define HODLR_KERNEL_LOG        2   /* log(r + a) */
#define HODLR_KERNEL_EXP        3   /* exp(-r) */
#define HODLR_KERNEL_SIGNED_INV 4   /* 1 / (x_i - x_j), 1D, needs diag_given */

typedef struct {
    int32_t kind;
    int32_t dim;              /* 1 or 2 */
    double a;
    double diag_shift;
    double diag_value;
    int32_t diag_given;
    int32_t reserved_;
} hodlr_kernel;

typedef struct {
    double ms_norms;          /* squared norms of every block and leaf, leaves */
    double ms_factors;        /* randomised truncated SVDs of the blocks */
    double ms_total;          /* the whole call, the operator's upload included */
    int32_t max_rank;
    int32_t max_sketch;       /* widest sketch used */
    int32_t sketch_rounds;    /* passes over a level's pending blocks (retries included) */
    int32_t exact_residual;   /* 1: the truncation residual was computed exactly (eps < 1e-6) */
} hodlr_build_report;

/* Build the eps-HODLR operator of a kernel matrix on GPU `device`
 * (Sect. 2-3): the tree of hodlr_tree_bounds for n and depth; leaves
 * D_i = A(I_i, I_i); every off-diagonal block B replaced by U V^T with
 * orthonormal U (eq. (3.1)) and the smallest rank p such that
 * ||B - U V^T||_F <= eps ||B||_F (Def. 2.2 in the Frobenius norm, so that
 * Lemma 2.4 holds), from a randomised truncated SVD whose residual is
 * computed (exactly, when eps < 1e-6) rather than estimated, so the rule
 * holds for the factors produced.  The matrix is evaluated on the fly on
 * the device and never stored.  ||A||_F^2 and ||A_b||_F^2 of the original
 * matrix (the nrmAll and nrm_k of Alg. "Adaptive-precision HODLR Format")
 * are computed exactly in fp64 and kept with the operator:
 * hodlr_assign_precision uses them when given neither xi nor norms2, and
 * hodlr_get_norms returns them.  points: n x dim fp64 on the host, point i
 * at points[i * dim] (deep-copied).  seed: the sketches' random numbers.
 * The new operator is uniform fp64, as from hodlr_create.  E_UNSUPPORTED
 * if a block needs a rank beyond the widest sketch (128 columns); report
 * may be NULL. */
hodlr_status hodlr_build_kernel(hodlr_op* out, int64_t n, int32_t depth, const double* points,
                                const hodlr_kernel* kernel, double eps, uint64_t seed, int32_t device,
                                hodlr_build_report* report);

/* The squared Frobenius norms kept by hodlr_build_kernel: 1 + nblocks
 * values, ||A||_F^2 then ||A_b||_F^2 in canonical order.  E_STATE for an
 * operator made by hodlr_create. */
hodlr_status hodlr_get_norms(hodlr_op op, double* norms2);

/* ---- operator ------------------------------------------------------- */

/* Create an operator from fp64 leaves (2^depth blocks, leaf i is m_i x m_i
 * column-major with leading dimension ld_leaves[i] >= m_i) and the
 * 2^(depth+1)-2 off-diagonal blocks in canonical order (rank <= min(r_b,
 * c_b); rank 0 allowed).  depth >= 0, n >= 1.  device >= 0 uploads the
 * operator to that GPU; device = -1 builds a host-only handle (tree, rule,
 * packing and export work; products return E_STATE).  The new operator is
 * uniform fp64 (every u_k = fp64) with fp64 accumulation, i.e. the
 * same-GPU uniform-precision baseline. */
hodlr_status hodlr_create(hodlr_op* out, int64_t n, int32_t depth, const int64_t* leaf_bounds,
                          const double* const* leaves, const int64_t* ld_leaves,
                          const hodlr_lowrank* blocks, int32_t device);

/* Adaptive precision (Alg. "Adaptive-precision HODLR Format", eq. (3.3)):
 * for each level k, xi_k = sqrt(nrm_k / nrmAll), u'_k = eps / (2^(k/2) xi_k)
 * (2^(k/2) evaluated as sqrt(2^k)), and u_k is the largest unit roundoff
 * <= u'_k among fp64 and `allowed` (n_allowed entries of hodlr_dtype).
 * xi: NULL, or depth values xi_1..xi_depth (finite, >= 0) used as given,
 * e.g. the algorithm's values computed elsewhere from the original matrix;
 * the decisions then depend on nothing else.  Without xi they come from
 * the norms.  norms2: NULL, or 1 + nblocks values: ||A||_F^2 followed by
 * ||A_b||_F^2 of the original blocks in canonical order (nrm_k is their
 * maximum over level k).  With NULL the norms are computed from the stored
 * fp64 factors and leaves (the H~ of Thm. 3.1); they are not needed when
 * xi is given without HODLR_PER_BLOCK.  If no format meets u'_k the level is fp64
 * and marked insufficient; if xi_k = 0 the coarsest allowed format is used.
 * Accumulation: fp64 if eps < 1e-7, else fp32, unless a HODLR_ACC_* flag
 * forces it.  The factors are then quantised (round to nearest even, once,
 * from fp64; fp16/fp8 columns scaled by 2^e_j, e_j the largest integer with
 * max_i |F_ij| 2^e_j <= the format's largest finite value) and repacked.
 * E_RANGE if HODLR_NO_COLUMN_SCALE is set and a value overflows.
 * HODLR_PER_BLOCK: each block b of level k gets its own format, the same
 * rule with its own norm, xi_b = sqrt(||A_b||_F^2 / nrmAll) in place of
 * xi_k (never finer than the level's format; the global bound (3.5) still
 * holds, as the proof of Thm. 3.1 bounds every block separately).
 * hodlr_get_level keeps reporting the level rule; hodlr_get_block gives
 * each block's format.  hodlr_set_level_precisions returns to one format
 * per level. */
hodlr_status hodlr_assign_precision(hodlr_op op, double eps, const int32_t* allowed,
                                    int32_t n_allowed, const double* xi, const double* norms2,
                                    uint32_t flags);

/* Explicit per-level formats (Alg. "Mixed-precision HODLR Format"):
 * per_level[k-1] is level k's storage format.  Accumulation: fp64 when
 * every level is fp64, else fp32, unless a HODLR_ACC_* flag forces it. */
hodlr_status hodlr_set_level_precisions(hodlr_op op, const int32_t* per_level, uint32_t flags);

/* The last assignment of level k (1..depth): format, xi_k, u'_k and the
 * insufficient mark (xi and u' are 0 after create / set_level). */
hodlr_status hodlr_get_level(hodlr_op op, int32_t level, int32_t* dtype, double* xi,
                             double* u_prime, int32_t* insufficient);

hodlr_status hodlr_get_info(hodlr_op op, hodlr_info* info);
hodlr_status hodlr_get_block(hodlr_op op, int32_t block, hodlr_block_info* info);

/* Everything about an operator in one call: the hodlr_info fields, the
 * last assignment of every level (format, xi_k, u'_k and the insufficient
 * mark of Alg. "Adaptive-precision HODLR Format"; entries past depth are
 * 0), whether blocks carry their own formats (HODLR_PER_BLOCK), and which
 * contraction the matrix-core products run: leaf_stacked = 1 when, for
 * every leaf, the ranks of all its ancestor blocks (one per level) fit one
 * pass of stacked 16-row matrix-core tiles of one format (at most 64
 * rows, 32 with fp64 arithmetic), so T_b = V_b^T X is formed leaf by leaf
 * with X read once; 0 when it is formed per level over runs of rows.
 * leaf_bounds: NULL, or room for 2^depth + 1 values (leaf node boundaries,
 * Def. 2.1); ranks: NULL, or room for nblocks values (canonical order). */
#define HODLR_MAX_LEVELS 24
typedef struct {
    hodlr_info info;
    int32_t level_dtype[HODLR_MAX_LEVELS];
    int32_t insufficient[HODLR_MAX_LEVELS];
    double xi[HODLR_MAX_LEVELS];
    double u_prime[HODLR_MAX_LEVELS];
    int32_t per_block;
    int32_t leaf_stacked;
} hodlr_query_info;

hodlr_status hodlr_query(hodlr_op op, hodlr_query_info* q, int64_t* leaf_bounds, int32_t* ranks);

/* Stored codes of block b: u_codes gets r_b x rank codes (column-major,
 * ld = r_b, element size s(f) bytes: the format's bit patterns), u_exp the
 * rank column exponents e_j (value = decode(code) * 2^-e_j; all 0 when
 * unscaled); v_codes / v_exp likewise for V (c_b x rank).  Any pointer may
 * be NULL.  from_device = 1 reads the uploaded image back from the GPU
 * (device handles only); 0 re-derives it on the host with the same packer. */
hodlr_status hodlr_export_block(hodlr_op op, int32_t block, void* u_codes, int8_t* u_exp,
                                void* v_codes, int8_t* v_exp, int32_t from_device);

/* Y = A_H X (Alg. "HODLR_MATVEC").  xy_dtype is the dtype of both X and Y.
 *
 * HODLR_FP64 or HODLR_FP32: leaf products D_i X_i run in fp64; a level
 * stored in fp64 runs in fp64; other levels run in the accumulation
 * precision, with the stored codes converted in registers.  With nrhs < 8
 * the products are wavefront reductions (HBM-bound); with nrhs >= 8 they
 * run on the matrix cores (fp64 MFMA for leaves and fp64 levels, fp32 MFMA
 * for the others).
 *
 * HODLR_BF16 or HODLR_FP16: the product in that low working precision W
 * (Thm. 3.5 and the Sect. 4 experiment with u = u_W): the leaves (a W copy
 * made on the first such call), every stored generator value and T_b =
 * V_b^T X enter the arithmetic rounded to W (nearest even), products are
 * summed in fp32 on the matrix cores (v_mfma_f32_16x16x32_bf16 / _f16),
 * and Y is rounded to W once.  Any nrhs >= 1.  For fp16 a leaf entry or a
 * generator stored in fp64/fp32/bf16 outside the fp16 range gives
 * HODLR_E_RANGE (narrow stored formats are column-scaled into range); a
 * T_b or Y entry beyond the range becomes infinite.  Not available in
 * hodlr_matvec_batched.
 *
 * stream: NULL is the default stream.  The call only enqueues work, except
 * that the first call on a stream, or with a larger nrhs than before on
 * it, allocates that stream's workspace (and the first bf16 / fp16 call
 * after an assignment builds that format's operand and waits for it), so
 * such a call must not be made while the stream is being captured
 * (E_STATE for the operand; capture rules forbid the allocation).
 *
 * Graphs: the products may be captured into a HIP graph.  Such a graph
 * stays valid until the handle is destroyed or reassigned (assign or
 * set_level_precisions replace the device image it reads); workspaces that
 * later calls outgrow are kept, not freed, until hodlr_destroy. */
hodlr_status hodlr_matvec(hodlr_op op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          int32_t nrhs, int32_t xy_dtype, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of hodlr_matvec with HODLR_FP64 or HODLR_FP32 X and Y, the same
 * kernels and the same result bit for bit, with every workspace buffer
 * taken from one library-owned static device array of 64 MiB per GPU
 * (held from the first such call on a device until the process ends)
 * instead of a per-stream workspace.  Nothing is allocated: not by the
 * library, not by the runtime on its behalf.  A product whose workspace
 * exceeds 64 MiB gets E_ARG (the message gives the bytes needed); bf16 /
 * fp16 X gets E_UNSUPPORTED (that path needs a per-assignment operand).
 * All such calls on one GPU share the array: calls that can overlap in
 * time (different streams, other threads, other handles) race and give
 * wrong results; serialise them, e.g. on one stream.  The arrival
 * counters in the array are cleared by a fill kernel at the start of each
 * call, so a captured call replays correctly. */
hodlr_status hodlr_matvec_noalloc(hodlr_op op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                  int32_t nrhs, int32_t xy_dtype, hipStream_t stream);

/* count independent products Y_i = A_i X_i (each as hodlr_matvec defines
 * it; the paper treats one operator at a time, this is the batch of many).
 * Operators may differ in size, depth, ranks, formats, nrhs and dtype but
 * must live on one device; arrays have length count; each Y_i is
 * overwritten.  A handle may appear only once per batch (its workspace
 * serves one product at a time; E_ARG otherwise).  Operators that share a kernel variant (X/Y dtype,
 * accumulation, wave or matrix-core path, right-hand-side grouping) run
 * together: one persistent launch per phase walks a work list of all their
 * units (leaves, contraction items, T reductions, expansion tiles), so the
 * whole batch is a handful of launches.
 * The first call with a given signature (handles and their current images,
 * X/Y pointers, leading dimensions, nrhs, dtypes, stream) builds a plan:
 * it uploads the work lists (device memory held until a handle in it is
 * destroyed or, unless a caller's graph has recorded the plan's launches,
 * 32 newer plans evict it), picks the shape of every launch (one
 * variant's one phase) on `stream`: work order longest-first or as given,
 * 1, 2, 4 or 8 workgroups per compute unit, each candidate timed alone,
 * and captures the launches into a HIP graph.  Choices are cached by the
 * device's architecture and the launch's shape class, in memory and in the
 * text file HODLR_TUNE_CACHE (default $HOME/.cache/hodlr/batch_tune.txt;
 * "off": memory only), so plans of known shapes skip the timing;
 * HODLR_BATCH_TUNE=0 skips tuning.  Every shape gives the same result bit
 * for bit.  Later calls with the same signature replay that graph.  On a
 * stream that is being captured the launches are recorded into the
 * caller's graph instead; that needs a plan made by an earlier call outside
 * capture (E_STATE otherwise), since nothing may be allocated during a
 * capture.  Operators with HODLR_BF16 or HODLR_FP16 X/Y (the low working
 * precision of hodlr_matvec) are not part of the plan: their products run
 * one after another, after the planned launches, through the
 * single-operator launches on `stream`, with the same results as
 * hodlr_matvec; their operands in W are checked and built (once per
 * precision assignment) before any product is enqueued, and a capture finds
 * them only when an earlier call outside it built them (E_STATE otherwise).
 * Argument errors are reported before anything is enqueued. */
hodlr_status hodlr_matvec_batched(const hodlr_op* ops, int32_t count, const void* const* X,
                                  const int64_t* ldx, void* const* Y, const int64_t* ldy,
                                  const int32_t* nrhs, const int32_t* xy_dtype, hipStream_t stream);

/* Per-phase GPU timing.  capacity > 0 makes the next `capacity` products
 * of this handle record a HIP event pair around each of their kernel phases
 * on the launch stream (0 turns recording off and drops the records).
 * Phases: 0 padded copy of X (when a leaf size is not a multiple of 16, or,
 * for nrhs >= 8, when X's columns are not 16-byte aligned), 1 contraction
 * (T = V^T X for every block), 2 expansion and leaves (Y = D X + U T),
 * 3 sum of the contraction's partial results into T (nrhs >= 8 only; below
 * that the contraction's last workgroup per block does it inside phase 1).
 * hodlr_profile_read synchronises on the recorded
 * events and returns, per phase, the summed duration in milliseconds and
 * the number of launches timed; it then clears the records. */
hodlr_status hodlr_profile(hodlr_op op, int32_t capacity);
hodlr_status hodlr_profile_read(hodlr_op op, double* ms_per_phase, int64_t* launches_per_phase);

/* ---- LU factorization and solves (Sect. 3.4) ------------------------ */

typedef struct {
    double ms_factor;         /* the factorization on the host (image upload excluded) */
    double norm_l;            /* ||L||_F and ||U||_F of the factors (exact, not formed) */
    double norm_u;
    int32_t max_rank;         /* widest off-diagonal generator met, updates included */
    int32_t reserved_;
} hodlr_lu_report;

/* Factor the operator as stored, H = L U (Alg. "HODLR_LU"), and keep the
 * factors with it.  The input is the mixed-precision representation the
 * product uses: fp64 leaves and every generator decoded from its stored
 * format.  Runs in fp64 on the host: leaves by LU without pivoting (unit
 * lower L); for H = [[H11, U12 V12^T], [U21 V21^T, H22]] the factors of H11,
 * then U's block (1,2) = (L11^-1 U12) V12^T and L's block (2,1) =
 * U21 (U11^-T V21)^T, then the Schur complement H22 - L21 U12 as a low-rank
 * update down H22's tree whose off-diagonal blocks are recompressed to the
 * smallest rank with ||B~ - B^||_F <= eps ||B~||_F (the truncation
 * assumption of Sect. 3.4; eps = 0 keeps every nonzero singular value), and
 * the factors of it.  The backward error then obeys Cor. "LU of
 * mixed-precision HODLR matrices": ||L U - H||_F <~ 2 (2^l - 1) eps ||H||_F
 * + 11 (2^l - 1) eps ||L||_F ||U||_F (with the representation's own error
 * against the original matrix added).  On a device handle the inverse
 * factors are also formed and uploaded for hodlr_solve (see there; about
 * twice the device memory of the fp64 operator).  Reassigning formats (hodlr_assign_
 * precision, hodlr_set_level_formats) or destroying the operator drops
 * them.  E_UNSUPPORTED on a zero pivot (no LU without pivoting);
 * E_ARG unless 0 <= eps < 1; report may be NULL. */
hodlr_status hodlr_lu(hodlr_op op, double eps, hodlr_lu_report* report);

/* X = U^-1 L^-1 B with the factors of hodlr_lu, on the GPU, on `stream`
 * (stream-ordered like hodlr_matvec).  B, X: n x nrhs column-major device
 * buffers, both HODLR_FP64 or both HODLR_FP32 (xy_dtype), leading
 * dimensions ldb, ldx >= n; B may alias X when ldb == ldx.  hodlr_lu forms
 * L^-1 and U^-1 as HODLR matrices of the same tree and ranks (the inverse of
 * a triangular HODLR matrix is one: L^-1's block (2,1) is
 * (-L22^-1 U21)(L11^-T Y21)^T, U^-1's block (1,2) is
 * (-U11^-1 X12)(U22^-T V12)^T, the leaves the inverses of the leaves'
 * triangular factors, all formed in fp64), and the solve is two fp64
 * products with fp64 accumulation, Z = L^-1 B then X = U^-1 Z (fp32 B is
 * widened first and X rounded once).  The operator owns an fp64 workspace
 * of 2 n nrhs doubles, grown (with a device synchronisation) when a call
 * needs more: calls that overlap on one operator race on it.  E_STATE
 * without factors or on a host-only handle. */
hodlr_status hodlr_solve(hodlr_op op, const void* B, int64_t ldb, void* X, int64_t ldx, int32_t nrhs,
                         int32_t xy_dtype, hipStream_t stream);

/* The factors as dense n x n column-major matrices (L unit lower, U upper
 * triangular), for checking; either pointer may be NULL.  E_STATE without
 * factors. */
hodlr_status hodlr_lu_dense(hodlr_op op, double* L, int64_t ldl, double* U, int64_t ldu);

hodlr_status hodlr_destroy(hodlr_op op);

const char* hodlr_status_string(hodlr_status s);
const char* hodlr_last_error_message(void);   /* thread-local detail of the last failure */
const char* hodlr_last_error(void);           /* the same string (earlier name) */

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H */
