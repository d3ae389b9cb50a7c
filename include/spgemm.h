/*
 * spgemm.h - C ABI of the MI355X (gfx950) sparse matrix-matrix product.
 *
 * The library computes C = A * B for row-major compressed sparse (CSR) FP64
 * matrices, row by row in the form the paper attributes to Gustavson
 * (Scharpff, Iglberger, Hager, Ruede, "Model-guided Performance Analysis of
 * the Sparse Matrix-Matrix Multiplication", arXiv:1303.1651, Section IV-A):
 * row r of C is the sum, over the stored a(r,c) of row r of A in stored
 * order, of a(r,c) times row c of B.
 *
 * Output contract (Section IV-B, the append/finalize interface): C is written
 * as one contiguous block, rows in increasing order and, inside a row, column
 * indices strictly increasing.  An entry exists in C exactly when some product
 * a(r,c) * b(c,x) was formed for it, whatever its value (a sum that cancels
 * to 0.0 is stored).  Each entry is accumulated from +0.0, one FP64 multiply
 * and one FP64 add per product, in A's column order (the listing of the
 * row-major computation kernel), unless SPGEMM_OPT_FAST is set, in which case
 * rows above the workgroup limit may add their products in another order
 * (values then agree to a few ulps, structure is still exact).
 *
 * Sizing (Section IV-B): the number of multiplications of a row is an upper
 * bound of its number of entries; the library reports the sum of these
 * bounds so that a caller can size C with one allocation, or the exact size
 * after the symbolic pass, or a learned estimate.
 *
 * Memory and ownership
 *   - Every matrix pointer in spgemm_csr is a DEVICE pointer owned by the
 *     caller.  The library never allocates device memory: the caller passes
 *     a workspace (size from spgemm_plan_workspace_size) and, where the
 *     plan reports one, a scratch buffer, both 256-byte aligned (as
 *     hipMalloc returns them).  Host-side plan objects are
 *     allocated with malloc and freed by spgemm_plan_destroy.
 *   - Row pointers are int64 (rows + 1 entries, row_ptr[0] == 0,
 *     non-decreasing, row_ptr[rows] == nnz).  Column indices are int32 in
 *     [0, cols), strictly increasing inside each row.  Values are FP64.
 *     cols must be < 2^31.
 *   - All work is enqueued on the caller's HIP stream.  Calls that return
 *     a size to the host (plan, symbolic, numeric) synchronise that stream.
 *
 * Errors are returned as spgemm_status; no call exits or throws.  A HIP
 * runtime error is reported as SPGEMM_E_HIP and its code is kept in the plan
 * (spgemm_plan_last_hip_error).
 */
#ifndef SPGEMM_H
#define SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spgemm_status {
    SPGEMM_OK = 0,
    SPGEMM_E_NULL = 1,            /* a required pointer is NULL                     */
    SPGEMM_E_DIM = 2,             /* A.cols != B.rows, negative sizes, or (found by
                                     the plan) nnz != row_ptr[rows] for A or B        */
    SPGEMM_E_NOT_CANONICAL = 3,   /* validate: unsorted/duplicate/out-of-range cols  */
    SPGEMM_E_INDEX_OVERFLOW = 4,  /* cols >= 2^31                                    */
    SPGEMM_E_WORKSPACE = 5,       /* workspace or scratch too small or not 256-byte aligned */
    SPGEMM_E_CAPACITY = 6,        /* C capacity too small; required size returned    */
    SPGEMM_E_NO_MODEL = 7,        /* learned sizing requested without a model        */
    SPGEMM_E_STATE = 8,           /* calls out of order (e.g. numeric before plan)   */
    SPGEMM_E_HIP = 9,             /* HIP runtime error                               */
    SPGEMM_E_INVALID = 10,        /* bad option value                                */
    SPGEMM_E_IO = 11,             /* model file could not be read or written         */
    SPGEMM_STATUS_INT_RANGE = 0x7fffffff  /* not a status: makes every int a value of the
                                             type, so that status_string may take any */
} spgemm_status;

/* A CSR matrix; pointers are device pointers.  val may be NULL where only
 * the structure is used (plan, symbolic).  nnz equals row_ptr[rows]. */
typedef struct spgemm_csr {
    int64_t rows, cols, nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} spgemm_csr;

/* How output rows are sized before the numeric pass. */
typedef enum spgemm_sizer {
    SPGEMM_SIZER_EXACT = 0,        /* two passes: symbolic (exact counts), scan, numeric      */
    SPGEMM_SIZER_UPPER_BOUND = 1,  /* one pass, per-row accumulators sized by the multiplication
                                      count (Section IV-B estimate)                         */
    SPGEMM_SIZER_LEARNED = 2       /* one pass, accumulators sized by the learned network;
                                      rows with no room spill to an arena, or with that full
                                      are computed again with their exact size              */
} spgemm_sizer;

enum {
    SPGEMM_OPT_FAST = 1,           /* allow reordered accumulation in workgroup-level rows  */
    SPGEMM_OPT_VALIDATE = 2,       /* check that A and B are canonical CSR                  */
    SPGEMM_OPT_TIMING = 4          /* time the tile kernel with HIP events (spgemm_info)    */
};

typedef struct spgemm_model spgemm_model;   /* learned row-size network (host object) */

/* Launch and tier parameters.  Zero fields take the library defaults; the
 * autotuner fills them for a workload family.  table_slots = -1 turns the
 * wave hash tier off (every row that is not merged goes to the workgroup
 * tier); merge_max_nnz = -1 turns the register-merge tier off; spill_ratio
 * = -1 sends every row that a learned one pass has no room for to the exact
 * path. */
typedef struct spgemm_tuning {
    int32_t table_slots;     /* largest LDS hash table of a wave: 256..4096, power of two   */
    int32_t stage_slots;     /* LDS staging of a wave tile (entries): 256..8192, with
                                12 * (table_slots + stage_slots) <= 147456 bytes          */
    int32_t merge_max_nnz;   /* register-merge tier: largest row (entries) it takes        */
    int32_t merge_lists;     /* register-merge tier: max stored entries of the A row (4/8) */
    float dense_ratio;       /* dense window used when column span <= ratio * capacity     */
    float margin;            /* learned sizing: capacity = pred * (1 + margin) + slack     */
    int32_t slack;
    int32_t blocks_per_cu;   /* workgroups per compute unit of the workgroup-tier kernel   */
    float spill_ratio;       /* learned one pass: spill arena = ratio * summed capacities
                                (at least 4096 entries), 0 < ratio <= 4; -1: no arena      */
    int32_t bitmap_cols;     /* workgroup tier: when B has at most this many columns
                                (<= 1,048,576), its rows keep a bitmap of their column
                                region in LDS (Section IV-B's dense row, one bit per
                                column) instead of a device table.  Opt-in (0 or -1:
                                device tables, the default): this path is disabled
                                pending a fault found in its first GPU run               */
    int32_t split_merge;     /* two-pass path: register-merge rows by the row-per-thread
                                kernel and hashed rows by tiles without the merge lists,
                                two launches each at its own occupancy (default); -1: one
                                tile kernel for both                                      */
} spgemm_tuning;

typedef struct spgemm_options {
    int32_t sizer;                    /* spgemm_sizer                                   */
    int32_t flags;                    /* SPGEMM_OPT_*                                   */
    const spgemm_model *model;        /* required for SPGEMM_SIZER_LEARNED              */
    const spgemm_tuning *tuning;      /* NULL: defaults                                 */
} spgemm_options;

/* Host-visible facts about a plan, filled by spgemm_plan. */
typedef struct spgemm_info {
    int64_t multiplications;   /* Section III count, sum over rows of the per-row bound
                                  (-1 until spgemm_symbolic for an EXACT plan whose rows
                                  all take the register merge: that pass counts them)   */
    int64_t c_capacity_hint;   /* entries to allocate for C: sum of per-row bounds
                                  (EXACT, UPPER_BOUND) or of learned capacities (LEARNED);
                                  -1 for an EXACT plan whose rows all take the register
                                  merge (the exact size comes from spgemm_symbolic)     */
    int64_t c_nnz;             /* exact nnz(C) once known (after symbolic or numeric), else -1 */
    size_t scratch_bytes;      /* scratch the numeric (and symbolic) call needs            */
    int64_t rows_merge, rows_hash, rows_global, rows_empty;  /* tier histogram          */
    int64_t overflow_rows;     /* one pass: rows computed again with their exact size
                                  (their wave tile had no room for them, the tile's rows
                                  sharing the sum of their capacities, and the spill arena
                                  was full)                                                */
    int64_t spilled_rows;      /* one pass: rows placed in the spill arena (a quarter of
                                  the summed capacities, LEARNED only) instead             */
    int64_t tiles;             /* wave tiles of the current pass                           */
    double tile_ms;            /* SPGEMM_OPT_TIMING: duration of the last pass's row kernels
                                  (wave tiles and workgroup-tier rows, one event pair)      */
    double tile_ms_total;      /* SPGEMM_OPT_TIMING: sum over the plan's passes            */
} spgemm_info;

typedef struct spgemm_plan spgemm_plan;

/* Device workspace needed by spgemm_plan for these operands (dims only). */
spgemm_status spgemm_plan_workspace_size(const spgemm_csr *A, const spgemm_csr *B,
                                         const spgemm_options *opts, size_t *bytes);

/* Validates descriptors, computes per-row features (entries of the A row,
 * multiplication count, longest selected B row, column span), runs the
 * learned sizer when asked, assigns tiers and tiles, and returns the sizes
 * the caller must provide.  `workspace` must stay alive and untouched until
 * the plan is destroyed.  Synchronises `stream`.  The plan keeps copies of
 * the descriptors (not of the data): A and B must not change until the plan
 * is destroyed. */
spgemm_status spgemm_plan_create(const spgemm_csr *A, const spgemm_csr *B,
                                 const spgemm_options *opts,
                                 void *workspace, size_t workspace_bytes,
                                 void *stream, spgemm_plan **out, spgemm_info *info);

/* Symbolic pass (SPGEMM_SIZER_EXACT only): exact entries per row of C and
 * their exclusive scan, written to c_row_ptr (device, rows + 1).  *c_nnz
 * (host) receives nnz(C).  Row r of C holds one entry per distinct column
 * among the selected rows of B (Section IV-A, the row-major algorithm: the
 * entries the dense temporary row receives); the scan gives the row
 * offsets of the output block that Section IV-B's append/finalize contract
 * fills in row order.  scratch: device, spgemm_info.scratch_bytes,
 * 256-byte aligned (SPGEMM_E_WORKSPACE otherwise).  Errors: SPGEMM_E_NULL,
 * SPGEMM_E_STATE (not an EXACT plan, or called twice), SPGEMM_E_HIP.
 * Synchronises `stream`. */
spgemm_status spgemm_symbolic(spgemm_plan *plan, void *scratch, size_t scratch_bytes,
                              int64_t *c_row_ptr, int64_t *c_nnz, void *stream);

/* Numeric pass: writes C, each entry accumulated from +0.0 by one FP64
 * multiply and one FP64 add per product in A's column order (Section IV-A,
 * the listing of the row-major kernel), each row's columns ascending
 * (Section IV-B, append/finalize).  For SPGEMM_SIZER_EXACT, c_row_ptr must hold the
 * result of spgemm_symbolic.  For the one-pass sizers it is written here:
 * the rows are computed into a padded buffer in `scratch` (laid out by the
 * capacities), counted, scanned into c_row_ptr and moved into C; when every
 * row of A has few enough entries to be merged in registers, the rows are
 * counted, scanned and merged straight into C instead (no scratch), all on
 * the device within this call.
 * c_col / c_val (device) have room for c_capacity entries.  If C needs more,
 * nothing past c_capacity is written, the call returns SPGEMM_E_CAPACITY and
 * *c_nnz holds the required size (call again with a larger C).  a_val and
 * b_val may be NULL to use the values in the plan's descriptors.
 * Synchronises `stream`. */
spgemm_status spgemm_numeric(spgemm_plan *plan, void *scratch, size_t scratch_bytes,
                             const double *a_val, const double *b_val,
                             int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                             int64_t c_capacity, int64_t *c_nnz, void *stream);

/* spgemm_numeric without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The scratch the numeric pass
 * needs (the workgroup-tier device tables; for the one-pass sizers also the
 * padded buffer and the spill arena) is taken from a static device array
 * of spgemm_numeric_static_limit() bytes (64 MiB) that the library holds
 * on every device it runs on until the process ends; its address is looked
 * up once per device on the first call there.  The call allocates nothing
 * and otherwise behaves as spgemm_numeric (same arguments, outputs and
 * errors).  Extra errors: SPGEMM_E_WORKSPACE when the padded buffer plus one
 * device table exceed the limit (when several tables do not fit, fewer
 * workgroup-tier workgroups run), SPGEMM_E_STATE when the current device is
 * not the one the plan was created on.  Every call on one device uses the
 * same array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  The counters are
 * read back into host stack memory.  Synchronises `stream`. */
spgemm_status spgemm_numeric_static(spgemm_plan *plan, const double *a_val, const double *b_val,
                                    int64_t *c_row_ptr, int32_t *c_col, double *c_val,
                                    int64_t c_capacity, int64_t *c_nnz, void *stream);
size_t spgemm_numeric_static_limit(void);

/* The pure computation kernel (Section IV-A), as a diagnostic beside the
 * complete product (Section IV-B measures storing as the difference): every
 * row of C is accumulated exactly as spgemm_numeric does (same order, same
 * rounding), but nothing of C is stored.  For each row r only its number of
 * entries (row_nnz[r], device int32, rows) and the largest magnitude of its
 * values (row_maxabs[r], device FP64, rows; 0 for an empty row) are written,
 * so the work cannot be skipped and can be checked.  Any sizer's plan;
 * products whose rows all take the register merge only (every row of A with
 * at most 16 entries and short outputs: the paper's five-point, nine-point
 * and random five-per-row test cases), SPGEMM_E_INVALID otherwise.  a_val
 * and b_val may be NULL (the descriptors' values).  Synchronises `stream`;
 * with SPGEMM_OPT_TIMING the kernel's time is in spgemm_info.tile_ms. */
spgemm_status spgemm_compute_only(spgemm_plan *plan, const double *a_val, const double *b_val,
                                  int32_t *row_nnz, double *row_maxabs, void *stream);

spgemm_status spgemm_plan_info(const spgemm_plan *plan, spgemm_info *info);
int spgemm_plan_last_hip_error(const spgemm_plan *plan);
void spgemm_plan_destroy(spgemm_plan *plan);
const char *spgemm_status_string(spgemm_status s);

/* ---------------------------------------------------------------- batched
 * Many independent products C_i = A_i * B_i (each as in spgemm_plan_create:
 * Section IV-A's C = A * B row by row) computed together: the instances are
 * laid side by side in one row space (A_i's columns shifted past the B rows
 * of the instances before it, the B_i stacked), so one plan and one
 * persistent numeric launch cover every row of every instance, and C comes
 * out as the concatenation of the C_i.  Not part of the paper.
 *
 * spgemm_batched_plan: A, B are host arrays of `count` descriptors (device
 * data; the data must stay unchanged in structure until the batch is
 * destroyed, values may change between runs).  Writes c_row_base (host,
 * count + 1): product i's row pointers go to c_row_pool[c_row_base[i] ..
 * c_row_base[i] + rows_i] (rows_i + 1 entries, relative to the product's
 * first entry).  *workspace_bytes: device workspace the batch needs.  Reads
 * descriptors only, no device work.  Errors: SPGEMM_E_DIM (A_i.cols !=
 * B_i.rows), SPGEMM_E_INDEX_OVERFLOW (total rows of A or B >= 2^31),
 * SPGEMM_E_NO_MODEL, SPGEMM_E_INVALID. */
typedef struct spgemm_batch spgemm_batch;

spgemm_status spgemm_batched_plan(int64_t count, const spgemm_csr *A, const spgemm_csr *B,
                                  const spgemm_options *opts,
                                  int64_t *c_row_base, size_t *workspace_bytes,
                                  spgemm_batch **out);

/* Binds the workspace (kept until destroy or the next reserve), builds the
 * concatenated operands in it, and plans them (features, learned or bound
 * sizing, tiers, tiles).  *c_capacity (host): entries the pools must hold
 * (sum of multiplication counts for EXACT and UPPER_BOUND, of learned
 * capacities for LEARNED; for EXACT when every row takes the register merge,
 * the exact total, from the symbolic pass run here); *scratch_bytes (host):
 * device scratch the runs need.  Synchronises `stream`. */
spgemm_status spgemm_batched_reserve(spgemm_batch *batch, void *workspace, size_t workspace_bytes,
                                     int64_t *c_capacity, size_t *scratch_bytes, void *stream);

/* Runs every product.  Entries of product i are written at c_col_pool /
 * c_val_pool[c_nnz_base[i] .. c_nnz_base[i] + c_nnz[i]) (c_nnz_base: host,
 * count + 1, c_nnz_base[count] = total; c_nnz: host, count).  The first run
 * (and any run with other pointers) takes the checked path and captures its
 * launches in a HIP graph; later runs with the same pointers replay it.
 * If the pools are too small: SPGEMM_E_CAPACITY with the total needed in
 * *c_required (may be NULL).  Synchronises `stream`. */
spgemm_status spgemm_batched(spgemm_batch *batch, void *scratch, size_t scratch_bytes,
                             int64_t *c_row_pool, int32_t *c_col_pool, double *c_val_pool,
                             int64_t c_capacity, int64_t *c_nnz_base, int64_t *c_nnz,
                             int64_t *c_required, void *stream);

/* 1 when the next spgemm_batched call with the same pointers replays a
 * captured graph. */
int spgemm_batched_uses_graph(const spgemm_batch *batch);
void spgemm_batched_destroy(spgemm_batch *batch);

/* ------------------------------------------------------ operand by columns
 * Section IV-A takes a right-hand operand stored by columns (CSC) by
 * converting it to rows first.  The arrays of a CSC matrix (column
 * pointers, row indices, values) are those of the CSR of its transpose, so
 * the conversion is a transpose: pass the CSC arrays of B as the CSR of B^T
 * (rows = B.cols, cols = B.rows) and get B in CSR.
 *
 * spgemm_transpose writes the CSR of M^T (M->cols rows, M->rows columns):
 * t_row_ptr (device, M->cols + 1 int64), t_col and t_val (device, M->nnz
 * each; t_val may be NULL, then no values are moved and M->val may be
 * NULL).  M must be canonical (see spgemm_csr); the columns of every row of
 * the transpose then come out strictly increasing.  scratch: device,
 * spgemm_transpose_scratch(M) bytes, 256-byte aligned.  Errors:
 * SPGEMM_E_NULL, SPGEMM_E_DIM (negative sizes, or row_ptr[rows] != nnz),
 * SPGEMM_E_INDEX_OVERFLOW (rows or cols >= 2^31), SPGEMM_E_WORKSPACE,
 * SPGEMM_E_NOT_CANONICAL (a column index outside [0, cols): such entries
 * are skipped and the output is not the transpose), SPGEMM_E_HIP,
 * SPGEMM_E_STATE.  Synchronises `stream`. */
size_t spgemm_transpose_scratch(const spgemm_csr *M);
spgemm_status spgemm_transpose(const spgemm_csr *M, int64_t *t_row_ptr, int32_t *t_col, double *t_val,
                               void *scratch, size_t scratch_bytes, void *stream);

/* ------------------------------------------------------------- learned sizer
 * A 3-32-32-1 perceptron (ReLU, logistic output, FP32, 1217 parameters)
 * mapping per-row features (entries of the A row, multiplication count,
 * longest selected B row; each as standardised log2(1 + x)) to the fraction
 * of the interval [longest B row, multiplication count] that nnz(C_row)
 * reaches.  Not part of the paper. */

/* Model from host arrays: theta[1217] (W1 32x3, b1, W2 32x32, b2, w3, b3),
 * mu[3], sd[3].  SPGEMM_E_INVALID when a parameter is not finite or an sd
 * is not positive (spgemm_model_load and spgemm_model_train report such a
 * model the same way).  A finite model whose prediction still overflows to
 * a NaN sizes that row by its multiplication count. */
spgemm_status spgemm_model_create(const float *theta, const float *mu, const float *sd,
                                  spgemm_model **out);
spgemm_status spgemm_model_get(const spgemm_model *m, float *theta, float *mu, float *sd);
spgemm_status spgemm_model_save(const spgemm_model *m, const char *path);
spgemm_status spgemm_model_load(const char *path, spgemm_model **out);
void spgemm_model_destroy(spgemm_model *m);

/* Features of every row of A*B on the device (int32, rows each): entries of
 * the A row, multiplication count (saturated at B.cols), longest selected B
 * row.  Used to build training sets.  Synchronises nothing. */
spgemm_status spgemm_row_features(const spgemm_csr *A, const spgemm_csr *B,
                                  int32_t *f_nnz_a, int32_t *f_ub, int32_t *f_maxb, void *stream);

/* Device parameter block of a model (theta, mu, sd as float32) and its
 * upload; used by spgemm_model_predict.  The upload synchronises `stream`. */
size_t spgemm_model_device_bytes(void);
spgemm_status spgemm_model_upload(const spgemm_model *m, void *dev_params, void *stream);

/* Training-set statistics: mu/sd (host, 3 each) of log2(1 + feature) over n
 * rows of device features.  scratch: device, spgemm_model_stats_scratch(n)
 * bytes.  Synchronises `stream`. */
size_t spgemm_model_stats_scratch(int64_t n);
spgemm_status spgemm_model_feature_stats(const int32_t *f_nnz_a, const int32_t *f_ub,
                                         const int32_t *f_maxb, int64_t n,
                                         float *mu, float *sd, void *scratch, void *stream);

/* Loss and gradient (device, float[1217]) of the network over n device
 * samples (features and exact row sizes).  scratch: device,
 * spgemm_model_grad_scratch(n) bytes.  *loss (host) is the mean squared
 * error over rows with UB > longest B row.  Synchronises `stream`. */
size_t spgemm_model_grad_scratch(int64_t n);
spgemm_status spgemm_model_loss_grad(const spgemm_model *m,
                                     const int32_t *f_nnz_a, const int32_t *f_ub,
                                     const int32_t *f_maxb, const int32_t *nnz_c, int64_t n,
                                     float *grad, void *scratch, float *loss, void *stream);

/* Mini-batch Adam training on the device (forward, backward and update
 * kernels of this library).  Batches are taken in order, batch_size rows
 * each, for `epochs` passes.  theta0, mu, sd (host) are the starting point
 * and the input standardisation; the trained model is returned in *out.
 * scratch: device, spgemm_model_train_scratch bytes.  loss_curve (host,
 * epochs) receives the loss of each epoch's last batch and may be NULL. */
typedef struct spgemm_train_params {
    int32_t epochs;
    int32_t batch_size;
    float lr, beta1, beta2, eps;
} spgemm_train_params;

size_t spgemm_model_train_scratch(int64_t n, int32_t batch_size);
spgemm_status spgemm_model_train(const float *theta0, const float *mu, const float *sd,
                                 const int32_t *f_nnz_a, const int32_t *f_ub,
                                 const int32_t *f_maxb, const int32_t *nnz_c, int64_t n,
                                 const spgemm_train_params *hp, void *scratch, size_t scratch_bytes,
                                 float *loss_curve, spgemm_model **out, void *stream);

/* Predicted nnz(C_row) (device float, n rows) from device features.
 * dev_params: device, spgemm_model_device_bytes() bytes, overwritten with
 * the model's parameters. */
spgemm_status spgemm_model_predict(const spgemm_model *m, const int32_t *f_nnz_a,
                                   const int32_t *f_ub, const int32_t *f_maxb, int64_t n,
                                   float *pred, void *dev_params, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPGEMM_H */
