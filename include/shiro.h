/*
 * shiro.h - C ABI of the per-rank, column-based (sparsity-aware) SpMM path.
 *
 * One rank p of P owns row panel A^(p,:) of a CSR matrix A (n_rows x n_cols)
 * in a 1D row partition.  Its work, on one GPU:
 *   1. partition    - take the panel and its column blocks A^(p,q)
 *                     (Sec. 2.2; Table 1: M rows per panel, K columns per block);
 *   2. select_rows  - Cols(A^(p,q)) for every q: the ascending unique column ids
 *                     of each block, compacted by prefix sum (Table 1; Sec. 3.1,
 *                     column-based scheme; Sec. 5.1 stage 1);
 *   3. pack_B       - gather exactly those rows of B into one contiguous buffer,
 *                     the payload of volume |Cols| * N * sz (Sec. 3.1 Eq. V_col;
 *                     Sec. 5.1 stage 3);
 *   4. spmm         - Y = A^(p,:) B over the packed rows, all blocks summed into
 *                     the panel's rows (Sec. 2.1; Sec. 2.2 stages 3-4; Sec. 5.1
 *                     stage 5);
 *   5. spmm_backward- gradients of a loss through step 4: dB = A^T dY and
 *                     dvals = (dY B^T) sampled at the nonzeros (the paper's GNN
 *                     training, Sec. 7.6, needs them; it does not describe them).
 *
 * Conventions shared by every call
 *  - Every call returns an int status: SHIRO_OK (0) or a negative SHIRO_ERR_*.
 *    Nothing throws across this boundary.  shiro_last_error() returns a
 *    thread-local text for the last failure of the calling thread.
 *  - d_* arguments are device pointers owned by the caller (for example
 *    allocated through PyTorch).  h_* arguments are host pointers.  The plan
 *    object and the arrays inside it are owned by the library and released by
 *    shiro_plan_destroy().
 *  - stream is a hipStream_t (NULL = the legacy default stream).  All device
 *    work is ordered on it.  Only shiro_partition, shiro_select_rows,
 *    shiro_prepare and shiro_autotune synchronise the stream or allocate; the
 *    per-call steps (pack_B, spmm, spmm_backward) neither allocate nor
 *    synchronise once shiro_prepare has run for their (N, dtype), so they can be
 *    captured into a HIP graph.
 *  - Matrices are row-major with a leading dimension (elements between rows):
 *    B is n_cols x N (ldb >= N), Bpacked is U x N, Y and dY are M x N, dB is
 *    n_cols x N.  Leading dimensions and base pointers that are multiples of
 *    16 bytes take the vector path; other values take a scalar path.
 *  - Sizes: n_rows, n_cols < 2^31; panel nonzeros < 2^31; all row * N address
 *    arithmetic is 64-bit.
 *  - The CSR is canonical: row_ptr non-decreasing from 0 to nnz, columns in
 *    [0, n_cols), strictly ascending inside each row.  It is verified on the
 *    device when SHIRO_CHECK_CSR is passed or the environment variable
 *    SHIRO_CHECK=1 is set (SHIRO_ERR_BAD_CSR on violation).  Without the check
 *    a malformed CSR gives unspecified results and may read out of bounds, so
 *    callers with untrusted input should pass the flag.
 *  - Determinism: every output is bitwise reproducible from run to run for a
 *    fixed plan and tuning; the default paths use no floating-point atomics.
 *  - A plan holds work buffers shared by its calls: calls on one plan must be
 *    ordered (one stream, or explicit events); concurrent calls on one plan
 *    race.  Different plans are independent.
 */
#ifndef SHIRO_H
#define SHIRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SHIRO_API __attribute__((visibility("default")))
#else
#define SHIRO_API
#endif

/* hipStream_t without requiring the HIP headers. */
typedef struct ihipStream_t* shiro_stream_t;

/* Opaque per-rank plan: the panel's pattern, its selection and derived
 * structures (work lists, transposed pattern, tuning).  Pattern-only: values
 * are passed to each compute call, so a plan is reused while the sparsity
 * pattern is unchanged (the paper reuses its offline analysis the same way,
 * Sec. 5.1 and Sec. 5.3). */
typedef struct shiro_plan_s* shiro_plan;

/* Caller-supplied device allocator (e.g. a framework's caching allocator).
 * alloc returns device memory of at least `bytes` bytes, aligned to 256
 * bytes, on the current device, or NULL; free receives the pointer and the
 * size it was allocated with. */
typedef void* (*shiro_alloc_fn)(size_t bytes, void* ctx);
typedef void (*shiro_free_fn)(void* ptr, size_t bytes, void* ctx);

typedef enum {
  SHIRO_F32 = 0,  /* IEEE binary32 */
  SHIRO_BF16 = 1  /* bfloat16 storage; arithmetic is float32, stores round to nearest even */
} shiro_dtype;

enum {
  SHIRO_OK = 0,
  SHIRO_ERR_INVALID_ARG = -1,   /* null pointer, bad size, p outside [0,P), ... */
  SHIRO_ERR_BAD_CSR = -2,       /* CSR check failed (check mode only)           */
  SHIRO_ERR_OOM = -3,           /* device allocation failed                     */
  SHIRO_ERR_HIP = -4,           /* a HIP runtime call failed                    */
  SHIRO_ERR_UNSUPPORTED = -5,   /* dtype pair or size outside what is built     */
  SHIRO_ERR_NOT_READY = -6,     /* call out of order (e.g. pack before select)  */
  SHIRO_ERR_CAPTURING = -7,     /* would allocate/synchronise during capture    */
  SHIRO_ERR_WORKSPACE = -8      /* fixed work area of an allocation-free call too small */
};

/* shiro_partition flags */
#define SHIRO_CHECK_CSR 1u

/* shiro_spmm modes */
#define SHIRO_MODE_BATCHED 0u   /* all column blocks in one persistent launch, row-merged */
#define SHIRO_MODE_PER_BLOCK 1u /* one launch per column block, summed in block order     */

/* shiro_aggregate_c flags */
#define SHIRO_AGG_ACCUMULATE 1u /* add the sums into Y instead of overwriting Y */

/* shiro_spmm_backward flags */
#define SHIRO_DB_OVERWRITE 1u /* dB rows at unique_cols are overwritten instead of added to */

/* shiro_prepare / shiro_autotune operation mask */
#define SHIRO_OP_SPMM 1u
#define SHIRO_OP_BACKWARD 2u
#define SHIRO_OP_PER_BLOCK 4u
#define SHIRO_OP_ROW_BASED 8u

typedef struct {
  int64_t n_rows, n_cols; /* global matrix shape                              */
  int32_t P, p;           /* partition and this rank                          */
  int64_t M, K;           /* ceil(n_rows/P) rows per panel, ceil(n_cols/P) cols per block */
  int64_t row_begin;      /* first global row of the panel                    */
  int64_t rows;           /* rows in this panel (M, or fewer for the last)    */
  int64_t nz_begin;       /* index of the panel's first nonzero in the CSR    */
  int64_t nnz;            /* nonzeros in the panel                            */
  int64_t U;              /* sum_q |Cols(A^(p,q))|, -1 before select_rows     */
} shiro_plan_info_t;

/* Tuning knobs of one kernel family (spmm, transposed spmm, sddmm, or the
 * row-based scheme's partial rows and sum). */
typedef struct {
  int32_t chunk;     /* merge-path items (rows + nonzeros) per wavefront       */
  int32_t lanes;     /* lanes sharing one dense row: 8, 16, 32 or 64 (tile width = lanes * 16 bytes) */
  int32_t unroll;    /* nonzeros in flight per lane group: 1, 2 or 4           */
  int32_t group_rows; /* 0: a wavefront per row; 1: each lane group of a
                       * wavefront owns its own rows; 2: each lane group walks
                       * its own chunks nonzero by nonzero across row ends;
                       * 3: the same walk with its index, row and value streams
                       * loaded a window of `lanes` nonzeros at a time (2 and 3
                       * not for the sampled product, SHIRO_KERNEL_SDDMM)      */
  int32_t xcd_remap; /* 1: give each XCD a contiguous range of work            */
  int32_t wg_per_cu; /* persistent grid: workgroups per compute unit           */
  int32_t lds_rows;  /* windowed walk (group_rows 3) of SHIRO_KERNEL_SPMM and
                      * SHIRO_KERNEL_SPMM_T only: the lds_rows most referenced
                      * rows of the gathered operand (Bpacked, resp. dY) are
                      * copied into each workgroup's LDS and read from there;
                      * 0 = off, at most 128 and 64 KB per workgroup          */
} shiro_tuning_t;

#define SHIRO_KERNEL_SPMM 0
#define SHIRO_KERNEL_SPMM_T 1
#define SHIRO_KERNEL_SDDMM 2
#define SHIRO_KERNEL_PARTIAL_C 3   /* row-based scheme: the owner's partial rows */
#define SHIRO_KERNEL_AGGREGATE_C 4 /* row-based scheme: their sum into the panel */

/* Library version, 10000*major + 100*minor + patch. */
SHIRO_API int shiro_version(void);

/* Hash of the sources this library was built from (16 hex digits of the
 * sha256 of every HIP source and header and of this header), so that a
 * caller can tell a library built from other sources.  Static string. */
SHIRO_API const char* shiro_build_hash(void);

/* Text of the calling thread's last error ("" if none).  Valid until the
 * thread's next failing call. */
SHIRO_API const char* shiro_last_error(void);

/* Build the plan of rank p (Sec. 2.2; Table 1).
 *   n_rows, n_cols: shape of A; nnz = d_row_ptr[n_rows].
 *   d_row_ptr: device int64[n_rows + 1]; d_col: device int32[nnz].  Only the
 *     panel's rows [p*M, min(n_rows,(p+1)*M)) and their nonzeros are read; the
 *     plan copies what it needs, so the caller may free them afterwards.
 *   P >= 1 processes, 0 <= p < P.  Panels and column blocks are contiguous,
 *     M = ceil(n_rows/P) rows and K = ceil(n_cols/P) columns; the last ones
 *     may be shorter (or empty).
 *   flags: SHIRO_CHECK_CSR validates the panel on the device first.
 * Synchronises the stream (reads the panel's nonzero range).  Errors:
 * INVALID_ARG, BAD_CSR, OOM, HIP, UNSUPPORTED (panel nnz >= 2^31). */
SHIRO_API int shiro_partition(int64_t n_rows, int64_t n_cols, int64_t nnz,
                              const int64_t* d_row_ptr, const int32_t* d_col, int32_t P,
                              int32_t p, uint32_t flags, shiro_stream_t stream,
                              shiro_plan* out_plan);

/* A plan over part of the panel's nonzeros: those k of panel p (counted
 * from the panel's first nonzero) with d_keep[k] == keep_value, in CSR
 * order, with the global shape, P and p of shiro_partition.  The joint
 * strategy (Sec. 5.1 step 2) splits each block into a row-based and a
 * column-based part; each part is a subset plan.  Compute calls take the
 * caller's whole value array (indexed like d_col, as for a full plan) and
 * read it through the subset's map; dvals of spmm_backward are written for
 * the subset's nonzeros only.  d_keep: device, one byte per panel nonzero.
 * The per-block spmm mode is not available on subset plans (UNSUPPORTED).
 * Other arguments and errors as shiro_partition. */
SHIRO_API int shiro_partition_subset(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                     const int64_t* d_row_ptr, const int32_t* d_col,
                                     const uint8_t* d_keep, uint8_t keep_value, int32_t P,
                                     int32_t p, uint32_t flags, shiro_stream_t stream,
                                     shiro_plan* out_plan);

SHIRO_API int shiro_plan_info(shiro_plan plan, shiro_plan_info_t* h_info);

/* Nonzeros of the panel in each column block, written to device int64[P]. */
SHIRO_API int shiro_block_nnz(shiro_plan plan, int64_t* d_block_nnz, shiro_stream_t stream);

/* Cols(A^(p,q)) for every block q (Table 1; Sec. 3.1; Sec. 5.1 stage 1).
 * Marks the column ids present in the panel, prefix-sums the marks and
 * compacts them, so that the plan holds
 *   unique_cols int32[U]: Cols_0, Cols_1, ... each ascending (global ids);
 *   block_off  int64[P+1]: block q's ids are unique_cols[block_off[q] ..
 *              block_off[q+1]);
 *   colmap     int32[nnz]: packed position of each panel nonzero's column,
 *              so unique_cols[colmap[k]] == col[k].
 * Writes U to *h_U_total and |Cols_q| to h_U_per_block[q] (nullable, P
 * entries).  Synchronises the stream to return U.  Idempotent. */
SHIRO_API int shiro_select_rows(shiro_plan plan, shiro_stream_t stream, int64_t* h_U_total,
                                int64_t* h_U_per_block);

/* Re-run the selection kernels of select_rows into the plan's arrays without
 * synchronising or allocating (the pattern is the plan's own copy, so the
 * result and U are unchanged).  Stream-ordered and capturable; lets a caller
 * time or graph-capture the whole path including the selection step.
 * NOT_READY before the first select_rows. */
SHIRO_API int shiro_refresh_selection(shiro_plan plan, shiro_stream_t stream);

/* Device views of the selection (owned by the plan; valid until destroy).
 * Any output pointer may be NULL.  NOT_READY before select_rows. */
SHIRO_API int shiro_plan_selection(shiro_plan plan, const int32_t** d_unique_cols,
                                   const int64_t** d_block_off, const int32_t** d_colmap);

/* Copy the selection into caller-owned device buffers (any may be NULL):
 * d_unique_cols int32[U], d_block_off int64[P+1], d_colmap int32[nnz].
 * Stream-ordered.  NOT_READY before select_rows. */
SHIRO_API int shiro_copy_selection(shiro_plan plan, int32_t* d_unique_cols, int64_t* d_block_off,
                                   int32_t* d_colmap, shiro_stream_t stream);

/* Pack (Sec. 3.1 Eq. V_col; Sec. 5.1 stage 3):
 *   Bpacked[u, 0:N] = B[unique_cols[u], 0:N] for u in [0, U), a bit-exact copy.
 * d_B: n_cols x N of dtype dt with leading dimension ldb >= N; d_Bpacked:
 * U x N with ldp >= N, same dtype, must not overlap d_B.  NOT_READY before
 * select_rows. */
SHIRO_API int shiro_pack_B(shiro_plan plan, const void* d_B, int64_t ldb, int32_t N,
                           shiro_dtype dt, void* d_Bpacked, int64_t ldp,
                           shiro_stream_t stream);

/* Local SpMM with aggregation over the column blocks (Sec. 2.1; Sec. 2.2
 * stages 3-4; Sec. 5.1 stage 5):
 *   Y[i, :] = sum_q sum_{k in row i of block q} vals[k] * Bpacked[colmap[k], :]
 * for the panel's rows i in [0, rows).  Y is overwritten (empty rows get 0).
 * d_vals: float32 values indexed like d_col of shiro_partition (global nonzero
 * index; the plan offsets by nz_begin).  Products and sums are float32; the
 * sum of each output element is taken in a fixed order.
 * Supported (in_dt -> out_dt): F32->F32, BF16->F32, BF16->BF16.
 * mode: SHIRO_MODE_BATCHED (one persistent launch over all blocks) or
 * SHIRO_MODE_PER_BLOCK (one launch per block, accumulated in block order).
 * NOT_READY before select_rows; CAPTURING if capture is active and the
 * structures for (N, dtype, mode) were not prepared. */
SHIRO_API int shiro_spmm(shiro_plan plan, const float* d_vals, const void* d_Bpacked,
                         int64_t ldp, int32_t N, shiro_dtype in_dt, void* d_Y, int64_t ldy,
                         shiro_dtype out_dt, uint32_t mode, shiro_stream_t stream);

/* Backward of Y = A Bpacked for a loss with upstream gradient dY (M x N);
 * the two gradients of <dY, A B> (the adjoint of the product of Sec. 2.1):
 *   dBpacked = A^T dY                       (U x N, overwritten; nullable)
 *   dB[unique_cols[u], :] += dBpacked[u, :] (n_cols x N, read-modify-write into
 *                                            the caller's buffer; nullable)
 *     or, with flags & SHIRO_DB_OVERWRITE,
 *   dB[unique_cols[u], :]  = dBpacked[u, :] (the other rows of dB are not
 *                                            touched: a zero-filled dB then
 *                                            holds the full gradient)
 *   dvals[k] = dY[i(k), :] . Bpacked[colmap[k], :]  (float32 per nonzero,
 *                                            indexed like d_vals; nullable)
 * A^T is applied through a transposed pattern built once per plan by a stable
 * radix sort (no atomics).  dt applies to dY, Bpacked, dBpacked and dB
 * (F32 or BF16; arithmetic float32).  Unknown flag bits: INVALID_ARG.
 * NOT_READY before select_rows. */
SHIRO_API int shiro_spmm_backward(shiro_plan plan, const float* d_vals, const void* d_dY,
                                  int64_t lddy, const void* d_Bpacked, int64_t ldp, int32_t N,
                                  shiro_dtype dt, void* d_dBpacked, int64_t lddbp, void* d_dB,
                                  int64_t lddb, float* d_dvals, uint32_t flags,
                                  shiro_stream_t stream);

/* Allocation-free form of shiro_spmm in SHIRO_MODE_BATCHED, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and kernels as shiro_spmm(..., SHIRO_MODE_BATCHED, ...), bit for bit; the
 * carry slots of rows cut by chunk boundaries live in a fixed 32 MiB device
 * array of the library (one per device, held until the process ends) instead
 * of the plan's buffer.  Makes no device or host allocation and does not
 * synchronise.  The plan must have been prepared for (N, in_dt) with
 * SHIRO_OP_SPMM under the tuning in force (NOT_READY otherwise); patterns
 * whose slots (2 * N floats per merge-path chunk) exceed the array return
 * SHIRO_ERR_WORKSPACE without launching anything.  Must be called with the
 * plan's device current (INVALID_ARG otherwise).  Every call on one device
 * shares that device's array and every slot a call reads it first writes, so
 * nothing needs clearing between calls; calls that overlap in time on one
 * device (different streams, or threads) race on the array and must be
 * ordered by the caller. */
SHIRO_API int shiro_spmm_noalloc(shiro_plan plan, const float* d_vals, const void* d_Bpacked,
                                 int64_t ldp, int32_t N, shiro_dtype in_dt, void* d_Y, int64_t ldy,
                                 shiro_dtype out_dt, shiro_stream_t stream);

/* ---- Row-based scheme (Table 1 Rows; Sec. 3.1 row-based scheme, Eq. V_row;
 * Sec. 5.1 stage 3 remote computation, stage 5 aggregation) -------------
 * Rows(A^(p,q)) is the set of panel rows with a nonzero in column block q.
 * The owner q of B^(q,:) computes the partial rows
 *   Cp[e, :] = sum_{k in row Rows_q[t] of block q} vals[k] * B[col[k], :]
 * for entry e = rblock_off[q] + t, and the receiver sums them into its rows
 *   Y[i, :] = sum over blocks q (ascending) of the entry of row i in block q.
 * On one GPU both sides run on the same device, with B given in full.
 *
 * shiro_select_c_rows builds the row-based structures (setup: allocates and
 * synchronises) and returns R = sum_q |Rows(A^(p,q))| in *h_R and, when
 * h_R_per_block is not NULL, |Rows(A^(p,q))| for q = 0..P-1. */
SHIRO_API int shiro_select_c_rows(shiro_plan plan, shiro_stream_t stream, int64_t* h_R,
                                  int64_t* h_R_per_block);

/* Copy Rows_0, Rows_1, ... (panel-local row ids, ascending within a block;
 * d_rows int32[R]) and rblock_off (d_rblock_off int64[P+1]) into
 * caller-owned device buffers (either may be NULL).  NOT_READY before
 * shiro_select_c_rows. */
SHIRO_API int shiro_copy_c_row_selection(shiro_plan plan, int32_t* d_rows, int64_t* d_rblock_off,
                                         shiro_stream_t stream);

/* The owner's partial rows: d_Cp (R x N, leading dimension ldc, out_dt)
 * overwritten from d_B (n_cols x N, ldb, in_dt; global rows) and d_vals
 * (float32, indexed like shiro_partition's d_col).  Float32 arithmetic, each
 * entry rounded once.  Pairs: F32->F32, BF16->F32, BF16->BF16.  NOT_READY
 * before shiro_select_c_rows; CAPTURING if capture is active and the
 * structures for (N, dtype) were not prepared (SHIRO_OP_ROW_BASED). */
SHIRO_API int shiro_partial_c(shiro_plan plan, const float* d_vals, const void* d_B, int64_t ldb,
                              int32_t N, shiro_dtype in_dt, void* d_Cp, int64_t ldc,
                              shiro_dtype out_dt, shiro_stream_t stream);

/* The receiver's sum: d_Y (rows x N, ldy, out_dt) overwritten with the sum
 * of each panel row's partial rows from d_Cp (R x N, ldc, in_dt), blocks in
 * ascending order; rows with no entry get 0.  With flags &
 * SHIRO_AGG_ACCUMULATE the sums are added to d_Y instead (rows with no
 * entry unchanged): the joint strategy adds the row-based part to the
 * column-based product.  Same pairs and errors as shiro_partial_c; unknown
 * flag bits: INVALID_ARG. */
SHIRO_API int shiro_aggregate_c(shiro_plan plan, const void* d_Cp, int64_t ldc, int32_t N,
                                shiro_dtype in_dt, void* d_Y, int64_t ldy, shiro_dtype out_dt,
                                uint32_t flags, shiro_stream_t stream);

/* ---- Joint row-column strategy (Sec. 5.2 problem; Sec. 5.3 minimum
 * weighted vertex cover by minimum s-t cut; Sec. 5.4 volumes) ------------
 * Host routines (the paper plans offline on the CPU, once per pattern).
 *
 * Minimum weighted vertex cover of a bipartite graph: left vertices are
 * rows of C (row-based sends), right vertices rows of B (column-based
 * fetches), edge e joins h_left[e] and h_right[e] (one per nonzero).
 * Costs h_w_left[n_left], h_w_right[n_right] (>= 0; NULL = all 1).  Writes
 * h_cover_left/right (1 = in the cover) and the cover's cost *h_weight.
 * Max flow by Dinic's algorithm.  Several optimal covers may exist; the one
 * returned is the source side of the minimum cut.  INVALID_ARG on bad sizes,
 * out-of-range endpoints or negative costs. */
SHIRO_API int shiro_mvc_bipartite(int64_t n_left, int64_t n_right, int64_t n_edges,
                                  const int32_t* h_left, const int32_t* h_right,
                                  const int64_t* h_w_left, const int64_t* h_w_right,
                                  uint8_t* h_cover_left, uint8_t* h_cover_right,
                                  int64_t* h_weight);

/* Joint plan of the panel: the cover above for every off-diagonal block
 * A^(p,q) (the diagonal block uses local B rows and is not planned), blocks
 * solved in parallel on n_threads host threads (0 = up to 16).
 * h_w_row: cost per panel row (rows entries, panel-local index), h_w_col:
 * cost per global column (n_cols entries); NULL = unit costs.
 * h_assign (nnz bytes, nullable): 1 for a nonzero computed row-based (its
 * row is in its block's cover), 0 for column-based (and for the diagonal
 * block).  h_stats (5*P int64, nullable): per block q, cover cost mu_q,
 * |Rows(A^(p,q))|, |Cols(A^(p,q))|, rows in the cover, columns in the cover
 * (mu and the cover counts are 0 for the diagonal block).  Copies the
 * pattern to the host and synchronises the stream. */
SHIRO_API int shiro_joint_plan(shiro_plan plan, const int64_t* h_w_row, const int64_t* h_w_col,
                               uint8_t* h_assign, int64_t* h_stats, int32_t n_threads,
                               shiro_stream_t stream);

/* Build everything the per-call steps need for (N, dtype, ops) - work lists
 * for the tuning in force, transposed pattern, per-nonzero row ids of the
 * nonzero walk, row-based structures, carry buffers - so later calls
 * neither allocate nor synchronise (required before graph capture; a tuning
 * set afterwards with another chunk needs another prepare).  Ops
 * other than SHIRO_OP_ROW_BASED need shiro_select_rows first (NOT_READY).
 * Synchronises the stream. */
SHIRO_API int shiro_prepare(shiro_plan plan, int32_t N, shiro_dtype dt, uint32_t ops,
                            shiro_stream_t stream);

/* Time candidate tunings of the kernels in `ops` on scratch data of the
 * plan's shape at width N and keep the fastest per kernel in the plan (the
 * median of nine runs ranks each candidate).  The backward is tuned in the
 * form autograd uses (dB rows overwritten, plus dvals), on a scratch dB of
 * n_cols x N; SHIRO_OP_ROW_BASED tunes the row-based partial rows (on a
 * scratch B of n_cols x N) and their sum.  If the environment variable
 * SHIRO_TUNE_CACHE names a file,
 * results are read from it (no timing for keys it holds) and new results are
 * appended (one line per key).  Allocates and synchronises. */
SHIRO_API int shiro_autotune(shiro_plan plan, int32_t N, shiro_dtype dt, uint32_t ops,
                             shiro_stream_t stream);

/* Read or override the tuning the plan uses for one kernel family
 * (SHIRO_KERNEL_*) at width N.  set validates the knobs (INVALID_ARG). */
SHIRO_API int shiro_get_tuning(shiro_plan plan, int32_t kernel, int32_t N, shiro_dtype dt,
                               shiro_tuning_t* h_tuning);
SHIRO_API int shiro_set_tuning(shiro_plan plan, int32_t kernel, int32_t N, shiro_dtype dt,
                               const shiro_tuning_t* h_tuning);

/* HIP graph capture of any sequence of pack_B / spmm / spmm_backward calls on
 * `stream`: begin, issue the calls, end; the instantiated graph is kept in the
 * plan under *h_graph_id and replayed by shiro_graph_launch.  Pointers and
 * sizes are frozen at capture.  Run shiro_prepare first. */
SHIRO_API int shiro_graph_begin(shiro_plan plan, shiro_stream_t stream);
SHIRO_API int shiro_graph_end(shiro_plan plan, shiro_stream_t stream, int32_t* h_graph_id);
SHIRO_API int shiro_graph_launch(shiro_plan plan, int32_t graph_id, shiro_stream_t stream);

/* Route the library's own device allocations (plan arrays, work lists,
 * carry and scratch buffers, autotuner buffers) through alloc/free instead
 * of hipMalloc/hipFree, so the caller's allocator owns all memory; both
 * NULL restores hipMalloc.  Process-wide; affects later allocations only
 * (each block is released through the allocator that made it).  One of the
 * two NULL: INVALID_ARG.  Allocation failures surface as OOM from the call
 * that allocates. */
SHIRO_API int shiro_set_allocator(shiro_alloc_fn alloc, shiro_free_fn free_fn, void* ctx);

/* Release the plan and everything it owns (synchronises the device first).
 * NULL is accepted. */
SHIRO_API int shiro_plan_destroy(shiro_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* SHIRO_H */
