/*
 * glu.h -- C ABI of the MI355X levelized sparse LU library.
 *
 * The library factorizes a square sparse matrix A (CSC, 0-based) as
 *     P A P^T = L U
 * with a fill-reducing symmetric permutation P chosen once by glu_analyze,
 * L unit lower triangular and U upper triangular, without numerical pivoting,
 * and solves A x = b with the factors.  This is the problem the paper states in
 * Section I (A x = b solved through A = LU and two triangular solves) with its
 * flow of Section II-C (ordering and symbolic analysis once on the host, the
 * numeric factorization on the GPU) and the opening of Section III (the numeric step is
 * repeated on a fixed pattern inside Newton iterations).
 *
 * Conventions for every entry point:
 *   - Matrices are CSC: colptr int64[n+1] (colptr[0] == 0), rowind int32[nnz]
 *     strictly increasing within each column, values float64[nnz] in the same
 *     order.  Explicit zeros are structural nonzeros.
 *   - Host arrays passed in are copied before the call returns; the library
 *     never keeps a caller pointer.  Device pointers (on_device / values_on_device
 *     = 1) must stay valid until the call returns (every call that takes them
 *     synchronizes its stream before returning).
 *   - The handle owns every allocation it makes, host and device; glu_destroy
 *     releases them.  Export buffers are allocated by the caller with the sizes
 *     glu_query reports.
 *   - Every function returns a glu_status code; no C++ exception crosses the
 *     ABI.  A failed analyze leaves the handle empty; a failed factor leaves it
 *     analyzed but not factored.
 *   - One handle must not be used by two threads at once.
 */
#ifndef GLU_H
#define GLU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GLU_OK = 0,
    GLU_ERR_ARG = -1,              /* bad pointer, size, unsorted/duplicate/out-of-range index */
    GLU_ERR_STATE = -2,            /* call out of order (e.g. solve before factor)             */
    GLU_ERR_ZERO_PIVOT = -3,       /* U(j,j) is zero or not finite; glu_failed_column gives j  */
    GLU_ERR_STRUCT_SINGULAR = -4,  /* a diagonal entry is absent from the filled pattern       */
    GLU_ERR_NOMEM = -5,            /* over max_device_bytes, or an allocation failed           */
    GLU_ERR_DEVICE = -6,           /* HIP runtime error, or no device on a host-only handle    */
    GLU_ERR_NONFINITE_INPUT = -7,  /* an input value is NaN or infinite                        */
    GLU_ERR_SCRATCH = -8           /* glu_solve_noalloc: n x nrhs too large for its scratch    */
} glu_status;

/* Fill-reducing ordering chosen by glu_analyze. */
enum { GLU_ORDER_AMD = 0, GLU_ORDER_NATURAL = 1, GLU_ORDER_USER = 2 };
/* Kernel mode forced on every level (Section III-B's three modes), or automatic. */
enum { GLU_MODE_AUTO = 0, GLU_MODE_SMALL_BLOCK = 1, GLU_MODE_LARGE_BLOCK = 2, GLU_MODE_STREAM = 3 };

/* Options; an all-zero struct (or NULL) selects every default. */
typedef struct {
    int32_t ordering;          /* GLU_ORDER_*; default AMD on the pattern of A + A^T          */
    int32_t force_mode;        /* GLU_MODE_*; default automatic choice per level             */
    int32_t stream_threshold;  /* levels with at most this many columns use stream mode
                                  (runs of them share one persistent launch); 0: default -1
                                  = no stream mode (the paper's switch point is 16)          */
    int32_t large_threshold;   /* levels with at most this many columns (and more than the
                                  stream threshold) use large-block mode (slices of 64
                                  entries); 0: default -1 = none                             */
    int64_t max_device_bytes;  /* refuse analyses whose device footprint exceeds this (0: no
                                  limit)                                                     */
    int32_t dense_tail;        /* trailing columns factorized as one dense block on the
                                  matrix cores: 0 = chosen by a cost model, -1 = never,
                                  m > 0 = exactly the last m columns                        */
    int32_t gpu_analysis;      /* 1: the relaxed dependency DAG and the levels of
                                  glu_analyze are computed on the device (same results);
                                  needs a device handle                                      */
    int32_t precision;         /* 0: FP64 factorization; 1: the mixed form -- the sparse
                                  levels in FP32 with FP32 arithmetic; a dense trailing block
                                  is updated in FP64 from the FP32 values and factorized in
                                  FP32 (the ROCm LAPACK no-pivot LU) from 8,192 columns on, in
                                  FP64 below; glu_solve refines in FP64 (residual b - A x and
                                  update) until the backward error is at most 1e-13,
                                  refactorizing in FP64 if refine_max_iters steps do not get
                                  there; stream mode is not available in this form          */
    int32_t refine_max_iters;  /* refinement steps per solve before the FP64 fallback (0: 10;
                                  -1: none, i.e. fall back unless the first solve is enough)  */
    int32_t dense_gemm;        /* bulk trailing updates of the dense block (plain GEMMs):
                                  0 = the ROCm BLAS library's DGEMM in its atomics-free,
                                  deterministic mode; 1 = this library's own FP64 MFMA
                                  kernel (every other dense step is always this library's)   */
    int32_t reserved[3];       /* must be zero                                              */
} glu_options;

/* Sizes and statistics of an analyzed (and possibly factored) handle. */
typedef struct {
    int32_t n;
    int32_t n_levels;          /* levels of the relaxed dependency DAG                        */
    int64_t nnz_a;             /* nonzeros of A                                              */
    int64_t nnz_lu;            /* nonzeros of A_s = L + U - I (diagonal counted once)         */
    int64_t nnz_l;             /* strictly lower entries                                     */
    int64_t nnz_u;             /* strictly upper entries                                     */
    int64_t n_dag_edges;       /* edges of the relaxed dependency DAG                         */
    int64_t macs;              /* multiply-adds of one numeric factorization: sum |L_j||U_j|  */
    int32_t n_levels_mode[3];  /* levels run in small-block, large-block and stream mode      */
    int32_t widest_level;
    int64_t n_tasks;           /* (level, target column) update tasks                         */
    int64_t n_work_items;      /* workgroups launched over all levels of one factorization    */
    int32_t n_solve_levels_l;  /* sparse levels of the forward (L) and backward (U) solves    */
    int32_t n_solve_levels_u;
    int32_t tail_m;            /* order of the dense trailing block (0: none)                 */
    int32_t n_exec_levels;     /* levels launched before the dense block (levels restricted
                                  to the columns before it)                                  */
    int64_t device_bytes;      /* device memory held by the handle                            */
    double t_order_ms;         /* host time of the last analyze, split by step                */
    double t_symbolic_ms;
    double t_levels_ms;        /* relaxed dependency detection + levelization                 */
    double t_plan_ms;          /* level plan, value map, solve schedule, upload               */
    double t_factor_ms;        /* device time of the last factor/refactor (events)            */
    double t_solve_ms;         /* device time of the last solve (events)                      */
    double t_update_ms;        /* device time of the level loop (normalisation + submatrix
                                  update launches) inside the last factor/refactor            */
    double t_dense_ms;         /* device time of the dense trailing block (gather, Schur-
                                  complement update, LU, scatter) and the pivot check       */
    double t_schur_ms;         /* part of t_dense_ms: gather and Schur-complement update of
                                  the dense block from the columns before it                 */
    int64_t schur_macs;        /* nonzero products of that update: sum_j |L(t:n,j)| |U(j,t:n)| */
    int64_t schur_steps;       /* (tile, source) steps of that update over 16 x 16 tiles     */
    int64_t schur_tiles;       /* nonempty tiles of that update                               */
    int64_t level_macs;        /* products applied by the sparse levels (target outside the
                                  dense block)                                                */
    int64_t tail_macs;         /* products inside the dense block (source column and target
                                  there): the method's own work of the block's LU             */
    int64_t level_nl;          /* L entries of the columns before the dense block             */
    int64_t level_nu;          /* U entries of the rows before the dense block                */
    int32_t precision;         /* 0 FP64, 1 the mixed form (FP32 factors, FP64 refinement)   */
    int32_t refine_iters;      /* refinement steps of the last solve (mixed form)            */
    int32_t fp64_fallback;     /* 1 if the last solve refactorized in FP64 (mixed form)      */
    int32_t reserved_info;
    double refine_berr;        /* backward error reached by the last solve's refinement      */
} glu_info;

typedef struct glu_handle glu_handle;

/* Create a handle bound to HIP device `device` (>= 0), or a host-only handle
 * (device = -1) that can analyze and export the symbolic results but not
 * factor.  opt may be NULL. */
int glu_create(glu_handle **out, int device, const glu_options *opt);

/* Ordering, symbolic fill, relaxed dependency DAG (Alg. 4), levelization, the
 * per-level kernel plan, then upload of the pattern and plan to the device.
 * colptr/rowind: host CSC pattern of A.  perm: host int32[n] with
 * perm[new] = old, read only when ordering == GLU_ORDER_USER (else NULL).
 * Errors: GLU_ERR_ARG (bad CSC or permutation), GLU_ERR_STRUCT_SINGULAR,
 * GLU_ERR_NOMEM, GLU_ERR_DEVICE.  Any previous analysis is discarded. */
int glu_analyze(glu_handle *h, int32_t n, const int64_t *colptr, const int32_t *rowind,
                const int32_t *perm);

/* Numeric factorization of the analyzed pattern with new values.
 * values: float64[nnz_a] in A's own CSC order (host pointer, or device pointer
 * when values_on_device = 1).  stream: a hipStream_t (NULL = the null stream).
 * Runs the value load, then the level-by-level right-looking factorization
 * (Alg. 2 with the submatrix update of Alg. 5, three kernel modes of
 * Section III-B), and synchronizes the stream to read the pivot status.
 * Part of the work runs on two streams the handle owns (forked from and
 * joined back to `stream` with events), so everything is complete when the
 * call returns.
 * Errors: GLU_ERR_STATE (not analyzed), GLU_ERR_NONFINITE_INPUT,
 * GLU_ERR_ZERO_PIVOT (glu_failed_column tells the column), GLU_ERR_DEVICE. */
int glu_factor(glu_handle *h, const double *values, int values_on_device, void *stream);

/* Same as glu_factor on the same pattern: the refactorization that the
 * opening of Section III describes, repeated inside Newton iterations with
 * new values on a fixed pattern, reusing the analysis; requires one earlier
 * successful glu_factor on this analysis.  Arguments and errors as
 * glu_factor. */
int glu_refactor(glu_handle *h, const double *values, int values_on_device, void *stream);

/* Solve A X = B for nrhs right-hand sides with the factors (the two triangular
 * solves of Section I: L y = P b, then U z = y, x = P^T z; the dense block's
 * rows by blocked substitution).  b: n x nrhs column-major with
 * leading dimension ldb >= n; x likewise with ldx; b may equal x.  Both host
 * pointers, or both device pointers when on_device = 1.  Each triangular solve
 * hands results between waves of one launch through bounded waits; a wait
 * that gives up (the device could not keep the launch resident) is reported
 * as GLU_ERR_DEVICE, never as a hang.
 * Errors: GLU_ERR_STATE (no successful factorization), GLU_ERR_ARG,
 * GLU_ERR_NOMEM, GLU_ERR_DEVICE. */
int glu_solve(glu_handle *h, int32_t nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
              int on_device, void *stream);

/* glu_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as glu_solve with on_device = 1, but every
 * scratch buffer (work vector, mailboxes, partial sums) lives in one static
 * device array of glu_solve_noalloc_capacity() doubles (64 MiB) per GPU,
 * held until the process ends; the call allocates nothing.  b and x are
 * device pointers (n x nrhs, column-major, ldb/ldx >= n; b may equal x).
 * Requires 2 ceil32(n nrhs) + ceil32(w nrhs) + ceil32(m nrhs) <= capacity
 * (w: cross-term work items of both substitutions, m: dense-block order;
 * ceil32 rounds up to 32),
 * else GLU_ERR_SCRATCH.  All calls on one GPU share the array: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialized by the caller.  Synchronizes the stream before returning.
 * Handles of the mixed form (precision = 1) are refused with GLU_ERR_ARG:
 * their refinement needs workspace of its own.
 * Errors: GLU_ERR_ARG, GLU_ERR_STATE, GLU_ERR_SCRATCH, GLU_ERR_DEVICE. */
int glu_solve_noalloc(glu_handle *h, int32_t nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
                      void *stream);

/* Capacity, in doubles, of glu_solve_noalloc's static scratch on each GPU. */
int64_t glu_solve_noalloc_capacity(void);

/* Batched factorization (many matrices of uneven size): the sparse levels of
 * several analyzed handles run together, one launch per level wavefront --
 * wavefront e holds level e of every handle that has one -- captured once
 * into a HIP graph at creation and replayed by every glu_batch_factor; the
 * rest of each factorization (dense block, pivot check) follows on a few
 * streams of the batch so that the handles' blocks overlap.  Each handle gets
 * exactly the factors glu_factor would give it with dense_gemm = 1 (same
 * kernels, same order per entry: a batch runs the dense blocks' bulk updates
 * on this library's kernel), and is solved afterwards with glu_solve or, all
 * together, with glu_batch_solve.  This is the batching of
 * the paper's motivating use, many Newton-iteration refactorizations
 * (Section III), on one device.
 * glu_batch_create: handles[count], all analyzed, distinct, on one device and
 * of one precision; they must outlive the batch, and a handle analyzed again
 * makes glu_batch_factor return GLU_ERR_STATE.  Errors: GLU_ERR_ARG,
 * GLU_ERR_STATE, GLU_ERR_NOMEM, GLU_ERR_DEVICE. */
typedef struct glu_batch glu_batch;
int glu_batch_create(glu_batch **out, glu_handle *const *handles, int32_t count);

/* Factorize every handle of the batch with its values[i] (float64[nnz_a] in
 * the handle's CSC order; host pointers, or device pointers when
 * values_on_device = 1), synchronizing the stream before returning.  Returns
 * the first failing handle's code (GLU_ERR_ZERO_PIVOT, GLU_ERR_NONFINITE_INPUT,
 * ...; that handle's glu_failed_column tells the column); the others are
 * factored. */
int glu_batch_factor(glu_batch *b, const double *const *values, int values_on_device, void *stream);

/* Solve A_i X_i = B_i for every handle i of the batch (factored by
 * glu_batch_factor or one by one), the solves running concurrently on the
 * batch's streams (forked from and joined to stream; synchronizes it before
 * returning).  bs[i], xs[i]: device pointers to column-major n_i x nrhs arrays
 * with leading dimensions ldb[i], ldx[i] >= n_i; for the mixed form xs[i] must
 * not alias bs[i].  The mixed form refines every handle as glu_solve does
 * (FP64 residual and update to backward error <= 1e-13, FP64 fallback), with
 * one host synchronisation per refinement round for the whole batch instead
 * of one per handle; glu_query gives each handle's refinement steps and
 * reached error.  Errors: GLU_ERR_ARG, GLU_ERR_STATE (a handle not factored,
 * or analyzed again), GLU_ERR_NOMEM, GLU_ERR_DEVICE. */
int glu_batch_solve(glu_batch *b, int32_t nrhs, const double *const *bs, const int64_t *ldb, double *const *xs,
                    const int64_t *ldx, void *stream);

/* Handles in the batch, level wavefronts, whether the wavefronts run as a
 * captured graph, and the device time of the last glu_batch_factor's level
 * wavefronts and of the whole call, and of the last glu_batch_solve (any
 * pointer may be NULL). */
int glu_batch_query(const glu_batch *b, int32_t *count, int32_t *n_wavefronts, int32_t *captured,
                    double *t_levels_ms, double *t_total_ms, double *t_solve_ms);

/* Release the batch (not its handles).  NULL is allowed. */
void glu_batch_destroy(glu_batch *b);

/* Sizes and timings. */
int glu_query(const glu_handle *h, glu_info *out);

/* Copy the symbolic results to caller buffers (any may be NULL):
 * perm int32[n] (perm[new] = old), lu_colptr int64[n+1], lu_rowind
 * int32[nnz_lu] (pattern of A_s for B = P A P^T), dag_ptr int64[n+1] and
 * dag_idx int32[n_dag_edges] (CSR: dag_idx[dag_ptr[k]..dag_ptr[k+1]) are the
 * columns k depends on, ascending), level_ptr int32[n_levels+1] and
 * level_cols int32[n] (columns of each level, ascending). */
int glu_export_symbolic(const glu_handle *h, int32_t *perm, int64_t *lu_colptr, int32_t *lu_rowind,
                        int64_t *dag_ptr, int32_t *dag_idx, int32_t *level_ptr,
                        int32_t *level_cols);

/* Copy the factor values (float64[nnz_lu], A_s order: L strictly below the
 * diagonal, U on and above) to a host buffer.  Requires a successful factor.
 * The factors of a dense trailing block are kept in the block by the
 * factorization and written into A_s order here first (synchronizes the
 * device).  Errors: GLU_ERR_ARG, GLU_ERR_STATE, GLU_ERR_DEVICE. */
int glu_export_factors(const glu_handle *h, double *lu_values);

/* Static pivoting and scaling before the ordering (MC64, the first step of
 * the preprocessing flow of Section II-C): a maximum-product transversal of
 * A by shortest augmenting paths, with the scalings from its dual variables.
 * Host only; needs no handle and no device.
 *   row_perm int32[n]: row_perm[j] is the row of A matched to column j, so the
 *       matrix Q A with (Q A)(j, :) = A(row_perm[j], :) has the matched
 *       entries on its diagonal and the largest product of diagonal
 *       magnitudes over all row permutations;
 *   row_scale, col_scale float64[n]: every entry of diag(row_scale) A
 *       diag(col_scale) has magnitude <= 1 and the matched ones 1 (up to
 *       rounding).
 * To solve A x = b through these: factor M = Q diag(row_scale) A
 * diag(col_scale), solve M y = Q (row_scale .* b) and take x = col_scale .* y.
 * Caller-owned output buffers of n elements.  Errors: GLU_ERR_ARG (bad CSC
 * or pointer), GLU_ERR_NONFINITE_INPUT, GLU_ERR_STRUCT_SINGULAR (an all-zero
 * column, or no perfect matching exists), GLU_ERR_NOMEM. */
int glu_mc64(int32_t n, const int64_t *colptr, const int32_t *rowind, const double *values, int32_t *row_perm,
             double *row_scale, double *col_scale);

/* Column of the last zero or non-finite pivot (in the permuted order), else -1. */
int32_t glu_failed_column(const glu_handle *h);

/* Static text for a status code. */
const char *glu_strerror(int code);

/* Release everything the handle owns.  NULL is allowed. */
void glu_destroy(glu_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* GLU_H */
