// Launchers of the HIP kernels (kernels.hip); all device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "analyze.hpp"

namespace glu {

struct FactorArgs {
    const int64_t* colptr;
    const int32_t* rowind;
    double* val;
    float* val32;  // the FP32 form's factor values (null: FP64)
    const int64_t* diag;
    const int64_t* amap;
    const int32_t* task_col;
    const int64_t* task_src_ptr;
    const int64_t* src_upos;
    const int64_t* src_dpos;
    const int32_t* src_llen;
    const int32_t* wi_task;
    const int64_t* wi_begin;
    const int64_t* wi_end;
    const int64_t* wi_ss;
    const int8_t* wi_whole;
    const int32_t* ss_lo;
    const int32_t* ss_hi;
    const int64_t* wi_s0;
    const int32_t* wi_nsrc;
    const int64_t* ss_up;
    const int64_t* ss_dp;
    // analysis maps (built on the device by launch_level_map)
    const int64_t* wi_pbase;
    const int64_t* wi_tbase;
    const int32_t* wi_ntouch;
    const uint8_t* touch_off;
    const uint16_t* pair_pos;  // target index | rank << 8 of every pair
};

// One factorization's share of a batched level wavefront (glu_batch_factor).
struct BatchEntry {
    int64_t boff;         // first workgroup of the entry in the launch
    int64_t wi0, nwi;     // the level's work items
    const int32_t* norm;  // the previous level's columns to normalise
    int32_t nnorm;
    int32_t h;            // index of the factorization's arguments
};

struct SolveArgs {
    int32_t n;
    int32_t nrhs;
    const double* val;
    const int64_t* diag;
    const int64_t* lrow_ptr;
    const int64_t* lrow_pos;
    const int32_t* lrow_col;
    const int64_t* urow_ptr;
    const int64_t* urow_pos;
    const int32_t* urow_col;
    double* y;  // n x nrhs work vector, column-major, leading dimension n
    // schedule-ordered entries of the sparse solves (Analysis::fs_*, bs_*)
    const int64_t* fs_ptr;
    const int32_t* fs_col;
    const double* fs_val;
    const int64_t* bs_ptr;
    const int32_t* bs_col;
    const double* bs_val;
};

// Schur-complement update of the dense block (schur.hip); see Analysis::sch_*.
struct SchurArgs {
    const SchurUnit* units;
    int64_t nunits;
    int64_t nheavy;  // the first nheavy units (the longest) get a block each
    const int32_t* pl;
    const int32_t* pu;
    double* LP;
    double* UP;
    int64_t lp_len, up_len;
    const int64_t* lpos;
    const int64_t* loff;
    const int64_t* upos;
    const int64_t* uoff;
    int64_t nl, nu;
};

hipError_t launch_zero(double* p, int64_t n, hipStream_t st);
// v64[i] = v32[i] (exact widening of the FP32 form's factors)
hipError_t launch_widen(const float* v32, double* v64, int64_t n, hipStream_t st);
// value load; also resets the status words and ncount int32 counters (the
// stream runs' tickets and completion counts).  With a dense block of m > 0
// columns starting at t, nnz_lu is the number of entries in the columns
// before it, and of its columns only the rows above t are cleared (tail_pos:
// the device copy of the analysis' tail_pos)
hipError_t launch_value_load(const FactorArgs& a, const double* avals, int64_t nnz_a, int64_t nnz_lu,
                             int32_t* status, int32_t* counters, int32_t ncount, int32_t t, int32_t m,
                             const int64_t* tail_pos, hipStream_t st);
// one level in small-block (wide levels, slices of up to 256 entries) or
// large-block mode (slices of up to 64), or a lone stream-mode level
hipError_t launch_level(const FactorArgs& a, int mode, int64_t wi0, int64_t nwi, const int32_t* norm_cols,
                        int32_t nnorm, hipStream_t st);
// a run of stream-mode levels in one persistent launch (Analysis::seg_*,
// device copies); counters: ticket and completion count of the run (zero);
// err: bit 4 set if a bounded wait gave up
hipError_t launch_level_stream(const FactorArgs& a, const int64_t* seg_start, const int64_t* seg_wi,
                               const int32_t* seg_norm, int32_t nseg, int64_t nitems, const int32_t* exec_cols,
                               int32_t* counters, int32_t* err, int32_t grid, hipStream_t st);
// level e of several factorizations in one launch: ent[nent] ordered by boff,
// nblocks workgroups in all (slices of at most 256 entries, any mode's plan)
hipError_t launch_level_batch(const FactorArgs* args, const BatchEntry* ent, int32_t nent, int64_t nblocks,
                              bool fp32, hipStream_t st);
// Touched-entry lists and pair positions of every work item (pattern only).
hipError_t launch_level_map(const FactorArgs& a, int64_t nwi, uint8_t* touch_off, uint16_t* pair_pos,
                            int32_t* wi_ntouch, int32_t* err, hipStream_t st);
hipError_t launch_finalize(const FactorArgs& a, const int32_t* norm_cols, int32_t nnorm, int32_t n,
                           int32_t* status, hipStream_t st);
hipError_t launch_solve_gather(int32_t n, int32_t nrhs, const double* b, int64_t ldb, const int32_t* perm,
                               double* y, hipStream_t st);
hipError_t launch_solve_scatter(int32_t n, int32_t nrhs, const double* y, const int32_t* perm, double* x,
                                int64_t ldx, hipStream_t st);
// a whole sparse substitution in one launch of at most grid blocks (a static
// walk when the grid is resident, else waves claim slots from an atomic
// ticket): forward (upper = false, rows 0..t-1 of the schedule) or backward;
// mail: n * nrhs doubles of scratch; tag: different on every call of a
// process; sync: three int32 of scratch (reset by the call); err: set
// non-zero if a bounded wait gave up
hipError_t launch_solve_all(const SolveArgs& sa, bool upper, const int32_t* rows, int32_t nslots, int32_t t,
                            double* mail, uint64_t tag, int32_t* sync, int32_t* err, int32_t grid,
                            hipStream_t st);
// iterative refinement (FP64): r = b - A x over A's row view, with
// norms[0] = ||A||_inf, norms[1 + 2c] = ||r_c||_inf, norms[2 + 2c] = ||x_c||_inf
// (1 + 2 nrhs doubles of scratch); then x += d
hipError_t launch_residual(int32_t n, int32_t nrhs, const int64_t* arow_ptr, const int32_t* arow_col,
                           const int64_t* arow_pos, const double* aval, const double* b, int64_t ldb,
                           const double* x, int64_t ldx, double* r, double* norms, hipStream_t st);
hipError_t launch_axpy_update(int32_t n, int32_t nrhs, const double* d, double* x, int64_t ldx, hipStream_t st);
// dst[x] = val[pos[x]] (the solves' values in schedule order, after a factorization)
hipError_t launch_gather_values(const double* val, const int64_t* pos, int64_t cnt, double* dst, hipStream_t st);
hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t st);
int max_chunk(int mode);  // largest work-item range the level kernel of a mode stages

// dense trailing block (dense_tail.hip)
// build the block in D (order M = m rounded up to whole 64-wide panels, the
// padding set to the identity) from the na entries of A inside it: A_s
// positions asrc (values read from val), local rows arow and columns acol
hipError_t launch_tail_gather(const double* val, const int64_t* asrc, const int32_t* arow, const int32_t* acol,
                              int64_t na, int32_t m, int32_t M, double* D, int64_t ld, hipStream_t st);
hipError_t launch_tail_scatter(const FactorArgs& a, const int64_t* tail_pos, int32_t t, int32_t m,
                               const double* D, int64_t ld, hipStream_t st);
// status[0] = min(status[0], t + i) for every pivot D(i, i), i < m, that is zero or not finite
hipError_t launch_dense_pivots(const double* D, int64_t ld, int32_t m, int32_t t, int32_t* status, hipStream_t st);
// the long tiles run on st, the short ones on aux (forked from and joined to
// st through ev_fork / ev_join)
hipError_t launch_schur(const SchurArgs& s, const double* val, double* D, int64_t ld, int32_t m, hipStream_t st,
                        hipStream_t aux, hipEvent_t ev_fork, hipEvent_t ev_join);
// no-pivot LU of the M x M block (M a multiple of 64); F: 2 * 64 * 64 doubles
// of scratch; aux: a second stream for the bulk of each outer update, forked
// from and joined to st through ev_fork / ev_join; blas: a handle from
// dense_blas_create (the bulk updates then run as library DGEMMs) or null
hipError_t launch_dense_lu(double* D, int64_t ld, int32_t M, double* F, hipStream_t st, hipStream_t aux,
                           hipEvent_t ev_fork, hipEvent_t ev_join, void* blas);
// FP32 LU without pivoting of the M x M block (the mixed form's large
// blocks): the block rounded to an FP32 copy S (M x M, packed), factored by
// the ROCm LAPACK library's no-pivot LU (blas: a handle from
// dense_blas_create; info: one int of device scratch, the library's status),
// and widened back into D exactly
hipError_t launch_dense_lu_fp32(double* D, int64_t ld, int32_t M, float* S, void* blas, int32_t* info,
                                hipStream_t st);
// blocks of at least this order take the FP32 LU in the mixed form
constexpr int32_t kFp32DenseMin = 8192;
// a dense-BLAS handle on the current device (deterministic mode), and its release
hipError_t dense_blas_create(void** blas);
void dense_blas_destroy(void* blas);
inline int32_t dense_padded(int32_t m) { return (m + 63) / 64 * 64; }
// forward-solve cross term of the tail rows (see Analysis::cross_*); part:
// nw * nrhs doubles of scratch
hipError_t launch_tail_cross_fwd(const SolveArgs& sa, int32_t t, int32_t m, const int64_t* tail_lsplit,
                                 const int32_t* cptr, const int32_t* crow, const int64_t* cq0, int32_t nw,
                                 double* part, hipStream_t st);
// backward-solve cross term of the rows before the tail (see Analysis::ux_*):
// y(rows[c]) -= sum of items [rptr[c], rptr[c+1]), item w = sum over
// [q0[w], q1[w]) of xv[q] y(xc[q]); y: n x nrhs; part: nw * nrhs doubles of scratch
hipError_t launch_tail_cross_bwd(const double* xv, const int32_t* xc, const int64_t* q0, const int64_t* q1,
                                 int32_t nw, const int32_t* rows, const int32_t* rptr, int32_t nrows, double* y,
                                 int32_t n, int32_t nrhs, double* part, hipStream_t st);
// triangular solve with the dense tail's unit lower (upper = false) or upper
// triangle; ticket: one int of scratch; mail: m * nrhs doubles of scratch;
// epoch: different on every call of a process (it tags the mailbox's sentinel)
hipError_t launch_dense_trsv(const double* D, int64_t ld, int32_t m, double* y, int64_t ldy, int32_t nrhs,
                             bool upper, int32_t* ticket, double* mail, int32_t epoch, int32_t* err,
                             hipStream_t st);

}  // namespace glu
