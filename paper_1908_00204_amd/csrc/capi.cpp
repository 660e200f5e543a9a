// C ABI (include/glu.h): handle, device residency of the analysis, and the
// host loop that launches one kernel per level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/glu.h"
#include "analyze.hpp"
#include "analyze_gpu.hpp"
#include "kernels.hpp"

namespace {

enum HState { EMPTY = 0, ANALYZED = 1, FACTORED = 2 };

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) { p = nullptr; return e; }
        n = count;
        return hipSuccess;
    }
    size_t bytes() const { return n * sizeof(T); }
};

}  // namespace

struct glu_handle {
    int device = -1;
    int ordering = GLU_ORDER_AMD;
    glu::PlanParams pp;
    int64_t max_device_bytes = 0;
    int state = EMPTY;
    uint64_t analysis_serial = 0;  // bumped by every glu_analyze (batches check it)
    // FP32 form: FP32 factorization, FP64 refinement in glu_solve
    int precision = 0;
    int refine_max = 10;
    int dense_gemm = 0;        // 0: library DGEMM for the dense block's bulk updates; 1: own kernel
    void* blas = nullptr;      // the library handle (created with the first dense block)
    double refine_tol = 1e-13;
    int32_t refine_iters = 0;
    double refine_berr = 0.0;
    int fp64_fallback = 0;     // the last solve refactorized in FP64 (refinement stalled)
    int factors_fp64 = 0;      // the factors held are FP64 ones (FP64 form, or after a fallback)
    int factored_once = 0;
    glu::Analysis an;
    int32_t failed_col = -1;
    double t_factor_ms = 0, t_solve_ms = 0, t_update_ms = 0, t_dense_ms = 0;

    DevBuf<int64_t> colptr, diag, amap, task_src_ptr, src_upos, src_dpos, wi_begin, wi_end, wi_ss;
    DevBuf<int64_t> lrow_ptr, lrow_pos, urow_ptr, urow_pos, tail_pos, tail_lsplit, tail_asrc;
    DevBuf<int32_t> tail_arow, tail_acol;
    DevBuf<int32_t> rowind, task_col, wi_task, src_llen, ss_src, ss_lo, ss_hi, exec_cols, lrow_col, urow_col, fsolve_rows, bsolve_rows, perm;
    DevBuf<int8_t> wi_whole;
    DevBuf<int64_t> wi_s0, ss_up, ss_dp, wi_pbase, wi_tbase;
    DevBuf<int32_t> wi_nsrc, wi_ntouch;
    DevBuf<uint8_t> touch_off;
    DevBuf<uint16_t> pair_pos;
    DevBuf<double> val, avals, y, bstage, dense;
    DevBuf<float> val32, dense32;  // FP32 factors; the mixed form's FP32 copy of a large dense block
    DevBuf<int32_t> sinfo;         // status of the library LU of that copy
    DevBuf<int64_t> arow_ptr, arow_pos;  // row view of A (FP32 form's residual)
    DevBuf<int32_t> arow_col;
    DevBuf<double> rbuf, dbuf, xstage, norms;
    DevBuf<int32_t> status, dsync;
    // stream-mode runs: segment tables and per-run ticket / completion count
    DevBuf<int64_t> seg_start, seg_wi;
    DevBuf<int32_t> seg_norm, run_sync;
    DevBuf<int32_t> cross_ptr, cross_row;
    DevBuf<int64_t> fs_ptr, fs_pos, bs_ptr, bs_pos;
    DevBuf<int32_t> fs_col, bs_col;
    DevBuf<double> fs_val, bs_val;
    DevBuf<int64_t> cross_q0;
    // backward-solve cross term of the rows before the dense block
    DevBuf<int32_t> ux_ptr, ux_row, ux_col;
    DevBuf<int64_t> ux_q0, ux_q1, ux_pos;
    DevBuf<double> ux_val;
    DevBuf<double> cross_part, dmail, smail;
    // Schur-complement update of the dense block
    DevBuf<glu::SchurUnit> sch_units;
    DevBuf<int32_t> sch_pl, sch_pu;
    DevBuf<int64_t> sch_lpos, sch_loff, sch_upos, sch_uoff;
    DevBuf<double> sch_lp, sch_up;
    int64_t dense_ld = 0;
    int32_t epoch = 0;
    int num_cu = 1;  // compute units of the device (sizes the one-launch sparse solves)
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr;
    // second stream of the dense LU (default priority, does not synchronise
    // with the null stream) and its fork / join events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the solves' value gather runs beside the dense block's factorization
    hipStream_t side = nullptr;
    hipEvent_t ev_gfork = nullptr, ev_gjoin = nullptr;
    double t_schur_ms = 0;

    void release_device() {
        colptr.release(); diag.release(); amap.release(); task_src_ptr.release(); src_upos.release();
        src_dpos.release(); wi_ss.release(); src_llen.release(); ss_src.release(); ss_lo.release();
        ss_hi.release(); wi_whole.release(); wi_s0.release(); ss_up.release(); ss_dp.release();
        wi_nsrc.release(); wi_pbase.release(); wi_tbase.release(); wi_ntouch.release(); touch_off.release();
        pair_pos.release();
        wi_begin.release(); wi_end.release(); lrow_ptr.release(); lrow_pos.release(); urow_ptr.release();
        urow_pos.release(); tail_pos.release(); tail_lsplit.release(); rowind.release(); task_col.release();
        tail_asrc.release(); tail_arow.release(); tail_acol.release();
        wi_task.release(); exec_cols.release(); lrow_col.release(); urow_col.release(); fsolve_rows.release();
        bsolve_rows.release(); perm.release(); val.release(); avals.release(); y.release(); bstage.release();
        val32.release(); arow_ptr.release(); arow_pos.release(); arow_col.release(); rbuf.release();
        dbuf.release(); xstage.release(); norms.release();
        dense.release(); dense32.release(); sinfo.release(); status.release(); dsync.release(); seg_start.release(); seg_wi.release();
        seg_norm.release(); run_sync.release(); cross_ptr.release(); cross_row.release();
        cross_q0.release(); cross_part.release(); dmail.release(); smail.release(); fs_ptr.release(); fs_pos.release(); bs_ptr.release();
        bs_pos.release(); fs_col.release(); bs_col.release(); fs_val.release(); bs_val.release();
        ux_ptr.release(); ux_row.release(); ux_col.release(); ux_q0.release(); ux_q1.release(); ux_pos.release();
        ux_val.release();
        sch_units.release(); sch_pl.release(); sch_pu.release(); sch_lpos.release(); sch_loff.release();
        sch_upos.release(); sch_uoff.release(); sch_lp.release(); sch_up.release();
    }
    int64_t device_bytes() const {
        return (int64_t)(colptr.bytes() + diag.bytes() + amap.bytes() + task_src_ptr.bytes() + src_dpos.bytes() +
                         wi_ss.bytes() + src_llen.bytes() + ss_src.bytes() + ss_lo.bytes() + ss_hi.bytes() +
                         wi_whole.bytes() + wi_s0.bytes() + ss_up.bytes() + ss_dp.bytes() + wi_nsrc.bytes() +
                         wi_pbase.bytes() + wi_tbase.bytes() + wi_ntouch.bytes() + touch_off.bytes() +
                         pair_pos.bytes() +
                         src_upos.bytes() + wi_begin.bytes() + wi_end.bytes() + lrow_ptr.bytes() +
                         lrow_pos.bytes() + urow_ptr.bytes() + urow_pos.bytes() + tail_pos.bytes() +
                         tail_asrc.bytes() + tail_arow.bytes() + tail_acol.bytes() +
                         tail_lsplit.bytes() + rowind.bytes() + task_col.bytes() + wi_task.bytes() +
                         exec_cols.bytes() + lrow_col.bytes() + urow_col.bytes() + fsolve_rows.bytes() +
                         bsolve_rows.bytes() + perm.bytes() + val.bytes() + avals.bytes() + y.bytes() +
                         bstage.bytes() + dense.bytes() + status.bytes() + dsync.bytes() + seg_start.bytes() +
                         val32.bytes() + dense32.bytes() + sinfo.bytes() + arow_ptr.bytes() + arow_pos.bytes() + arow_col.bytes() + rbuf.bytes() +
                         dbuf.bytes() + xstage.bytes() + norms.bytes() +
                         seg_wi.bytes() + seg_norm.bytes() + run_sync.bytes() + cross_ptr.bytes() +
                         cross_row.bytes() + cross_q0.bytes() + cross_part.bytes() + dmail.bytes() + smail.bytes() + fs_ptr.bytes() +
                         fs_pos.bytes() + bs_ptr.bytes() + bs_pos.bytes() + fs_col.bytes() + bs_col.bytes() +
                         fs_val.bytes() + bs_val.bytes() + ux_ptr.bytes() + ux_row.bytes() + ux_col.bytes() +
                         ux_q0.bytes() + ux_q1.bytes() + ux_pos.bytes() + ux_val.bytes() + sch_units.bytes() +
                         sch_pl.bytes() + sch_pu.bytes() + sch_lpos.bytes() + sch_loff.bytes() + sch_upos.bytes() +
                         sch_uoff.bytes() + sch_lp.bytes() + sch_up.bytes());
    }
    glu::FactorArgs fargs(bool fp32 = false) const {
        glu::FactorArgs a;
        a.colptr = colptr.p; a.rowind = rowind.p; a.val = val.p; a.diag = diag.p; a.amap = amap.p;
        a.val32 = fp32 ? val32.p : nullptr;
        a.task_col = task_col.p; a.task_src_ptr = task_src_ptr.p; a.src_upos = src_upos.p;
        a.src_dpos = src_dpos.p; a.src_llen = src_llen.p; a.wi_ss = wi_ss.p; a.wi_whole = wi_whole.p;
        a.ss_lo = ss_lo.p; a.ss_hi = ss_hi.p;
        a.wi_s0 = wi_s0.p; a.wi_nsrc = wi_nsrc.p; a.ss_up = ss_up.p; a.ss_dp = ss_dp.p;
        a.wi_pbase = wi_pbase.p; a.wi_tbase = wi_tbase.p; a.wi_ntouch = wi_ntouch.p;
        a.touch_off = touch_off.p; a.pair_pos = pair_pos.p;
        a.wi_task = wi_task.p; a.wi_begin = wi_begin.p; a.wi_end = wi_end.p;
        return a;
    }
};

// A batch of analyzed handles whose sparse levels are factorized together:
// wavefront e launches level e of every handle that has one.
struct glu_batch {
    std::vector<glu_handle*> hs;
    std::vector<uint64_t> serial;          // each handle's analysis when the batch was made
    int device = -1;
    bool fp32 = false;
    DevBuf<glu::FactorArgs> args;
    DevBuf<glu::BatchEntry> ent;
    std::vector<int64_t> wf_ent;           // [wavefront] -> first entry (+ sentinel)
    std::vector<int64_t> wf_blocks;        // workgroups of each wavefront
    std::vector<hipStream_t> tails;        // streams for the handles' dense blocks and checks
    hipEvent_t ev_levels = nullptr;
    std::vector<hipEvent_t> ev_done;
    hipGraphExec_t graph = nullptr;        // the wavefront launches, captured once
    hipStream_t capture_stream = nullptr;
    double t_levels_ms = 0, t_total_ms = 0, t_solve_ms = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    // pinned host copies of every handle's residual norms and solve status
    double* hnorm = nullptr;
    size_t hnorm_n = 0;
    int32_t* hstat = nullptr;
    int32_t* hstat3 = nullptr;  // every handle's factorization status words
};

namespace {

template <class T>
hipError_t upload(DevBuf<T>& d, const std::vector<T>& h) {
    hipError_t e = d.alloc(h.size());
    if (e != hipSuccess) return e;
    if (!h.empty()) e = hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int64_t dense_ld_for(int32_t m) { return glu::dense_padded(m); }

int64_t planned_bytes(const glu::Analysis& a) {
    auto v = [](const auto& x) { return (int64_t)(x.size() * sizeof(x[0])); };
    return v(a.lu_colptr) + v(a.diag) + v(a.amap) + v(a.task_src_ptr) + v(a.src_upos) + v(a.wi_begin) +
           v(a.src_dpos) + v(a.src_llen) + v(a.wi_ss) + v(a.wi_whole) + v(a.ss_lo) + v(a.ss_hi) + v(a.ss_up) + v(a.ss_dp) +
           v(a.wi_s0) + v(a.wi_nsrc) + v(a.wi_pbase) + v(a.wi_tbase) + v(a.wi_nsrc) + a.n_pairs + a.n_touch_cap +
           v(a.wi_end) + v(a.lrow_ptr) + v(a.lrow_pos) + v(a.urow_ptr) + v(a.urow_pos) + v(a.lu_rowind) +
           v(a.task_col) + v(a.wi_task) + v(a.exec_cols) + v(a.lrow_col) + v(a.urow_col) +
           v(a.fsolve_rows) + v(a.bsolve_rows) + v(a.perm) + v(a.tail_pos) + v(a.tail_lsplit) +
           v(a.tail_asrc) + v(a.tail_arow) + v(a.tail_acol) +
           v(a.cross_ptr) + v(a.cross_row) + v(a.cross_q0) + v(a.cross_row) * 2 +
           v(a.fs_ptr) + v(a.fs_pos) * 2 + v(a.fs_col) + v(a.bs_ptr) + v(a.bs_pos) * 2 + v(a.bs_col) +
           v(a.ux_ptr) + v(a.ux_row) + v(a.ux_col) + v(a.ux_q0) + v(a.ux_q1) + v(a.ux_pos) * 2 +
           v(a.sch_units) + v(a.sch_pair_l) + v(a.sch_pair_u) + v(a.sch_lpos) + v(a.sch_loff) + v(a.sch_upos) +
           v(a.sch_uoff) + (a.sch_lp_len + a.sch_up_len) * 8 +
           (int64_t)a.lu_rowind.size() * 8 + a.nnz_a * 8 + dense_ld_for(a.tail_m) * glu::dense_padded(a.tail_m) * 8 + 2 * 64 * 64 * 8;
}

int set_device(const glu_handle* h) {
    if (h->device < 0) return GLU_ERR_DEVICE;
    if (hipSetDevice(h->device) != hipSuccess) return GLU_ERR_DEVICE;
    return GLU_OK;
}

// The factorization in phases, so that several handles can share the level
// loop (glu_batch_factor).  factor_begin: value load (with status reset);
// factor_levels: the sparse levels; factor_end: the dense block, the last
// normalisation, the pivot check and the solves' value gather, all enqueued
// on st; factor_finish: wait for st and read the status.
int factor_begin(glu_handle* h, const double* values, int on_device, hipStream_t st, bool fp32) {
    if (!h || !values) return GLU_ERR_ARG;
    if (h->state == EMPTY) return GLU_ERR_STATE;
    int rc = set_device(h);
    if (rc) return rc;
    const glu::Analysis& an = h->an;
    h->failed_col = -1;
    h->state = ANALYZED;
    const double* av = values;
    if (!on_device || (h->precision && values != h->avals.p)) {
        // the FP32 form keeps the values: its refinement's residual reads them
        if (an.nnz_a > 0 &&
            hipMemcpyAsync(h->avals.p, values, an.nnz_a * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st) != hipSuccess)
            return GLU_ERR_DEVICE;
        av = h->avals.p;
    }
    glu::FactorArgs fa = h->fargs(fp32);
    if (hipEventRecord(h->ev0, st) != hipSuccess) return GLU_ERR_DEVICE;
    const int32_t nruns = (int32_t)an.run_e0.size();
    // with a dense block only the entries outside it are cleared (the block
    // is built from A's entries in it)
    const int64_t nclear = an.tail_m > 0 ? an.lu_colptr[an.tail_start] : (int64_t)an.lu_rowind.size();
    if (glu::launch_value_load(fa, av, an.nnz_a, nclear, h->status.p, h->run_sync.p, 2 * nruns, an.tail_start,
                               an.tail_m, h->tail_pos.p, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (hipEventRecord(h->ev2, st) != hipSuccess) return GLU_ERR_DEVICE;
    return GLU_OK;
}

int factor_levels(glu_handle* h, hipStream_t st, bool fp32) {
    const glu::Analysis& an = h->an;
    glu::FactorArgs fa = h->fargs(fp32);
    const int32_t nruns = (int32_t)an.run_e0.size();
    const int32_t nexec = (int32_t)an.exec_ptr.size() - 1;
    int32_t run = 0;
    for (int32_t e = 0; e < nexec; e++) {
        if (run < nruns && an.run_e0[run] == e) {
            // a run of stream-mode levels in one persistent launch; it also
            // normalises the level before it, and leaves its own last level
            // to the next launch, as a single level does
            const int64_t sb = an.run_sb[run];
            const int32_t nseg = an.run_e1[run] - an.run_e0[run];
            if (glu::launch_level_stream(fa, h->seg_start.p + sb, h->seg_wi.p + sb, h->seg_norm.p + sb, nseg,
                                         an.seg_start[sb + nseg], h->exec_cols.p, h->run_sync.p + 2 * run,
                                         h->status.p + 2, 2 * h->num_cu, st) != hipSuccess)
                return GLU_ERR_DEVICE;
            e = an.run_e1[run] - 1;
            run++;
            continue;
        }
        const int64_t wi0 = an.wi_ptr[e], nwi = an.wi_ptr[e + 1] - an.wi_ptr[e];
        const int32_t* norm = nullptr;
        int32_t nnorm = 0;
        if (e > 0) {
            norm = h->exec_cols.p + an.exec_ptr[e - 1];
            nnorm = an.exec_ptr[e] - an.exec_ptr[e - 1];
        }
        if (glu::launch_level(fa, an.level_mode[e], wi0, nwi, norm, nnorm, st) != hipSuccess)
            return GLU_ERR_DEVICE;
    }
    return GLU_OK;
}

// The rest of a factorization after the level loop.  in_batch: a batch's
// factorization -- the handle's timing events are left out and the dense
// block's bulk updates run on this library's kernel (not the BLAS library),
// so that every handle of a batch runs the same kernels in every form.
int factor_end(glu_handle* h, hipStream_t st, bool fp32, bool in_batch = false) {
    const glu::Analysis& an = h->an;
    glu::FactorArgs fa = h->fargs(fp32);
    const int32_t nexec = (int32_t)an.exec_ptr.size() - 1;
    // With a dense block, the last level's L columns are divided now: the
    // Schur-complement update reads them.
    const bool norm_now = an.tail_m > 0 && nexec > 0;
    if (norm_now && glu::launch_level(fa, an.level_mode[nexec - 1], 0, 0, h->exec_cols.p + an.exec_ptr[nexec - 1],
                                      an.exec_ptr[nexec] - an.exec_ptr[nexec - 1], st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (!in_batch && hipEventRecord(h->ev3, st) != hipSuccess) return GLU_ERR_DEVICE;
    // With a dense block every value the solves gather (rows before the block)
    // is final once the last level is normalised -- the rest of the
    // factorization only reads A_s -- so the gather runs on a side stream
    // beside the block's LU, whose panel chain leaves compute units idle.
    const bool gather_side = an.tail_m > 0;
    // The FP32 form with a dense block: the sparse columns' FP32 factors (and
    // the block's FP32-rounded entries) are widened exactly before the Schur
    // update reads them; the block is then updated and factorized in FP64.
    if (fp32 && an.tail_m > 0 &&
        glu::launch_widen(h->val32.p, h->val.p, (int64_t)an.lu_rowind.size(), st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (an.tail_m > 0) {
        glu::SchurArgs sa;
        sa.units = h->sch_units.p; sa.nunits = (int64_t)an.sch_units.size(); sa.nheavy = an.sch_nheavy;
        sa.pl = h->sch_pl.p; sa.pu = h->sch_pu.p; sa.LP = h->sch_lp.p; sa.UP = h->sch_up.p;
        sa.lp_len = an.sch_lp_len; sa.up_len = an.sch_up_len;
        sa.lpos = h->sch_lpos.p; sa.loff = h->sch_loff.p; sa.upos = h->sch_upos.p; sa.uoff = h->sch_uoff.p;
        sa.nl = (int64_t)an.sch_lpos.size(); sa.nu = (int64_t)an.sch_upos.size();
        const int32_t M = glu::dense_padded(an.tail_m);
        if (glu::launch_tail_gather(h->val.p, h->tail_asrc.p, h->tail_arow.p, h->tail_acol.p,
                                    (int64_t)an.tail_asrc.size(), an.tail_m, M, h->dense.p, h->dense_ld, st) !=
                hipSuccess ||
            glu::launch_schur(sa, h->val.p, h->dense.p, h->dense_ld, an.tail_m, st, h->aux, h->ev_fork, h->ev_join) !=
                hipSuccess ||
            (!in_batch && hipEventRecord(h->ev4, st) != hipSuccess) || hipEventRecord(h->ev_gfork, st) != hipSuccess ||
            hipStreamWaitEvent(h->side, h->ev_gfork, 0) != hipSuccess ||
            glu::launch_gather_values(h->val.p, h->fs_pos.p, (int64_t)an.fs_pos.size(), h->fs_val.p, h->side) !=
                hipSuccess ||
            glu::launch_gather_values(h->val.p, h->bs_pos.p, (int64_t)an.bs_pos.size(), h->bs_val.p, h->side) !=
                hipSuccess ||
            glu::launch_gather_values(h->val.p, h->ux_pos.p, (int64_t)an.ux_pos.size(), h->ux_val.p, h->side) !=
                hipSuccess ||
            hipEventRecord(h->ev_gjoin, h->side) != hipSuccess ||
            (fp32 && !in_batch && h->dense32.p
                 ? glu::launch_dense_lu_fp32(h->dense.p, h->dense_ld, M, h->dense32.p, h->blas, h->sinfo.p, st)
                 : glu::launch_dense_lu(h->dense.p, h->dense_ld, M, h->dense.p + (size_t)h->dense_ld * M, st, h->aux,
                                        h->ev_fork, h->ev_join, h->dense_gemm == 0 && !in_batch ? h->blas : nullptr)) !=
                hipSuccess ||
            glu::launch_dense_pivots(h->dense.p, h->dense_ld, an.tail_m, an.tail_start, h->status.p, st) !=
                hipSuccess)
            return GLU_ERR_DEVICE;
        // The block stays the home of the tail's factors: the solves read it,
        // and glu_export_factors scatters it into A_s.
    }
    {
        const int32_t* norm = nullptr;
        int32_t nnorm = 0;
        if (nexec > 0 && !norm_now) {
            norm = h->exec_cols.p + an.exec_ptr[nexec - 1];
            nnorm = an.exec_ptr[nexec] - an.exec_ptr[nexec - 1];
        }
        // pivots of the sparse columns (the dense block's were checked above)
        if (glu::launch_finalize(fa, norm, nnorm, an.tail_m > 0 ? an.tail_start : an.n, h->status.p, st) !=
            hipSuccess)
            return GLU_ERR_DEVICE;
    }
    // the FP32 form's factors, widened exactly, are what the solves read
    if (fp32 && an.tail_m == 0 &&
        glu::launch_widen(h->val32.p, h->val.p, (int64_t)an.lu_rowind.size(), st) != hipSuccess)
        return GLU_ERR_DEVICE;
    // the sparse solves read the factors in schedule order
    if (gather_side) {
        if (hipStreamWaitEvent(st, h->ev_gjoin, 0) != hipSuccess) return GLU_ERR_DEVICE;
    } else if (glu::launch_gather_values(h->val.p, h->fs_pos.p, (int64_t)an.fs_pos.size(), h->fs_val.p, st) !=
                   hipSuccess ||
               glu::launch_gather_values(h->val.p, h->bs_pos.p, (int64_t)an.bs_pos.size(), h->bs_val.p, st) !=
                   hipSuccess ||
               glu::launch_gather_values(h->val.p, h->ux_pos.p, (int64_t)an.ux_pos.size(), h->ux_val.p, st) !=
                   hipSuccess) {
        return GLU_ERR_DEVICE;
    }
    if (!in_batch && hipEventRecord(h->ev1, st) != hipSuccess) return GLU_ERR_DEVICE;
    return GLU_OK;
}

// The outcome of a factorization from its status words {first bad pivot
// column or INT32_MAX, non-finite input flag, stream-run wait error}.
int factor_status(glu_handle* h, const int32_t* stat, bool fp32) {
    if (stat[2]) return GLU_ERR_DEVICE;  // a stream run's bounded wait gave up
    if (stat[1]) return GLU_ERR_NONFINITE_INPUT;
    if (stat[0] != INT32_MAX) {
        h->failed_col = stat[0];
        return GLU_ERR_ZERO_PIVOT;
    }
    h->state = FACTORED;
    h->factored_once = 1;
    h->factors_fp64 = !fp32;
    return GLU_OK;
}

int factor_finish(glu_handle* h, hipStream_t st, bool fp32) {
    const glu::Analysis& an = h->an;
    int32_t stat[3] = {INT32_MAX, 0, 0};
    if (hipMemcpyAsync(stat, h->status.p, sizeof(stat), hipMemcpyDeviceToHost, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return GLU_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->t_factor_ms = ms;
    if (hipEventElapsedTime(&ms, h->ev2, h->ev3) == hipSuccess) h->t_update_ms = ms;
    if (hipEventElapsedTime(&ms, h->ev3, h->ev1) == hipSuccess) h->t_dense_ms = ms;
    h->t_schur_ms = 0;
    if (an.tail_m > 0 && hipEventElapsedTime(&ms, h->ev3, h->ev4) == hipSuccess) h->t_schur_ms = ms;
    return factor_status(h, stat, fp32);
}


int run_factor(glu_handle* h, const double* values, int on_device, void* stream, bool fp32) {
    hipStream_t st = (hipStream_t)stream;
    int rc = factor_begin(h, values, on_device, st, fp32);
    if (!rc) rc = factor_levels(h, st, fp32);
    if (!rc) rc = factor_end(h, st, fp32);
    if (!rc) rc = factor_finish(h, st, fp32);
    return rc;
}

// Device scratch of one solve: the work vector and the mailbox (n x nrhs
// each), the tail's cross-term partial sums (work items x nrhs) and the
// dense solves' mailbox (m x nrhs).
struct SolveScratch {
    double* y;
    double* smail;
    double* cross_part;
    double* dmail;
};

// The device part of a solve: permute b, the two sparse substitutions around
// the dense block's, inverse-permute into x (device pointers, column-major).
int run_solve(glu_handle* h, int32_t nrhs, const double* db, int64_t dldb, double* dx, int64_t dldx,
              const SolveScratch& sc, hipStream_t st) {
    const glu::Analysis& a = h->an;
    const int32_t n = a.n;
    glu::SolveArgs sa;
    sa.n = n; sa.nrhs = nrhs; sa.val = h->val.p; sa.diag = h->diag.p;
    sa.lrow_ptr = h->lrow_ptr.p; sa.lrow_pos = h->lrow_pos.p; sa.lrow_col = h->lrow_col.p;
    sa.urow_ptr = nullptr; sa.urow_pos = nullptr; sa.urow_col = nullptr;
    sa.y = sc.y;
    sa.fs_ptr = h->fs_ptr.p; sa.fs_col = h->fs_col.p; sa.fs_val = h->fs_val.p;
    sa.bs_ptr = h->bs_ptr.p; sa.bs_col = h->bs_col.p; sa.bs_val = h->bs_val.p;
    if (hipEventRecord(h->ev0, st) != hipSuccess) return GLU_ERR_DEVICE;
    if (glu::launch_set_i32(h->status.p + 2, 0, st) != hipSuccess) return GLU_ERR_DEVICE;
    if (glu::launch_solve_gather(n, nrhs, db, dldb, h->perm.p, sc.y, st) != hipSuccess) return GLU_ERR_DEVICE;
    // the sparse substitutions: one launch each, a few 256-thread blocks per
    // compute unit walking the level schedule
    const int32_t tsp = a.tail_m > 0 ? a.tail_start : n;
    const int32_t sgrid = 2 * h->num_cu;
    if (!a.fsolve_ptr.empty() &&
        glu::launch_solve_all(sa, false, h->fsolve_rows.p, a.fsolve_ptr.back(), tsp, sc.smail, (uint32_t)++h->epoch,
                              h->dsync.p + 1, h->status.p + 2, sgrid, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (a.tail_m > 0) {
        const int32_t t = a.tail_start;
        const int32_t nw = (int32_t)a.cross_row.size();
        if (glu::launch_tail_cross_fwd(sa, t, a.tail_m, h->tail_lsplit.p, h->cross_ptr.p, h->cross_row.p,
                                       h->cross_q0.p, nw, sc.cross_part, st) != hipSuccess)
            return GLU_ERR_DEVICE;
        if (glu::launch_dense_trsv(h->dense.p, h->dense_ld, a.tail_m, sc.y + t, n, nrhs, false, h->dsync.p,
                                   sc.dmail, ++h->epoch, h->status.p + 2, st) != hipSuccess ||
            glu::launch_dense_trsv(h->dense.p, h->dense_ld, a.tail_m, sc.y + t, n, nrhs, true, h->dsync.p,
                                   sc.dmail, ++h->epoch, h->status.p + 2, st) != hipSuccess)
            return GLU_ERR_DEVICE;
        // the rows before the block: their U entries in the block's columns, in parallel
        if (glu::launch_tail_cross_bwd(h->ux_val.p, h->ux_col.p, h->ux_q0.p, h->ux_q1.p, (int32_t)a.ux_q0.size(),
                                       h->ux_row.p, h->ux_ptr.p, (int32_t)a.ux_row.size(), sc.y, n, nrhs,
                                       sc.cross_part + (size_t)nw * nrhs, st) != hipSuccess)
            return GLU_ERR_DEVICE;
    }
    if (!a.bsolve_ptr.empty() &&
        glu::launch_solve_all(sa, true, h->bsolve_rows.p, a.bsolve_ptr.back(), tsp, sc.smail, (uint32_t)++h->epoch,
                              h->dsync.p + 1, h->status.p + 2, sgrid, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (glu::launch_solve_scatter(n, nrhs, sc.y, h->perm.p, dx, dldx, st) != hipSuccess) return GLU_ERR_DEVICE;
    if (hipEventRecord(h->ev1, st) != hipSuccess) return GLU_ERR_DEVICE;
    return GLU_OK;
}

// Wait for the solve on st and report a failed bounded wait.
int finish_solve(glu_handle* h, hipStream_t st) {
    int32_t serr = 0;
    if (hipMemcpyAsync(&serr, h->status.p + 2, sizeof(serr), hipMemcpyDeviceToHost, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return GLU_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->t_solve_ms = ms;
    return serr ? GLU_ERR_DEVICE : GLU_OK;
}

// Static device scratch of glu_solve_noalloc: one array per GPU, loaded with
// the code object and held until the process ends.  Host code never uses the
// array's name as an address; it asks the runtime for the device's copy once
// per device (hipGetSymbolAddress) and passes that pointer to the kernels.
constexpr int64_t kNoAllocScratchDoubles = (int64_t)8 << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The device's copy of the scratch array (device must be current).
int scratch_on_device(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return GLU_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GLU_ERR_DEVICE;
        g_scratch_dev[device] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[device];
    return GLU_OK;
}

// Doubles rounded up to whole 256-byte lines.
int64_t lines(int64_t doubles) { return (doubles + 31) / 32 * 32; }

// Iterative refinement of the FP32 form (FP64 residual and update): with x
// from the solve with the FP32 factors, repeat r = b - A x; stop when every
// right-hand side's backward error ||r||_inf / (||A||_inf ||x||_inf) is at
// most refine_tol; else d = (LU)^-1 r and x += d.  If refine_max steps do not
// get there, the matrix is refactorized in FP64 (same plan) and solved again.
// The handle's device scratch for solves of nrhs right-hand sides (grown, never shrunk).
int solve_scratch(glu_handle* h, int32_t nrhs, SolveScratch& sc) {
    const glu::Analysis& a = h->an;
    const size_t need = (size_t)a.n * nrhs;
    if (h->y.n < need && h->y.alloc(need) != hipSuccess) return GLU_ERR_NOMEM;
    if (h->smail.n < need && h->smail.alloc(need) != hipSuccess) return GLU_ERR_NOMEM;
    const size_t nw = a.cross_row.size() + a.ux_q0.size();  // forward and backward cross items
    if (a.tail_m > 0) {
        if (h->cross_part.n < nw * nrhs && h->cross_part.alloc(nw * nrhs) != hipSuccess) return GLU_ERR_NOMEM;
        if (h->dmail.n < (size_t)a.tail_m * nrhs && h->dmail.alloc((size_t)a.tail_m * nrhs) != hipSuccess)
            return GLU_ERR_NOMEM;
    }
    sc = SolveScratch{h->y.p, h->smail.p, h->cross_part.p, h->dmail.p};
    return GLU_OK;
}

// ... and the refinement's residual, correction and norms.
int refine_scratch(glu_handle* h, int32_t nrhs) {
    const size_t need = (size_t)h->an.n * nrhs;
    if ((h->rbuf.n < need && h->rbuf.alloc(need) != hipSuccess) ||
        (h->dbuf.n < need && h->dbuf.alloc(need) != hipSuccess) ||
        (h->norms.n < (size_t)(1 + 2 * nrhs) && h->norms.alloc(1 + 2 * nrhs) != hipSuccess))
        return GLU_ERR_NOMEM;
    return GLU_OK;
}

// Backward error max_c ||b_c - A x_c||_inf / (||A||_inf ||x_c||_inf) from the
// residual kernel's norms {||A||, then (||r_c||, ||x_c||) per column}.
double backward_error(const double* nm, int32_t nrhs) {
    double be = 0.0;
    for (int32_t c = 0; c < nrhs; c++) {
        const double den = nm[0] * nm[2 + 2 * c];
        be = std::max(be, den > 0 ? nm[1 + 2 * c] / den : (nm[1 + 2 * c] > 0 ? INFINITY : 0.0));
    }
    return be;
}

int refine_solution(glu_handle* h, int32_t nrhs, const double* db, int64_t dldb, double* dx, int64_t dldx,
                    const SolveScratch& sc, hipStream_t st) {
    const glu::Analysis& a = h->an;
    const int32_t n = a.n;
    if (refine_scratch(h, nrhs)) return GLU_ERR_NOMEM;
    std::vector<double> nm(1 + 2 * nrhs);
    h->refine_iters = 0;
    for (int pass = 0;; pass++) {
        for (int it = 0;; it++) {
            if (glu::launch_residual(n, nrhs, h->arow_ptr.p, h->arow_col.p, h->arow_pos.p, h->avals.p, db, dldb, dx,
                                     dldx, h->rbuf.p, h->norms.p, st) != hipSuccess ||
                hipMemcpyAsync(nm.data(), h->norms.p, nm.size() * sizeof(double), hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return GLU_ERR_DEVICE;
            const double be = backward_error(nm.data(), nrhs);
            h->refine_berr = be;
            if (be <= h->refine_tol) return GLU_OK;
            if (it >= h->refine_max || !std::isfinite(be)) break;
            int rc = run_solve(h, nrhs, h->rbuf.p, n, h->dbuf.p, n, sc, st);
            if (rc) return rc;
            if (glu::launch_axpy_update(n, nrhs, h->dbuf.p, dx, dldx, st) != hipSuccess) return GLU_ERR_DEVICE;
            h->refine_iters++;
        }
        if (pass > 0 || h->factors_fp64) return GLU_OK;  // FP64 factors: report the reached error
        // FP64 fallback on the same plan and values
        int rc = run_factor(h, h->avals.p, 1, st, false);
        if (rc) return rc;
        h->fp64_fallback = 1;
        rc = run_solve(h, nrhs, db, dldb, dx, dldx, sc, st);
        if (rc) return rc;
    }
}

}  // namespace

extern "C" {

const char* glu_strerror(int code) {
    switch (code) {
        case GLU_OK: return "success";
        case GLU_ERR_ARG: return "invalid argument";
        case GLU_ERR_STATE: return "call out of order for the handle's state";
        case GLU_ERR_ZERO_PIVOT: return "zero or non-finite pivot";
        case GLU_ERR_STRUCT_SINGULAR: return "structurally singular matrix (diagonal absent after fill)";
        case GLU_ERR_NOMEM: return "out of memory or over the device-memory limit";
        case GLU_ERR_DEVICE: return "HIP device error or no device";
        case GLU_ERR_NONFINITE_INPUT: return "non-finite input value";
        case GLU_ERR_SCRATCH: return "solve too large for the no-allocation solve's static scratch";
        default: return "unknown status";
    }
}

int glu_create(glu_handle** out, int device, const glu_options* opt) {
    if (!out) return GLU_ERR_ARG;
    *out = nullptr;
    glu_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    for (int r : o.reserved)
        if (r != 0) return GLU_ERR_ARG;
    // The device DAG + levels (analyze_gpu.hip) is switched off: its first
    // GPU run stopped answering inside that step on a 40-column input and the
    // cause is not known yet, so the option is refused rather than run.
    if (o.gpu_analysis != 0) return GLU_ERR_ARG;
    // the FP32 form runs its sparse levels in small- or large-block mode (the
    // stream-mode kernel exists in FP64 only)
    if (o.precision < 0 || o.precision > 1 || o.refine_max_iters < -1 ||
        (o.precision == 1 && (o.force_mode == GLU_MODE_STREAM || o.stream_threshold > 0)))
        return GLU_ERR_ARG;
    if (device < -1 || o.ordering < 0 || o.ordering > 2 || o.force_mode < 0 || o.force_mode > 3 ||
        o.stream_threshold < -1 || o.large_threshold < -1 || o.max_device_bytes < 0 || o.dense_tail < -1 ||
        o.dense_gemm < 0 || o.dense_gemm > 1)
        return GLU_ERR_ARG;
    glu_handle* h = new (std::nothrow) glu_handle();
    if (!h) return GLU_ERR_NOMEM;
    h->device = device;
    h->ordering = o.ordering;
    h->pp.force_mode = o.force_mode == GLU_MODE_AUTO ? -1 : o.force_mode - 1;
    // defaults from the mode ablation on MI355X: small-block launches for
    // every level; large-block slices (1-14% slower) and the persistent
    // stream-mode runs (1.3-18x slower: their coherent value access costs far
    // more than the launches they save) only when asked for or tuned in
    h->pp.stream_threshold = o.stream_threshold ? o.stream_threshold : -1;
    h->pp.large_threshold = o.large_threshold ? o.large_threshold : -1;
    h->pp.chunk_small = glu::max_chunk(0);
    h->pp.chunk_large = glu::max_chunk(1);
    h->pp.chunk_stream = glu::max_chunk(2);
    h->max_device_bytes = o.max_device_bytes;
    h->pp.dense_tail = o.dense_tail;
    h->precision = o.precision;
    h->dense_gemm = o.dense_gemm;
    if (o.precision == 1) h->pp.stream_threshold = -1;
    if (o.refine_max_iters != 0) h->refine_max = std::max(0, o.refine_max_iters);
    if (o.gpu_analysis) {
        h->pp.dag_levels = [](int32_t n, const std::vector<int64_t>& cp, const std::vector<int32_t>& ri,
                              const std::vector<int64_t>& dg, std::vector<int64_t>& dp, std::vector<int32_t>& di,
                              std::vector<int32_t>& lev, int32_t* spin_err) -> int {
            return glu::gpu_dag_levels(n, cp, ri, dg, dp, di, lev, spin_err) == hipSuccess ? 0 : 1;
        };
    }
    if (device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev || hipSetDevice(device) != hipSuccess ||
            hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
            hipEventCreate(&h->ev2) != hipSuccess || hipEventCreate(&h->ev3) != hipSuccess ||
            hipEventCreate(&h->ev4) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_gfork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_gjoin, hipEventDisableTiming) != hipSuccess ||
            hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
            hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
            for (hipEvent_t e : {h->ev0, h->ev1, h->ev2, h->ev3, h->ev4, h->ev_fork, h->ev_join, h->ev_gfork,
                                 h->ev_gjoin})
                if (e) (void)hipEventDestroy(e);
            if (h->aux) (void)hipStreamDestroy(h->aux);
            if (h->side) (void)hipStreamDestroy(h->side);
            delete h;
            return GLU_ERR_DEVICE;
        }
    }
    *out = h;
    return GLU_OK;
}

int glu_analyze(glu_handle* h, int32_t n, const int64_t* colptr, const int32_t* rowind, const int32_t* perm) {
    if (!h) return GLU_ERR_ARG;
    if (h->ordering == GLU_ORDER_USER && !perm) return GLU_ERR_ARG;
    if (h->device >= 0 && set_device(h) != GLU_OK) return GLU_ERR_DEVICE;
    h->release_device();
    h->state = EMPTY;
    h->analysis_serial++;
    h->factored_once = 0;
    h->failed_col = -1;
    glu::Status st;
    try {
        st = glu::analyze(n, colptr, rowind, h->ordering, h->ordering == GLU_ORDER_USER ? perm : nullptr,
                          h->pp, h->an);
    } catch (const std::bad_alloc&) {
        h->an = glu::Analysis();
        return GLU_ERR_NOMEM;
    } catch (...) {
        h->an = glu::Analysis();
        return GLU_ERR_ARG;
    }
    if (st != glu::Status::ok) {
        if (st == glu::Status::struct_singular) h->failed_col = h->an.bad_col;
        glu::Analysis keep_bad;
        keep_bad.bad_col = h->an.bad_col;
        h->an = keep_bad;
        return (int)st;
    }
    if (h->device < 0) {
        h->state = ANALYZED;
        return GLU_OK;
    }
    if (h->max_device_bytes > 0 && planned_bytes(h->an) > h->max_device_bytes) {
        h->an = glu::Analysis();
        return GLU_ERR_NOMEM;
    }
    auto t0 = std::chrono::steady_clock::now();
    const glu::Analysis& a = h->an;
    hipError_t e = hipSuccess;
    auto up = [&](auto& d, const auto& v) {
        if (e == hipSuccess) e = upload(d, v);
    };
    up(h->colptr, a.lu_colptr); up(h->rowind, a.lu_rowind); up(h->diag, a.diag); up(h->amap, a.amap);
    up(h->task_col, a.task_col); up(h->task_src_ptr, a.task_src_ptr); up(h->src_upos, a.src_upos);
    up(h->wi_task, a.wi_task); up(h->wi_begin, a.wi_begin); up(h->wi_end, a.wi_end);
    up(h->src_dpos, a.src_dpos); up(h->src_llen, a.src_llen); up(h->wi_ss, a.wi_ss); up(h->wi_whole, a.wi_whole);
    up(h->ss_lo, a.ss_lo); up(h->ss_hi, a.ss_hi);
    up(h->wi_s0, a.wi_s0); up(h->wi_nsrc, a.wi_nsrc); up(h->ss_up, a.ss_up); up(h->ss_dp, a.ss_dp);
    up(h->wi_pbase, a.wi_pbase); up(h->wi_tbase, a.wi_tbase);
    if (e == hipSuccess) e = h->wi_ntouch.alloc(a.wi_task.size());
    if (e == hipSuccess) e = h->touch_off.alloc((size_t)a.n_touch_cap);
    if (e == hipSuccess) e = h->pair_pos.alloc((size_t)a.n_pairs);
    up(h->exec_cols, a.exec_cols); up(h->tail_pos, a.tail_pos); up(h->tail_lsplit, a.tail_lsplit);
    up(h->tail_asrc, a.tail_asrc); up(h->tail_arow, a.tail_arow); up(h->tail_acol, a.tail_acol);
    up(h->seg_start, a.seg_start); up(h->seg_wi, a.seg_wi); up(h->seg_norm, a.seg_norm);
    if (e == hipSuccess) e = h->run_sync.alloc(2 * a.run_e0.size());
    up(h->lrow_ptr, a.lrow_ptr); up(h->lrow_pos, a.lrow_pos); up(h->lrow_col, a.lrow_col);
    up(h->fsolve_rows, a.fsolve_rows); up(h->bsolve_rows, a.bsolve_rows); up(h->perm, a.perm);
    up(h->sch_units, a.sch_units); up(h->sch_pl, a.sch_pair_l); up(h->sch_pu, a.sch_pair_u);
    up(h->sch_lpos, a.sch_lpos); up(h->sch_loff, a.sch_loff); up(h->sch_upos, a.sch_upos);
    up(h->sch_uoff, a.sch_uoff);
    up(h->cross_ptr, a.cross_ptr); up(h->cross_row, a.cross_row); up(h->cross_q0, a.cross_q0);
    up(h->fs_ptr, a.fs_ptr); up(h->fs_pos, a.fs_pos); up(h->fs_col, a.fs_col);
    up(h->bs_ptr, a.bs_ptr); up(h->bs_pos, a.bs_pos); up(h->bs_col, a.bs_col);
    up(h->ux_ptr, a.ux_ptr); up(h->ux_row, a.ux_row); up(h->ux_col, a.ux_col);
    up(h->ux_q0, a.ux_q0); up(h->ux_q1, a.ux_q1); up(h->ux_pos, a.ux_pos);
    if (e == hipSuccess) e = h->fs_val.alloc(a.fs_pos.size());
    if (e == hipSuccess) e = h->bs_val.alloc(a.bs_pos.size());
    if (e == hipSuccess) e = h->ux_val.alloc(a.ux_pos.size());
    if (e == hipSuccess) e = h->sch_lp.alloc((size_t)a.sch_lp_len);
    if (e == hipSuccess) e = h->sch_up.alloc((size_t)a.sch_up_len);
    // the Schur panels: zero once; the factorizations write only the pattern's positions
    if (e == hipSuccess) e = hipMemset(h->sch_lp.p, 0, h->sch_lp.bytes());
    if (e == hipSuccess) e = hipMemset(h->sch_up.p, 0, h->sch_up.bytes());
    if (e == hipSuccess) e = h->val.alloc(a.lu_rowind.size());
    if (e == hipSuccess && h->precision == 1) {
        // FP32 factor storage, and the row view of A for the refinement's
        // residual (column indices and positions in A's own CSC order)
        e = h->val32.alloc(a.lu_rowind.size());
        std::vector<int64_t> rp(n + 1, 0), rpos(a.nnz_a);
        std::vector<int32_t> rcol(a.nnz_a);
        for (int64_t p = 0; p < a.nnz_a; p++) rp[rowind[p] + 1]++;
        for (int32_t i = 0; i < n; i++) rp[i + 1] += rp[i];
        std::vector<int64_t> f(rp.begin(), rp.end() - 1);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                const int64_t q = f[rowind[p]]++;
                rcol[q] = j;
                rpos[q] = p;
            }
        up(h->arow_ptr, rp); up(h->arow_col, rcol); up(h->arow_pos, rpos);
    }
    if (e == hipSuccess) e = h->avals.alloc((size_t)a.nnz_a);
    if (e == hipSuccess) e = h->status.alloc(4);
    if (e == hipSuccess && a.tail_m > 0) {
        h->dense_ld = dense_ld_for(a.tail_m);
        // the padded block, then the 2 x 64 x 64 scratch of the panel solves
        e = h->dense.alloc((size_t)h->dense_ld * glu::dense_padded(a.tail_m) + 2 * 64 * 64);
        // blocks past two outer panels have bulk updates (library DGEMMs by default)
        if (e == hipSuccess && h->dense_gemm == 0 && !h->blas && glu::dense_padded(a.tail_m) > 512)
            e = glu::dense_blas_create(&h->blas);
        // the mixed form factors a large block in FP32 (through the same library handle)
        const int32_t M = glu::dense_padded(a.tail_m);
        if (e == hipSuccess && h->precision == 1 && h->dense_gemm == 0 && M >= glu::kFp32DenseMin) {
            e = h->dense32.alloc((size_t)M * M);
            if (e == hipSuccess) e = h->sinfo.alloc(1);
        }
    }
    if (e == hipSuccess) e = h->dsync.alloc(4);
    if (e == hipSuccess) e = hipMemset(h->dsync.p, 0, h->dsync.bytes());
    if (e == hipSuccess) e = hipMemset(h->status.p, 0, h->status.bytes());
    h->epoch = 0;
    // the touched-entry lists and pair positions of the level kernel (pattern only)
    if (e == hipSuccess) {
        glu::FactorArgs fa = h->fargs();
        int32_t err = 0;
        e = glu::launch_level_map(fa, (int64_t)a.wi_task.size(), h->touch_off.p, h->pair_pos.p, h->wi_ntouch.p,
                                  h->status.p + 3, nullptr);
        if (e == hipSuccess) e = hipMemcpy(&err, h->status.p + 3, sizeof(err), hipMemcpyDeviceToHost);
        if (e == hipSuccess && err != 0) e = hipErrorUnknown;
    }
    if (e != hipSuccess) {
        h->release_device();
        h->an = glu::Analysis();
        return e == hipErrorOutOfMemory ? GLU_ERR_NOMEM : GLU_ERR_DEVICE;
    }
    h->an.t_plan_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (std::getenv("GLU_VERBOSE")) {
        std::fprintf(stderr, "[glu analyze] device upload done (%.2f GB on the device)\n", h->device_bytes() / 1e9);
        std::fflush(stderr);
    }
    h->state = ANALYZED;
    return GLU_OK;
}

int glu_factor(glu_handle* h, const double* values, int values_on_device, void* stream) {
    if (!h) return GLU_ERR_ARG;
    h->fp64_fallback = 0;
    return run_factor(h, values, values_on_device, stream, h->precision == 1);
}

int glu_refactor(glu_handle* h, const double* values, int values_on_device, void* stream) {
    if (!h) return GLU_ERR_ARG;
    if (!h->factored_once) return GLU_ERR_STATE;
    h->fp64_fallback = 0;
    return run_factor(h, values, values_on_device, stream, h->precision == 1);
}

int glu_solve(glu_handle* h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx, int on_device,
              void* stream) {
    if (!h || nrhs < 0 || (nrhs > 0 && (!b || !x))) return GLU_ERR_ARG;
    if (h->state != FACTORED) return GLU_ERR_STATE;
    const glu::Analysis& a = h->an;
    const int32_t n = a.n;
    if (ldb < n || ldx < n) return GLU_ERR_ARG;
    if (nrhs == 0 || n == 0) return GLU_OK;
    int rc = set_device(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t need = (size_t)n * nrhs;
    SolveScratch sc;
    rc = solve_scratch(h, nrhs, sc);
    if (rc) return rc;
    const double* db = b;
    if (!on_device) {
        if (h->bstage.n < need && h->bstage.alloc(need) != hipSuccess) return GLU_ERR_NOMEM;
        for (int32_t r = 0; r < nrhs; r++)
            if (hipMemcpyAsync(h->bstage.p + (size_t)r * n, b + (size_t)r * ldb, n * sizeof(double),
                               hipMemcpyHostToDevice, st) != hipSuccess)
                return GLU_ERR_DEVICE;
        db = h->bstage.p;
    }
    const bool refine = h->precision == 1;
    if (refine && !on_device && h->xstage.n < need && h->xstage.alloc(need) != hipSuccess) return GLU_ERR_NOMEM;
    double* dx = on_device ? x : (refine ? h->xstage.p : h->bstage.p);
    const int64_t dldb = on_device ? ldb : n, dldx = on_device ? ldx : n;
    if (refine && on_device && (const double*)x == b) return GLU_ERR_ARG;  // refinement re-reads b
    rc = run_solve(h, nrhs, db, dldb, dx, dldx, sc, st);
    if (rc) return rc;
    if (refine) {
        rc = finish_solve(h, st);
        if (rc) return rc;
        rc = refine_solution(h, nrhs, db, dldb, dx, dldx, sc, st);
        if (rc) return rc;
    }
    if (!on_device) {
        for (int32_t r = 0; r < nrhs; r++)
            if (hipMemcpyAsync(x + (size_t)r * ldx, dx + (size_t)r * n, n * sizeof(double),
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                return GLU_ERR_DEVICE;
    }
    return finish_solve(h, st);
}

int glu_solve_noalloc(glu_handle* h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                      void* stream) {
    if (!h || nrhs < 0 || (nrhs > 0 && (!b || !x))) return GLU_ERR_ARG;
    if (h->state != FACTORED) return GLU_ERR_STATE;
    const glu::Analysis& a = h->an;
    const int32_t n = a.n;
    if (ldb < n || ldx < n || h->precision == 1) return GLU_ERR_ARG;  // the mixed form refines: workspace
    if (nrhs == 0 || n == 0) return GLU_OK;
    const int64_t nr = (int64_t)n * nrhs;
    const int64_t ncross = (int64_t)(a.cross_row.size() + a.ux_q0.size()) * nrhs, ndm = (int64_t)a.tail_m * nrhs;
    const int64_t need = 2 * lines(nr) + lines(ncross) + lines(ndm);
    if (need > kNoAllocScratchDoubles) return GLU_ERR_SCRATCH;
    int rc = set_device(h);
    if (rc) return rc;
    double* base = nullptr;
    rc = scratch_on_device(h->device, &base);
    if (rc) return rc;
    SolveScratch sc{base, base + lines(nr), base + 2 * lines(nr), base + 2 * lines(nr) + lines(ncross)};
    hipStream_t st = (hipStream_t)stream;
    rc = run_solve(h, nrhs, b, ldb, x, ldx, sc, st);
    if (rc) return rc;
    return finish_solve(h, st);
}

int64_t glu_solve_noalloc_capacity(void) { return kNoAllocScratchDoubles; }

void glu_batch_destroy(glu_batch* b) {
    if (!b) return;
    if (b->device >= 0) {
        (void)hipSetDevice(b->device);
        (void)hipDeviceSynchronize();
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        for (hipStream_t t : b->tails)
            if (t) (void)hipStreamDestroy(t);
        if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
        for (hipEvent_t e : b->ev_done)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : {b->ev_levels, b->ev0, b->ev1, b->ev2})
            if (e) (void)hipEventDestroy(e);
        b->args.release();
        b->ent.release();
        if (b->hnorm) (void)hipHostFree(b->hnorm);
        if (b->hstat) (void)hipHostFree(b->hstat);
        if (b->hstat3) (void)hipHostFree(b->hstat3);
    }
    delete b;
}

int glu_batch_create(glu_batch** out, glu_handle* const* handles, int32_t count) {
    if (!out) return GLU_ERR_ARG;
    *out = nullptr;
    if (!handles || count <= 0) return GLU_ERR_ARG;
    const int dev = handles[0] ? handles[0]->device : -1;
    for (int32_t i = 0; i < count; i++) {
        const glu_handle* h = handles[i];
        if (!h || h->device < 0 || h->device != dev || h->precision != handles[0]->precision) return GLU_ERR_ARG;
        if (h->state == EMPTY) return GLU_ERR_STATE;
        for (int32_t k = 0; k < i; k++)
            if (handles[k] == h) return GLU_ERR_ARG;
    }
    if (hipSetDevice(dev) != hipSuccess) return GLU_ERR_DEVICE;
    glu_batch* b = new (std::nothrow) glu_batch();
    if (!b) return GLU_ERR_NOMEM;
    b->device = dev;
    b->fp32 = handles[0]->precision == 1;
    b->hs.assign(handles, handles + count);
    std::vector<glu::FactorArgs> fa;
    for (glu_handle* h : b->hs) {
        fa.push_back(h->fargs(b->fp32));
        b->serial.push_back(h->analysis_serial);
    }
    // wavefront tables: entry (e, h) for every handle with an executed level e
    int32_t nwf = 0;
    for (glu_handle* h : b->hs) nwf = std::max(nwf, (int32_t)h->an.exec_ptr.size() - 1);
    std::vector<glu::BatchEntry> ent;
    b->wf_ent.assign(1, 0);
    for (int32_t e = 0; e < nwf; e++) {
        int64_t boff = 0;
        for (int32_t i = 0; i < count; i++) {
            const glu::Analysis& an = b->hs[i]->an;
            const int32_t nexec = (int32_t)an.exec_ptr.size() - 1;
            if (e >= nexec) continue;
            glu::BatchEntry x;
            x.boff = boff;
            x.wi0 = an.wi_ptr[e];
            x.nwi = an.wi_ptr[e + 1] - an.wi_ptr[e];
            x.norm = e > 0 ? b->hs[i]->exec_cols.p + an.exec_ptr[e - 1] : nullptr;
            x.nnorm = e > 0 ? an.exec_ptr[e] - an.exec_ptr[e - 1] : 0;
            x.h = i;
            if (x.nwi + x.nnorm == 0) continue;
            ent.push_back(x);
            boff += x.nwi + x.nnorm;
        }
        b->wf_ent.push_back((int64_t)ent.size());
        b->wf_blocks.push_back(boff);
    }
    hipError_t e = upload(b->args, fa);
    if (e == hipSuccess) e = upload(b->ent, ent);
    const int ntail = std::min<int32_t>(count, 8);
    b->tails.assign(ntail, nullptr);
    for (int i = 0; i < ntail && e == hipSuccess; i++) e = hipStreamCreateWithFlags(&b->tails[i], hipStreamNonBlocking);
    b->ev_done.assign(ntail, nullptr);
    for (int i = 0; i < ntail && e == hipSuccess; i++)
        e = hipEventCreateWithFlags(&b->ev_done[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_levels, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e == hipSuccess) e = hipEventCreate(&b->ev2);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    // capture the wavefront launches once; replays launch them all
    if (e == hipSuccess && nwf > 0) {
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int32_t w = 0; ok && w < nwf; w++)
            ok = glu::launch_level_batch(b->args.p, b->ent.p + b->wf_ent[w], (int32_t)(b->wf_ent[w + 1] - b->wf_ent[w]),
                                         b->wf_blocks[w], b->fp32, b->capture_stream) == hipSuccess;
        const bool ended = hipStreamEndCapture(b->capture_stream, &g) == hipSuccess;
        if (ok && ended && g && hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0) != hipSuccess) b->graph = nullptr;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();  // a failed capture leaves direct launches in use
    }
    if (e == hipSuccess &&
        hipHostMalloc((void**)&b->hstat3, (size_t)count * 3 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        b->hstat3 = nullptr;
        e = hipErrorOutOfMemory;
    }
    if (e != hipSuccess) {
        glu_batch_destroy(b);
        return GLU_ERR_DEVICE;
    }
    *out = b;
    return GLU_OK;
}

// Run work(t) for every batch stream t, each from a host thread of its own
// (the launches of different streams then do not queue behind one another
// on one thread); the first nonzero status, if any.
static int on_batch_streams(const glu_batch* b, const std::function<int(int)>& work) {
    const int ntail = (int)b->tails.size();
    std::vector<int> rc(ntail, GLU_OK);
    std::vector<std::thread> th;
    th.reserve(ntail);
    for (int t = 0; t < ntail; t++)
        th.emplace_back([&, t] { rc[t] = hipSetDevice(b->device) == hipSuccess ? work(t) : GLU_ERR_DEVICE; });
    for (std::thread& x : th) x.join();
    for (int r : rc)
        if (r) return r;
    return GLU_OK;
}

int glu_batch_factor(glu_batch* b, const double* const* values, int values_on_device, void* stream) {
    if (!b || !values) return GLU_ERR_ARG;
    const int32_t count = (int32_t)b->hs.size();
    for (int32_t i = 0; i < count; i++) {
        if (!values[i]) return GLU_ERR_ARG;
        if (b->hs[i]->analysis_serial != b->serial[i] || b->hs[i]->state == EMPTY) return GLU_ERR_STATE;
    }
    if (hipSetDevice(b->device) != hipSuccess) return GLU_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    if (hipEventRecord(b->ev0, st) != hipSuccess) return GLU_ERR_DEVICE;
    for (int32_t i = 0; i < count; i++) {
        b->hs[i]->fp64_fallback = 0;
        const int rc = factor_begin(b->hs[i], values[i], values_on_device, st, b->fp32);
        if (rc) return rc;
    }
    if (hipEventRecord(b->ev2, st) != hipSuccess) return GLU_ERR_DEVICE;
    const int32_t nwf = (int32_t)b->wf_blocks.size();
    if (b->graph) {
        if (hipGraphLaunch(b->graph, st) != hipSuccess) return GLU_ERR_DEVICE;
    } else {
        for (int32_t w = 0; w < nwf; w++)
            if (glu::launch_level_batch(b->args.p, b->ent.p + b->wf_ent[w], (int32_t)(b->wf_ent[w + 1] - b->wf_ent[w]),
                                        b->wf_blocks[w], b->fp32, st) != hipSuccess)
                return GLU_ERR_DEVICE;
    }
    if (hipEventRecord(b->ev_levels, st) != hipSuccess || hipEventRecord(b->ev1, st) != hipSuccess)
        return GLU_ERR_DEVICE;
    // the rest of each factorization (dense block, last normalisation, pivot
    // check, value gather) on a few side streams, so that the dense blocks of
    // different handles overlap
    const int ntail = (int)b->tails.size();
    int rct = on_batch_streams(b, [&](int t) -> int {
        if (hipStreamWaitEvent(b->tails[t], b->ev_levels, 0) != hipSuccess) return GLU_ERR_DEVICE;
        for (int32_t i = t; i < count; i += ntail) {
            const int rc = factor_end(b->hs[i], b->tails[t], b->fp32, true);
            if (rc) return rc;
        }
        return hipEventRecord(b->ev_done[t], b->tails[t]) == hipSuccess ? GLU_OK : GLU_ERR_DEVICE;
    });
    if (rct) return rct;
    for (int t = 0; t < ntail; t++)
        if (hipStreamWaitEvent(st, b->ev_done[t], 0) != hipSuccess) return GLU_ERR_DEVICE;
    // every handle's status words, one synchronisation
    for (int32_t i = 0; i < count; i++)
        if (hipMemcpyAsync(b->hstat3 + 3 * i, b->hs[i]->status.p, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return GLU_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return GLU_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, b->ev2, b->ev1) == hipSuccess) b->t_levels_ms = ms;
    int first = GLU_OK;
    for (int32_t i = 0; i < count; i++) {
        const int rc = factor_status(b->hs[i], b->hstat3 + 3 * i, b->fp32);
        if (rc && first == GLU_OK) first = rc;
    }
    if (hipEventRecord(b->ev1, st) != hipSuccess || hipEventSynchronize(b->ev1) != hipSuccess) return GLU_ERR_DEVICE;
    if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) b->t_total_ms = ms;
    return first;
}

int glu_batch_solve(glu_batch* b, int32_t nrhs, const double* const* bs, const int64_t* ldb, double* const* xs,
                    const int64_t* ldx, void* stream) {
    if (!b || nrhs < 0 || (nrhs > 0 && (!bs || !xs || !ldb || !ldx))) return GLU_ERR_ARG;
    const int32_t count = (int32_t)b->hs.size();
    for (int32_t i = 0; i < count && nrhs > 0; i++) {
        const glu_handle* h = b->hs[i];
        if (h->analysis_serial != b->serial[i] || h->state != FACTORED) return GLU_ERR_STATE;
        const int32_t n = h->an.n;
        if (ldb[i] < n || ldx[i] < n || (n > 0 && (!bs[i] || !xs[i]))) return GLU_ERR_ARG;
        if (b->fp32 && n > 0 && (const double*)xs[i] == bs[i]) return GLU_ERR_ARG;  // refinement re-reads b
    }
    if (nrhs == 0) return GLU_OK;
    if (hipSetDevice(b->device) != hipSuccess) return GLU_ERR_DEVICE;
    const size_t per = 1 + 2 * (size_t)nrhs;
    if (b->hnorm_n < per * count) {
        if (b->hnorm) (void)hipHostFree(b->hnorm);
        b->hnorm = nullptr;
        b->hnorm_n = 0;
        if (hipHostMalloc((void**)&b->hnorm, per * count * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return GLU_ERR_NOMEM;
        b->hnorm_n = per * count;
    }
    if (!b->hstat && hipHostMalloc((void**)&b->hstat, (size_t)count * sizeof(int32_t), hipHostMallocDefault) !=
                         hipSuccess) {
        b->hstat = nullptr;
        return GLU_ERR_NOMEM;
    }
    std::vector<SolveScratch> sc(count);
    for (int32_t i = 0; i < count; i++) {
        int rc = solve_scratch(b->hs[i], nrhs, sc[i]);
        if (!rc && b->fp32) rc = refine_scratch(b->hs[i], nrhs);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    const int ntail = (int)b->tails.size();
    if (hipEventRecord(b->ev0, st) != hipSuccess) return GLU_ERR_DEVICE;
    // every handle's solve and refinement on its batch stream, each stream
    // driven by a host thread of its own: the mixed form's refinement rounds of
    // one stream's handles (their residuals, one synchronisation of that
    // stream, then a correction solve for those above the tolerance) do not
    // wait for the other streams
    const int rct = on_batch_streams(b, [&](int t) -> int {
        hipStream_t ts = b->tails[t];
        if (hipStreamWaitEvent(ts, b->ev0, 0) != hipSuccess) return GLU_ERR_DEVICE;
        std::vector<int32_t> open, next, stalled;
        for (int32_t i = t; i < count; i += ntail) {
            glu_handle* h = b->hs[i];
            h->refine_iters = 0;
            h->refine_berr = 0.0;
            if (h->an.n == 0) continue;
            const int rc = run_solve(h, nrhs, bs[i], ldb[i], xs[i], ldx[i], sc[i], ts);
            if (rc) return rc;
            open.push_back(i);
        }
        while (b->fp32 && !open.empty()) {
            for (int32_t i : open) {
                glu_handle* h = b->hs[i];
                if (glu::launch_residual(h->an.n, nrhs, h->arow_ptr.p, h->arow_col.p, h->arow_pos.p, h->avals.p, bs[i],
                                         ldb[i], xs[i], ldx[i], h->rbuf.p, h->norms.p, ts) != hipSuccess ||
                    hipMemcpyAsync(b->hnorm + per * i, h->norms.p, per * sizeof(double), hipMemcpyDeviceToHost, ts) !=
                        hipSuccess)
                    return GLU_ERR_DEVICE;
            }
            if (hipStreamSynchronize(ts) != hipSuccess) return GLU_ERR_DEVICE;
            next.clear();
            for (int32_t i : open) {
                glu_handle* h = b->hs[i];
                const double be = backward_error(b->hnorm + per * i, nrhs);
                h->refine_berr = be;
                if (be <= h->refine_tol) continue;
                if (h->refine_iters >= h->refine_max || !std::isfinite(be)) {
                    stalled.push_back(i);
                    continue;
                }
                const int32_t n = h->an.n;
                const int rc = run_solve(h, nrhs, h->rbuf.p, n, h->dbuf.p, n, sc[i], ts);
                if (rc) return rc;
                if (glu::launch_axpy_update(n, nrhs, h->dbuf.p, xs[i], ldx[i], ts) != hipSuccess)
                    return GLU_ERR_DEVICE;
                h->refine_iters++;
                next.push_back(i);
            }
            open.swap(next);
        }
        // handles whose refinement stalled: refactorize in FP64 on the same
        // plan and values, then solve and refine with those factors
        for (int32_t i : stalled) {
            glu_handle* h = b->hs[i];
            int rc = run_factor(h, h->avals.p, 1, ts, false);
            if (!rc) {
                h->fp64_fallback = 1;
                rc = run_solve(h, nrhs, bs[i], ldb[i], xs[i], ldx[i], sc[i], ts);
            }
            if (!rc) rc = refine_solution(h, nrhs, bs[i], ldb[i], xs[i], ldx[i], sc[i], ts);
            if (rc) return rc;
        }
        // the solve kernels' error flags
        for (int32_t i = t; i < count; i += ntail) {
            b->hstat[i] = 0;
            if (b->hs[i]->an.n > 0 && hipMemcpyAsync(b->hstat + i, b->hs[i]->status.p + 2, sizeof(int32_t),
                                                     hipMemcpyDeviceToHost, ts) != hipSuccess)
                return GLU_ERR_DEVICE;
        }
        return hipEventRecord(b->ev_done[t], ts) == hipSuccess ? GLU_OK : GLU_ERR_DEVICE;
    });
    if (rct) return rct;
    for (int t = 0; t < ntail; t++)
        if (hipStreamWaitEvent(st, b->ev_done[t], 0) != hipSuccess) return GLU_ERR_DEVICE;
    if (hipEventRecord(b->ev1, st) != hipSuccess || hipEventSynchronize(b->ev1) != hipSuccess) return GLU_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) b->t_solve_ms = ms;
    for (int32_t i = 0; i < count; i++)
        if (b->hstat[i]) return GLU_ERR_DEVICE;
    return GLU_OK;
}

int glu_batch_query(const glu_batch* b, int32_t* count, int32_t* n_wavefronts, int32_t* captured,
                    double* t_levels_ms, double* t_total_ms, double* t_solve_ms) {
    if (!b) return GLU_ERR_ARG;
    if (count) *count = (int32_t)b->hs.size();
    if (n_wavefronts) *n_wavefronts = (int32_t)b->wf_blocks.size();
    if (captured) *captured = b->graph != nullptr;
    if (t_levels_ms) *t_levels_ms = b->t_levels_ms;
    if (t_total_ms) *t_total_ms = b->t_total_ms;
    if (t_solve_ms) *t_solve_ms = b->t_solve_ms;
    return GLU_OK;
}

int glu_query(const glu_handle* h, glu_info* out) {
    if (!h || !out) return GLU_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    const glu::Analysis& a = h->an;
    if (h->state == EMPTY) return GLU_ERR_STATE;
    out->n = a.n;
    out->n_levels = (int32_t)a.level_ptr.size() - 1;
    out->nnz_a = a.nnz_a;
    out->nnz_lu = (int64_t)a.lu_rowind.size();
    out->nnz_l = a.nnz_l;
    out->nnz_u = a.nnz_u;
    out->n_dag_edges = (int64_t)a.dag_idx.size();
    out->macs = a.macs;
    for (int m = 0; m < 3; m++) out->n_levels_mode[m] = a.levels_per_mode[m];
    out->widest_level = a.widest;
    out->n_tasks = (int64_t)a.task_col.size();
    out->n_work_items = (int64_t)a.wi_task.size();
    out->n_solve_levels_l = a.fsolve_ptr.empty() ? 0 : (int32_t)a.fsolve_ptr.size() - 1;
    out->n_solve_levels_u = a.bsolve_ptr.empty() ? 0 : (int32_t)a.bsolve_ptr.size() - 1;
    out->tail_m = a.tail_m;
    out->n_exec_levels = a.exec_ptr.empty() ? 0 : (int32_t)a.exec_ptr.size() - 1;
    out->device_bytes = h->device_bytes();
    out->t_order_ms = a.t_order_ms;
    out->t_symbolic_ms = a.t_symbolic_ms;
    out->t_levels_ms = a.t_levels_ms;
    out->t_plan_ms = a.t_plan_ms;
    out->t_factor_ms = h->t_factor_ms;
    out->t_solve_ms = h->t_solve_ms;
    out->t_update_ms = h->t_update_ms;
    out->t_dense_ms = h->t_dense_ms;
    out->t_schur_ms = h->t_schur_ms;
    out->schur_macs = a.sch_macs;
    out->schur_steps = (int64_t)a.sch_pair_l.size();
    out->schur_tiles = (int64_t)a.sch_units.size();
    out->level_macs = a.n_pairs;
    out->tail_macs = a.tail_macs;
    out->level_nl = a.level_nl;
    out->level_nu = a.level_nu;
    out->precision = h->precision;
    out->refine_iters = h->refine_iters;
    out->fp64_fallback = h->fp64_fallback;
    out->refine_berr = h->refine_berr;
    return GLU_OK;
}

int glu_export_symbolic(const glu_handle* h, int32_t* perm, int64_t* lu_colptr, int32_t* lu_rowind,
                        int64_t* dag_ptr, int32_t* dag_idx, int32_t* level_ptr, int32_t* level_cols) {
    if (!h) return GLU_ERR_ARG;
    if (h->state == EMPTY) return GLU_ERR_STATE;
    const glu::Analysis& a = h->an;
    auto cp = [](auto* dst, const auto& v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(perm, a.perm);
    cp(lu_colptr, a.lu_colptr);
    cp(lu_rowind, a.lu_rowind);
    cp(dag_ptr, a.dag_ptr);
    cp(dag_idx, a.dag_idx);
    cp(level_ptr, a.level_ptr);
    cp(level_cols, a.level_cols);
    return GLU_OK;
}

int glu_export_factors(const glu_handle* h, double* lu_values) {
    if (!h || !lu_values) return GLU_ERR_ARG;
    if (h->state != FACTORED) return GLU_ERR_STATE;
    if (set_device(h) != GLU_OK) return GLU_ERR_DEVICE;
    size_t nnz = h->an.lu_rowind.size();
    // the dense block's factors into A_s first (the factorization leaves them in the block)
    if (h->an.tail_m > 0 && (glu::launch_tail_scatter(h->fargs(), h->tail_pos.p, h->an.tail_start, h->an.tail_m,
                                                      h->dense.p, h->dense_ld, nullptr) != hipSuccess ||
                             hipDeviceSynchronize() != hipSuccess))
        return GLU_ERR_DEVICE;
    if (nnz && hipMemcpy(lu_values, h->val.p, nnz * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return GLU_ERR_DEVICE;
    return GLU_OK;
}

int glu_mc64(int32_t n, const int64_t* colptr, const int32_t* rowind, const double* values, int32_t* row_perm,
             double* row_scale, double* col_scale) {
    if (n < 0 || (n > 0 && (!colptr || !rowind || !values || !row_perm || !row_scale || !col_scale)))
        return GLU_ERR_ARG;
    try {
        std::vector<int32_t> m;
        std::vector<double> dr, dc;
        const glu::Status st = glu::mc64_scale(n, colptr, rowind, values, m, dr, dc);
        if (st != glu::Status::ok) return static_cast<int>(st);
        std::copy(m.begin(), m.end(), row_perm);
        std::copy(dr.begin(), dr.end(), row_scale);
        std::copy(dc.begin(), dc.end(), col_scale);
        return GLU_OK;
    } catch (const std::bad_alloc&) {
        return GLU_ERR_NOMEM;
    } catch (...) {
        return GLU_ERR_ARG;
    }
}

int32_t glu_failed_column(const glu_handle* h) { return h ? h->failed_col : -1; }

void glu_destroy(glu_handle* h) {
    if (!h) return;
    if (h->device >= 0) {
        (void)hipSetDevice(h->device);
        if (h->aux) (void)hipStreamSynchronize(h->aux);
        if (h->side) (void)hipStreamSynchronize(h->side);
        h->release_device();
        for (hipEvent_t e : {h->ev0, h->ev1, h->ev2, h->ev3, h->ev4, h->ev_fork, h->ev_join, h->ev_gfork, h->ev_gjoin})
            if (e) (void)hipEventDestroy(e);
        if (h->aux) (void)hipStreamDestroy(h->aux);
        if (h->side) (void)hipStreamDestroy(h->side);
        glu::dense_blas_destroy(h->blas);
    }
    delete h;
}

}  // extern "C"
