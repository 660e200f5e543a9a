// Host-side analysis: ordering, symbolic fill, relaxed dependency DAG,
// levelization and the per-level kernel plan that the HIP kernels execute.
#pragma once

#include <cstdint>
#include <vector>

namespace glu {

enum class Status : int {
    ok = 0,
    arg = -1,
    state = -2,
    zero_pivot = -3,
    struct_singular = -4,
    nomem = -5,
    device = -6,
    nonfinite = -7,
};

// Validate a CSC pattern: colptr[0] == 0, nondecreasing, rows in range and
// strictly increasing within each column.
Status validate_csc(int32_t n, const int64_t* colptr, const int32_t* rowind);

// Maximum-product transversal with row and column scaling (MC64 of the
// paper's preprocessing, Section II-C).  row_of_col[j] is the row of A matched
// to column j; Dr A Dc has every magnitude <= 1 and the matched ones 1.
Status mc64_scale(int32_t n, const int64_t* colptr, const int32_t* rowind, const double* values,
                  std::vector<int32_t>& row_of_col, std::vector<double>& rscale, std::vector<double>& cscale);

// Approximate minimum degree ordering of the pattern of A + A^T (perm[new] = old).
std::vector<int32_t> amd_order(int32_t n, const int64_t* colptr, const int32_t* rowind);

// Kernel modes of the paper's Section III-B, per level.
enum Mode : int32_t { MODE_SMALL = 0, MODE_LARGE = 1, MODE_STREAM = 2 };

// Entries of one work item of the forward-solve cross term.
constexpr int32_t CROSS_CHUNK = 2048;

// Tile edge of the Schur-complement update of the dense block.
constexpr int32_t SCH_TS = 16;
// Tiles with at least this many pairs get a whole workgroup in the update.
constexpr int64_t SCH_HEAVY = 4096;
// XCDs of the GPU (each with its own L2); the update's tiles are grouped by it.
constexpr int SCH_XCDS = 8;

// One tile of the Schur-complement update: rows [i0, i0 + SCH_TS) and columns
// [k0, k0 + SCH_TS) of the dense block, the pair range [pb, pe) and the first
// double of its row tile's L panel and its column tile's U panel.
struct SchurUnit {
    int32_t i0, k0;
    int64_t pb, pe;
    int64_t lbase, ubase;
};

// Dependency DAG + levels computed elsewhere (the device): returns 0 on
// success; same outputs as the host steps.
using DagLevelsFn = int (*)(int32_t n, const std::vector<int64_t>& lu_colptr, const std::vector<int32_t>& lu_rowind,
                            const std::vector<int64_t>& diag, std::vector<int64_t>& dag_ptr,
                            std::vector<int32_t>& dag_idx, std::vector<int32_t>& level_of, int32_t* spin_err);

struct PlanParams {
    DagLevelsFn dag_levels = nullptr;  // null: the host computes the DAG and levels
    int32_t force_mode = -1;         // -1 auto, else a Mode
    int32_t stream_threshold = -1;   // width <= this: stream mode (-1: none)
    int32_t large_threshold = -1;    // width <= this (and > stream): large-block mode (-1: none)
    int32_t chunk_small = 256;       // max target entries staged per work item, per mode
    int32_t chunk_large = 1024;
    int32_t chunk_stream = 512;
    int32_t stream_min_run = 2;      // shortest run of stream levels given one persistent launch
    bool xcd_items = true;           // group a level's items by XCD (shared first source column)
    // dense trailing block: 0 = chosen by the cost model, < 0 = never,
    // > 0 = exactly this many trailing columns
    int32_t dense_tail = 0;
};

struct Analysis {
    int32_t n = 0;
    int64_t nnz_a = 0;
    std::vector<int32_t> perm, pinv;  // perm[new] = old, pinv[old] = new

    // Filled pattern A_s of B = P A P^T (CSC, rows ascending).
    std::vector<int64_t> lu_colptr;
    std::vector<int32_t> lu_rowind;
    std::vector<int64_t> diag;        // position of A_s(j,j)
    std::vector<int64_t> amap;        // A entry p -> position in A_s

    // Relaxed dependency DAG (Alg. 4) and levels.
    std::vector<int64_t> dag_ptr;
    std::vector<int32_t> dag_idx;
    std::vector<int32_t> level_of, level_ptr, level_cols;

    // Row views: L rows (for the forward solve), U rows (subcolumns of each column).
    std::vector<int64_t> lrow_ptr, lrow_pos;
    std::vector<int32_t> lrow_col;
    std::vector<int64_t> urow_ptr, urow_pos;
    std::vector<int32_t> urow_col;

    // Dense trailing block: columns [tail_start, n) are factorized as one dense
    // m x m block once every column before it has applied its update
    // (m = n - tail_start, 0 when there is no dense tail).
    int32_t tail_start = 0;
    int32_t tail_m = 0;
    std::vector<int64_t> tail_pos;        // [c] first position of column t+c with row >= t
    // The entries of A inside the block (the block's initial values): A_s
    // position, local row and local column, in A's order.  The block is built
    // from these alone (zeros elsewhere), so the value load need not clear the
    // rest of the block's part of A_s.
    std::vector<int64_t> tail_asrc;
    std::vector<int32_t> tail_arow, tail_acol;
    std::vector<int64_t> tail_lsplit;     // [c] first lrow entry of row t+c with column >= t
    // Forward-solve cross term of the tail rows, y(t+c) -= L(t+c, 0:t) y(0:t),
    // cut into work items of at most CROSS_CHUNK entries: row tail c owns items
    // [cross_ptr[c], cross_ptr[c+1]), item w starts at lrow entry cross_q0[w].
    std::vector<int32_t> cross_ptr;
    std::vector<int32_t> cross_row;
    std::vector<int64_t> cross_q0;
    // Backward-solve cross term of the rows before the tail, y(j) -= U(j, t:n)
    // x(t:n), applied in parallel once the tail is solved (the backward walk
    // then visits only the entries in columns < t): the entries row by row
    // (ux_pos: positions in A_s, ux_col: columns), cut into work items of at
    // most CROSS_CHUNK entries [ux_q0[w], ux_q1[w]); row ux_row[c] owns items
    // [ux_ptr[c], ux_ptr[c+1]).
    std::vector<int32_t> ux_ptr, ux_row, ux_col;
    std::vector<int64_t> ux_q0, ux_q1, ux_pos;

    // Executed sparse levels: the levels restricted to columns < tail_start
    // (empty restrictions dropped), ascending columns.
    std::vector<int32_t> exec_ptr, exec_cols;

    // Numeric plan: per executed level, update tasks (level, target column k)
    // with their sources (U entries of column k whose row j is in the level),
    // and work items (task, range of column-k positions staged by one workgroup).
    std::vector<int32_t> level_mode;
    std::vector<int64_t> task_ptr;        // [level] -> first task
    std::vector<int32_t> task_col;        // target column k
    std::vector<int64_t> task_src_ptr;    // [task] -> first source
    std::vector<int64_t> src_upos;        // position of U(j,k) in A_s (row j is the source)
    std::vector<int64_t> src_dpos;        // position of the source's pivot A_s(j,j)
    std::vector<int32_t> src_llen;        // |L(:,j)| of the source
    std::vector<int64_t> wi_ptr;          // [level] -> first work item
    std::vector<int32_t> wi_task;
    std::vector<int64_t> wi_begin, wi_end;
    // Work items that cover only part of their task's target range list the
    // sources whose L rows fall in the slice, ascending: entries
    // [wi_ss[w], wi_ss[w] + wi_nsrc[w]) of ss_src (source offset within the
    // task) and ss_lo/ss_hi (sub-range of L(:,j) as offsets from its first L
    // entry).  Within a level, work items are ordered by decreasing pair count.
    // wi_whole[w] = 1 when the slice covers every row the task touches (then
    // all sources apply with their whole L columns and the list is empty).
    std::vector<int64_t> wi_ss;
    std::vector<int8_t> wi_whole;
    std::vector<int32_t> ss_src, ss_lo, ss_hi;
    // What a work item needs without a second dependent load: the task's first
    // source (wi_s0), the number of sources it applies (wi_nsrc), and for
    // listed sources the positions of U(j,k) and of the pivot (ss_up, ss_dp).
    std::vector<int64_t> wi_s0;
    std::vector<int32_t> wi_nsrc;
    std::vector<int64_t> ss_up, ss_dp;
    // Per work item: the first index of its (source, L-row) pairs in the
    // pair-position map (wi_pbase) and the first slot of its touched-entry
    // list (wi_tbase; room for min(slice length, pairs) entries).  The maps
    // themselves are built on the device at analysis: the slice entries that
    // some pair updates (offsets from the slice start, ascending) and, for
    // every pair in the level kernel's order, the index of its target there.
    std::vector<int64_t> wi_pbase, wi_tbase;
    int64_t n_pairs = 0, n_touch_cap = 0;

    // Stream-mode runs: maximal runs of at least two consecutive executed
    // levels in stream mode, each run in one persistent launch.  Run r covers
    // executed levels [run_e0[r], run_e1[r]) and segments [run_sb[r],
    // run_sb[r] + run_e1[r] - run_e0[r]] of the segment arrays: segment s of
    // the run (level e = run_e0 + s) is the level's work items (the first is
    // seg_wi[s], the count seg_wi[s+1] - seg_wi[s]) followed by the columns of
    // level e-1 to normalise (exec_cols from seg_norm[s]); seg_start[s] is the
    // segment's first item index within the run (seg_start[nseg] = items).
    std::vector<int32_t> run_e0, run_e1;
    std::vector<int64_t> run_sb;
    std::vector<int64_t> seg_start, seg_wi;
    std::vector<int32_t> seg_norm;

    // Schur-complement update of the dense block from the sparse columns,
    // S = A_s(t:n, t:n) - L(t:n, 0:t) U(0:t, t:n), applied after the sparse
    // levels (no sparse level reads or writes the block, so its updates can
    // wait).  The block is cut into SCH_TS x SCH_TS tiles.  Row tile I keeps a
    // dense panel of the L entries in its rows, one SCH_TS-wide row per source
    // column j that has any (ascending j); column tile K keeps the same for U.
    // A tile's update walks the sources present in both its panels in
    // ascending j (pairs of panel row indices), so every entry of the block
    // receives its products in ascending source order.
    std::vector<int64_t> sch_lpos, sch_loff;  // L entry position in A_s -> offset in the L panels
    std::vector<int64_t> sch_upos, sch_uoff;  // U entry position -> offset in the U panels
    int64_t sch_lp_len = 0, sch_up_len = 0;   // panel sizes (doubles)
    std::vector<SchurUnit> sch_units;         // nonempty tiles, most pairs first
    int64_t sch_nheavy = 0;                   // leading units with at least SCH_HEAVY pairs
    std::vector<int32_t> sch_pair_l, sch_pair_u;
    int64_t sch_macs = 0;                     // nonzero products of the update

    // Solve schedules over rows < tail_start: forward levels over rows of L,
    // backward levels over rows of U.
    std::vector<int32_t> fsolve_ptr, fsolve_rows;
    std::vector<int32_t> bsolve_ptr, bsolve_rows;
    // The solves' factor entries in schedule order: slot w (the w-th row of
    // fsolve_rows / bsolve_rows) owns entries [fs_ptr[w], fs_ptr[w+1]) of L's
    // row (columns before it) or [bs_ptr[w], bs_ptr[w+1]) of U's row (columns
    // after it); *_pos is the entry's position in A_s (its value is gathered
    // there after every factorization) and *_col its column.
    std::vector<int64_t> fs_ptr, fs_pos, bs_ptr, bs_pos;
    std::vector<int32_t> fs_col, bs_col;

    int64_t nnz_l = 0, nnz_u = 0, macs = 0;
    // products whose source and target lie in the dense block, and the L / U
    // entries of the columns / rows before it
    int64_t tail_macs = 0, level_nl = 0, level_nu = 0;
    int32_t widest = 0;
    int32_t levels_per_mode[3] = {0, 0, 0};
    double t_order_ms = 0, t_symbolic_ms = 0, t_levels_ms = 0, t_plan_ms = 0;
    int32_t bad_col = -1;
};

// The whole host analysis.  perm_in: NULL for AMD / natural, else user perm.
Status analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, int ordering,
               const int32_t* perm_in, const PlanParams& pp, Analysis& out);

}  // namespace glu
