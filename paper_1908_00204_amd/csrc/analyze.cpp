// Host analysis for the levelized right-looking factorization.
//
//  * symbolic fill of B = P A P^T without pivoting: for each column j, the
//    rows reachable from struct(B(:,j)) through the graph of L's earlier
//    columns (Section II-A: the symbolic analysis that precedes Alg. 1/Alg. 2),
//    by depth-first search with symmetric pruning (Eisenstat and Liu): once
//    L(j,i) and U(i,j) are both nonzero, every row of L(:,i) below j is also a
//    row of L(:,j), so later searches only need L(:,i)'s rows up to j;
//  * relaxed dependency detection (Alg. 4): column k depends on i < k when
//    A_s(i,k) != 0 and L(:,i) has an entry below the diagonal ("look up"), or
//    when A_s(k,i) != 0 ("look left");
//  * levelization (Section II-C): level(k) = 1 + max level of its dependencies;
//  * the level plan executed by the kernels (Section III-B): per level, the
//    submatrix update of Alg. 5 regrouped by target column, one of the three
//    kernel modes chosen by the level's width, and the solve schedules.
#include "analyze.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <functional>
#include <numeric>
#include <thread>

namespace glu {

namespace {

// First position in [first, last) whose value is >= key (or > key when
// strict), searched by doubling steps from `first`: cheap when the answer is
// near the start, as it is for cursors that only move forward.
const int32_t* gallop(const int32_t* first, const int32_t* last, int32_t key, bool strict) {
    auto before = [&](int32_t v) { return strict ? v <= key : v < key; };
    if (first >= last || !before(*first)) return first;
    std::ptrdiff_t lo = 0, step = 1, n = last - first;
    while (lo + step < n && before(first[lo + step])) {
        lo += step;
        step <<= 1;
    }
    const int32_t* b = first + lo + 1;
    const int32_t* e = first + std::min(n, lo + step + 1);
    return strict ? std::upper_bound(b, e, key) : std::lower_bound(b, e, key);
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Progress of a long analysis on stderr, one line per finished step, when the
// environment sets GLU_VERBOSE (a million-column analysis takes minutes).
void progress(const char* step, std::chrono::steady_clock::time_point start) {
    static const bool on = std::getenv("GLU_VERBOSE") != nullptr;
    if (!on) return;
    std::fprintf(stderr, "[glu analyze] %s done at %.1f s\n", step, ms_since(start) / 1e3);
    std::fflush(stderr);
}

// Host threads for the plan: GLU_PLAN_THREADS if set, else the hardware's
// (at most 16).
int plan_threads() {
    static const int nt = [] {
        const char* e = std::getenv("GLU_PLAN_THREADS");
        int v = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
        return std::max(1, std::min(v, 16));
    }();
    return nt;
}

// work(r) for r in [0, count), on count host threads; the first exception a
// worker throws (an allocation failure) is rethrown here after all joined.
void run_parallel(int count, const std::function<void(int)>& work) {
    if (count <= 1) {
        if (count == 1) work(0);
        return;
    }
    std::vector<std::exception_ptr> err(count);
    std::vector<std::thread> th;
    th.reserve(count);
    for (int r = 0; r < count; r++)
        th.emplace_back([&, r] {
            try {
                work(r);
            } catch (...) {
                err[r] = std::current_exception();
            }
        });
    for (std::thread& x : th) x.join();
    for (const std::exception_ptr& e : err)
        if (e) std::rethrow_exception(e);
}

// Column-wise pattern of B = P A P^T (rows unsorted; only reachability is needed).
void permuted_pattern(int32_t n, const int64_t* colptr, const int32_t* rowind,
                      const std::vector<int32_t>& perm, const std::vector<int32_t>& pinv,
                      std::vector<int64_t>& bp, std::vector<int32_t>& bi) {
    bp.assign(n + 1, 0);
    for (int32_t j = 0; j < n; j++) bp[j + 1] = bp[j] + (colptr[perm[j] + 1] - colptr[perm[j]]);
    bi.resize(bp[n]);
    for (int32_t j = 0; j < n; j++) {
        int32_t oj = perm[j];
        int64_t q = bp[j];
        for (int64_t p = colptr[oj]; p < colptr[oj + 1]; p++) bi[q++] = pinv[rowind[p]];
    }
}

// Pruned depth-first symbolic factorization.
Status symbolic(int32_t n, const std::vector<int64_t>& bp, const std::vector<int32_t>& bi,
                Analysis& a) {
    a.lu_colptr.assign(n + 1, 0);
    a.diag.assign(n, -1);
    a.lu_rowind.clear();
    a.lu_rowind.reserve(bp[n] * 4 + 16);
    std::vector<int32_t> visited(n, -1);
    std::vector<int64_t> plen(n, -1);          // pruned length of L(:,i) for the search
    std::vector<int32_t> stack_node(n), reach;
    std::vector<int64_t> stack_next(n);
    reach.reserve(n);
    for (int32_t j = 0; j < n; j++) {
        reach.clear();
        for (int64_t p = bp[j]; p < bp[j + 1]; p++) {
            int32_t r0 = bi[p];
            if (visited[r0] == j) continue;
            int32_t top = 0;
            stack_node[0] = r0;
            visited[r0] = j;
            stack_next[0] = (r0 < j) ? a.diag[r0] + 1 : 0;
            while (top >= 0) {
                int32_t v = stack_node[top];
                bool pushed = false;
                if (v < j) {
                    int64_t end = a.diag[v] + 1 + plen[v];
                    for (int64_t q = stack_next[top]; q < end; q++) {
                        int32_t c = a.lu_rowind[q];
                        if (visited[c] == j) continue;
                        stack_next[top] = q + 1;
                        visited[c] = j;
                        ++top;
                        stack_node[top] = c;
                        stack_next[top] = (c < j) ? a.diag[c] + 1 : 0;
                        pushed = true;
                        break;
                    }
                }
                if (!pushed) {
                    reach.push_back(v);
                    --top;
                }
            }
        }
        std::sort(reach.begin(), reach.end());
        int64_t base = a.lu_colptr[j];
        for (size_t q = 0; q < reach.size(); q++) {
            if (reach[q] == j) a.diag[j] = base + (int64_t)q;
            a.lu_rowind.push_back(reach[q]);
        }
        a.lu_colptr[j + 1] = base + (int64_t)reach.size();
        if (a.diag[j] < 0) {
            a.bad_col = j;
            return Status::struct_singular;
        }
        plen[j] = a.lu_colptr[j + 1] - a.diag[j] - 1;
        // symmetric pruning of the columns i with U(i,j) != 0 and L(j,i) != 0
        for (int64_t q = base; q < a.diag[j]; q++) {
            int32_t i = a.lu_rowind[q];
            int64_t lb = a.diag[i] + 1, le = a.diag[i] + 1 + plen[i];
            if (le - lb <= 0) continue;
            const int32_t* rb = a.lu_rowind.data();
            const int32_t* it = std::lower_bound(rb + lb, rb + le, j);
            if (it != rb + le && *it == j) plen[i] = (it - (rb + lb)) + 1;
        }
    }
    return Status::ok;
}

// True when the pattern of A (CSC, rows ascending) equals that of A^T.
bool pattern_symmetric(int32_t n, const int64_t* colptr, const int32_t* rowind) {
    std::vector<int64_t> tp(n + 1, 0);
    for (int64_t p = 0; p < colptr[n]; p++) tp[rowind[p] + 1]++;
    for (int32_t i = 0; i < n; i++) {
        tp[i + 1] += tp[i];
        if (tp[i + 1] != colptr[i + 1]) return false;
    }
    std::vector<int32_t> ti(colptr[n]);
    std::vector<int64_t> f(tp.begin(), tp.end() - 1);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) ti[f[rowind[p]]++] = j;
    return std::equal(ti.begin(), ti.end(), rowind);
}

// Symbolic fill of a structurally symmetric B.  The directed graph of B is
// then symmetric, so (i, j) is filled iff an undirected path joins i and j
// through vertices smaller than both (the fill-path lemma), which is the fill
// of the Cholesky factor: struct(L) is the elimination-tree structure and
// struct(U) = struct(L)^T.  Row i of L is the union of the tree paths from
// each k < i with B(i,k) != 0 up to i (row subtrees, Liu), so two walks
// (count, then fill) and one transposition give every column sorted, in
// O(nnz(L)) instead of the depth-first searches.  The diagonal (j,j) is in
// the reach of column j iff B(j,j) != 0 or B has an entry above it in column
// j (then a path j -> i -> j through i < j exists); the smallest column
// without either is structurally singular, as in the searches.
Status symbolic_symmetric(int32_t n, const std::vector<int64_t>& bp, const std::vector<int32_t>& bi,
                          Analysis& a) {
    for (int32_t j = 0; j < n; j++) {
        bool has = false;
        for (int64_t p = bp[j]; p < bp[j + 1] && !has; p++) has = bi[p] <= j;
        if (!has) {
            a.bad_col = j;
            return Status::struct_singular;
        }
    }
    // elimination tree (path compression through the ancestor links)
    std::vector<int32_t> parent(n, -1), anc(n, -1);
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = bp[i]; p < bp[i + 1]; p++) {
            int32_t r = bi[p];
            if (r >= i) continue;
            while (anc[r] != -1 && anc[r] != i) {
                const int32_t nx = anc[r];
                anc[r] = i;
                r = nx;
            }
            if (anc[r] == -1) {
                anc[r] = i;
                parent[r] = i;
            }
        }
    std::vector<int32_t>().swap(anc);
    std::vector<int32_t> mark(n, -1);
    std::vector<int64_t> lcnt(n, 0), ucnt(n, 0);  // |L(:,r)| and |U(:,i)| = |L(i,:)|
    for (int32_t i = 0; i < n; i++) {
        mark[i] = i;
        for (int64_t p = bp[i]; p < bp[i + 1]; p++)
            for (int32_t r = bi[p]; r < i && mark[r] != i; r = parent[r]) {
                mark[r] = i;
                lcnt[r]++;
                ucnt[i]++;
            }
    }
    a.lu_colptr.assign(n + 1, 0);
    a.diag.assign(n, -1);
    for (int32_t j = 0; j < n; j++) {
        a.diag[j] = a.lu_colptr[j] + ucnt[j];
        a.lu_colptr[j + 1] = a.diag[j] + 1 + lcnt[j];
    }
    a.lu_rowind.assign((size_t)a.lu_colptr[n], 0);
    int32_t* ri = a.lu_rowind.data();
    std::vector<int64_t> lf(n);  // L cursors: rows arrive ascending
    for (int32_t j = 0; j < n; j++) {
        ri[a.diag[j]] = j;
        lf[j] = a.diag[j] + 1;
    }
    std::fill(mark.begin(), mark.end(), -1);
    for (int32_t i = 0; i < n; i++) {
        mark[i] = i;
        for (int64_t p = bp[i]; p < bp[i + 1]; p++)
            for (int32_t r = bi[p]; r < i && mark[r] != i; r = parent[r]) {
                mark[r] = i;
                ri[lf[r]++] = i;
            }
    }
    // U(:,i) = rows r of L(i,:): transpose the L columns, r ascending
    std::vector<int64_t>& uf = lf;
    for (int32_t j = 0; j < n; j++) uf[j] = a.lu_colptr[j];
    for (int32_t r = 0; r < n; r++)
        for (int64_t q = a.diag[r] + 1; q < a.lu_colptr[r + 1]; q++) ri[uf[ri[q]]++] = r;
    return Status::ok;
}

// Dense trailing block.  Columns [t, n) whose filled pattern is nearly dense
// are better factorized as one dense block on the matrix cores than column by
// column: the submatrix update of a dense column moves about 20 bytes per
// multiply-add, a blocked dense LU moves a few bytes per hundred.  t minimises
//   T(t) = dense(n - t) - sparse_saved(t)
// with dense(m) = (2/3 m^3 flops) / R_dense + ceil(m/64) * T_panel
//                 + 16 m^2 bytes / BW (gather and scatter of the block),
// sparse_saved(t) = sum_{j >= t} macs_j * C_mac + (levels lying entirely at or
//                   beyond t) * T_level,
// and a tail is used only if T(t) < 0.  The constants are measured orders of
// magnitude on MI355X, not tuned per matrix.
// Schur-complement plan of the dense block (see Analysis::sch_*).
// Workgroups are dispatched to the GPU's XCDs round-robin (workgroup b runs on
// XCD b mod SCH_XCDS), and each XCD has its own L2.  The long tiles (one block
// each, blocks [0, nheavy)) of one tile row read the same L panel, so each XCD
// takes a contiguous range of them in row-major order.  The short tiles keep
// their longest-first order.  Within a tile the pair order is unchanged, so
// the results are too.
void xcd_order(std::vector<SchurUnit>& units, int64_t nheavy) {
    std::vector<SchurUnit> v(units.begin(), units.begin() + nheavy);
    std::sort(v.begin(), v.end(),
              [](const SchurUnit& x, const SchurUnit& y) { return x.i0 != y.i0 ? x.i0 < y.i0 : x.k0 < y.k0; });
    // XCD x receives v[range x]; block b takes the next unit of XCD b mod SCH_XCDS
    std::vector<size_t> head(SCH_XCDS), end(SCH_XCDS);
    for (int x = 0; x < SCH_XCDS; x++) {
        head[x] = (size_t)nheavy * x / SCH_XCDS;
        end[x] = (size_t)nheavy * (x + 1) / SCH_XCDS;
    }
    for (int64_t blk = 0; blk < nheavy; blk++) {
        int x = (int)(blk % SCH_XCDS);
        if (head[x] == end[x])  // this XCD's range is used up: take from the longest rest
            for (int y = 0; y < SCH_XCDS; y++)
                if (end[y] - head[y] > end[x] - head[x]) x = y;
        units[blk] = v[head[x]++];
    }
}

void build_schur_plan(Analysis& a, const std::vector<int64_t>& ltail) {
    const int32_t t = a.tail_start, m = a.tail_m;
    a.sch_lpos.clear(); a.sch_loff.clear(); a.sch_upos.clear(); a.sch_uoff.clear();
    a.sch_units.clear(); a.sch_pair_l.clear(); a.sch_pair_u.clear();
    a.sch_lp_len = a.sch_up_len = 0;
    a.sch_macs = 0;
    a.sch_nheavy = 0;
    if (m == 0 || t == 0) return;
    const int32_t TS = SCH_TS;
    const int32_t nt = (m + TS - 1) / TS;
    const int32_t* ri = a.lu_rowind.data();
    // U entries of row j in columns >= t: the tail of row j's U view
    std::vector<int64_t> utail(t);
    for (int32_t j = 0; j < t; j++)
        utail[j] = std::lower_bound(a.urow_col.begin() + a.urow_ptr[j], a.urow_col.begin() + a.urow_ptr[j + 1], t) -
                   a.urow_col.begin();
    // distinct row tiles of L(t:n, j) and column tiles of U(j, t:n), each with
    // the source's row index inside that tile's panel
    std::vector<int64_t> rt_ptr(t + 1, 0), ct_ptr(t + 1, 0);
    std::vector<int32_t> rt_tile, rt_idx, ct_tile, ct_idx;
    std::vector<int64_t> cntI(nt, 0), cntK(nt, 0);
    for (int32_t j = 0; j < t; j++) {
        int32_t last = -1;
        for (int64_t q = ltail[j]; q < a.lu_colptr[j + 1]; q++) {
            const int32_t I = (ri[q] - t) / TS;
            if (I != last) {
                rt_tile.push_back(I);
                rt_idx.push_back((int32_t)cntI[I]++);
                last = I;
            }
        }
        rt_ptr[j + 1] = (int64_t)rt_tile.size();
        last = -1;
        for (int64_t q = utail[j]; q < a.urow_ptr[j + 1]; q++) {
            const int32_t K = (a.urow_col[q] - t) / TS;
            if (K != last) {
                ct_tile.push_back(K);
                ct_idx.push_back((int32_t)cntK[K]++);
                last = K;
            }
        }
        ct_ptr[j + 1] = (int64_t)ct_tile.size();
        a.sch_macs += (int64_t)(a.lu_colptr[j + 1] - ltail[j]) * (a.urow_ptr[j + 1] - utail[j]);
    }
    // panel bases
    std::vector<int64_t> lbase(nt + 1, 0), ubase(nt + 1, 0);
    for (int32_t I = 0; I < nt; I++) {
        lbase[I + 1] = lbase[I] + cntI[I] * TS;
        ubase[I + 1] = ubase[I] + cntK[I] * TS;
    }
    a.sch_lp_len = lbase[nt];
    a.sch_up_len = ubase[nt];
    // value maps into the panels
    for (int32_t j = 0; j < t; j++) {
        int64_t r = rt_ptr[j];
        for (int64_t q = ltail[j]; q < a.lu_colptr[j + 1]; q++) {
            const int32_t I = (ri[q] - t) / TS;
            while (rt_tile[r] != I) r++;
            a.sch_lpos.push_back(q);
            a.sch_loff.push_back(lbase[I] + (int64_t)rt_idx[r] * TS + (ri[q] - t - I * TS));
        }
        int64_t c = ct_ptr[j];
        for (int64_t q = utail[j]; q < a.urow_ptr[j + 1]; q++) {
            const int32_t k = a.urow_col[q];
            const int32_t K = (k - t) / TS;
            while (ct_tile[c] != K) c++;
            a.sch_upos.push_back(a.urow_pos[q]);
            a.sch_uoff.push_back(ubase[K] + (int64_t)ct_idx[c] * TS + (k - t - K * TS));
        }
    }
    // pairs per tile, ascending j inside a tile (counting sort over tiles).
    // Host threads take ranges of sources of about equal pair counts; each
    // writes its sources' pairs after those of the earlier ranges in every
    // tile, so the lists are the ones a single pass gives.
    const size_t ntt = (size_t)nt * nt;
    std::vector<int32_t> jcut(1, 0);
    {
        std::vector<int64_t> wpre(t + 1, 0);
        for (int32_t j = 0; j < t; j++)
            wpre[j + 1] = wpre[j] + (rt_ptr[j + 1] - rt_ptr[j]) * (ct_ptr[j + 1] - ct_ptr[j]) + 1;
        const int nth = plan_threads();
        for (int r = 1; r < nth; r++) {
            int32_t j = (int32_t)(std::lower_bound(wpre.begin(), wpre.end(), wpre[t] * r / nth) - wpre.begin());
            jcut.push_back(std::min(std::max(j, jcut.back()), t));
        }
        jcut.push_back(t);
    }
    const int nparts = (int)jcut.size() - 1;
    std::vector<std::vector<int64_t>> cur(nparts);
    run_parallel(nparts, [&](int r) {
        cur[r].assign(ntt, 0);
        for (int32_t j = jcut[r]; j < jcut[r + 1]; j++)
            for (int64_t x = rt_ptr[j]; x < rt_ptr[j + 1]; x++)
                for (int64_t y = ct_ptr[j]; y < ct_ptr[j + 1]; y++) cur[r][(size_t)rt_tile[x] * nt + ct_tile[y]]++;
    });
    std::vector<int64_t> tile_ptr(ntt + 1, 0);
    for (size_t q = 0; q < ntt; q++) {
        int64_t o = tile_ptr[q];
        for (int r = 0; r < nparts; r++) {  // counts -> each range's first slot in tile q
            const int64_t c = cur[r][q];
            cur[r][q] = o;
            o += c;
        }
        tile_ptr[q + 1] = o;
    }
    a.sch_pair_l.resize(tile_ptr[ntt]);
    a.sch_pair_u.resize(tile_ptr[ntt]);
    run_parallel(nparts, [&](int r) {
        std::vector<int64_t>& f = cur[r];
        for (int32_t j = jcut[r]; j < jcut[r + 1]; j++)
            for (int64_t x = rt_ptr[j]; x < rt_ptr[j + 1]; x++)
                for (int64_t y = ct_ptr[j]; y < ct_ptr[j + 1]; y++) {
                    const int64_t o = f[(size_t)rt_tile[x] * nt + ct_tile[y]]++;
                    a.sch_pair_l[o] = rt_idx[x];
                    a.sch_pair_u[o] = ct_idx[y];
                }
        std::vector<int64_t>().swap(f);
    });
    for (int32_t I = 0; I < nt; I++)
        for (int32_t K = 0; K < nt; K++) {
            const size_t q = (size_t)I * nt + K;
            if (tile_ptr[q + 1] == tile_ptr[q]) continue;
            a.sch_units.push_back({I * TS, K * TS, tile_ptr[q], tile_ptr[q + 1], lbase[I], ubase[K]});
        }
    // longest tiles first, so that they start first
    std::stable_sort(a.sch_units.begin(), a.sch_units.end(),
                     [](const SchurUnit& x, const SchurUnit& y) { return x.pe - x.pb > y.pe - y.pb; });
    a.sch_nheavy = 0;
    while (a.sch_nheavy < (int64_t)a.sch_units.size() &&
           a.sch_units[a.sch_nheavy].pe - a.sch_units[a.sch_nheavy].pb >= SCH_HEAVY)
        a.sch_nheavy++;
    xcd_order(a.sch_units, a.sch_nheavy);
}

void choose_tail(Analysis& a, const PlanParams& pp, const std::vector<int64_t>& ucount) {
    const int32_t n = a.n;
    int32_t m = 0;
    if (pp.dense_tail > 0) {
        m = std::min(pp.dense_tail, n);
    } else if (pp.dense_tail == 0 && n >= 256) {
        const double R_dense = 25e12, T_panel = 25e-6, BW = 4e12, C_mac = 1e-11, T_level = 15e-6;
        std::vector<double> cost_from(n + 1, 0.0);  // sum over j >= t of the sparse per-column cost
        for (int32_t j = n - 1; j >= 0; j--) {
            double lj = (double)(a.lu_colptr[j + 1] - a.diag[j] - 1);
            double uj = (double)ucount[j];
            cost_from[j] = cost_from[j + 1] + lj * uj * C_mac;
        }
        const int32_t nlev = (int32_t)a.level_ptr.size() - 1;
        std::vector<int32_t> lev_min(nlev);
        for (int32_t l = 0; l < nlev; l++) lev_min[l] = a.level_cols[a.level_ptr[l]];
        std::sort(lev_min.begin(), lev_min.end());
        double best = 0.0;
        // The block is capped at 34,816 columns (9.7 GB).  On a 10^6-node
        // circuit with 400 supply rails, where the model reaches the cap, forced
        // sizes of 32,768 / 33,792 / 34,816 / 35,840 / 36,864 / 38,912 / 40,960
        // columns refactorize in 745 / 652 / 602 / 617 / 655 / 750 / 853 ms: the
        // per-product sparse cost below overstates what the levels and the
        // deferred Schur update cost once the block holds the rails' fill.
        const int32_t mmax = std::min(n, 34816);
        for (int32_t mm = 128; mm <= mmax; mm += 64) {
            int32_t t = n - mm;
            double md = (double)mm;
            double dense = (2.0 / 3.0) * md * md * md / R_dense + std::ceil(md / 64.0) * T_panel +
                           16.0 * md * md / BW;
            int64_t gone = lev_min.end() - std::lower_bound(lev_min.begin(), lev_min.end(), t);
            double saved = cost_from[t] + (double)gone * T_level;
            if (dense - saved < best) {
                best = dense - saved;
                m = mm;
            }
        }
    }
    a.tail_m = m;
    a.tail_start = n - m;
    a.tail_pos.resize(m);
    for (int32_t c = 0; c < m; c++) {
        int32_t k = a.tail_start + c;
        const int32_t* b = a.lu_rowind.data() + a.lu_colptr[k];
        const int32_t* e = a.lu_rowind.data() + a.lu_colptr[k + 1];
        a.tail_pos[c] = a.lu_colptr[k] + (std::lower_bound(b, e, a.tail_start) - b);
    }
}

}  // namespace

Status validate_csc(int32_t n, const int64_t* colptr, const int32_t* rowind) {
    if (n < 0 || (n > 0 && (!colptr || !rowind))) return Status::arg;
    if (n == 0) return Status::ok;
    if (colptr[0] != 0) return Status::arg;
    for (int32_t j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return Status::arg;
        int32_t last = -1;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t r = rowind[p];
            if (r < 0 || r >= n || r <= last) return Status::arg;
            last = r;
        }
    }
    return Status::ok;
}

Status analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, int ordering,
               const int32_t* perm_in, const PlanParams& pp, Analysis& a) {
    a = Analysis();
    Status st = validate_csc(n, colptr, rowind);
    if (st != Status::ok) return st;
    a.n = n;
    a.nnz_a = n ? colptr[n] : 0;

    // ---- ordering
    const auto t_start = std::chrono::steady_clock::now();
    auto t0 = t_start;
    if (ordering == 2) {
        if (!perm_in) return Status::arg;
        a.perm.assign(perm_in, perm_in + n);
    } else if (ordering == 1) {
        a.perm.resize(n);
        std::iota(a.perm.begin(), a.perm.end(), 0);
    } else if (ordering == 0) {
        a.perm = amd_order(n, colptr, rowind);
    } else {
        return Status::arg;
    }
    a.pinv.assign(n, -1);
    for (int32_t i = 0; i < n; i++) {
        int32_t o = a.perm[i];
        if (o < 0 || o >= n || a.pinv[o] != -1) return Status::arg;
        a.pinv[o] = i;
    }
    a.t_order_ms = ms_since(t0);
    progress("ordering", t_start);

    // ---- symbolic fill
    t0 = std::chrono::steady_clock::now();
    std::vector<int64_t> bp;
    std::vector<int32_t> bi;
    permuted_pattern(n, colptr, rowind, a.perm, a.pinv, bp, bi);
    st = pattern_symmetric(n, colptr, rowind) ? symbolic_symmetric(n, bp, bi, a) : symbolic(n, bp, bi, a);
    if (st != Status::ok) return st;
    const int64_t nnz = a.lu_colptr[n];
    // value map: A entry (r, c) -> position of B(pinv[r], pinv[c]) in A_s
    a.amap.resize(a.nnz_a);
    for (int32_t c = 0; c < n; c++) {
        int32_t jc = a.pinv[c];
        const int32_t* rb = a.lu_rowind.data() + a.lu_colptr[jc];
        const int32_t* re = a.lu_rowind.data() + a.lu_colptr[jc + 1];
        for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
            const int32_t* it = std::lower_bound(rb, re, a.pinv[rowind[p]]);
            a.amap[p] = it - a.lu_rowind.data();
        }
    }
    a.t_symbolic_ms = ms_since(t0);
    progress("symbolic fill", t_start);

    // ---- relaxed dependency DAG (Alg. 4): merge of two ascending lists per k,
    // U(:,k)'s rows with a non-empty L column ("look up") and row k of L
    // ("look left", from a column-only transposition of L freed afterwards)
    t0 = std::chrono::steady_clock::now();
    std::vector<char> lnonempty(n);
    std::vector<int64_t> ucount(n, 0);  // |U(i,:)| per row, for the dense-block cost model
    for (int32_t j = 0; j < n; j++) {
        lnonempty[j] = a.diag[j] + 1 < a.lu_colptr[j + 1];
        for (int64_t p = a.lu_colptr[j]; p < a.diag[j]; p++) ucount[a.lu_rowind[p]]++;
    }
    a.nnz_u = 0;
    for (int32_t i = 0; i < n; i++) a.nnz_u += ucount[i];
    a.nnz_l = (int64_t)a.lu_rowind.size() - n - a.nnz_u;
    int32_t nlev = 0;
    if (pp.dag_levels) {
        // the same two steps on the device (bit-identical results)
        int32_t spin_err = 0;
        if (pp.dag_levels(n, a.lu_colptr, a.lu_rowind, a.diag, a.dag_ptr, a.dag_idx, a.level_of, &spin_err) != 0 ||
            spin_err != 0)
            return Status::device;
        for (int32_t k = 0; k < n; k++) nlev = std::max(nlev, a.level_of[k] + 1);
    } else {
        std::vector<int64_t> lptr(n + 1, 0);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = a.diag[j] + 1; p < a.lu_colptr[j + 1]; p++) lptr[a.lu_rowind[p] + 1]++;
        for (int32_t i = 0; i < n; i++) lptr[i + 1] += lptr[i];
        std::vector<int32_t> lcol((size_t)a.nnz_l);
        {
            std::vector<int64_t> lf(lptr.begin(), lptr.end() - 1);
            for (int32_t j = 0; j < n; j++)  // ascending j keeps each row sorted
                for (int64_t p = a.diag[j] + 1; p < a.lu_colptr[j + 1]; p++) lcol[lf[a.lu_rowind[p]]++] = j;
        }
        a.dag_ptr.assign(n + 1, 0);
        for (int pass = 0; pass < 2; pass++) {
            if (pass == 1) a.dag_idx.assign((size_t)a.dag_ptr[n], 0);
            int64_t cnt = 0;
            for (int32_t k = 0; k < n; k++) {
                int64_t p = a.lu_colptr[k], pe = a.diag[k];  // look up: U(:,k)
                int64_t q = lptr[k], qe = lptr[k + 1];       // look left: row k of L
                while (p < pe || q < qe) {
                    int32_t iu = INT32_MAX, il = INT32_MAX;
                    while (p < pe && !lnonempty[a.lu_rowind[p]]) p++;
                    if (p < pe) iu = a.lu_rowind[p];
                    if (q < qe) il = lcol[q];
                    if (iu == INT32_MAX && il == INT32_MAX) break;
                    const int32_t i = std::min(iu, il);
                    if (pass == 1) a.dag_idx[(size_t)cnt] = i;
                    cnt++;
                    if (iu == i) p++;
                    if (il == i) q++;
                }
                if (pass == 0) a.dag_ptr[k + 1] = cnt;
            }
        }
        // ---- levelization
        a.level_of.assign(n, 0);
        for (int32_t k = 0; k < n; k++) {
            int32_t l = 0;
            for (int64_t e = a.dag_ptr[k]; e < a.dag_ptr[k + 1]; e++)
                l = std::max(l, a.level_of[a.dag_idx[e]] + 1);
            a.level_of[k] = l;
            nlev = std::max(nlev, l + 1);
        }
    }
    a.level_ptr.assign(nlev + 1, 0);
    for (int32_t k = 0; k < n; k++) a.level_ptr[a.level_of[k] + 1]++;
    for (int32_t l = 0; l < nlev; l++) a.level_ptr[l + 1] += a.level_ptr[l];
    a.level_cols.resize(n);
    {
        std::vector<int32_t> f(a.level_ptr.begin(), a.level_ptr.end() - 1);
        for (int32_t k = 0; k < n; k++) a.level_cols[f[a.level_of[k]]++] = k;
    }
    a.t_levels_ms = ms_since(t0);
    progress("dependency DAG and levels", t_start);

    // ---- dense trailing block
    choose_tail(a, pp, ucount);
    std::vector<int64_t>().swap(ucount);
    a.tail_asrc.clear(); a.tail_arow.clear(); a.tail_acol.clear();
    if (a.tail_m > 0) {
        const int32_t t = a.tail_start;
        for (int32_t c = 0; c < n; c++) {
            const int32_t jc = a.pinv[c];
            if (jc < t) continue;
            for (int64_t p = colptr[c]; p < colptr[c + 1]; p++) {
                const int32_t r = a.pinv[rowind[p]];
                if (r < t) continue;
                a.tail_asrc.push_back(a.amap[p]);
                a.tail_arow.push_back(r - t);
                a.tail_acol.push_back(jc - t);
            }
        }
    }

    // ---- row views of L and U outside the dense block (the block is dense
    // on the device; nothing reads its entries by row): L rows before the
    // block whole, L rows of the block up to its first column (the forward
    // solve's cross term), U rows before the block whole
    {
        const int32_t t = a.tail_start;
        a.lrow_ptr.assign(n + 1, 0);
        a.urow_ptr.assign(n + 1, 0);
        for (int32_t j = 0; j < t; j++) {
            for (int64_t p = a.lu_colptr[j]; p < a.diag[j]; p++) a.urow_ptr[a.lu_rowind[p] + 1]++;
            for (int64_t p = a.diag[j] + 1; p < a.lu_colptr[j + 1]; p++) a.lrow_ptr[a.lu_rowind[p] + 1]++;
        }
        for (int32_t j = t; j < n; j++)
            for (int64_t p = a.lu_colptr[j]; p < a.diag[j] && a.lu_rowind[p] < t; p++)
                a.urow_ptr[a.lu_rowind[p] + 1]++;
        for (int32_t i = 0; i < n; i++) {
            a.urow_ptr[i + 1] += a.urow_ptr[i];
            a.lrow_ptr[i + 1] += a.lrow_ptr[i];
        }
        a.urow_pos.resize(a.urow_ptr[n]);
        a.urow_col.resize(a.urow_ptr[n]);
        a.lrow_pos.resize(a.lrow_ptr[n]);
        a.lrow_col.resize(a.lrow_ptr[n]);
        std::vector<int64_t> uf(a.urow_ptr.begin(), a.urow_ptr.end() - 1);
        std::vector<int64_t> lf(a.lrow_ptr.begin(), a.lrow_ptr.end() - 1);
        for (int32_t j = 0; j < n; j++) {  // ascending j keeps each row view sorted
            for (int64_t p = a.lu_colptr[j]; p < a.diag[j]; p++) {
                const int32_t r = a.lu_rowind[p];
                if (r >= t) break;
                a.urow_col[uf[r]] = j;
                a.urow_pos[uf[r]++] = p;
            }
            if (j >= t) continue;
            for (int64_t p = a.diag[j] + 1; p < a.lu_colptr[j + 1]; p++) {
                const int32_t r = a.lu_rowind[p];
                a.lrow_col[lf[r]] = j;
                a.lrow_pos[lf[r]++] = p;
            }
        }
    }

    progress("dense block choice and row views", t_start);
    // ---- executed levels: each level restricted to columns before the tail
    const int32_t t = a.tail_start;
    std::vector<int32_t> exec_of(nlev, -1);
    a.exec_ptr.assign(1, 0);
    a.exec_cols.clear();
    for (int32_t l = 0; l < nlev; l++) {
        int32_t cnt = 0;
        for (int32_t q = a.level_ptr[l]; q < a.level_ptr[l + 1]; q++)
            if (a.level_cols[q] < t) { a.exec_cols.push_back(a.level_cols[q]); cnt++; }
        if (cnt > 0) {
            exec_of[l] = (int32_t)a.exec_ptr.size() - 1;
            a.exec_ptr.push_back((int32_t)a.exec_cols.size());
        }
    }
    const int32_t nexec = (int32_t)a.exec_ptr.size() - 1;

    // ---- level plan
    t0 = std::chrono::steady_clock::now();
    a.level_mode.resize(nexec);
    a.widest = 0;
    for (int32_t l = 0; l < nlev; l++) a.widest = std::max(a.widest, a.level_ptr[l + 1] - a.level_ptr[l]);
    for (int32_t e = 0; e < nexec; e++) {
        int32_t w = a.exec_ptr[e + 1] - a.exec_ptr[e];
        int32_t m;
        if (pp.force_mode >= 0) m = pp.force_mode;
        else if (pp.stream_threshold >= 0 && w <= pp.stream_threshold) m = MODE_STREAM;
        else if (pp.large_threshold >= 0 && w <= pp.large_threshold) m = MODE_LARGE;
        else m = MODE_SMALL;
        a.level_mode[e] = m;
        a.levels_per_mode[m]++;
    }
    // multiply-adds of the whole factorization (sparse levels and dense tail
    // alike), the part inside the dense block (source and target there), and
    // the L and U entries of the columns / rows before the block
    a.macs = 0;
    a.tail_macs = 0;
    {
        std::vector<int64_t> lc(n);
        for (int32_t j = 0; j < n; j++) lc[j] = a.lu_colptr[j + 1] - a.diag[j] - 1;
        for (int32_t k = 0; k < n; k++)
            for (int64_t p = a.lu_colptr[k]; p < a.diag[k]; p++) {
                const int32_t j = a.lu_rowind[p];
                a.macs += lc[j];
                if (j >= t) a.tail_macs += lc[j];
            }
        a.level_nl = 0;
        for (int32_t j = 0; j < t; j++) a.level_nl += lc[j];
        a.level_nu = a.urow_ptr[t];  // U rows before the block are whole in the row view
    }
    // ltail[j]: first position of column j with row >= t.  A source j < t
    // updates a target column k >= t only in rows < t inside the levels (its
    // rows >= t go to the Schur-complement update of the dense block).
    std::vector<int64_t> ltail(t);
    for (int32_t j = 0; j < t; j++)
        ltail[j] = std::lower_bound(a.lu_rowind.begin() + a.diag[j] + 1, a.lu_rowind.begin() + a.lu_colptr[j + 1],
                                    t) - a.lu_rowind.begin();
    auto level_llen = [&](int32_t j, int32_t k) -> int32_t {
        return (int32_t)((k >= t ? ltail[j] : a.lu_colptr[j + 1]) - a.diag[j] - 1);
    };
    // update entries (executed level of j, k, position of U(j,k)) for sources
    // j < t with L rows to apply in the levels, grouped by executed level with
    // a stable counting sort; inside a level they stay ordered by (k, j)
    std::vector<int64_t> ecount(nexec + 1, 0);
    for (int32_t k = 0; k < n; k++)
        for (int64_t p = a.lu_colptr[k]; p < a.diag[k]; p++) {
            int32_t j = a.lu_rowind[p];
            if (j >= t || level_llen(j, k) == 0) continue;
            ecount[exec_of[a.level_of[j]] + 1]++;
        }
    for (int32_t e = 0; e < nexec; e++) ecount[e + 1] += ecount[e];
    std::vector<int64_t> ent_pos(ecount[nexec]);
    std::vector<int32_t> ent_col(ecount[nexec]);
    {
        std::vector<int64_t> f(ecount.begin(), ecount.end() - 1);
        for (int32_t k = 0; k < n; k++)
            for (int64_t p = a.lu_colptr[k]; p < a.diag[k]; p++) {
                int32_t j = a.lu_rowind[p];
                if (j >= t || level_llen(j, k) == 0) continue;
                int64_t s = f[exec_of[a.level_of[j]]]++;
                ent_pos[s] = p;
                ent_col[s] = k;
            }
    }
    progress("level plan: update entries", t_start);
    a.src_upos = ent_pos;
    a.src_dpos.resize(ent_pos.size());
    a.src_llen.resize(ent_pos.size());
    for (size_t q = 0; q < ent_pos.size(); q++) {
        int32_t j = a.lu_rowind[ent_pos[q]];
        a.src_dpos[q] = a.diag[j];
        a.src_llen[q] = level_llen(j, ent_col[q]);
    }
    a.task_ptr.assign(nexec + 1, 0);
    a.wi_ptr.assign(nexec + 1, 0);
    a.task_col.clear();
    a.task_src_ptr.clear();
    a.wi_task.clear();
    a.wi_begin.clear();
    a.wi_end.clear();
    a.wi_ss.clear();
    a.wi_whole.clear();
    a.wi_s0.clear();
    a.wi_nsrc.clear();
    a.ss_up.clear();
    a.ss_dp.clear();
    a.ss_src.clear();
    a.ss_lo.clear();
    a.ss_hi.clear();
    const int32_t* ri = a.lu_rowind.data();
    // Tasks and work items of a range [sa, sb) of the update entries (cut at
    // task boundaries), with task and piece indices local to the range; the
    // ranges are planned on host threads and concatenated in entry order,
    // which gives the same arrays as one pass over all entries.
    struct Piece { int32_t slice, src, lo, hi; };
    struct RangePlan {
        std::vector<int32_t> task_col, wi_task, wi_nsrc, ss_src, ss_lo, ss_hi;
        std::vector<int64_t> task_src_ptr, wi_begin, wi_end, wi_ss, wi_s0, ss_up, ss_dp;
        std::vector<int8_t> wi_whole;
    };
    auto level_of_entry = [&](int64_t x) {  // the executed level holding entry x
        return (int32_t)(std::upper_bound(ecount.begin(), ecount.end(), x) - ecount.begin()) - 1;
    };
    auto plan_entries = [&](int64_t sa, int64_t sb, RangePlan& o) {
        std::vector<int64_t> sl_cnt;
        std::vector<Piece> pieces;
        int32_t e = sa < sb ? level_of_entry(sa) : 0;
        {
            for (int64_t s = sa; s < sb;) {
                while (ecount[e + 1] <= s) e++;
                const int64_t chunk = a.level_mode[e] == MODE_SMALL ? pp.chunk_small
                                      : a.level_mode[e] == MODE_LARGE ? pp.chunk_large : pp.chunk_stream;
                int32_t k = ent_col[s];
                int64_t s2 = s;
                while (s2 < ecount[e + 1] && ent_col[s2] == k) s2++;
                int32_t tk = (int32_t)o.task_col.size();
                o.task_col.push_back(k);
                o.task_src_ptr.push_back(s);
                // span of target rows the task touches: the union of its sources' L rows
                int32_t rmin = INT32_MAX, rmax = -1;
                int64_t pairs = 0;
                for (int64_t q = s; q < s2; q++) {
                    int64_t l0 = a.src_dpos[q] + 1, l1 = l0 + a.src_llen[q];
                    rmin = std::min(rmin, ri[l0]);
                    rmax = std::max(rmax, ri[l1 - 1]);
                    pairs += a.src_llen[q];
                }
                const int64_t pb = std::lower_bound(ri + ent_pos[s] + 1, ri + a.lu_colptr[k + 1], rmin) - ri;
                const int64_t pe = std::upper_bound(ri + pb, ri + a.lu_colptr[k + 1], rmax) - ri;
                // slice length: the mode's cap, shortened for deep tasks (many sources
                // per target entry) so that a slice holds about kPairsPerSlice updates
                const int64_t kPairsPerSlice = 4096;
                const int64_t span = pe - pb;
                int64_t ch = chunk;
                while (ch > 32 && pairs * ch > kPairsPerSlice * span) ch >>= 1;
                if (span <= ch) {
                    o.wi_task.push_back(tk);
                    o.wi_begin.push_back(pb);
                    o.wi_end.push_back(pe);
                    o.wi_ss.push_back((int64_t)o.ss_src.size());
                    o.wi_whole.push_back(1);
                    o.wi_s0.push_back(s);
                    o.wi_nsrc.push_back((int32_t)(s2 - s));
                    s = s2;
                    continue;
                }
                const int32_t nsl = (int32_t)((span + ch - 1) / ch);
                // pieces: maximal runs of a source's L rows inside one slice
                pieces.clear();
                for (int64_t q = s; q < s2; q++) {
                    const int64_t l0 = a.src_dpos[q] + 1, l1 = l0 + a.src_llen[q];
                    int64_t x = l0;
                    int64_t tp = pb;  // target position cursor (rows of L(:,j) are rows of column k)
                    while (x < l1) {
                        tp = gallop(ri + tp, ri + pe, ri[x], false) - ri;
                        const int32_t sl = (int32_t)((tp - pb) / ch);
                        const int32_t slice_last_row = ri[std::min(pe, pb + (int64_t)(sl + 1) * ch) - 1];
                        const int64_t y = gallop(ri + x, ri + l1, slice_last_row, true) - ri;
                        pieces.push_back({sl, (int32_t)(q - s), (int32_t)(x - l0), (int32_t)(y - l0)});
                        x = y;
                    }
                }
                // group by slice, keeping ascending source order inside a slice
                sl_cnt.assign(nsl + 1, 0);
                for (const Piece& pc : pieces) sl_cnt[pc.slice + 1]++;
                for (int32_t i = 0; i < nsl; i++) sl_cnt[i + 1] += sl_cnt[i];
                const int64_t base = (int64_t)o.ss_src.size();
                o.ss_src.resize(base + pieces.size());
                o.ss_lo.resize(base + pieces.size());
                o.ss_hi.resize(base + pieces.size());
                o.ss_up.resize(base + pieces.size());
                o.ss_dp.resize(base + pieces.size());
                {
                    std::vector<int64_t> f(sl_cnt.begin(), sl_cnt.end() - 1);
                    for (const Piece& pc : pieces) {
                        const int64_t x = base + f[pc.slice]++;
                        o.ss_src[x] = pc.src;
                        o.ss_up[x] = a.src_upos[s + pc.src];
                        o.ss_dp[x] = a.src_dpos[s + pc.src];
                        o.ss_lo[x] = pc.lo;
                        o.ss_hi[x] = pc.hi;
                    }
                }
                for (int32_t i = 0; i < nsl; i++) {
                    if (sl_cnt[i + 1] == sl_cnt[i]) continue;  // no source touches this slice
                    o.wi_task.push_back(tk);
                    o.wi_begin.push_back(pb + (int64_t)i * ch);
                    o.wi_end.push_back(std::min(pe, pb + (int64_t)(i + 1) * ch));
                    o.wi_ss.push_back(base + sl_cnt[i]);
                    o.wi_whole.push_back(0);
                    o.wi_s0.push_back(s);
                    o.wi_nsrc.push_back((int32_t)(sl_cnt[i + 1] - sl_cnt[i]));
                }
                s = s2;
            }
        }
    };
    {
        // entry ranges of about equal size, one per host thread, each cut
        // moved forward to the next task boundary
        const int nth = plan_threads();
        const int64_t total = ecount[nexec];
        std::vector<int64_t> cut(1, 0);
        for (int r = 1; r < nth; r++) {
            int64_t x = std::max(total * r / nth, cut.back());
            if (x < total) {
                const int32_t e = level_of_entry(x);
                while (x > ecount[e] && x < ecount[e + 1] && ent_col[x] == ent_col[x - 1]) x++;
            }
            cut.push_back(std::min(x, total));
        }
        cut.push_back(total);
        std::vector<RangePlan> parts(cut.size() - 1);
        run_parallel((int)parts.size(), [&](int r) { plan_entries(cut[r], cut[r + 1], parts[r]); });
        for (size_t r = 0; r < parts.size(); r++) {
            RangePlan& o = parts[r];
            const int32_t task_off = (int32_t)a.task_col.size();
            const int64_t ss_off = (int64_t)a.ss_src.size();
            a.task_col.insert(a.task_col.end(), o.task_col.begin(), o.task_col.end());
            a.task_src_ptr.insert(a.task_src_ptr.end(), o.task_src_ptr.begin(), o.task_src_ptr.end());
            for (int32_t x : o.wi_task) a.wi_task.push_back(x + task_off);
            a.wi_begin.insert(a.wi_begin.end(), o.wi_begin.begin(), o.wi_begin.end());
            a.wi_end.insert(a.wi_end.end(), o.wi_end.begin(), o.wi_end.end());
            for (int64_t x : o.wi_ss) a.wi_ss.push_back(x + ss_off);
            a.wi_whole.insert(a.wi_whole.end(), o.wi_whole.begin(), o.wi_whole.end());
            a.wi_s0.insert(a.wi_s0.end(), o.wi_s0.begin(), o.wi_s0.end());
            a.wi_nsrc.insert(a.wi_nsrc.end(), o.wi_nsrc.begin(), o.wi_nsrc.end());
            a.ss_src.insert(a.ss_src.end(), o.ss_src.begin(), o.ss_src.end());
            a.ss_lo.insert(a.ss_lo.end(), o.ss_lo.begin(), o.ss_lo.end());
            a.ss_hi.insert(a.ss_hi.end(), o.ss_hi.begin(), o.ss_hi.end());
            a.ss_up.insert(a.ss_up.end(), o.ss_up.begin(), o.ss_up.end());
            a.ss_dp.insert(a.ss_dp.end(), o.ss_dp.begin(), o.ss_dp.end());
            o = RangePlan();  // release the part
        }
        // per level: its first task (tasks are in entry order) and first item
        // (items are in task order)
        for (int32_t e = 0; e <= nexec; e++) {
            a.task_ptr[e] = std::lower_bound(a.task_src_ptr.begin(), a.task_src_ptr.end(), ecount[e]) -
                            a.task_src_ptr.begin();
            a.wi_ptr[e] = std::lower_bound(a.wi_task.begin(), a.wi_task.end(), (int32_t)a.task_ptr[e]) -
                          a.wi_task.begin();
        }
    }
    a.task_src_ptr.push_back(ecount[nexec]);
    a.wi_ss.push_back((int64_t)a.ss_src.size());
    progress("level plan: tasks and slices", t_start);
    // stream-mode runs (Section III-B's stream mode): consecutive narrow
    // levels share one persistent launch
    a.run_e0.clear(); a.run_e1.clear(); a.run_sb.clear();
    a.seg_start.clear(); a.seg_wi.clear(); a.seg_norm.clear();
    for (int32_t e = 0; e < nexec;) {
        if (a.level_mode[e] != MODE_STREAM) { e++; continue; }
        int32_t e1 = e;
        while (e1 < nexec && a.level_mode[e1] == MODE_STREAM) e1++;
        if (e1 - e >= std::max(1, pp.stream_min_run)) {
            a.run_e0.push_back(e);
            a.run_e1.push_back(e1);
            a.run_sb.push_back((int64_t)a.seg_start.size());
            int64_t items = 0;
            for (int32_t x = e; x < e1; x++) {
                const int64_t nwi = a.wi_ptr[x + 1] - a.wi_ptr[x];
                const int32_t nn = x > 0 ? a.exec_ptr[x] - a.exec_ptr[x - 1] : 0;
                a.seg_start.push_back(items);
                a.seg_wi.push_back(a.wi_ptr[x]);
                a.seg_norm.push_back(x > 0 ? a.exec_ptr[x - 1] : 0);
                items += nwi + nn;
            }
            a.seg_start.push_back(items);
            a.seg_wi.push_back(a.wi_ptr[e1]);
            a.seg_norm.push_back(0);
        }
        e = e1;
    }
    // pair and touched-entry map offsets of every work item
    progress("level plan: stream runs", t_start);
    {
        const size_t nw = a.wi_task.size();
        a.wi_pbase.assign(nw + 1, 0);
        a.wi_tbase.assign(nw + 1, 0);
        for (size_t w = 0; w < nw; w++) {
            int64_t np = 0;
            if (a.wi_whole[w]) {
                for (int64_t q = 0; q < a.wi_nsrc[w]; q++) np += a.src_llen[a.wi_s0[w] + q];
            } else {
                for (int64_t e = a.wi_ss[w]; e < a.wi_ss[w + 1]; e++) np += a.ss_hi[e] - a.ss_lo[e];
            }
            a.wi_pbase[w + 1] = a.wi_pbase[w] + np;
            a.wi_tbase[w + 1] = a.wi_tbase[w] + std::min<int64_t>(np, a.wi_end[w] - a.wi_begin[w]);
        }
        a.n_pairs = a.wi_pbase[nw];
        a.n_touch_cap = a.wi_tbase[nw];
        progress("level plan: map offsets", t_start);
        // Within a level, items run most pairs first: the dispatcher starts
        // waves in item order, so the long items start early and the short
        // ones fill the end of the launch.  Items write disjoint entries, so
        // the order changes no result.  Each item keeps its map offsets; the
        // sentinels at index nw stay in place.
        //
        // XCD placement (pp.xcd_items): workgroup b of a launch runs on XCD
        // b mod SCH_XCDS, each XCD with its own L2, and the items of a level
        // that share their first source column read the same L column.  Such
        // items are grouped, the groups (heaviest first) go to the XCD with
        // the fewest pairs so far (longest processing time first), each
        // XCD's items run longest first, and the launch order deals them out
        // so that item position b lands on XCD b mod SCH_XCDS.
        std::vector<int64_t> ord;
        std::vector<int64_t> t64;
        std::vector<int32_t> t32;
        std::vector<int8_t> t8;
        auto npairs = [&](int64_t x) { return a.wi_pbase[x + 1] - a.wi_pbase[x]; };
        for (int32_t e = 0; e < nexec; e++) {
            const int64_t w0 = a.wi_ptr[e], w1 = a.wi_ptr[e + 1];
            ord.resize((size_t)(w1 - w0));
            for (int64_t w = w0; w < w1; w++) ord[(size_t)(w - w0)] = w;
            std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return npairs(x) > npairs(y); });
            if (pp.xcd_items && w1 - w0 >= 2 * SCH_XCDS) {
                // group key: the item's first source column
                auto first_src = [&](int64_t x) -> int32_t {
                    const int64_t sidx = a.wi_whole[x] ? a.wi_s0[x] : a.wi_s0[x] + a.ss_src[a.wi_ss[x]];
                    return a.lu_rowind[a.src_upos[sidx]];
                };
                std::vector<std::pair<int32_t, int64_t>> key((size_t)(w1 - w0));  // (source, item)
                for (int64_t w = w0; w < w1; w++) key[(size_t)(w - w0)] = {first_src(w), w};
                std::sort(key.begin(), key.end());
                struct Group { int64_t load, b, e; };  // key[b, e)
                std::vector<Group> groups;
                for (size_t q = 0; q < key.size();) {
                    size_t q2 = q;
                    int64_t load = 0;
                    while (q2 < key.size() && key[q2].first == key[q].first) load += npairs(key[q2++].second);
                    groups.push_back({load, (int64_t)q, (int64_t)q2});
                    q = q2;
                }
                std::stable_sort(groups.begin(), groups.end(), [](const Group& x, const Group& y) { return x.load > y.load; });
                std::vector<int64_t> xload(SCH_XCDS, 0);
                std::vector<std::vector<int64_t>> bucket(SCH_XCDS);
                for (const Group& g : groups) {
                    const int x = (int)(std::min_element(xload.begin(), xload.end()) - xload.begin());
                    xload[x] += g.load;
                    for (int64_t q = g.b; q < g.e; q++) bucket[x].push_back(key[(size_t)q].second);
                }
                for (auto& bk : bucket)
                    std::stable_sort(bk.begin(), bk.end(), [&](int64_t x, int64_t y) { return npairs(x) > npairs(y); });
                std::vector<size_t> head(SCH_XCDS, 0);
                for (size_t pos = 0; pos < ord.size(); pos++) {
                    int x = (int)(pos % SCH_XCDS);
                    if (head[x] == bucket[x].size())  // this XCD's share is used up: the fullest rest
                        for (int y = 0; y < SCH_XCDS; y++)
                            if (bucket[y].size() - head[y] > bucket[x].size() - head[x]) x = y;
                    ord[pos] = bucket[x][head[x]++];
                }
            }
            auto perm64 = [&](std::vector<int64_t>& v) {
                t64.resize(ord.size());
                for (size_t i = 0; i < ord.size(); i++) t64[i] = v[(size_t)ord[i]];
                std::copy(t64.begin(), t64.end(), v.begin() + w0);
            };
            auto perm32 = [&](std::vector<int32_t>& v) {
                t32.resize(ord.size());
                for (size_t i = 0; i < ord.size(); i++) t32[i] = v[(size_t)ord[i]];
                std::copy(t32.begin(), t32.end(), v.begin() + w0);
            };
            t8.resize(ord.size());
            for (size_t i = 0; i < ord.size(); i++) t8[i] = a.wi_whole[(size_t)ord[i]];
            std::copy(t8.begin(), t8.end(), a.wi_whole.begin() + w0);
            perm32(a.wi_task);
            perm64(a.wi_begin);
            perm64(a.wi_end);
            perm64(a.wi_ss);
            perm64(a.wi_s0);
            perm32(a.wi_nsrc);
            perm64(a.wi_pbase);
            perm64(a.wi_tbase);
        }
    }

    progress("level plan", t_start);
    build_schur_plan(a, ltail);
    progress("Schur-complement plan", t_start);
    if (std::getenv("GLU_VERBOSE") && !a.sch_units.empty()) {
        int64_t ph = 0, pl = 0, pmax = 0;
        for (size_t u = 0; u < a.sch_units.size(); u++) {
            const int64_t np = a.sch_units[u].pe - a.sch_units[u].pb;
            ((int64_t)u < a.sch_nheavy ? ph : pl) += np;
            pmax = std::max(pmax, np);
        }
        std::fprintf(stderr,
                     "[glu analyze] Schur tiles: %lld long (%lld pairs, longest %lld), %lld short (%lld pairs); "
                     "panels %lld + %lld rows\n",
                     (long long)a.sch_nheavy, (long long)ph, (long long)pmax,
                     (long long)(a.sch_units.size() - a.sch_nheavy), (long long)pl,
                     (long long)(a.sch_lp_len / SCH_TS), (long long)(a.sch_up_len / SCH_TS));
    }

    // ---- solve schedules over rows before the tail (the tail is solved densely)
    {
        std::vector<int32_t> lv(n, 0);
        int32_t nl = 0;
        for (int32_t i = 0; i < t; i++) {
            int32_t l = 0;
            for (int64_t q = a.lrow_ptr[i]; q < a.lrow_ptr[i + 1]; q++) l = std::max(l, lv[a.lrow_col[q]] + 1);
            lv[i] = l;
            nl = std::max(nl, l + 1);
        }
        a.fsolve_ptr.assign(nl + 1, 0);
        for (int32_t i = 0; i < t; i++) a.fsolve_ptr[lv[i] + 1]++;
        for (int32_t l = 0; l < nl; l++) a.fsolve_ptr[l + 1] += a.fsolve_ptr[l];
        a.fsolve_rows.resize(t);
        std::vector<int32_t> f(a.fsolve_ptr.begin(), a.fsolve_ptr.end() - 1);
        for (int32_t i = 0; i < t; i++) a.fsolve_rows[f[lv[i]]++] = i;
    }
    {
        // tail columns are solved first, so they count as done (level -1)
        std::vector<int32_t> lv(n, -1);
        int32_t nl = 0;
        for (int32_t j = t - 1; j >= 0; j--) {
            int32_t l = 0;
            for (int64_t q = a.urow_ptr[j]; q < a.urow_ptr[j + 1]; q++) l = std::max(l, lv[a.urow_col[q]] + 1);
            lv[j] = l;
            nl = std::max(nl, l + 1);
        }
        a.bsolve_ptr.assign(nl + 1, 0);
        for (int32_t j = 0; j < t; j++) a.bsolve_ptr[lv[j] + 1]++;
        for (int32_t l = 0; l < nl; l++) a.bsolve_ptr[l + 1] += a.bsolve_ptr[l];
        a.bsolve_rows.resize(t);
        std::vector<int32_t> f(a.bsolve_ptr.begin(), a.bsolve_ptr.end() - 1);
        for (int32_t j = 0; j < t; j++) a.bsolve_rows[f[lv[j]]++] = j;
    }
    // the solves' entries in schedule order
    // (a row's entries [rptr[row], rend(row)): the forward rows before the tail
    // have no column >= t; the backward rows stop at their first column >= t)
    std::vector<int64_t> usplit(t);
    for (int32_t j = 0; j < t; j++) {
        const int32_t* b = a.urow_col.data() + a.urow_ptr[j];
        const int32_t* e = a.urow_col.data() + a.urow_ptr[j + 1];
        usplit[j] = a.urow_ptr[j] + (std::lower_bound(b, e, t) - b);
    }
    auto schedule_entries = [&](const std::vector<int32_t>& rows, const std::vector<int64_t>& rptr,
                                const std::vector<int64_t>& rpos, const std::vector<int32_t>& rcol,
                                const std::vector<int64_t>* rend, std::vector<int64_t>& ptr,
                                std::vector<int64_t>& pos, std::vector<int32_t>& col) {
        auto end = [&](int32_t r) { return rend ? (*rend)[r] : rptr[r + 1]; };
        ptr.assign(rows.size() + 1, 0);
        for (size_t w = 0; w < rows.size(); w++) ptr[w + 1] = ptr[w] + (end(rows[w]) - rptr[rows[w]]);
        pos.resize(ptr.back());
        col.resize(ptr.back());
        for (size_t w = 0; w < rows.size(); w++) {
            int64_t x = ptr[w];
            for (int64_t q = rptr[rows[w]]; q < end(rows[w]); q++, x++) {
                pos[x] = rpos[q];
                col[x] = rcol[q];
            }
        }
    };
    schedule_entries(a.fsolve_rows, a.lrow_ptr, a.lrow_pos, a.lrow_col, nullptr, a.fs_ptr, a.fs_pos, a.fs_col);
    schedule_entries(a.bsolve_rows, a.urow_ptr, a.urow_pos, a.urow_col, &usplit, a.bs_ptr, a.bs_pos, a.bs_col);
    // the backward cross term U(j, t:n) x(t:n) of the rows before the tail
    a.ux_ptr.assign(1, 0);
    a.ux_row.clear(); a.ux_col.clear(); a.ux_q0.clear(); a.ux_q1.clear(); a.ux_pos.clear();
    for (int32_t j = 0; j < t; j++) {
        const int64_t q1 = a.urow_ptr[j + 1];
        if (usplit[j] == q1) continue;
        const int64_t base = (int64_t)a.ux_pos.size();
        for (int64_t q = usplit[j]; q < q1; q++) {
            a.ux_pos.push_back(a.urow_pos[q]);
            a.ux_col.push_back(a.urow_col[q]);
        }
        const int64_t len = q1 - usplit[j];
        for (int64_t o = 0; o < len; o += CROSS_CHUNK) {
            a.ux_q0.push_back(base + o);
            a.ux_q1.push_back(base + std::min<int64_t>(o + CROSS_CHUNK, len));
        }
        a.ux_row.push_back(j);
        a.ux_ptr.push_back((int32_t)a.ux_q0.size());
    }
    // split of every tail row's L row into columns before / inside the tail
    a.tail_lsplit.resize(a.tail_m);
    for (int32_t c = 0; c < a.tail_m; c++) {
        int32_t i = t + c;
        const int32_t* b = a.lrow_col.data() + a.lrow_ptr[i];
        const int32_t* e = a.lrow_col.data() + a.lrow_ptr[i + 1];
        a.tail_lsplit[c] = a.lrow_ptr[i] + (std::lower_bound(b, e, t) - b);
    }
    a.cross_ptr.assign(a.tail_m + 1, 0);
    a.cross_row.clear();
    a.cross_q0.clear();
    for (int32_t c = 0; c < a.tail_m; c++) {
        for (int64_t q = a.lrow_ptr[t + c]; q < a.tail_lsplit[c]; q += CROSS_CHUNK) {
            a.cross_row.push_back(c);
            a.cross_q0.push_back(q);
        }
        a.cross_ptr[c + 1] = (int32_t)a.cross_row.size();
    }
    (void)nnz;
    a.t_plan_ms = ms_since(t0);
    progress("solve schedules", t_start);
    return Status::ok;
}

}  // namespace glu
