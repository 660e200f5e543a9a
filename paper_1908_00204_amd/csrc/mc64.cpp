// Maximum-product transversal and scaling (the MC64 step of the paper's
// preprocessing, Section II-C), written from the published method (Duff and
// Koster, SIAM J. Matrix Anal. Appl. 22(4), 2001: a weighted bipartite
// matching by shortest augmenting paths, with the dual variables giving the
// scaling).
//
// Rows are matched to columns so that the product of the matched magnitudes
// is largest: with c(i,j) = log max_k |a(k,j)| - log |a(i,j)| >= 0 this is a
// minimum-cost perfect matching.  For each column in turn, a Dijkstra search
// over reduced costs c(i,j) - u(i) - v(j) >= 0 finds the cheapest augmenting
// path to a free row; the duals are then updated so that the reduced costs
// stay non-negative and are zero on the matched pairs.  Scaling: with
// Dr(i) = exp(u(i)), Dc(j) = exp(v(j)) / max_k |a(k,j)|, every entry of
// Dr A Dc has magnitude at most 1 and the matched ones exactly 1 (up to
// rounding).  Row permutation: row perm[j] of A is matched to column j, so
// (Q A)(j,j) = A(perm[j], j) is the matched entry.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <limits>
#include <queue>
#include <utility>
#include <vector>

#include "analyze.hpp"

namespace glu {

Status mc64_scale(int32_t n, const int64_t* colptr, const int32_t* rowind, const double* values,
                  std::vector<int32_t>& row_of_col, std::vector<double>& rscale, std::vector<double>& cscale) {
    Status st = validate_csc(n, colptr, rowind);
    if (st != Status::ok) return st;
    if (n > 0 && !values) return Status::arg;
    const double inf = std::numeric_limits<double>::infinity();
    // costs, column by column
    std::vector<double> cost(n > 0 ? colptr[n] : 0), cmax(n, 0.0);
    for (int32_t j = 0; j < n; j++) {
        double mx = 0.0;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            if (!std::isfinite(values[p])) return Status::nonfinite;
            mx = std::max(mx, std::fabs(values[p]));
        }
        if (mx == 0.0) return Status::struct_singular;  // an empty (or all-zero) column
        cmax[j] = mx;
        const double lm = std::log(mx);
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++)
            cost[p] = values[p] != 0.0 ? lm - std::log(std::fabs(values[p])) : inf;
    }
    std::vector<double> u(n, 0.0), v(n, 0.0);        // row and column duals
    std::vector<int32_t> col_of_row(n, -1);
    row_of_col.assign(n, -1);
    // initial duals and a cheap matching: v(j) = min_i c(i,j), then match a
    // column to a free row where the reduced cost is zero
    for (int32_t j = 0; j < n; j++) {
        double mn = inf;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) mn = std::min(mn, cost[p]);
        v[j] = mn;
    }
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            const int32_t i = rowind[p];
            if (col_of_row[i] < 0 && cost[p] - v[j] == 0.0) {
                col_of_row[i] = j;
                row_of_col[j] = i;
                break;
            }
        }
    // shortest augmenting paths for the unmatched columns
    std::vector<double> dist(n, inf);
    std::vector<int32_t> pred_col(n, -1), touched, settled;  // pred_col[i]: column reaching row i
    std::vector<char> done(n, 0);
    using QE = std::pair<double, int32_t>;
    for (int32_t j0 = 0; j0 < n; j0++) {
        if (row_of_col[j0] >= 0) continue;
        std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
        touched.clear();
        // relax the edges of column j from distance dj
        auto relax = [&](int32_t j, double dj) {
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                if (cost[p] == inf) continue;
                const int32_t i = rowind[p];
                if (done[i]) continue;
                const double nd = dj + (cost[p] - u[i] - v[j]);
                if (nd < dist[i]) {
                    if (dist[i] == inf) touched.push_back(i);
                    dist[i] = nd;
                    pred_col[i] = j;
                    pq.push({nd, i});
                }
            }
        };
        relax(j0, 0.0);
        int32_t free_row = -1;
        double dfree = inf;
        settled.clear();
        while (!pq.empty()) {
            const auto [d, i] = pq.top();
            pq.pop();
            if (done[i] || d > dist[i]) continue;
            done[i] = 1;
            settled.push_back(i);
            if (col_of_row[i] < 0) {
                free_row = i;
                dfree = d;
                break;
            }
            // continue through the column matched to row i (zero reduced cost)
            relax(col_of_row[i], d);
        }
        if (free_row < 0) {
            for (int32_t i : touched) { dist[i] = inf; done[i] = 0; pred_col[i] = -1; }
            return Status::struct_singular;  // no perfect matching
        }
        // dual update: a column reached at distance d and a row settled at
        // distance d both move by dfree - d (the root column j0 by dfree), which
        // keeps every reduced cost non-negative and makes the path's edges tight
        v[j0] += dfree;
        for (int32_t i : settled) {
            const double delta = dfree - dist[i];
            if (delta > 0) {
                u[i] -= delta;
                if (col_of_row[i] >= 0) v[col_of_row[i]] += delta;
            }
        }
        for (int32_t i = free_row; i >= 0;) {
            const int32_t j = pred_col[i];
            const int32_t iprev = row_of_col[j];
            row_of_col[j] = i;
            col_of_row[i] = j;
            i = (j == j0) ? -1 : iprev;
        }
        for (int32_t i : touched) { dist[i] = inf; done[i] = 0; pred_col[i] = -1; }
    }
    // make every matched reduced cost exactly zero (v(j) = c(m(j), j) - u(m(j)))
    for (int32_t j = 0; j < n; j++) {
        const int32_t i = row_of_col[j];
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++)
            if (rowind[p] == i) { v[j] = cost[p] - u[i]; break; }
    }
    rscale.resize(n);
    cscale.resize(n);
    for (int32_t i = 0; i < n; i++) rscale[i] = std::exp(u[i]);
    for (int32_t j = 0; j < n; j++) cscale[j] = std::exp(v[j]) / cmax[j];
    return Status::ok;
}

}  // namespace glu
