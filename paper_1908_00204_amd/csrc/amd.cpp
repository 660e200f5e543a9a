// Approximate minimum degree ordering on the pattern of A + A^T.
//
// The paper names AMD as the fill-reducing step of its preprocessing
// (Section II-C) and gives no detail.  This is an implementation written from
// the published method (Amestoy, Davis and Duff, SIAM J. Matrix Anal. Appl.
// 17(4), 1996): elimination on a quotient graph of variables and elements,
// approximate external degrees
//     d_i = min(n_left - 1, d_i_old + |L_p \ i|,
//               |A_i \ i| + |L_p \ i| + sum_{e in E_i \ p} |L_e \ L_p|),
// and element absorption (an element whose variables all lie in L_p is
// absorbed by p).  Rows whose degree exceeds max(16, min(5 sqrt(n), 40 d)),
// d the mean degree, are treated as dense: they are left out of the
// elimination and ordered last, in ascending index.  (The published default
// cut is 10 sqrt(n); the lower cut also removes the high-degree supply-rail
// nodes of circuit matrices, which otherwise enter almost every pivot's
// element and make the elimination both slow and worse.  On a million-node
// circuit 5 sqrt(n) = 5,000 is the degree of a rail wired to 0.5% of the
// nodes, so the cut also follows the mean degree.)
//
// Deterministic tie-break: among variables of minimum approximate degree, the
// smallest original index is eliminated first.  Supervariable detection and
// mass elimination are not implemented (a quality-neutral speed device).
#include <algorithm>
#include <cmath>
#include <set>
#include <utility>
#include <vector>

#include "analyze.hpp"

namespace glu {

std::vector<int32_t> amd_order(int32_t n, const int64_t* colptr, const int32_t* rowind) {
    std::vector<int32_t> perm;
    perm.reserve(n);
    if (n <= 0) return perm;

    // symmetric adjacency without the diagonal, deduplicated
    std::vector<int64_t> cnt(n + 1, 0);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i != j) { cnt[i + 1]++; cnt[j + 1]++; }
        }
    for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    std::vector<int32_t> adj(cnt[n]);
    std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
            int32_t i = rowind[p];
            if (i != j) { adj[fillp[i]++] = j; adj[fillp[j]++] = i; }
        }
    std::vector<std::vector<int32_t>> adjV(n), adjE(n), Le(n);
    for (int32_t i = 0; i < n; i++) {
        std::vector<int32_t>& a = adjV[i];
        a.assign(adj.begin() + cnt[i], adj.begin() + cnt[i + 1]);
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<int32_t>().swap(adj);

    enum : int8_t { VAR = 0, ELEM = 1, ABSORBED = 2, DENSE = 3 };
    std::vector<int8_t> state(n, VAR);
    // dense-row cut: max(16, min(5 sqrt(n), 40 x the mean degree))
    int64_t deg_sum = 0;
    for (int32_t i = 0; i < n; i++) deg_sum += (int64_t)adjV[i].size();
    const double mean_deg = (double)deg_sum / (double)n;
    const double dense_lim = std::max(16.0, std::min(5.0 * std::sqrt((double)n), 40.0 * mean_deg));
    std::vector<int32_t> dense;
    for (int32_t i = 0; i < n; i++)
        if ((double)adjV[i].size() > dense_lim) { state[i] = DENSE; dense.push_back(i); }
    int32_t nleft = n - (int32_t)dense.size();
    std::vector<int64_t> deg(n, 0);
    std::set<std::pair<int64_t, int32_t>> heap;
    for (int32_t i = 0; i < n; i++) {
        if (state[i] != VAR) continue;
        auto& a = adjV[i];
        a.erase(std::remove_if(a.begin(), a.end(), [&](int32_t v) { return state[v] == DENSE; }),
                a.end());
        deg[i] = (int64_t)a.size();
        heap.insert({deg[i], i});
    }

    std::vector<int32_t> mark(n, -1), wstamp(n, -1);
    std::vector<int64_t> w(n, 0);
    std::vector<int32_t> Lp;
    int32_t step = 0;
    while (!heap.empty()) {
        const int32_t p = heap.begin()->second;
        heap.erase(heap.begin());
        perm.push_back(p);
        nleft--;
        step++;
        // L_p = (A_p u union of L_e over e in E_p) \ {p}, restricted to live variables
        Lp.clear();
        mark[p] = step;
        for (int32_t v : adjV[p])
            if (state[v] == VAR && mark[v] != step) { mark[v] = step; Lp.push_back(v); }
        for (int32_t e : adjE[p]) {
            if (state[e] != ELEM) continue;
            for (int32_t v : Le[e])
                if (state[v] == VAR && mark[v] != step) { mark[v] = step; Lp.push_back(v); }
            state[e] = ABSORBED;
            std::vector<int32_t>().swap(Le[e]);
        }
        state[p] = ELEM;
        std::vector<int32_t>().swap(adjV[p]);
        std::vector<int32_t>().swap(adjE[p]);
        std::sort(Lp.begin(), Lp.end());
        Le[p] = Lp;
        for (int32_t i : Lp) heap.erase({deg[i], i});
        // |L_e \ L_p| for every other element adjacent to a variable of L_p
        for (int32_t i : Lp) {
            for (int32_t e : adjE[i]) {
                if (state[e] != ELEM || e == p) continue;
                if (wstamp[e] != step) {
                    // a live element keeps all its variables: eliminating any of
                    // them absorbs the element, so |L_e| is its list's length
                    w[e] = (int64_t)Le[e].size();
                    wstamp[e] = step;
                }
                w[e] -= 1;
            }
        }
        const int64_t lp1 = (int64_t)Lp.size() - 1;
        for (int32_t i : Lp) {
            auto& ei = adjE[i];
            int64_t ext = 0;
            size_t o = 0;
            for (size_t q = 0; q < ei.size(); q++) {
                int32_t e = ei[q];
                if (state[e] != ELEM || e == p) continue;
                if (w[e] <= 0) {  // L_e is inside L_p: absorbed by p
                    state[e] = ABSORBED;
                    std::vector<int32_t>().swap(Le[e]);
                    continue;
                }
                ext += w[e];
                ei[o++] = e;
            }
            ei.resize(o);
            ei.push_back(p);
            auto& ai = adjV[i];
            ai.erase(std::remove_if(ai.begin(), ai.end(),
                                    [&](int32_t v) { return state[v] != VAR || mark[v] == step; }),
                     ai.end());
            int64_t d = (int64_t)ai.size() + lp1 + ext;
            d = std::min(d, deg[i] + lp1);
            d = std::min(d, (int64_t)nleft - 1);
            if (d < 0) d = 0;
            deg[i] = d;
            heap.insert({d, i});
        }
    }
    for (int32_t i : dense) perm.push_back(i);
    return perm;
}

}  // namespace glu
