// Approximate minimum degree ordering on the pattern of A + A^T.
//
// The paper names AMD as the fill-reducing step of its preprocessing
// (Section II-C) and gives no detail.  This is an implementation written from
// the published method (Amestoy, Davis and Duff, SIAM J. Matrix Anal. Appl.
// 17(4), 1996): elimination on a quotient graph of variables and elements
// with
//  * supervariables: variables with the same element and variable
//    neighbourhoods are indistinguishable (found by hashing the two lists),
//    are merged into one weighted variable and eliminated together;
//  * mass elimination: a variable whose only neighbour left is the new
//    element is eliminated together with the pivot (no extra fill);
//  * element absorption: the pivot absorbs every element it belonged to, and
//    (aggressive absorption) every element whose variables all lie in L_p;
//  * approximate external degrees, weighted by supervariable size,
//        d_i = min(n_left - |i|, d_i_old + |L_p \ i|,
//                  |A_i \ i| + |L_p \ i| + sum_{e in E_i \ p} |L_e \ L_p|).
// Rows whose degree exceeds max(16, min(5 sqrt(n), 40 d)), d the mean degree,
// are treated as dense: they are left out of the elimination and ordered
// last, in ascending index.  (The published default cut is 10 sqrt(n); the
// lower cut also removes the high-degree supply-rail nodes of circuit
// matrices, which otherwise enter almost every pivot's element and make the
// elimination both slow and worse.  On a million-node circuit 5 sqrt(n) =
// 5,000 is the degree of a rail wired to 0.5% of the nodes, so the cut also
// follows the mean degree.)
//
// Deterministic: among supervariables of minimum approximate degree the one
// with the smallest principal index is eliminated first; a supervariable's
// principal is its smallest member, and a pivot block lists the pivot's
// members, then those of the variables mass-eliminated with it, each in
// ascending index.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <set>
#include <utility>
#include <vector>

#include "analyze.hpp"

namespace glu {

namespace {

enum : int8_t { VAR = 0, ELEM = 1, ABSORBED = 2, MERGED = 3, ELIMINATED = 4, DENSE = 5 };

}  // namespace

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
    {
        std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
        for (int32_t j = 0; j < n; j++)
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                int32_t i = rowind[p];
                if (i != j) { adj[fillp[i]++] = j; adj[fillp[j]++] = i; }
            }
    }
    std::vector<std::vector<int32_t>> adjV(n), adjE(n), Le(n);
    for (int32_t i = 0; i < n; i++) {
        std::vector<int32_t>& a = adjV[i];
        a.assign(adj.begin() + cnt[i], adj.begin() + cnt[i + 1]);
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<int32_t>().swap(adj);

    std::vector<int8_t> state(n, VAR);
    // dense-row cut: max(16, min(5 sqrt(n), 40 x the mean degree))
    int64_t deg_sum = 0;
    for (int32_t i = 0; i < n; i++) deg_sum += (int64_t)adjV[i].size();
    const double mean_deg = (double)deg_sum / (double)n;
    const double dense_lim = std::max(16.0, std::min(5.0 * std::sqrt((double)n), 40.0 * mean_deg));
    std::vector<int32_t> dense;
    for (int32_t i = 0; i < n; i++)
        if ((double)adjV[i].size() > dense_lim) { state[i] = DENSE; dense.push_back(i); }
    int64_t nleft = n - (int64_t)dense.size();

    std::vector<int64_t> nv(n, 1);        // supervariable weight (principal variables)
    std::vector<int64_t> deg(n, 0);       // approximate external degree (variables)
    std::vector<int64_t> edeg(n, 0);      // weighted |L_e| (elements)
    std::vector<std::vector<int32_t>> members(n);  // variables merged into a principal
    std::set<std::pair<int64_t, int32_t>> heap;
    for (int32_t i = 0; i < n; i++) {
        if (state[i] != VAR) continue;
        auto& a = adjV[i];
        a.erase(std::remove_if(a.begin(), a.end(), [&](int32_t v) { return state[v] == DENSE; }),
                a.end());
        deg[i] = (int64_t)a.size();
        heap.insert({deg[i], i});
    }

    std::vector<int32_t> mark(n, -1), wstamp(n, -1), cmpmark(n, -1);
    std::vector<int64_t> w(n, 0), ext(n, 0), aw(n, 0);
    std::vector<uint64_t> hsh(n, 0);
    std::vector<int32_t> Lp, block, bucket_order;
    int32_t step = 0, cmpstamp = 0;
    auto emit = [&](int32_t v) {
        perm.push_back(v);
        std::vector<int32_t>& mv = members[v];
        std::sort(mv.begin(), mv.end());
        for (int32_t u : mv) perm.push_back(u);
        std::vector<int32_t>().swap(mv);
    };
    while (!heap.empty()) {
        const int32_t p = heap.begin()->second;
        heap.erase(heap.begin());
        step++;
        nleft -= nv[p];
        // L_p = (A_p u union of L_e over e in E_p) \ {p}, live principal variables
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
        int64_t dp = 0;
        for (int32_t i : Lp) {
            dp += nv[i];
            heap.erase({deg[i], i});
        }
        // |L_e \ L_p| (weighted) for every other element adjacent to L_p
        for (int32_t i : Lp) {
            for (int32_t e : adjE[i]) {
                if (state[e] != ELEM) continue;
                if (wstamp[e] != step) { w[e] = edeg[e]; wstamp[e] = step; }
                w[e] -= nv[i];
            }
        }
        // clean the lists of L_p's variables, external degrees, mass elimination
        block.clear();
        for (int32_t i : Lp) {
            auto& ei = adjE[i];
            int64_t x = 0;
            size_t o = 0;
            for (size_t q = 0; q < ei.size(); q++) {
                const int32_t e = ei[q];
                if (state[e] != ELEM) continue;
                if (w[e] <= 0) {  // L_e lies inside L_p: absorbed by p
                    state[e] = ABSORBED;
                    std::vector<int32_t>().swap(Le[e]);
                    continue;
                }
                x += w[e];
                ei[o++] = e;
            }
            ei.resize(o);
            auto& ai = adjV[i];
            int64_t a = 0;
            o = 0;
            for (size_t q = 0; q < ai.size(); q++) {
                const int32_t v = ai[q];
                if (state[v] != VAR || mark[v] == step) continue;
                a += nv[v];
                ai[o++] = v;
            }
            ai.resize(o);
            if (ei.empty() && ai.empty()) {  // adjacent to p alone: eliminate with p
                state[i] = ELIMINATED;
                block.push_back(i);
                dp -= nv[i];
                nleft -= nv[i];
                continue;
            }
            ext[i] = x;
            aw[i] = a;
            uint64_t h = (uint64_t)p;
            for (int32_t e : ei) h += (uint64_t)e * 0x9E3779B97F4A7C15ull;
            for (int32_t v : ai) h += (uint64_t)v * 0xC2B2AE3D27D4EB4Full + 0x165667B19E3779F9ull;
            hsh[i] = h;
        }
        {
            size_t o = 0;
            for (int32_t i : Lp)
                if (state[i] == VAR) Lp[o++] = i;
            Lp.resize(o);
        }
        // supervariables: equal hashes, then equal element and variable lists
        bucket_order.assign(Lp.begin(), Lp.end());
        std::sort(bucket_order.begin(), bucket_order.end(), [&](int32_t x, int32_t y) {
            return hsh[x] != hsh[y] ? hsh[x] < hsh[y] : x < y;
        });
        for (size_t s = 0; s < bucket_order.size();) {
            size_t e = s + 1;
            while (e < bucket_order.size() && hsh[bucket_order[e]] == hsh[bucket_order[s]]) e++;
            for (size_t a = s; a < e; a++) {
                const int32_t i = bucket_order[a];
                if (state[i] != VAR) continue;
                cmpstamp++;
                for (int32_t x : adjE[i]) cmpmark[x] = cmpstamp;
                for (int32_t x : adjV[i]) cmpmark[x] = cmpstamp;
                for (size_t b = a + 1; b < e; b++) {
                    const int32_t j = bucket_order[b];
                    if (state[j] != VAR || adjE[j].size() != adjE[i].size() ||
                        adjV[j].size() != adjV[i].size())
                        continue;
                    bool same = true;
                    for (int32_t x : adjE[j]) if (cmpmark[x] != cmpstamp) { same = false; break; }
                    if (same)
                        for (int32_t x : adjV[j]) if (cmpmark[x] != cmpstamp) { same = false; break; }
                    if (!same) continue;
                    // i < j (bucket sorted by index): j joins i
                    nv[i] += nv[j];
                    nv[j] = 0;
                    state[j] = MERGED;
                    members[i].push_back(j);
                    members[i].insert(members[i].end(), members[j].begin(), members[j].end());
                    std::vector<int32_t>().swap(members[j]);
                    std::vector<int32_t>().swap(adjE[j]);
                    std::vector<int32_t>().swap(adjV[j]);
                }
            }
            s = e;
        }
        // the new element, degrees of its variables
        {
            size_t o = 0;
            for (int32_t i : Lp)
                if (state[i] == VAR) Lp[o++] = i;
            Lp.resize(o);
        }
        for (int32_t i : Lp) {
            const int64_t lpi = dp - nv[i];
            int64_t d = aw[i] + lpi + ext[i];
            d = std::min(d, deg[i] + lpi);
            d = std::min(d, nleft - nv[i]);
            if (d < 0) d = 0;
            deg[i] = d;
            adjE[i].push_back(p);
            heap.insert({d, i});
        }
        Le[p] = Lp;
        edeg[p] = dp;
        // pivot block: p's supervariable, then the mass-eliminated ones
        emit(p);
        std::sort(block.begin(), block.end());
        for (int32_t v : block) emit(v);
    }
    for (int32_t i : dense) perm.push_back(i);
    return perm;
}

}  // namespace glu
