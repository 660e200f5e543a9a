// HIP kernels for gfx950 (MI355X): value load, the level-by-level right-looking
// numeric factorization and the triangular solves (one launch each, walking
// the level schedule).
//
// Factorization (Alg. 2 with the submatrix update of Alg. 5, run level by level
// over the levels of the relaxed dependency DAG of Alg. 4).  For the columns j
// of one level the submatrix update is
//     A_s(i,k) -= L(i,j) * U(j,k)   for k with U(j,k) != 0, i in struct(L(:,j)),
// where L(i,j) = A_s(i,j) / A_s(j,j) (Alg. 2's normalisation).  The kernels
// regroup one level's update by target column k: a work item owns a contiguous
// range of column k's entries and applies every source j of the level that hits
// k, in ascending j, so concurrent columns of a level never write the same
// entry (no atomics, bitwise repeatable).  The two-level parallelism of
// Section III-B (subcolumns of a column, elements of a subcolumn) becomes:
// work items over (subcolumn k, element range), lanes over the rows of L(:,j).
//
// The normalisation is fused: an update task reads the not yet divided A_s(i,j)
// and divides it by the pivot itself (IEEE division, the same operation and
// result as the stored L(i,j)), and the stored column L(:,j) of a level is
// divided in the next level's launch (no column of the next level reads or
// writes it) or in the final launch.
//
// Kernel modes follow the paper's three level types (Section III-B): wide
// levels run small workgroups (one wave64, "small block"), medium levels run
// 256-lane workgroups ("large block"), and narrow levels ("stream" mode, at most
// 16 columns) split every subcolumn into many element ranges so that the whole
// device works on few columns at once -- one launch per level in all modes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "mailbox.hpp"

namespace glu {

namespace {

constexpr int kChunk = 256;  // largest target slice a work item stages in LDS
constexpr int kChunkLarge = 64;  // slices of large-block mode: more work items per column
constexpr int64_t kMaxGrid = (int64_t)1 << 24;  // workgroups per launch of the one-wave kernels
static_assert(kChunk <= 256, "slice offsets and touched-entry indices are stored as bytes");

__device__ __forceinline__ int32_t lds_lower_bound(const int32_t* s, int32_t len, int32_t key) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (s[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t gl_lower_bound(const int32_t* __restrict__ r, int64_t lo, int64_t hi,
                                                  int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (r[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class T>
__global__ void k_fill(T* __restrict__ v, int64_t n, T x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) v[i] = x;
}

// Zero the entries of column t + c above row t (block c, c < m): the part of
// the dense block's columns that the sparse levels update.
template <class T>
__global__ void k_fill_heads(const int64_t* __restrict__ colptr, const int64_t* __restrict__ tail_pos, int32_t t,
                             int32_t m, T* __restrict__ v) {
    const int32_t c = blockIdx.x;
    if (c >= m) return;
    for (int64_t p = colptr[t + c] + threadIdx.x; p < tail_pos[c]; p += blockDim.x) v[p] = (T)0;
}

__global__ void k_status_reset(int32_t* status, int32_t* counters, int32_t ncount) {
    if (threadIdx.x == 0) {
        status[0] = INT32_MAX;  // smallest failed pivot column
        status[1] = 0;          // non-finite input seen
        status[2] = 0;          // synchronisation error (a bounded wait gave up)
    }
    for (int32_t i = threadIdx.x; i < ncount; i += blockDim.x) counters[i] = 0;
}

// a5: value load, A_s.val[amap[p]] = A.val[p] (fill entries were zeroed before)
// (in the FP32 form the value is rounded to float here: the factorization's
// only conversion of the input)
template <class T>
__global__ void k_scatter_values(const double* __restrict__ a, const int64_t* __restrict__ amap,
                                 int64_t nnz_a, T* __restrict__ v, int32_t* __restrict__ status) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; p < nnz_a; p += stride) {
        const double x = a[p];
        const T y = (T)x;
        bad |= !isfinite(x) || !isfinite(y);
        v[amap[p]] = y;
    }
    if (bad) atomicOr(&status[1], 1);
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        int32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}


// Metadata of the sources of one batch of a work item, one source per lane:
// its L range [qb, qe) (restricted to the slice), U(j,k) and its pivot.  Sources are all of the task's (whole) or the item's listed
// subset, in ascending order.
template <class T = double>
struct Batch {
    int64_t qb, qe;
    T u, d;
};

template <class T = double>
__device__ __forceinline__ Batch<T> load_batch(const FactorArgs& args, const T* __restrict__ val, bool whole,
                                               int64_t s0, int64_t e0s, int64_t nsrc, int64_t ib, int lane,
                                               bool with_values) {
    Batch<T> B = {0, 0, (T)0, (T)0};
    if (ib + lane < nsrc) {
        int64_t up, dp;
        int32_t lo, hi;
        if (whole) {
            const int64_t s = s0 + ib + lane;
            lo = 0;
            hi = args.src_llen[s];
            up = args.src_upos[s];
            dp = args.src_dpos[s];
        } else {
            const int64_t e = e0s + ib + lane;
            lo = args.ss_lo[e];
            hi = args.ss_hi[e];
            up = args.ss_up[e];
            dp = args.ss_dp[e];
        }
        if (with_values) {
            B.u = val[up];
            B.d = val[dp];
        }
        B.qb = dp + 1 + lo;
        B.qe = dp + 1 + hi;
    }
    return B;
}

// Position q in A_s of pair e (e < total) of a batch whose per-lane counts are
// cnt with inclusive prefix incl, and the lane that holds its source.  Every
// lane must be active (the shuffles); lanes past the end get a clamped pair.
__device__ __forceinline__ int64_t pair_position(int32_t e, int32_t total, int32_t cnt, int32_t incl, int64_t qb,
                                                 int32_t& src) {
    const int32_t ec = min(e, total - 1);
    src = 0;  // number of lanes whose inclusive count is <= ec
#pragma unroll
    for (int st = 32; st > 0; st >>= 1)
        if (__shfl(incl, src + st - 1, 64) <= ec) src += st;
    const int32_t excl = __shfl(incl, src, 64) - __shfl(cnt, src, 64);
    return __shfl(qb, src, 64) + (ec - excl);
}

// Analysis pass over work items [wi0, wi0 + nwi) (pattern only, no values):
// for each slice, the entries its pairs touch (offsets from the slice start,
// ascending, written at touch_off + wi_tbase) and their count, and for every
// pair, in the order the level kernel enumerates them (pair_pos + wi_pbase):
// the index of its target in that list (low byte) and its rank among the
// lanes of its 64-pair step that hit the same target (high byte; lane order).
// A pair whose row is missing from its slice sets err (the plan would be
// inconsistent).
__global__ __launch_bounds__(64) void k_level_map(const FactorArgs args, int64_t wi0, int64_t nwi,
                                                  uint8_t* __restrict__ touch_off, uint16_t* __restrict__ pair_pos,
                                                  int32_t* __restrict__ wi_ntouch, int32_t* __restrict__ err) {
    constexpr int CH = kChunk;
    const int32_t* __restrict__ rowind = args.rowind;
    const int lane = threadIdx.x;
    const int64_t wi = wi0 + blockIdx.x;
    if ((int64_t)blockIdx.x >= nwi) return;
    __shared__ int32_t srow[CH];
    __shared__ int32_t sidx[CH];
    const int64_t pb = args.wi_begin[wi];
    const int32_t len = (int32_t)(args.wi_end[wi] - pb);
    const int64_t s0 = args.wi_s0[wi], nsrc = args.wi_nsrc[wi], e0s = args.wi_ss[wi];
    const bool whole = args.wi_whole[wi] != 0;
    for (int32_t x = lane; x < CH; x += 64) {
        srow[x] = x < len ? rowind[pb + x] : INT32_MAX;
        sidx[x] = 0;
    }
    __syncthreads();
    // pass 0 marks touched entries, pass 1 writes each pair's index
    for (int pass = 0; pass < 2; pass++) {
        int64_t pdone = 0;
        for (int64_t ib = 0; ib < nsrc; ib += 64) {
            const Batch<> B = load_batch<double>(args, nullptr, whole, s0, e0s, nsrc, ib, lane, false);
            const int32_t cnt = (int32_t)(B.qe - B.qb);
            const int32_t incl = wave_incl_scan(cnt, lane);
            const int32_t total = __shfl(incl, 63, 64);
            for (int32_t e0 = 0; e0 < total; e0 += 64) {
                int32_t src;
                const int64_t q = pair_position(e0 + lane, total, cnt, incl, B.qb, src);
                int32_t tgt = -1;  // this lane's target index (pass 1), -1 for none
                if (e0 + lane < total) {
                    const int32_t i = rowind[q];
                    const int32_t p = lds_lower_bound(srow, len, i);
                    const bool found = p < len && srow[p] == i;
                    if (!found) atomicOr(err, 8);
                    if (pass == 0) {
                        if (found) sidx[p] = 1;
                    } else {
                        tgt = found ? sidx[p] : 0;
                    }
                }
                if (pass == 1) {
                    // rank: earlier lanes of this step with the same target
                    int32_t rank = 0;
                    for (int s = 0; s < 64; s++) {
                        const int32_t ts = __shfl(tgt, s, 64);
                        if (s < lane && tgt >= 0 && ts == tgt) rank++;
                    }
                    if (tgt >= 0) pair_pos[args.wi_pbase[wi] + pdone + e0 + lane] = (uint16_t)(tgt | (rank << 8));
                }
            }
            pdone += total;
        }
        __syncthreads();
        if (pass == 0) {
            // exclusive prefix over the marks: lane owns entries 4 lane .. 4 lane + 3
            int32_t m[CH / 64], sum = 0;
#pragma unroll
            for (int k = 0; k < CH / 64; k++) {
                m[k] = sidx[(CH / 64) * lane + k];
                sum += m[k];
            }
            const int32_t incl2 = wave_incl_scan(sum, lane);
            int32_t run = incl2 - sum;
#pragma unroll
            for (int k = 0; k < CH / 64; k++) {
                const int32_t x = (CH / 64) * lane + k;
                if (m[k]) touch_off[args.wi_tbase[wi] + run] = (uint8_t)x;
                sidx[x] = run;
                run += m[k];
            }
            if (lane == 63) wi_ntouch[wi] = incl2;
            __syncthreads();
        }
    }
}

// Value access of the level kernels.  The per-level launches use plain loads
// and stores (kernel boundaries order the levels).  The persistent
// stream-mode kernel hands values between levels inside one launch, across
// the XCDs' separate L2 caches, so it reads and writes every factor value
// with agent-scope relaxed atomics (served by the device-wide coherence
// point, never by a stale L2 line) and orders them with a completion counter.
template <bool COH, class T>
__device__ __forceinline__ T vload(const T* p) {
    if constexpr (COH) {
        static_assert(sizeof(T) == 8, "coherent access is used by the FP64 stream kernel only");
        return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const uint64_t*>(p),
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    } else {
        return *p;
    }
}
template <bool COH, class T>
__device__ __forceinline__ void vstore(T* p, T x) {
    if constexpr (COH) {
        static_assert(sizeof(T) == 8, "coherent access is used by the FP64 stream kernel only");
        __hip_atomic_store(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(x), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        *p = x;
    }
}

// Metadata of one batch of sources, as load_batch, with the values read
// through vload.
template <bool COH, class T>
__device__ __forceinline__ Batch<T> load_batch_v(const FactorArgs& args, const T* __restrict__ val, bool whole,
                                                 int64_t s0, int64_t e0s, int64_t nsrc, int64_t ib, int lane) {
    Batch<T> B = load_batch<T>(args, nullptr, whole, s0, e0s, nsrc, ib, lane, false);
    if (ib + lane < nsrc) {
        const int64_t up = whole ? args.src_upos[s0 + ib + lane] : args.ss_up[e0s + ib + lane];
        const int64_t dp = whole ? args.src_dpos[s0 + ib + lane] : args.ss_dp[e0s + ib + lane];
        B.u = vload<COH>(val + up);
        B.d = vload<COH>(val + dp);
    }
    return B;
}

// Divide the L entries of column j by its pivot (one wave).
template <bool COH, class T>
__device__ __forceinline__ void normalise_column(const FactorArgs& args, T* __restrict__ val, int32_t j, int lane) {
    const int64_t dj = args.diag[j];
    const T d = vload<COH>(val + dj);
    for (int64_t q = dj + 1 + lane; q < args.colptr[j + 1]; q += 64) vstore<COH>(val + q, vload<COH>(val + q) / d);
}

// One work item (one wave): a slice of target column k (at most CH entries)
// and every source j of the level with U(j,k) != 0 whose L rows reach the
// slice, taken in ascending j.  Only the entries of the slice that some pair
// updates are staged in LDS (their offsets come from the analysis map), and
// every pair carries the index of its target in that list, so no row index
// is read or searched.  The (source, L-row) pairs are flattened: metadata for
// 64 sources is loaded one per lane, a wave prefix sum over their L lengths
// numbers the pairs, and lane e of each step handles pair e.  Pairs are
// applied in pair order, and lanes of one step that hit the same target entry
// are applied lowest lane first, so every entry receives its updates in
// ascending source order -- the sequential order of Alg. 2 within a level --
// and the result is bitwise repeatable.
template <int CH, bool COH, class T>
__device__ __forceinline__ void level_work_item(const FactorArgs& args, T* __restrict__ val, int64_t wi, int lane,
                                                T* __restrict__ sval, uint8_t* __restrict__ soff) {
    // everything about the work item is one level of independent loads
    const int64_t pb = args.wi_begin[wi];
    const int32_t nt = args.wi_ntouch[wi];
    const int64_t tb = args.wi_tbase[wi];
    const int64_t pbase = args.wi_pbase[wi];
    const int64_t s0 = args.wi_s0[wi];
    const int64_t nsrc = args.wi_nsrc[wi];
    const bool whole = args.wi_whole[wi] != 0;
    const int64_t e0s = args.wi_ss[wi];
    // the first batch's metadata and the touched entries are fetched together
    Batch<T> B = COH ? load_batch_v<COH, T>(args, val, whole, s0, e0s, nsrc, 0, lane)
                     : load_batch<T>(args, val, whole, s0, e0s, nsrc, 0, lane, true);
    constexpr int SPL = CH / 64;
    {
        int32_t off[SPL];
        T vv[SPL];
#pragma unroll
        for (int k = 0; k < SPL; k++) {
            const int32_t x = lane + 64 * k;
            off[k] = x < nt ? (int32_t)args.touch_off[tb + x] : 0;
        }
#pragma unroll
        for (int k = 0; k < SPL; k++)
            if (lane + 64 * k < nt) vv[k] = vload<COH>(val + pb + off[k]);
#pragma unroll
        for (int k = 0; k < SPL; k++) {
            const int32_t x = lane + 64 * k;
            if (x < nt) {
                sval[x] = vv[k];
                soff[x] = (uint8_t)off[k];
            }
        }
    }
    __syncthreads();
    int64_t pdone = 0;
    for (int64_t ib = 0; ib < nsrc; ib += 64) {
        if (ib > 0)
            B = COH ? load_batch_v<COH, T>(args, val, whole, s0, e0s, nsrc, ib, lane)
                    : load_batch<T>(args, val, whole, s0, e0s, nsrc, ib, lane, true);
        const int32_t cnt = (int32_t)(B.qe - B.qb);
        const int32_t incl = wave_incl_scan(cnt, lane);
        const int32_t total = __shfl(incl, 63, 64);
        // Steps of 64 pairs, software-pipelined two steps deep: the global
        // loads of steps s+1 and s+2 are in flight during the LDS work of step
        // s.  The step loop is uniform across the wave and every shuffle runs
        // with all lanes active.
        struct Pair {
            int32_t pos;  // target index | rank << 8, or -1
            T a, u, d;
        };
        auto fetch = [&](int32_t e0, Pair& P) {
            const int32_t e = e0 + lane;
            int32_t src;
            const int64_t q = pair_position(e, total, cnt, incl, B.qb, src);
            P.pos = -1;
            P.a = (T)0;
            if (e < total) {
                P.pos = args.pair_pos[pbase + pdone + e];
                P.a = vload<COH>(val + q);
            }
            P.u = __shfl(B.u, src, 64);
            P.d = __shfl(B.d, src, 64);
        };
        auto apply = [&](int32_t pos, T l, T uu) {
            // lanes sharing an entry go in rank order, i.e. lowest lane first
            bool pending = pos >= 0;
            const int32_t t = pos & 0xff, rank = pos >> 8;
            for (int32_t r = 0; __ballot(pending); r++) {
                if (pending && rank == r) {
                    sval[t] = fma(-l, uu, sval[t]);
                    pending = false;
                }
            }
        };
        Pair PA, PB;
        if (total > 0) fetch(0, PA);
        if (total > 64) fetch(64, PB);
        for (int32_t e0 = 0; e0 < total; e0 += 128) {
            {
                const int32_t pos = PA.pos;
                const T l = PA.a / PA.d, uu = PA.u;
                if (e0 + 128 < total) fetch(e0 + 128, PA);
                apply(pos, l, uu);
            }
            if (e0 + 64 < total) {
                const int32_t pos = PB.pos;
                const T l = PB.a / PB.d, uu = PB.u;
                if (e0 + 192 < total) fetch(e0 + 192, PB);
                apply(pos, l, uu);
            }
        }
        pdone += total;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SPL; k++) {
        const int32_t x = lane + 64 * k;
        if (x < nt) vstore<COH>(val + pb + soff[x], sval[x]);
    }
}

// Large-block mode: one launch per level, one wave per block.  Blocks
// [0, nwi) are work items (level_work_item); blocks [nwi, nwi + nnorm) divide
// the L columns of the previous level by their pivots.
template <int CH, class T>
__global__ __launch_bounds__(64) void k_level(const FactorArgs args, T* __restrict__ val, int64_t wi0, int64_t nwi,
                                              const int32_t* __restrict__ norm_cols, int32_t nnorm) {
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    if (b >= nwi) {
        const int64_t c = b - nwi;
        if (c < nnorm) normalise_column<false>(args, val, norm_cols[c], lane);
        return;
    }
    __shared__ T sval[CH];
    __shared__ uint8_t soff[CH];
    level_work_item<CH, false, T>(args, val, wi0 + b, lane, sval, soff);
}

// Batched level wavefront: level e of many factorizations in one launch
// (glu_batch_factor).  Entry x covers workgroups [ent[x].boff, ent[x+1].boff):
// handle ent[x].h's work items [wi0, wi0 + nwi) of its level e, then the
// normalisation of its level e-1's columns.  Each workgroup finds its entry by
// binary search and runs the same work item as k_level with that handle's
// arguments, so every factorization gets the same results as alone.
template <int CH, class T>
__global__ __launch_bounds__(64) void k_level_batch(const FactorArgs* __restrict__ args,
                                                    const BatchEntry* __restrict__ ent, int32_t nent) {
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    int32_t x = 0;
    for (int32_t st = 1 << 20; st > 0; st >>= 1)
        if (x + st < nent && ent[x + st].boff <= b) x += st;
    const BatchEntry E = ent[x];
    const FactorArgs a = args[E.h];
    T* val;
    if constexpr (sizeof(T) == 4) val = a.val32; else val = a.val;
    const int64_t off = b - E.boff;
    if (off >= E.nwi) {
        if (off - E.nwi < E.nnorm) normalise_column<false>(a, val, E.norm[off - E.nwi], lane);
        return;
    }
    __shared__ T sval[CH];
    __shared__ uint8_t soff[CH];
    level_work_item<CH, false, T>(a, val, E.wi0 + off, lane, sval, soff);
}

// Stream mode: a run of consecutive narrow levels (at most the stream
// threshold of columns each) in one persistent launch instead of one launch
// per level.  The run is a sequence of segments, one per level e: the level's
// work items, then the normalisation of level e-1's columns (which no item of
// level e reads or writes); seg[s] is the first item index of segment s.
// Waves claim items one at a time, in increasing order, from an atomic
// ticket; an item of segment s starts once `done` (items finished) reaches
// seg[s], i.e. once every earlier level has finished, and counts itself
// into `done` when its values are stored.  The earliest unfinished item
// belongs to a running wave and waits for nothing unfinished, so the run
// progresses whether or not the whole grid is resident.  Every wait is
// bounded; a wait that gives up sets bit 4 of err and the wave leaves.
template <int CH>
__global__ __launch_bounds__(64) void k_level_stream(const FactorArgs args, const int64_t* __restrict__ seg,
                                                     int32_t nseg, const int64_t* __restrict__ wi_first,
                                                     const int32_t* __restrict__ norm_first,
                                                     const int32_t* __restrict__ exec_cols, int32_t* ticket,
                                                     int32_t* done, int32_t* err) {
    __shared__ double sval[CH];
    __shared__ uint8_t soff[CH];
    const int lane = threadIdx.x;
    const int64_t total = seg[nseg];
    for (;;) {
        int64_t g = 0;
        if (lane == 0) g = atomicAdd(ticket, 1);
        g = __shfl(g, 0, 64);
        if (g >= total) return;
        int32_t s = 0;  // segment of item g: seg[s] <= g < seg[s + 1]
        for (int32_t st = 1 << 20; st > 0; st >>= 1)
            if (s + st < nseg && seg[s + st] <= g) s += st;
        const int64_t need = seg[s];
        int ok = 1;
        if (lane == 0) {
            for (int it = 0; __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need;) {
                if (++it > kMailSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    atomicOr(err, 4);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (!__shfl(ok, 0, 64)) return;
        const int64_t nwi_s = wi_first[s + 1] - wi_first[s];
        const int64_t x = g - need;
        if (x < nwi_s)
            level_work_item<CH, true, double>(args, args.val, wi_first[s] + x, lane, sval, soff);
        else
            normalise_column<true>(args, args.val, exec_cols[norm_first[s] + (x - nwi_s)], lane);
        // every store of this wave has reached the coherence point before the
        // item is counted
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) __hip_atomic_fetch_add(done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// Normalise the last level's columns and check every pivot.
template <class T>
__global__ void k_finalize(const FactorArgs args, T* __restrict__ val, const int32_t* __restrict__ norm_cols,
                           int32_t nnorm, int32_t n, int32_t* __restrict__ status) {
    const int64_t* __restrict__ colptr = args.colptr;
    const int64_t* __restrict__ diag = args.diag;
    int64_t b = blockIdx.x;
    if (b < nnorm) {
        int32_t j = norm_cols[b];
        int64_t dj = diag[j];
        const T d = val[dj];
        for (int64_t q = dj + 1 + threadIdx.x; q < colptr[j + 1]; q += blockDim.x) val[q] = val[q] / d;
        return;
    }
    int64_t j = (b - nnorm) * blockDim.x + threadIdx.x;
    if (j < n) {
        const T d = val[diag[j]];
        if (d == (T)0 || !isfinite(d)) atomicMin(&status[0], (int32_t)j);
    }
}

// FP32 form: the factors widened to FP64 for the solves (exact conversion)
__global__ void k_widen(const float* __restrict__ v32, double* __restrict__ v64, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) v64[i] = (double)v32[i];
}

// ---------------------------------------------------------------- solves

__global__ void k_gather_perm(int32_t n, int32_t nrhs, const double* __restrict__ b, int64_t ldb,
                              const int32_t* __restrict__ perm, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = perm[i];
    for (int32_t r = 0; r < nrhs; r++) y[(int64_t)r * n + i] = b[(int64_t)r * ldb + o];
}

__global__ void k_scatter_perm(int32_t n, int32_t nrhs, const double* __restrict__ y,
                               const int32_t* __restrict__ perm, double* __restrict__ x, int64_t ldx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = perm[i];
    for (int32_t r = 0; r < nrhs; r++) x[(int64_t)r * ldx + o] = y[(int64_t)r * n + i];
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Dot product of the schedule-ordered entries [b, e) with the mailbox copy of
// the work vector, one wave: four independent loads per lane in flight (each
// value polled until it is final), then a fixed reduction tree.
__device__ __forceinline__ double row_dot_mail(const double* __restrict__ v, const int32_t* __restrict__ col,
                                               const double* mail, int64_t b, int64_t e, int lane, uint64_t sentinel,
                                               int32_t* err) {
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    for (int64_t x = b + lane; x < e; x += 256) {
        const bool h1 = x + 64 < e, h2 = x + 128 < e, h3 = x + 192 < e;
        const double v0 = v[x], v1 = h1 ? v[x + 64] : 0.0, v2 = h2 ? v[x + 128] : 0.0, v3 = h3 ? v[x + 192] : 0.0;
        const int32_t c0 = col[x], c1 = h1 ? col[x + 64] : c0, c2 = h2 ? col[x + 128] : c0, c3 = h3 ? col[x + 192] : c0;
        const int64_t idx[4] = {c0, c1, c2, c3};
        const bool use[4] = {true, h1, h2, h3};
        double yv[4];
        mail_read<4>(mail, idx, use, sentinel, yv, err);
        const double y0 = yv[0], y1 = yv[1], y2 = yv[2], y3 = yv[3];
        acc0 = fma(v0, y0, acc0);
        acc1 = h1 ? fma(v1, y1, acc1) : acc1;
        acc2 = h2 ? fma(v2, y2, acc2) : acc2;
        acc3 = h3 ? fma(v3, y3, acc3) : acc3;
    }
    return wave_sum((acc0 + acc1) + (acc2 + acc3));
}

// Both sparse substitutions in one launch each: a grid of a few blocks per
// compute unit walks the whole schedule, one wave per row as in the per-level
// kernels.  A row's inputs are rows of earlier levels, i.e. earlier slots,
// read from the mailbox copy of the work vector (mail, n doubles per
// right-hand side) and polled until published; each row publishes its result
// there.
//
// Slot assignment.  When the whole grid is resident, wave q takes slots
// q, q + W, q + 2W, ... (W waves): no shared counter at all.  The earliest
// unfinished slot always has its inputs and its wave has finished its own
// earlier slots, so the walk progresses -- but only if that wave is running.
// Beside other kernels the grid may not all be resident, so the blocks first
// agree on a mode: each block counts itself in on arrival; the last to arrive
// selects the static walk, while a block that has waited for the others for
// a while selects the dynamic one, whichever comes first (one compare-and-
// swap).  In the dynamic walk every wave takes its next slot from an atomic
// ticket (handed out in increasing order), so the earliest unfinished slot
// belongs to a running wave whatever is resident.  sync: [0] ticket,
// [1] blocks arrived, [2] mode (0 undecided, 1 static, 2 dynamic), zeroed
// before the launch.
constexpr int kArriveSpinLimit = 1 << 13;

__device__ __forceinline__ int32_t solve_walk_mode(int32_t* sync, int32_t* err) {
    __shared__ int32_t smode;
    if (threadIdx.x == 0) {
        const int32_t a = atomicAdd(&sync[1], 1);
        if (a == (int32_t)gridDim.x - 1) atomicCAS(&sync[2], 0, 1);
        int32_t m = 0;
        for (int it = 0;; it++) {
            m = __hip_atomic_load(&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (m != 0) break;
            if (it > kArriveSpinLimit) {
                atomicCAS(&sync[2], 0, 2);
                m = __hip_atomic_load(&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        smode = m;
    }
    __syncthreads();
    return smode;
}

// Next slot of a wave in the dynamic walk: one ticket, broadcast from lane 0.
__device__ __forceinline__ int32_t wave_ticket(int32_t* ticket, int lane) {
    int32_t w = 0;
    if (lane == 0) w = atomicAdd(ticket, 1);
    return __shfl(w, 0, 64);
}

__global__ __launch_bounds__(256) void k_fsolve_all(const SolveArgs sa, const int32_t* __restrict__ rows,
                                                   int32_t nslots, double* mail, uint64_t sentinel, int32_t* sync,
                                                   int32_t* err) {
    const int lane = threadIdx.x & 63;
    const bool dyn = solve_walk_mode(sync, err) == 2;
    const int32_t nw = (int32_t)((gridDim.x * blockDim.x) >> 6);
    int32_t w = dyn ? wave_ticket(sync, lane) : (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    while (w < nslots) {
        const int32_t i = rows[w];
        const int64_t b = sa.fs_ptr[w], e = sa.fs_ptr[w + 1];
        for (int32_t r = 0; r < sa.nrhs; r++) {
            double* yr = sa.y + (int64_t)r * sa.n;
            double* mr = mail + (int64_t)r * sa.n;
            const double acc = row_dot_mail(sa.fs_val, sa.fs_col, mr, b, e, lane, sentinel, err);
            if (lane == 0) {
                const double x = yr[i] - acc;
                yr[i] = x;
                mail_put(mr, i, x);
            }
        }
        w = dyn ? wave_ticket(sync, lane) : w + nw;
    }
}

__global__ __launch_bounds__(256) void k_bsolve_all(const SolveArgs sa, const int32_t* __restrict__ rows,
                                                   int32_t nslots, double* mail, uint64_t sentinel, int32_t* sync,
                                                   int32_t* err) {
    const int lane = threadIdx.x & 63;
    const bool dyn = solve_walk_mode(sync, err) == 2;
    const int32_t nw = (int32_t)((gridDim.x * blockDim.x) >> 6);
    int32_t w = dyn ? wave_ticket(sync, lane) : (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    while (w < nslots) {
        const int32_t j = rows[w];
        const int64_t b = sa.bs_ptr[w], e = sa.bs_ptr[w + 1];
        const double d = sa.val[sa.diag[j]];
        for (int32_t r = 0; r < sa.nrhs; r++) {
            double* yr = sa.y + (int64_t)r * sa.n;
            double* mr = mail + (int64_t)r * sa.n;
            const double acc = row_dot_mail(sa.bs_val, sa.bs_col, mr, b, e, lane, sentinel, err);
            if (lane == 0) {
                const double x = (yr[j] - acc) / d;
                yr[j] = x;
                mail_put(mr, j, x);
            }
        }
        w = dyn ? wave_ticket(sync, lane) : w + nw;
    }
}

// Mailbox before a substitution: the sentinel for rows [0, t) (to be solved),
// the current work vector for rows [t, n) (final already); the walk's
// synchronisation words restart at 0.
__global__ void k_mail_prep(double* __restrict__ mail, const double* __restrict__ y, int32_t n, int32_t t,
                            int32_t nrhs, uint64_t sentinel, int32_t* sync) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < 3) sync[x] = 0;
    if (x >= (int64_t)n * nrhs) return;
    const int32_t i = (int32_t)(x % n);
    reinterpret_cast<uint64_t*>(mail)[x] = i < t ? sentinel : (uint64_t)__double_as_longlong(y[x]);
}

__global__ void k_gather_values(const double* __restrict__ val, const int64_t* __restrict__ pos, int64_t cnt,
                                 double* __restrict__ dst) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; x < cnt; x += stride) dst[x] = val[pos[x]];
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
    if (threadIdx.x == 0) p[0] = v;
}

// ---------------------------------------------------------------- iterative refinement

// Non-negative doubles order like their bit patterns as unsigned integers,
// so a maximum of them is an atomic integer maximum.
// Largest of the wave's values (non-negative doubles compared by bit pattern,
// which orders them numerically and puts a NaN above every number).
__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// r = b - A x in FP64 over the rows of A (its row view: arow_ptr / arow_col,
// values at arow_pos in A's own CSC value order), 16 lanes per row (a supply
// rail's row holds thousands of entries: one lane per row would walk them one
// dependent load after another), 16 rows per block, grid.y = right-hand side;
// norms[0] = max_i sum_k |a_ik| (= ||A||_inf), norms[1 + 2c] = ||r_c||_inf,
// norms[2 + 2c] = ||x_c||_inf, reduced per wave and block (as bit patterns)
// before one atomic per block and norm.  norms must be zero before.
__global__ __launch_bounds__(256) void k_residual(int32_t n, const int64_t* __restrict__ arow_ptr,
                                                  const int32_t* __restrict__ arow_col,
                                                  const int64_t* __restrict__ arow_pos, const double* __restrict__ aval,
                                                  const double* __restrict__ b, int64_t ldb,
                                                  const double* __restrict__ x, int64_t ldx, double* __restrict__ r,
                                                  double* __restrict__ norms, int32_t c0) {
    constexpr int G = 16;
    __shared__ unsigned long long red[3][4];
    const int32_t c = c0 + (int32_t)blockIdx.y;
    const int gl = threadIdx.x % G;
    const int32_t i = (int32_t)blockIdx.x * (256 / G) + (int32_t)(threadIdx.x / G);
    const double* xc = x + (int64_t)c * ldx;
    double acc = 0.0, arow = 0.0;
    if (i < n) {
        for (int64_t q = arow_ptr[i] + gl; q < arow_ptr[i + 1]; q += G) {
            const double a = aval[arow_pos[q]];
            acc = fma(a, xc[arow_col[q]], acc);
            arow += fabs(a);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, G);
        arow += __shfl_xor(arow, off, G);
    }
    unsigned long long ma = 0, mr = 0, mx = 0;
    if (i < n && gl == 0) {
        const double ri = b[(int64_t)c * ldb + i] - acc;
        r[(int64_t)c * n + i] = ri;
        ma = (unsigned long long)__double_as_longlong(arow);
        mr = (unsigned long long)__double_as_longlong(fabs(ri));
        mx = (unsigned long long)__double_as_longlong(fabs(xc[i]));
    }
    ma = wave_max_bits(ma);
    mr = wave_max_bits(mr);
    mx = wave_max_bits(mx);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = ma;
        red[1][w] = mr;
        red[2][w] = mx;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        unsigned long long m = red[k][0];
        for (int v = 1; v < 4; v++) m = red[k][v] > m ? red[k][v] : m;
        double* dst = k == 0 ? &norms[0] : &norms[k + 2 * c];
        if (k > 0 || c == 0) atomicMax(reinterpret_cast<unsigned long long*>(dst), m);
    }
}

// x += d (the refinement step, FP64)
__global__ void k_axpy_update(int32_t n, int32_t nrhs, const double* __restrict__ d, double* __restrict__ x,
                              int64_t ldx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nrhs) return;
    const int32_t i = (int32_t)(t % n), c = (int32_t)(t / n);
    x[(int64_t)c * ldx + i] += d[(int64_t)c * n + i];
}

__global__ void k_zero_f64(double* p, int32_t n) {
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

inline unsigned grid_for(int64_t n, int bs, int64_t cap = 1 << 20) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill<double><<<grid_for(n, 256, 8192), 256, 0, st>>>(p, n, 0.0);
    return hipGetLastError();
}

hipError_t launch_widen(const float* v32, double* v64, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_widen<<<grid_for(n, 256, 8192), 256, 0, st>>>(v32, v64, n);
    return hipGetLastError();
}

hipError_t launch_value_load(const FactorArgs& a, const double* avals, int64_t nnz_a, int64_t nnz_lu,
                             int32_t* status, int32_t* counters, int32_t ncount, int32_t t, int32_t m,
                             const int64_t* tail_pos, hipStream_t st) {
    k_status_reset<<<1, 256, 0, st>>>(status, counters, ncount);
    // with a dense block, only the entries outside it are cleared: the
    // columns before it whole (nnz_lu holds their count then) and the rows
    // above it in its columns
    if (a.val32) {
        k_fill<float><<<grid_for(nnz_lu, 256, 8192), 256, 0, st>>>(a.val32, nnz_lu, 0.0f);
        if (m > 0) k_fill_heads<float><<<(unsigned)m, 256, 0, st>>>(a.colptr, tail_pos, t, m, a.val32);
        if (nnz_a > 0)
            k_scatter_values<float><<<grid_for(nnz_a, 256, 8192), 256, 0, st>>>(avals, a.amap, nnz_a, a.val32, status);
    } else {
        k_fill<double><<<grid_for(nnz_lu, 256, 8192), 256, 0, st>>>(a.val, nnz_lu, 0.0);
        if (m > 0) k_fill_heads<double><<<(unsigned)m, 256, 0, st>>>(a.colptr, tail_pos, t, m, a.val);
        if (nnz_a > 0)
            k_scatter_values<double><<<grid_for(nnz_a, 256, 8192), 256, 0, st>>>(avals, a.amap, nnz_a, a.val, status);
    }
    return hipGetLastError();
}

hipError_t launch_level(const FactorArgs& a, int mode, int64_t wi0, int64_t nwi, const int32_t* norm_cols,
                        int32_t nnorm, hipStream_t st) {
    // the mode shapes the plan's slices (at most max_chunk(mode) entries);
    // every work item is one wave
    if (nwi + nnorm <= 0) return hipSuccess;
    // at most kMaxGrid workgroups per launch (the grid's thread count must
    // stay below 2^32); the normalisation blocks ride with the last chunk
    int64_t w0 = 0;
    do {
        const int64_t cnt = std::min<int64_t>(nwi - w0, kMaxGrid);
        const bool last = w0 + cnt >= nwi;
        const int32_t nn = last ? nnorm : 0;
        if (cnt + nn > 0) {
            const unsigned g = (unsigned)(cnt + nn);
            if (a.val32) {
                if (mode == MODE_LARGE)
                    k_level<kChunkLarge, float><<<g, 64, 0, st>>>(a, a.val32, wi0 + w0, cnt, norm_cols, nn);
                else
                    k_level<kChunk, float><<<g, 64, 0, st>>>(a, a.val32, wi0 + w0, cnt, norm_cols, nn);
            } else {
                if (mode == MODE_LARGE)
                    k_level<kChunkLarge, double><<<g, 64, 0, st>>>(a, a.val, wi0 + w0, cnt, norm_cols, nn);
                else
                    k_level<kChunk, double><<<g, 64, 0, st>>>(a, a.val, wi0 + w0, cnt, norm_cols, nn);
            }
        }
        w0 += cnt;
    } while (w0 < nwi);
    return hipGetLastError();
}

hipError_t launch_level_batch(const FactorArgs* args, const BatchEntry* ent, int32_t nent, int64_t nblocks,
                              bool fp32, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
    if (fp32)
        k_level_batch<kChunk, float><<<(unsigned)nblocks, 64, 0, st>>>(args, ent, nent);
    else
        k_level_batch<kChunk, double><<<(unsigned)nblocks, 64, 0, st>>>(args, ent, nent);
    return hipGetLastError();
}

hipError_t launch_level_stream(const FactorArgs& a, const int64_t* seg_start, const int64_t* seg_wi,
                               const int32_t* seg_norm, int32_t nseg, int64_t nitems, const int32_t* exec_cols,
                               int32_t* counters, int32_t* err, int32_t grid, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(grid, nitems));
    k_level_stream<kChunk><<<(unsigned)g, 64, 0, st>>>(a, seg_start, nseg, seg_wi, seg_norm, exec_cols, counters,
                                                       counters + 1, err);
    return hipGetLastError();
}

hipError_t launch_level_map(const FactorArgs& a, int64_t nwi, uint8_t* touch_off, uint16_t* pair_pos,
                            int32_t* wi_ntouch, int32_t* err, hipStream_t st) {
    if (nwi <= 0) return hipSuccess;
    for (int64_t w0 = 0; w0 < nwi; w0 += kMaxGrid) {
        const int64_t cnt = std::min<int64_t>(nwi - w0, kMaxGrid);
        k_level_map<<<(unsigned)cnt, 64, 0, st>>>(a, w0, cnt, touch_off, pair_pos, wi_ntouch, err);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const FactorArgs& a, const int32_t* norm_cols, int32_t nnorm, int32_t n,
                           int32_t* status, hipStream_t st) {
    int64_t grid = nnorm + (n + 255) / 256;
    if (grid <= 0) return hipSuccess;
    if (a.val32)
        k_finalize<float><<<(unsigned)grid, 256, 0, st>>>(a, a.val32, norm_cols, nnorm, n, status);
    else
        k_finalize<double><<<(unsigned)grid, 256, 0, st>>>(a, a.val, norm_cols, nnorm, n, status);
    return hipGetLastError();
}

hipError_t launch_solve_gather(int32_t n, int32_t nrhs, const double* b, int64_t ldb, const int32_t* perm,
                               double* y, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_gather_perm<<<grid_for(n, 256), 256, 0, st>>>(n, nrhs, b, ldb, perm, y);
    return hipGetLastError();
}

hipError_t launch_solve_scatter(int32_t n, int32_t nrhs, const double* y, const int32_t* perm, double* x,
                                int64_t ldx, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_scatter_perm<<<grid_for(n, 256), 256, 0, st>>>(n, nrhs, y, perm, x, ldx);
    return hipGetLastError();
}

hipError_t launch_solve_all(const SolveArgs& sa, bool upper, const int32_t* rows, int32_t nslots, int32_t t,
                            double* mail, uint64_t tag, int32_t* sync, int32_t* err, int32_t grid,
                            hipStream_t st) {
    if (nslots <= 0) return hipSuccess;
    const int64_t nm = (int64_t)sa.n * sa.nrhs;
    const uint64_t sentinel = mail_sentinel(tag);
    k_mail_prep<<<grid_for(nm, 256, 1 << 30), 256, 0, st>>>(mail, sa.y, sa.n, t, sa.nrhs, sentinel, sync);
    const int32_t g = std::max(1, std::min(grid, (nslots + 3) / 4));
    if (upper)
        k_bsolve_all<<<g, 256, 0, st>>>(sa, rows, nslots, mail, sentinel, sync, err);
    else
        k_fsolve_all<<<g, 256, 0, st>>>(sa, rows, nslots, mail, sentinel, sync, err);
    return hipGetLastError();
}

hipError_t launch_residual(int32_t n, int32_t nrhs, const int64_t* arow_ptr, const int32_t* arow_col,
                           const int64_t* arow_pos, const double* aval, const double* b, int64_t ldb,
                           const double* x, int64_t ldx, double* r, double* norms, hipStream_t st) {
    k_zero_f64<<<1, 64, 0, st>>>(norms, 1 + 2 * nrhs);
    for (int32_t c0 = 0; n > 0 && c0 < nrhs; c0 += 65535) {
        const dim3 grid((unsigned)((n + 15) / 16), (unsigned)std::min(nrhs - c0, 65535));
        k_residual<<<grid, 256, 0, st>>>(n, arow_ptr, arow_col, arow_pos, aval, b, ldb, x, ldx, r, norms, c0);
    }
    return hipGetLastError();
}

hipError_t launch_axpy_update(int32_t n, int32_t nrhs, const double* d, double* x, int64_t ldx, hipStream_t st) {
    const int64_t nt = (int64_t)n * nrhs;
    if (nt > 0) k_axpy_update<<<grid_for(nt, 256, 1 << 30), 256, 0, st>>>(n, nrhs, d, x, ldx);
    return hipGetLastError();
}

hipError_t launch_gather_values(const double* val, const int64_t* pos, int64_t cnt, double* dst, hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    k_gather_values<<<grid_for(cnt, 256, 8192), 256, 0, st>>>(val, pos, cnt, dst);
    return hipGetLastError();
}

hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t st) {
    k_set_i32<<<1, 64, 0, st>>>(p, v);
    return hipGetLastError();
}

int max_chunk(int mode) { return mode == MODE_LARGE ? kChunkLarge : kChunk; }

}  // namespace glu
