// Schur-complement update of the dense trailing block from the sparse columns
// on gfx950.
//
// Once the sparse levels have produced L(t:n, 0:t) and U(0:t, t:n), the block
// still owes S = A_s(t:n, t:n) - L(t:n, 0:t) U(0:t, t:n) (the submatrix update
// of Alg. 2 / Alg. 5 from every column before t).  No sparse level reads the
// block, so these products are deferred and applied here (two kernels side by
// side: long tiles and short ones), with every entry receiving its products in
// ascending source order j, one fused multiply-add at a time -- the order of
// the column-by-column algorithm.
//
// The block is tiled 16 x 16.  For a tile, the host lists the sources j that
// have L rows in the tile's rows and U columns in its columns (ascending j), as
// row indices into two dense panels built here from the sparse values: the row
// tile's L panel (one 16-wide row per source) and the column tile's U panel.
// A zero in a panel row contributes fma(-0, u, s) = s exactly, so the dense
// tile update equals the sparse sequence of products.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace glu {

namespace {

constexpr int TS = SCH_TS;
static_assert(TS == 16, "a tile is one 16 x 16 MFMA accumulator");

__global__ void k_panel_scatter(const double* __restrict__ val, const int64_t* __restrict__ pos,
                                const int64_t* __restrict__ off, int64_t cnt, double* __restrict__ P) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; x < cnt; x += stride) P[off[x]] = val[pos[x]];
}

constexpr int CPH = 64;    // pairs per staged chunk of a long tile
constexpr int HSTAGE = 8;  // chunks of a long tile in flight
// Short tiles: small chunks and a short pipeline keep the kernel at 62 VGPRs
// (7 waves per SIMD); many resident tiles hide the memory latency better than
// a deep pipeline per wave (at 112 VGPRs and 4 waves per SIMD, with 4-pair
// chunks four deep, the update took a third longer).
constexpr int SPL = 2;     // pairs per quarter-wave in a chunk of a short tile (chunk: 4 SPL pairs)
constexpr int SST = 2;     // chunks of a short tile whose values are in flight

typedef double v4d __attribute__((ext_vector_type(4)));

// S -= L21 U12 on 16 x 16 tiles of the dense block D (column-major, leading
// dimension ld) on the FP64 matrix cores.  v_mfma_f64_16x16x4f64 applies 4
// pairs per instruction: lane l supplies the U entry of column l % 16 and the
// negated L entry of row l % 16 for pair l / 16 of the group, and its
// accumulator v holds S(row l % 16, column l / 16 + 4 v).  Measured on gfx950,
// the instruction accumulates the 4 products of each entry as 4 fused
// multiply-adds in ascending k, so every entry still receives its products in
// list order (ascending source), one rounding each, as a one-FMA-per-pair loop
// would; a zero panel entry is an exact no-op.
__device__ __forceinline__ v4d tile_load(const double* __restrict__ D, int64_t ld, int32_t i0, int32_t k0, int32_t m,
                                         int lane) {
    const int32_t r = i0 + (lane & 15);
    v4d acc;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int32_t c = k0 + (lane >> 4) + 4 * v;
        acc[v] = (r < m && c < m) ? D[r + (int64_t)c * ld] : 0.0;
    }
    return acc;
}

__device__ __forceinline__ void tile_store(const v4d& acc, double* __restrict__ D, int64_t ld, int32_t i0, int32_t k0,
                                           int32_t m, int lane) {
    const int32_t r = i0 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int32_t c = k0 + (lane >> 4) + 4 * v;
        if (r < m && c < m) D[r + (int64_t)c * ld] = acc[v];
    }
}

// The long tiles, units [0, nheavy), one block each: all 256 threads stream
// the tile's panel rows through LDS, HSTAGE chunks of CPH pairs in flight in
// registers (the panel-row indices HSTAGE chunks further ahead), and wave 0
// runs the MFMAs: one accumulator chain per tile, as the pair order demands.
// A long tile's time is its chain, so the deep prefetch keeps the staging
// ahead of it while other tiles load the memory system.
__global__ __launch_bounds__(256, 2) void k_schur_long(const SchurUnit* __restrict__ units,
                                                       const int32_t* __restrict__ pl, const int32_t* __restrict__ pu,
                                                       const double* __restrict__ LP, const double* __restrict__ UP,
                                                       double* __restrict__ D, int64_t ld, int32_t m) {
    __shared__ double2 sbuf[2][CPH][TS];  // [buffer][pair][L row as 8 double2 | U row as 8 double2]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const SchurUnit un = units[blockIdx.x];
    const int64_t np = un.pe - un.pb;
    const int64_t nch = (np + CPH - 1) / CPH;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    if (w == 0) acc = tile_load(D, ld, un.i0, un.k0, m, lane);
    // thread t stages 64 bytes of pair x = t / 4 of each chunk: the L row
    // (t % 4 < 2) or the U row, double2 parts 4 (t % 2) .. 4 (t % 2) + 3
    const int x = tid >> 2, h = (tid >> 1) & 1, part = 4 * (tid & 1);
    const double* pbase = h ? UP + un.ubase : LP + un.lbase;
    const int32_t* pidx = h ? pu : pl;
    // Loads are issued unconditionally (clamped to the tile's last pair and to
    // panel row 0) and their results selected, and the loop runs whole groups
    // of HSTAGE chunks with no branch in its body: loads under a branch end
    // the compiler's tracking of the loads in flight, and it then waits for
    // all of them at the top of every chunk.
    auto load_idx = [&](int64_t ch) -> int32_t {
        const int64_t p = un.pb + ch * CPH + x;
        const int32_t v = pidx[p < un.pe ? p : un.pe - 1];
        return p < un.pe ? v : -1;
    };
    auto load_val = [&](int32_t ix, double2 (&v)[4]) {
        const double2* src = reinterpret_cast<const double2*>(pbase + (int64_t)max(ix, 0) * TS) + part;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double2 t = src[q];
            v[q] = ix >= 0 ? t : make_double2(0.0, 0.0);
        }
    };
    int32_t X[HSTAGE];
    double2 V[HSTAGE][4];
#pragma unroll
    for (int k = 0; k < HSTAGE; k++) X[k] = load_idx(k);
#pragma unroll
    for (int k = 0; k < HSTAGE; k++) {
        load_val(X[k], V[k]);
        X[k] = load_idx(k + HSTAGE);
    }
    static_assert(HSTAGE % 2 == 0, "chunk k of a group uses LDS buffer k % 2");
    for (int64_t ch0 = 0; ch0 < nch; ch0 += HSTAGE) {
#pragma unroll
        for (int k = 0; k < HSTAGE; k++) {
            const int64_t ch = ch0 + k;
            const int bsel = k & 1;
#pragma unroll
            for (int q = 0; q < 4; q++) sbuf[bsel][x][h * 8 + part + q] = V[k][q];
            load_val(X[k], V[k]);  // chunk ch + HSTAGE
            X[k] = load_idx(ch + 2 * HSTAGE);
            __syncthreads();  // chunk ch is in LDS; wave 0 finished chunk ch - 1
            if (w == 0) {
                // chunks past the end, and the end of the last one, were
                // staged as zero rows: exact no-ops; every operand is read
                // before the first MFMA
                const double* cb = reinterpret_cast<const double*>(sbuf[bsel]) + grp * 2 * TS + col;
                double ua[CPH / 4], la[CPH / 4];
#pragma unroll
                for (int q = 0; q < CPH / 4; q++) {
                    ua[q] = cb[q * 8 * TS + TS];
                    la[q] = -cb[q * 8 * TS];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < CPH / 4; q++)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[q], la[q], acc, 0, 0, 0);
            }
        }
    }
    if (w == 0) tile_store(acc, D, ld, un.i0, un.k0, m, lane);
}

// The short tiles, units [first, nunits), one per wave, four to a block.  A
// wave loads its lanes' operands straight from the panels: lane l takes pair
// 4 s + l / 16 of each chunk (s < SPL), column l % 16 of its U row and row
// l % 16 of its L row.  The loads form a two-step pipeline: the values of the
// next SST chunks are in flight, loaded from panel-row indices that were
// fetched SST chunks before them, so a wait for an index never waits for the
// value loads issued after it (the memory counters retire in order).
__global__ __launch_bounds__(256) void k_schur_short(const SchurUnit* __restrict__ units, int64_t nunits,
                                                     int64_t first, const int32_t* __restrict__ pl,
                                                     const int32_t* __restrict__ pu, const double* __restrict__ LP,
                                                     const double* __restrict__ UP, double* __restrict__ D,
                                                     int64_t ld, int32_t m) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int col = lane & 15, grp = lane >> 4;
    // the wave's unit, in scalar registers (the wave index is uniform)
    const int64_t uidx = first + (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(tid >> 6);
    if (uidx >= nunits) return;  // (no block-wide barrier follows)
    const SchurUnit un = units[uidx];
    constexpr int CP = 4 * SPL;
    const int32_t np = (int32_t)(un.pe - un.pb);  // a short tile has fewer than 2^31 pairs
    const int32_t nch = (np + CP - 1) / CP;
    v4d acc = tile_load(D, ld, un.i0, un.k0, m, lane);
    // uniform bases; per-lane 32-bit byte offsets (a panel has fewer than
    // 2^25 rows of 128 bytes)
    const int32_t* plb = pl + un.pb;
    const int32_t* pub = pu + un.pb;
    const char* lb = reinterpret_cast<const char*>(LP + un.lbase);
    const char* ub = reinterpret_cast<const char*>(UP + un.ubase);
    const uint32_t cofs = 8u * (uint32_t)col;
    // Every load is issued unconditionally (a pair past the tile's end reads
    // its last pair's entries, a missing row reads row 0 of the panel) and the
    // result is then selected: loads under a branch end the compiler's
    // tracking of the in-flight loads, and it waits for all of them there.
    auto load_idx = [&](int32_t ch, int32_t (&il)[SPL], int32_t (&iu)[SPL]) {
#pragma unroll
        for (int s4 = 0; s4 < SPL; s4++) {
            const int32_t p = ch * CP + 4 * s4 + grp;
            const int32_t q = p < np ? p : np - 1;
            const int32_t a = plb[q], b = pub[q];
            il[s4] = p < np ? a : -1;
            iu[s4] = p < np ? b : -1;
        }
    };
    auto load_val = [&](const int32_t (&il)[SPL], const int32_t (&iu)[SPL], double (&A)[SPL], double (&B)[SPL]) {
#pragma unroll
        for (int s4 = 0; s4 < SPL; s4++) {
            const double u = *reinterpret_cast<const double*>(ub + ((uint32_t)max(iu[s4], 0) * 128u + cofs));
            const double l = *reinterpret_cast<const double*>(lb + ((uint32_t)max(il[s4], 0) * 128u + cofs));
            A[s4] = iu[s4] >= 0 ? u : 0.0;
            B[s4] = il[s4] >= 0 ? -l : 0.0;
        }
    };
    int32_t IL[SST][SPL], IU[SST][SPL];
    double A[SST][SPL], B[SST][SPL];
#pragma unroll
    for (int k = 0; k < SST; k++) load_idx(k, IL[k], IU[k]);
#pragma unroll
    for (int k = 0; k < SST; k++) {
        load_val(IL[k], IU[k], A[k], B[k]);
        load_idx(k + SST, IL[k], IU[k]);
    }
    // whole groups of SST chunks, so that the loop body is one straight block:
    // the chunks past the end hold zero operands (exact no-ops)
    for (int32_t ch0 = 0; ch0 < nch; ch0 += SST) {
#pragma unroll
        for (int k = 0; k < SST; k++) {
#pragma unroll
            for (int s4 = 0; s4 < SPL; s4++)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k][s4], B[k][s4], acc, 0, 0, 0);
            load_val(IL[k], IU[k], A[k], B[k]);  // chunk ch0 + k + SST
            load_idx(ch0 + k + 2 * SST, IL[k], IU[k]);
        }
    }
    tile_store(acc, D, ld, un.i0, un.k0, m, lane);
}

inline unsigned grid_for(int64_t n, int bs, int64_t cap = 1 << 16) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_schur(const SchurArgs& s, const double* val, double* D, int64_t ld, int32_t m, hipStream_t st,
                        hipStream_t aux, hipEvent_t ev_fork, hipEvent_t ev_join) {
    if (s.nunits <= 0) return hipSuccess;
    // the panels' entries outside the pattern are zero from their allocation
    // on, and every factorization rewrites the same positions
    if (s.nl > 0) k_panel_scatter<<<grid_for(s.nl, 256), 256, 0, st>>>(val, s.lpos, s.loff, s.nl, s.LP);
    if (s.nu > 0) k_panel_scatter<<<grid_for(s.nu, 256), 256, 0, st>>>(val, s.upos, s.uoff, s.nu, s.UP);
    // the short tiles on aux beside the long ones on st (disjoint tiles); the
    // long tiles are launched first, so that their blocks find room first.
    // Without long tiles the short ones stay on st (no fork and join).
    const int64_t nlight = s.nunits - s.nheavy;
    const bool fork = s.nheavy > 0 && nlight > 0;
    if (fork && (hipEventRecord(ev_fork, st) != hipSuccess || hipStreamWaitEvent(aux, ev_fork, 0) != hipSuccess))
        return hipErrorUnknown;
    if (s.nheavy > 0) k_schur_long<<<(unsigned)s.nheavy, 256, 0, st>>>(s.units, s.pl, s.pu, s.LP, s.UP, D, ld, m);
    if (nlight > 0) {
        k_schur_short<<<(unsigned)((nlight + 3) / 4), 256, 0, fork ? aux : st>>>(s.units, s.nunits, s.nheavy, s.pl,
                                                                                s.pu, s.LP, s.UP, D, ld, m);
        if (fork && (hipEventRecord(ev_join, aux) != hipSuccess || hipStreamWaitEvent(st, ev_join, 0) != hipSuccess))
            return hipErrorUnknown;
    }
    return hipGetLastError();
}

}  // namespace glu
