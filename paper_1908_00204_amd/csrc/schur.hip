// Schur-complement update of the dense trailing block from the sparse columns
// on gfx950.
//
// Once the sparse levels have produced L(t:n, 0:t) and U(0:t, t:n), the block
// still owes S = A_s(t:n, t:n) - L(t:n, 0:t) U(0:t, t:n) (the submatrix update
// of Alg. 2 / Alg. 5 from every column before t).  No sparse level reads the
// block, so these products are deferred and applied here in one launch, with
// every entry receiving its products in ascending source order j, one fused
// multiply-add at a time -- the order of the column-by-column algorithm.
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

constexpr int CP = 32;     // pairs per chunk of a short tile
constexpr int CPH = 64;    // pairs per staged chunk of a long tile
constexpr int HSTAGE = 4;  // chunks in flight for a long tile

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
//
// Blocks [0, nheavy) each take one long tile: all 256 threads stream its panel
// rows through LDS, HSTAGE chunks of CPH pairs in flight in registers (the
// panel-row indices HSTAGE chunks further ahead), and wave 0 runs the MFMAs.
// Later blocks give each of their 4 waves its own short tile; a wave loads its
// lanes' operands straight from the panels, three chunks ahead.
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

__global__ __launch_bounds__(256, 3) void k_schur(const SchurUnit* __restrict__ units, int64_t nunits, int64_t nheavy,
                                               const int32_t* __restrict__ pl, const int32_t* __restrict__ pu,
                                               const double* __restrict__ LP, const double* __restrict__ UP,
                                               double* __restrict__ D, int64_t ld, int32_t m) {
    __shared__ double2 sbuf[2][CPH][TS];  // [buffer][pair][L row as 8 double2 | U row as 8 double2]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const bool heavy = (int64_t)blockIdx.x < nheavy;
    const int64_t uidx = heavy ? (int64_t)blockIdx.x : nheavy + ((int64_t)blockIdx.x - nheavy) * 4 + w;
    if (uidx >= nunits) return;  // (light blocks only: no block-wide barrier follows)
    const SchurUnit un = units[uidx];
    const int64_t np = un.pe - un.pb;
    if (heavy) {
        const int64_t nch = (np + CPH - 1) / CPH;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        if (w == 0) acc = tile_load(D, ld, un.i0, un.k0, m, lane);
        // thread t stages 64 bytes of pair x = t / 4 of each chunk: the L row
        // (t % 4 < 2) or the U row, double2 parts 4 (t % 2) .. 4 (t % 2) + 3
        const int x = tid >> 2, h = (tid >> 1) & 1, part = 4 * (tid & 1);
        const double* pbase = h ? UP + un.ubase : LP + un.lbase;
        const int32_t* pidx = h ? pu : pl;
        auto load_idx = [&](int64_t ch) -> int32_t {
            const int64_t p = un.pb + ch * CPH + x;
            return (ch < nch && p < un.pe) ? pidx[p] : -1;
        };
        auto load_val = [&](int32_t ix, double2 (&v)[4]) {
            if (ix >= 0) {
                const double2* src = reinterpret_cast<const double2*>(pbase + (int64_t)ix * TS) + part;
#pragma unroll
                for (int q = 0; q < 4; q++) v[q] = src[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++) v[q] = make_double2(0.0, 0.0);
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
        for (int64_t ch0 = 0; ch0 < nch; ch0 += HSTAGE) {
#pragma unroll
            for (int k = 0; k < HSTAGE; k++) {
                const int64_t ch = ch0 + k;
                if (ch < nch) {  // uniform over the block
                    const int bsel = (int)(ch & 1);
#pragma unroll
                    for (int q = 0; q < 4; q++) sbuf[bsel][x][h * 8 + part + q] = V[k][q];
                    load_val(X[k], V[k]);  // chunk ch + HSTAGE
                    X[k] = load_idx(ch + 2 * HSTAGE);
                    __syncthreads();  // chunk ch is in LDS; wave 0 finished chunk ch - 1
                    if (w == 0) {
                        // a partial last chunk was staged with zero rows: exact
                        // no-ops; every operand is read before the first MFMA
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
        }
        if (w == 0) tile_store(acc, D, ld, un.i0, un.k0, m, lane);
    } else {
        const int64_t nch = (np + CP - 1) / CP;
        v4d acc = tile_load(D, ld, un.i0, un.k0, m, lane);
        const double* lb = LP + un.lbase + col;
        const double* ub = UP + un.ubase + col;
        // operands of one chunk: pair grp + 4 s of the chunk, s < CP / 4
        auto load = [&](int64_t ch, double (&A)[CP / 4], double (&B)[CP / 4]) {
#pragma unroll
            for (int s4 = 0; s4 < CP / 4; s4++) {
                const int64_t p = un.pb + ch * CP + 4 * s4 + grp;
                const bool ok = p < un.pe;
                const int32_t il = ok ? pl[p] : 0, iu = ok ? pu[p] : 0;
                A[s4] = ok ? ub[(int64_t)iu * TS] : 0.0;
                B[s4] = ok ? -lb[(int64_t)il * TS] : 0.0;
            }
        };
        auto step = [&](const double (&A)[CP / 4], const double (&B)[CP / 4]) {
#pragma unroll
            for (int s4 = 0; s4 < CP / 4; s4++) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s4], B[s4], acc, 0, 0, 0);
        };
        double A0[CP / 4], B0[CP / 4], A1[CP / 4], B1[CP / 4], A2[CP / 4], B2[CP / 4];
        load(0, A0, B0);
        load(1, A1, B1);
        load(2, A2, B2);
        for (int64_t ch = 0; ch < nch; ch += 3) {
            step(A0, B0);
            load(ch + 3, A0, B0);
            if (ch + 1 < nch) {
                step(A1, B1);
                load(ch + 4, A1, B1);
            }
            if (ch + 2 < nch) {
                step(A2, B2);
                load(ch + 5, A2, B2);
            }
        }
        tile_store(acc, D, ld, un.i0, un.k0, m, lane);
    }
}

inline unsigned grid_for(int64_t n, int bs, int64_t cap = 1 << 16) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_schur(const SchurArgs& s, const double* val, double* D, int64_t ld, int32_t m, hipStream_t st) {
    if (s.nunits <= 0) return hipSuccess;
    // the panels' entries outside the pattern are zero from their allocation
    // on, and every factorization rewrites the same positions
    if (s.nl > 0) k_panel_scatter<<<grid_for(s.nl, 256), 256, 0, st>>>(val, s.lpos, s.loff, s.nl, s.LP);
    if (s.nu > 0) k_panel_scatter<<<grid_for(s.nu, 256), 256, 0, st>>>(val, s.upos, s.uoff, s.nu, s.UP);
    const int64_t nlight = s.nunits - s.nheavy;
    const int64_t grid = s.nheavy + (nlight + 3) / 4;
    k_schur<<<(unsigned)grid, 256, 0, st>>>(s.units, s.nunits, s.nheavy, s.pl, s.pu, s.LP, s.UP, D, ld, m);
    return hipGetLastError();
}

}  // namespace glu
