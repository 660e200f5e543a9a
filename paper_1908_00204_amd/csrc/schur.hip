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
static_assert(TS == 16, "the tile kernel maps 64 lanes to 2 x 2 entries of a 16 x 16 tile");

__global__ void k_panel_scatter(const double* __restrict__ val, const int64_t* __restrict__ pos,
                                const int64_t* __restrict__ off, int64_t cnt, double* __restrict__ P) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; x < cnt; x += stride) P[off[x]] = val[pos[x]];
}

constexpr int CP = 32;  // pairs per staged chunk

// One wave per tile; lane (rp, cp) owns rows i0 + 2rp + {0,1} and columns
// k0 + 2cp + {0,1} of the dense block D (column-major, leading dimension ld).
// The tile's pairs stream through LDS in chunks of CP: for staging, lane
// (q, h) of the wave loads the L (h = 0) or U (h = 1) panel row of pair q of a
// chunk (128 contiguous bytes), so each panel row is read once per tile.
// Three chunks are in flight in registers while the wave computes on an
// earlier one from LDS, which hides the memory latency of the long tiles.
__global__ __launch_bounds__(64) void k_schur(const SchurUnit* __restrict__ units, const int32_t* __restrict__ pl,
                                              const int32_t* __restrict__ pu, const double* __restrict__ LP,
                                              const double* __restrict__ UP, double* __restrict__ D, int64_t ld,
                                              int32_t m) {
    __shared__ double2 buf[2][CP][TS];  // [buffer][pair][L row as 8 double2 | U row as 8 double2]
    const SchurUnit un = units[blockIdx.x];
    const int lane = threadIdx.x;
    const int rp = lane & 7, cp = lane >> 3;
    const int32_t r = un.i0 + 2 * rp;
    const int32_t c = un.k0 + 2 * cp;
    const bool r0ok = r < m, r1ok = r + 1 < m, c0ok = c < m, c1ok = c + 1 < m;
    double* d0 = D + r + (int64_t)c * ld;
    double* d1 = d0 + ld;
    double s00 = (r0ok && c0ok) ? d0[0] : 0.0;
    double s10 = (r1ok && c0ok) ? d0[1] : 0.0;
    double s01 = (r0ok && c1ok) ? d1[0] : 0.0;
    double s11 = (r1ok && c1ok) ? d1[1] : 0.0;

    const int q = lane >> 1, h = lane & 1;
    const double* pbase = h ? UP + un.ubase : LP + un.lbase;
    const int32_t* pidx = h ? pu : pl;
    const int64_t np = un.pe - un.pb;
    const int64_t nch = (np + CP - 1) / CP;
    auto load = [&](int64_t ch, double2(&R)[8]) {
        const int64_t p = un.pb + ch * CP + q;
        if (ch < nch && p < un.pe) {
            const double2* src = reinterpret_cast<const double2*>(pbase + (int64_t)pidx[p] * TS);
#pragma unroll
            for (int k = 0; k < 8; k++) R[k] = src[k];
        } else {
#pragma unroll
            for (int k = 0; k < 8; k++) R[k] = make_double2(0.0, 0.0);
        }
    };
    auto step = [&](int64_t ch, double2(&R)[8]) {
        // chunk ch sits in R: move it to LDS, refill R with chunk ch + 3, then
        // apply the chunk's pairs in order
        const int bsel = (int)(ch & 1);
        __syncthreads();  // earlier reads of this buffer are done
#pragma unroll
        for (int k = 0; k < 8; k++) buf[bsel][q][h * 8 + k] = R[k];
        __syncthreads();
        load(ch + 3, R);
        const int cnt = (int)min<int64_t>(CP, np - ch * CP);
        auto apply = [&](const double2& l, const double2& u) {
            s00 = fma(-l.x, u.x, s00);
            s10 = fma(-l.y, u.x, s10);
            s01 = fma(-l.x, u.y, s01);
            s11 = fma(-l.y, u.y, s11);
        };
        if (cnt == CP) {
            // groups of 8 pairs; the LDS reads of group g + 1 are issued
            // before the multiply-adds of group g
            double2 la[8], ua[8], lb[8], ub[8];
#pragma unroll
            for (int x = 0; x < 8; x++) {
                la[x] = buf[bsel][x][rp];
                ua[x] = buf[bsel][x][8 + cp];
            }
#pragma unroll
            for (int g = 0; g < CP / 8; g += 2) {
#pragma unroll
                for (int x = 0; x < 8; x++) {
                    lb[x] = buf[bsel][8 * (g + 1) + x][rp];
                    ub[x] = buf[bsel][8 * (g + 1) + x][8 + cp];
                }
#pragma unroll
                for (int x = 0; x < 8; x++) apply(la[x], ua[x]);
                if (g + 2 < CP / 8) {
#pragma unroll
                    for (int x = 0; x < 8; x++) {
                        la[x] = buf[bsel][8 * (g + 2) + x][rp];
                        ua[x] = buf[bsel][8 * (g + 2) + x][8 + cp];
                    }
                }
#pragma unroll
                for (int x = 0; x < 8; x++) apply(lb[x], ub[x]);
            }
        } else {
            for (int x = 0; x < cnt; x++) apply(buf[bsel][x][rp], buf[bsel][x][8 + cp]);
        }
    };
    double2 RA[8], RB[8], RC[8];
    load(0, RA);
    load(1, RB);
    load(2, RC);
    for (int64_t ch = 0; ch < nch; ch += 3) {
        step(ch, RA);
        if (ch + 1 < nch) step(ch + 1, RB);
        if (ch + 2 < nch) step(ch + 2, RC);
    }
    if (r0ok && c0ok) d0[0] = s00;
    if (r1ok && c0ok) d0[1] = s10;
    if (r0ok && c1ok) d1[0] = s01;
    if (r1ok && c1ok) d1[1] = s11;
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
    if (launch_zero(s.LP, s.lp_len, st) != hipSuccess || launch_zero(s.UP, s.up_len, st) != hipSuccess)
        return hipGetLastError();
    if (s.nl > 0) k_panel_scatter<<<grid_for(s.nl, 256), 256, 0, st>>>(val, s.lpos, s.loff, s.nl, s.LP);
    if (s.nu > 0) k_panel_scatter<<<grid_for(s.nu, 256), 256, 0, st>>>(val, s.upos, s.uoff, s.nu, s.UP);
    k_schur<<<(unsigned)s.nunits, 64, 0, st>>>(s.units, s.pl, s.pu, s.LP, s.UP, D, ld, m);
    return hipGetLastError();
}

}  // namespace glu
