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

// One wave per tile; lane (rp, cp) owns rows i0 + 2rp + {0,1} and columns
// k0 + 2cp + {0,1} of the dense block D (column-major, leading dimension ld).
__global__ __launch_bounds__(64) void k_schur(const SchurUnit* __restrict__ units, const int32_t* __restrict__ pl,
                                              const int32_t* __restrict__ pu, const double* __restrict__ LP,
                                              const double* __restrict__ UP, double* __restrict__ D, int64_t ld,
                                              int32_t m) {
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
    const double* lp = LP + un.lbase + 2 * rp;
    const double* up = UP + un.ubase + 2 * cp;
    constexpr int B = 8;
    int64_t p = un.pb;
    for (; p + B <= un.pe; p += B) {
        double2 l[B], u[B];
#pragma unroll
        for (int x = 0; x < B; x++) {
            l[x] = *reinterpret_cast<const double2*>(lp + (int64_t)pl[p + x] * TS);
            u[x] = *reinterpret_cast<const double2*>(up + (int64_t)pu[p + x] * TS);
        }
#pragma unroll
        for (int x = 0; x < B; x++) {
            s00 = fma(-l[x].x, u[x].x, s00);
            s10 = fma(-l[x].y, u[x].x, s10);
            s01 = fma(-l[x].x, u[x].y, s01);
            s11 = fma(-l[x].y, u[x].y, s11);
        }
    }
    for (; p < un.pe; p++) {
        const double2 l = *reinterpret_cast<const double2*>(lp + (int64_t)pl[p] * TS);
        const double2 u = *reinterpret_cast<const double2*>(up + (int64_t)pu[p] * TS);
        s00 = fma(-l.x, u.x, s00);
        s10 = fma(-l.y, u.x, s10);
        s01 = fma(-l.x, u.y, s01);
        s11 = fma(-l.y, u.y, s11);
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
