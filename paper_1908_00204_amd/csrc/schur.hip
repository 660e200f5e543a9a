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

constexpr int CP = 32;     // pairs per staged chunk
constexpr int HSTAGE = 8;  // chunks in flight for a long tile

// The 2 x 2 block of lane (rp, cp): s00..s11 of rows 2rp, 2rp+1 and columns
// 2cp, 2cp+1 of the tile, updated with the cnt pairs staged in buf (each a
// 16-wide L row as 8 double2, then the U row) in order.  Full chunks read the
// next 8 pairs from LDS before the multiply-adds of the current 8.
struct TileAcc {
    double s00, s10, s01, s11;
    __device__ __forceinline__ void apply(const double2& l, const double2& u) {
        s00 = fma(-l.x, u.x, s00);
        s10 = fma(-l.y, u.x, s10);
        s01 = fma(-l.x, u.y, s01);
        s11 = fma(-l.y, u.y, s11);
    }
    __device__ __forceinline__ void chunk(const double2 (*buf)[TS], int cnt, int rp, int cp) {
        if (cnt == CP) {
            double2 la[8], ua[8], lb[8], ub[8];
#pragma unroll
            for (int x = 0; x < 8; x++) {
                la[x] = buf[x][rp];
                ua[x] = buf[x][8 + cp];
            }
#pragma unroll
            for (int g = 0; g < CP / 8; g += 2) {
#pragma unroll
                for (int x = 0; x < 8; x++) {
                    lb[x] = buf[8 * (g + 1) + x][rp];
                    ub[x] = buf[8 * (g + 1) + x][8 + cp];
                }
#pragma unroll
                for (int x = 0; x < 8; x++) apply(la[x], ua[x]);
                if (g + 2 < CP / 8) {
#pragma unroll
                    for (int x = 0; x < 8; x++) {
                        la[x] = buf[8 * (g + 2) + x][rp];
                        ua[x] = buf[8 * (g + 2) + x][8 + cp];
                    }
                }
#pragma unroll
                for (int x = 0; x < 8; x++) apply(lb[x], ub[x]);
            }
        } else {
            for (int x = 0; x < cnt; x++) apply(buf[x][rp], buf[x][8 + cp]);
        }
    }
};

// S -= L21 U12 on 16 x 16 tiles of the dense block D (column-major, leading
// dimension ld); lane (rp, cp) of the computing wave owns rows i0 + 2rp + {0,1}
// and columns k0 + 2cp + {0,1}.  A tile's pairs are applied in list order
// (ascending source).  Blocks [0, nheavy) each take one long tile: all 256
// threads stream its panel rows through LDS, HSTAGE chunks of CP pairs in
// flight in registers (the panel-row indices HSTAGE chunks further ahead), and
// wave 0 computes.  Later blocks give each of their 4 waves its own short
// tile, streamed the same way three chunks deep.
__global__ __launch_bounds__(256) void k_schur(const SchurUnit* __restrict__ units, int64_t nunits, int64_t nheavy,
                                               const int32_t* __restrict__ pl, const int32_t* __restrict__ pu,
                                               const double* __restrict__ LP, const double* __restrict__ UP,
                                               double* __restrict__ D, int64_t ld, int32_t m) {
    __shared__ double2 sbuf[4][2][CP][TS];  // [wave][buffer][pair][L row | U row]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rp = lane & 7, cp = lane >> 3;
    const bool heavy = (int64_t)blockIdx.x < nheavy;
    const int64_t uidx = heavy ? (int64_t)blockIdx.x : nheavy + ((int64_t)blockIdx.x - nheavy) * 4 + w;
    if (uidx >= nunits) return;  // (light blocks only: no block-wide barrier follows)
    const SchurUnit un = units[uidx];
    const int32_t r = un.i0 + 2 * rp;
    const int32_t c = un.k0 + 2 * cp;
    const bool r0ok = r < m, r1ok = r + 1 < m, c0ok = c < m, c1ok = c + 1 < m;
    double* d0 = D + r + (int64_t)c * ld;
    double* d1 = d0 + ld;
    const bool computes = !heavy || w == 0;
    TileAcc acc = {0.0, 0.0, 0.0, 0.0};
    if (computes) {
        acc.s00 = (r0ok && c0ok) ? d0[0] : 0.0;
        acc.s10 = (r1ok && c0ok) ? d0[1] : 0.0;
        acc.s01 = (r0ok && c1ok) ? d1[0] : 0.0;
        acc.s11 = (r1ok && c1ok) ? d1[1] : 0.0;
    }
    const int64_t np = un.pe - un.pb;
    const int64_t nch = (np + CP - 1) / CP;
    if (heavy) {
        // thread t stages 32 bytes of pair x = t / 8 of each chunk: the L row
        // (t % 8 < 4) or the U row, double2 parts 2 (t % 4) and 2 (t % 4) + 1
        const int x = tid >> 3, h = (tid >> 2) & 1, part = 2 * (tid & 3);
        const double* pbase = h ? UP + un.ubase : LP + un.lbase;
        const int32_t* pidx = h ? pu : pl;
        double2(*buf)[CP][TS] = sbuf[0];
        auto load_idx = [&](int64_t ch) -> int32_t {
            const int64_t p = un.pb + ch * CP + x;
            return (ch < nch && p < un.pe) ? pidx[p] : -1;
        };
        auto load_val = [&](int32_t ix, double2& v0, double2& v1) {
            if (ix >= 0) {
                const double2* src = reinterpret_cast<const double2*>(pbase + (int64_t)ix * TS) + part;
                v0 = src[0];
                v1 = src[1];
            } else {
                v0 = v1 = make_double2(0.0, 0.0);
            }
        };
        int32_t X[HSTAGE];
        double2 V0[HSTAGE], V1[HSTAGE];
#pragma unroll
        for (int k = 0; k < HSTAGE; k++) X[k] = load_idx(k);
#pragma unroll
        for (int k = 0; k < HSTAGE; k++) {
            load_val(X[k], V0[k], V1[k]);
            X[k] = load_idx(k + HSTAGE);
        }
        for (int64_t ch0 = 0; ch0 < nch; ch0 += HSTAGE) {
#pragma unroll
            for (int k = 0; k < HSTAGE; k++) {
                const int64_t ch = ch0 + k;
                if (ch < nch) {  // uniform over the block
                    const int bsel = (int)(ch & 1);
                    buf[bsel][x][h * 8 + part] = V0[k];
                    buf[bsel][x][h * 8 + part + 1] = V1[k];
                    load_val(X[k], V0[k], V1[k]);     // chunk ch + HSTAGE
                    X[k] = load_idx(ch + 2 * HSTAGE);
                    __syncthreads();  // chunk ch is in LDS; wave 0 finished chunk ch - 1
                    if (w == 0) acc.chunk(buf[bsel], (int)min<int64_t>(CP, np - ch * CP), rp, cp);
                }
            }
        }
    } else {
        // lane (q, hq) stages the L (hq = 0) or U row of pair q of a chunk
        const int q = lane >> 1, hq = lane & 1;
        const double* pbase = hq ? UP + un.ubase : LP + un.lbase;
        const int32_t* pidx = hq ? pu : pl;
        double2(*buf)[CP][TS] = sbuf[w];
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
            // one wave owns this buffer: its LDS operations complete in order
            const int bsel = (int)(ch & 1);
#pragma unroll
            for (int k = 0; k < 8; k++) buf[bsel][q][hq * 8 + k] = R[k];
            __builtin_amdgcn_wave_barrier();
            load(ch + 3, R);
            acc.chunk(buf[bsel], (int)min<int64_t>(CP, np - ch * CP), rp, cp);
            __builtin_amdgcn_wave_barrier();
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
    }
    if (computes) {
        if (r0ok && c0ok) d0[0] = acc.s00;
        if (r1ok && c0ok) d0[1] = acc.s10;
        if (r0ok && c1ok) d1[0] = acc.s01;
        if (r1ok && c1ok) d1[1] = acc.s11;
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
    if (launch_zero(s.LP, s.lp_len, st) != hipSuccess || launch_zero(s.UP, s.up_len, st) != hipSuccess)
        return hipGetLastError();
    if (s.nl > 0) k_panel_scatter<<<grid_for(s.nl, 256), 256, 0, st>>>(val, s.lpos, s.loff, s.nl, s.LP);
    if (s.nu > 0) k_panel_scatter<<<grid_for(s.nu, 256), 256, 0, st>>>(val, s.upos, s.uoff, s.nu, s.UP);
    const int64_t nlight = s.nunits - s.nheavy;
    const int64_t grid = s.nheavy + (nlight + 3) / 4;
    k_schur<<<(unsigned)grid, 256, 0, st>>>(s.units, s.nunits, s.nheavy, s.pl, s.pu, s.LP, s.UP, D, ld, m);
    return hipGetLastError();
}

}  // namespace glu
