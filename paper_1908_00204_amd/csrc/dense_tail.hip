// Dense trailing block of the factorization on gfx950.
//
// Late in the factorization of circuit matrices the remaining submatrix is
// dense (the wide-to-narrow level profile of Section III-B ends in levels of
// one column whose subcolumns cover the whole remaining matrix).  Once every
// column before t has applied its submatrix update, the block A_s(t:n, t:n)
// holds the Schur complement; its LU without pivoting is the same L and U the
// column-by-column algorithm produces (up to rounding order), so it is
// gathered into a dense m x m column-major buffer and factorized blockwise:
//   for each 64-wide panel:  LU of the diagonal block (one workgroup, LDS),
//   L21 = A21 U11^-1 and U12 = L11^-1 A12 (workgroups over 64-row / 64-column
//   blocks), A22 -= L21 U12 on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// Entries outside the filled pattern stay exactly zero (one factor of each of
// their products is an exact zero), so scattering the block back to A_s loses
// nothing.  The block stays resident for the dense part of the solves.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cstdint>

#include "kernels.hpp"
#include "mailbox.hpp"

namespace glu {

namespace {

constexpr int NB = 64;       // panel width
constexpr int SLD = NB + 1;  // padded leading dimension of 64x64 LDS blocks
constexpr int ALD = 72;      // LDS leading dimension of the GEMM's L21 tile (k-major)
constexpr int BLD = 68;      // LDS leading dimension of the GEMM's U12 tile (column-major)

typedef double v4d __attribute__((ext_vector_type(4)));

// Column c of the block: zero, or the identity's column for the padding
// columns m..M-1 (whole 64-wide panels).  Each entry is written once.
__global__ __launch_bounds__(256) void k_tail_init(int32_t m, int32_t M, double* __restrict__ D, int64_t ld) {
    const int32_t c = blockIdx.x;
    if (c >= M) return;
    double* col = D + (int64_t)c * ld;
    for (int32_t r = threadIdx.x; r < M; r += blockDim.x) col[r] = (r == c && c >= m) ? 1.0 : 0.0;
}

// The entries of A inside the block (A_s position, local row and column):
// the block's initial values.
__global__ __launch_bounds__(256) void k_tail_avals(const int64_t* __restrict__ src, const int32_t* __restrict__ row,
                                                    const int32_t* __restrict__ col, int64_t na,
                                                    const double* __restrict__ val, double* __restrict__ D,
                                                    int64_t ld) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < na) D[row[x] + (int64_t)col[x] * ld] = val[src[x]];
}

__global__ __launch_bounds__(256) void k_tail_scatter(const int64_t* __restrict__ colptr,
                                                      const int32_t* __restrict__ rowind,
                                                      double* __restrict__ val,
                                                      const int64_t* __restrict__ tail_pos, int32_t t,
                                                      int32_t m, const double* __restrict__ D, int64_t ld) {
    const int32_t c = blockIdx.x;
    if (c >= m) return;
    const double* col = D + (int64_t)c * ld;
    const int32_t k = t + c;
    for (int64_t p = tail_pos[c] + threadIdx.x; p < colptr[k + 1]; p += blockDim.x) val[p] = col[rowind[p] - t];
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// One elimination step c of the LU without pivoting of a 64 x 64 block held
// by one wave in a 2-D cyclic layout: lane 16p + q holds A(4i + p, 16j + q)
// in a[i][j].  The pivot row (row c) travels across the four 16-lane rows of
// the wave with ds_bpermute, and each multiplier across a 16-lane row with a
// DPP row broadcast.  The lanes of column c scale their entries below the
// pivot into L by the pivot's reciprocal (refined by two Newton steps; the
// other lanes multiply by 1, an exact no-op), so the broadcast value is the
// multiplier itself and the stored L entry is the one the update uses.
template <int C>
__device__ __forceinline__ void lu_step(double (&a)[16][4], int p, int q) {
    constexpr int ic = C >> 2, pc = C & 3, jc = C >> 4, qc = C & 15;
    const double piv = readlane_f64(a[ic][jc], 16 * pc + qc);
    double rp = __builtin_amdgcn_rcp(piv);
    double e = fma(-piv, rp, 1.0);
    rp = fma(rp, e, rp);
    e = fma(-piv, rp, 1.0);
    rp = fma(rp, e, rp);
    double u[4];  // pivot row entries of this lane's columns; zero at columns <= c
    const int addr = (16 * pc + q) * 4;
#pragma unroll
    for (int j = jc; j < 4; j++) {
        const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(a[ic][j]));
        const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(a[ic][j]));
        u[j] = __hiloint2double(hi, lo);
    }
    u[jc] = q > qc ? u[jc] : 0.0;
    const double f = q == qc ? rp : 1.0;
    const double f0 = p > pc ? f : 1.0;  // rows <= c of column c stay U
#pragma unroll
    for (int i = ic; i < 16; i++) {
        a[i][jc] *= (i == ic ? f0 : f);
        double l = __builtin_amdgcn_mov_dpp(a[i][jc], 0x150 + qc, 0xF, 0xF, true);  // row_newbcast:qc
        if (i == ic) l = p > pc ? l : 0.0;
#pragma unroll
        for (int j = jc; j < 4; j++) a[i][j] = fma(-l, u[j], a[i][j]);
    }
}

template <int C>
struct LuSteps {
    static __device__ __forceinline__ void run(double (&a)[16][4], int p, int q) {
        lu_step<C>(a, p, q);
        LuSteps<C + 1>::run(a, p, q);
    }
};
template <>
struct LuSteps<NB - 1> {
    static __device__ __forceinline__ void run(double (&)[16][4], int, int) {}
};

// LU without pivoting of the 64 x 64 block T (LDS, T[r * SLD + c]) by wave 0,
// then every thread of the block stores it to A (column-major, leading
// dimension ld) and to the side buffer the next triangular solves read: F
// row-major and F + NB*NB column-major.
__device__ __forceinline__ void lds_lu_store(double* T, int tid, int nthreads, double* __restrict__ A, int64_t ld,
                                             double* __restrict__ F) {
    if (tid < 64) {
        const int p = tid >> 4, q = tid & 15;
        double a[16][4];
#pragma unroll
        for (int i = 0; i < 16; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) a[i][j] = T[(4 * i + p) * SLD + 16 * j + q];
        LuSteps<0>::run(a, p, q);
#pragma unroll
        for (int i = 0; i < 16; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) T[(4 * i + p) * SLD + 16 * j + q] = a[i][j];
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += nthreads) {
        const int r = e & 63, c = e >> 6;
        const double v = T[r * SLD + c];
        A[r + (int64_t)c * ld] = v;
        F[NB * NB + e] = v;
        F[e] = T[c * SLD + r];  // row c, column r
    }
}

// LU of the first 64 x 64 diagonal block in place.
__global__ __launch_bounds__(256) void k_dense_diag(double* __restrict__ D, int64_t ld, double* __restrict__ F) {
    __shared__ double T[NB * SLD];
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) T[(e & 63) * SLD + (e >> 6)] = D[(e & 63) + (int64_t)(e >> 6) * ld];
    __syncthreads();
    lds_lu_store(T, tid, 256, D, ld, F);
}

// Broadcast lane G of each group of four lanes to the whole group (DPP
// quad_perm [G,G,G,G]), as two 32-bit moves.
template <int G>
__device__ __forceinline__ double quad_bcast(double x) {
    constexpr int ctrl = G * 0x55;
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double quad_bcast(double x, int g0) {
    switch (g0) {
        case 0: return quad_bcast<0>(x);
        case 1: return quad_bcast<1>(x);
        case 2: return quad_bcast<2>(x);
        default: return quad_bcast<3>(x);
    }
}

constexpr int QS = 18;      // LDS stride of one lane group's 16 entries (even: 16-byte reads)
constexpr int QL = 4 * QS;  // LDS stride of one step's entries

// Block rows of L21 = A21 U11^-1 (blockIdx < nrb) and block columns of
// U12 = L11^-1 A12 (blockIdx >= nrb) for the panel at kb, 4 waves per 64 x 64
// block.  The rows of L21 (columns of U12) are independent: lane (i, g) of
// the block, i = 16 w + lane / 4 and g = lane % 4, holds entries 4k + g,
// k < 16, of row (column) i, so the four lanes of one row form a DPP quad.
// Step c of the substitution finishes entry c on lane g = c % 4 of every
// quad, broadcasts it within the quad, and each lane updates its later
// entries with the step's row of U11 (column of L11), read from LDS where it
// is stored grouped by g.  L21 divides by the pivot with its reciprocal and
// one residual correction.
__global__ __launch_bounds__(256) void k_dense_trsm(double* __restrict__ D, int64_t ld, int32_t kb, int32_t nrb,
                                                    const double* __restrict__ F) {
    __shared__ double S[NB * QL];  // step c: S[c*QL + g*QS + k] = U11(c, 4k+g) or L11(4k+g, c), else 0
    __shared__ double T[NB * 68];  // U12 staging, T[j * 68 + r] = A12(r, j)
    __shared__ double rd[NB];      // 1 / U11(c, c)
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int g = lane & 3, i = 16 * w + (lane >> 2);
    const bool lower = (int32_t)blockIdx.x < nrb;
    double x[16];
    if (lower) {
#pragma unroll
        for (int j = 0; j < 16; j++) {  // F row-major: F[c * NB + col] = U11(c, col) for col >= c
            const int e = tid + 256 * j, c = e >> 6, col = e & 63;
            S[c * QL + (col & 3) * QS + (col >> 2)] = col >= c ? F[e] : 0.0;
        }
        if (tid < NB) rd[tid] = 1.0 / F[tid * NB + tid];
        const double* A21 = D + (kb + NB + (int64_t)blockIdx.x * NB + i) + (int64_t)kb * ld;
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = A21[(int64_t)(4 * k + g) * ld];
    } else {
#pragma unroll
        for (int j = 0; j < 16; j++) {  // F + NB*NB column-major: [c * NB + r] = L11(r, c) for r > c
            const int e = tid + 256 * j, c = e >> 6, r = e & 63;
            S[c * QL + (r & 3) * QS + (r >> 2)] = r > c ? F[NB * NB + e] : 0.0;
        }
        const double* A12 = D + kb + (kb + NB + (int64_t)((int32_t)blockIdx.x - nrb) * NB) * ld;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j, r = e & 63, col = e >> 6;
            T[col * 68 + r] = A12[r + (int64_t)col * ld];
        }
    }
    __syncthreads();
    if (lower) {
#pragma unroll
        for (int c = 0; c < NB; c++) {
            const int k0 = c >> 2, g0 = c & 3;
            const double* srow = S + c * QL + g * QS;
            const double dg = S[c * QL + g0 * QS + k0], r = rd[c];
            const double q0 = x[k0] * r;
            const double q = fma(fma(-q0, dg, x[k0]), r, q0);
            x[k0] = g == g0 ? q : x[k0];
            const double xc = quad_bcast(x[k0], g0);
            const double xu = fma(-xc, srow[k0], x[k0]);
            x[k0] = g > g0 ? xu : x[k0];
#pragma unroll
            for (int k = k0 + 1; k < 16; k++) x[k] = fma(-xc, srow[k], x[k]);
        }
        double* A21 = D + (kb + NB + (int64_t)blockIdx.x * NB + i) + (int64_t)kb * ld;
#pragma unroll
        for (int k = 0; k < 16; k++) A21[(int64_t)(4 * k + g) * ld] = x[k];
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = T[i * 68 + 4 * k + g];
#pragma unroll
        for (int c = 0; c < NB - 1; c++) {
            const int k0 = c >> 2, g0 = c & 3;
            const double* scol = S + c * QL + g * QS;
            const double xc = quad_bcast(x[k0], g0);
            // rows 4k + g <= c meet stored zeros: exact no-ops
#pragma unroll
            for (int k = k0; k < 16; k++) x[k] = fma(-scol[k], xc, x[k]);
        }
        __syncthreads();  // every lane has read its column from T
#pragma unroll
        for (int k = 0; k < 16; k++) T[i * 68 + 4 * k + g] = x[k];
        __syncthreads();
        double* A12 = D + kb + (kb + NB + (int64_t)((int32_t)blockIdx.x - nrb) * NB) * ld;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j, r = e & 63, col = e >> 6;
            A12[r + (int64_t)col * ld] = T[col * 68 + r];
        }
    }
}

// A rectangle of 64x64 output tiles of the trailing update: rows r0 + 64 tr,
// columns c0 + 64 tc, tr < ntr, tc < ntc.
struct TileRegion {
    int32_t r0, c0, ntr, ntc;
};

// C -= A B on the 64x64 tiles of up to two regions, with A = D(rows, ka : ka+K)
// (L columns) and B = D(ka : ka+K, cols) (U rows), K a multiple of 64.
// 4 waves per tile, each a 32x32 quadrant of 2x2 MFMA tiles; v_mfma_f64_16x16x4f64
// takes lane l's first operand as P[l%16][l/16] and second as Q[l/16][l%16] and
// returns D[l/16 + 4v][l%16] in accumulator v (layout measured on gfx950).  P
// is U (16 columns x 4 k) and Q is L (4 k x 16 rows), so for each v the 16 lanes
// of a quarter-wave hold 16 consecutive rows of one column and the
// read-modify-write of C is coalesced.  K runs in chunks of 64 staged through
// LDS, the next chunk prefetched into registers during the current one's MFMAs;
// the C tile is fetched at the start.  With fuse set, tile (0,0) of region 0
// is the next panel's diagonal block: its block finishes the tile in LDS and
// factors it (the next panel then starts with its solves).
__global__ __launch_bounds__(256) void k_dense_update(double* __restrict__ D, int64_t ld, int32_t ka, int32_t K,
                                                      TileRegion g0, TileRegion g1, int32_t fuse,
                                                      double* __restrict__ F) {
    __shared__ double As[NB * ALD];  // As[k * ALD + r] = L(r0 + r, ka + k0 + k)
    __shared__ double Bs[NB * BLD];  // Bs[c * BLD + k] = U(ka + k0 + k, c0 + c)
    const int tid = threadIdx.x;
    int32_t t = blockIdx.x;
    TileRegion g = g0;
    if (t >= g0.ntr * g0.ntc) {
        t -= g0.ntr * g0.ntc;
        g = g1;
    }
    const int32_t r0 = g.r0 + NB * (t % g.ntr), c0 = g.c0 + NB * (t / g.ntr);
    const int lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int i = lane & 15, kq = lane >> 4;
    double cv[2][2][4];
#pragma unroll
    for (int sc = 0; sc < 2; sc++)
#pragma unroll
        for (int sr = 0; sr < 2; sr++)
#pragma unroll
            for (int v = 0; v < 4; v++)
                cv[sc][sr][v] = D[(r0 + wr * 32 + sr * 16 + i) + (int64_t)(c0 + wc * 32 + sc * 16 + kq + 4 * v) * ld];
    double ar[16], br[16];
    auto load_chunk = [&](int32_t k0) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j;
            ar[j] = D[(r0 + (e & 63)) + (int64_t)(ka + k0 + (e >> 6)) * ld];
            br[j] = D[(ka + k0 + (e & 63)) + (int64_t)(c0 + (e >> 6)) * ld];
        }
    };
    v4d acc[2][2];
    for (int x = 0; x < 2; x++)
        for (int y = 0; y < 2; y++) acc[x][y] = (v4d){0.0, 0.0, 0.0, 0.0};
    load_chunk(0);
    for (int32_t k0 = 0; k0 < K; k0 += NB) {
        __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int e = tid + 256 * j;
            As[(e >> 6) * ALD + (e & 63)] = ar[j];
            Bs[(e >> 6) * BLD + (e & 63)] = br[j];
        }
        __syncthreads();
        if (k0 + NB < K) load_chunk(k0 + NB);
#pragma unroll
        for (int k4 = 0; k4 < NB; k4 += 4) {
            const int kk = k4 + kq;
            double p[2], q[2];
#pragma unroll
            for (int sc = 0; sc < 2; sc++) p[sc] = Bs[(wc * 32 + sc * 16 + i) * BLD + kk];
#pragma unroll
            for (int sr = 0; sr < 2; sr++) q[sr] = As[kk * ALD + wr * 32 + sr * 16 + i];
#pragma unroll
            for (int sc = 0; sc < 2; sc++)
#pragma unroll
                for (int sr = 0; sr < 2; sr++)
                    acc[sc][sr] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[sc], q[sr], acc[sc][sr], 0, 0, 0);
        }
    }
    if (fuse && blockIdx.x == 0) {
        __syncthreads();  // every wave is done with As / Bs
        double* Tt = As;  // Tt[r * SLD + c], local row r and column c of the tile
#pragma unroll
        for (int sc = 0; sc < 2; sc++)
#pragma unroll
            for (int sr = 0; sr < 2; sr++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    Tt[(wr * 32 + sr * 16 + i) * SLD + wc * 32 + sc * 16 + kq + 4 * v] = cv[sc][sr][v] - acc[sc][sr][v];
        __syncthreads();
        lds_lu_store(Tt, tid, 256, D + r0 + (int64_t)c0 * ld, ld, F);
        return;
    }
#pragma unroll
    for (int sc = 0; sc < 2; sc++)
#pragma unroll
        for (int sr = 0; sr < 2; sr++)
#pragma unroll
            for (int v = 0; v < 4; v++)
                D[(r0 + wr * 32 + sr * 16 + i) + (int64_t)(c0 + wc * 32 + sc * 16 + kq + 4 * v) * ld] =
                    cv[sc][sr][v] - acc[sc][sr][v];
}

// ---------------------------------------------------------------- dense solves

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Read N mailbox values (base + 4 i, i < N; indices at or past lim read as 0)
// once none is the sentinel (mailbox.hpp).  The dense triangular solves hand
// each block's results to the later blocks this way.
template <int N>
__device__ __forceinline__ void mail_get(const double* mail, int64_t base, int64_t lim, uint64_t sentinel,
                                         double (&v)[N], int32_t* err) {
    int64_t idx[N];
    bool use[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        idx[i] = base + 4 * i;
        use[i] = idx[i] < lim;
    }
    mail_read<N>(mail, idx, use, sentinel, v, err);
}

// Forward substitution on the dense tail (unit lower triangle of D), rows in
// 64-row blocks taken in ticket order; block b first subtracts the finished
// blocks to its left (reading their results from the mailbox), then solves
// its diagonal block in one wave and publishes.  y: tail part of the work
// vector(s); mail: m x nrhs mailbox.  Everything that does not depend on
// another block is loaded before the waits: wave 0 holds its lane's row of the
// diagonal block in registers, and each 64-column chunk of the block's rows is
// fetched before its results are polled.  The diagonal solve broadcasts each
// solved entry with v_readlane.
__global__ __launch_bounds__(256) void k_dense_fwd(const double* __restrict__ D, int64_t ld, int32_t m,
                                                   double* __restrict__ y, int64_t ldy, int32_t nrhs,
                                                   int32_t* ticket, double* mail, int32_t epoch, int32_t* err) {
    __shared__ int32_t sblk;
    __shared__ double part[4][64];
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    if (tid == 0) sblk = atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t blk = sblk;
    const int32_t r0 = blk * 64;
    const int32_t nr = min(64, m - r0);
    const bool rok = lane < nr;
    const int32_t row = r0 + (rok ? lane : 0);
    const uint64_t sentinel = mail_sentinel((uint32_t)epoch);
    double drow[NB];
    if (q == 0) {
#pragma unroll
        for (int c = 0; c < NB; c++) drow[c] = (rok && c < nr) ? D[row + (int64_t)(r0 + c) * ld] : 0.0;
    }
    for (int32_t r = 0; r < nrhs; r++) {
        double* yr = y + (int64_t)r * ldy;
        double* mr = mail + (int64_t)r * m;
        double acc = 0.0;
        for (int32_t cb = 0; cb < blk; cb++) {
            double dv[16], yv[16];
#pragma unroll
            for (int i = 0; i < 16; i++) dv[i] = D[row + (int64_t)(cb * 64 + q + 4 * i) * ld];
            mail_get<16>(mr, cb * 64 + q, m, sentinel, yv, err);
#pragma unroll
            for (int i = 0; i < 16; i++) acc += dv[i] * yv[i];
        }
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0) {
            double x = rok ? yr[row] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]) : 0.0;
#pragma unroll
            for (int c = 0; c < NB - 1; c++) {
                const double xc = readlane_f64(x, c);
                const double xu = fma(-drow[c], xc, x);
                x = lane > c ? xu : x;
            }
            if (rok) {
                yr[row] = x;
                mail_put(mr, row, x);
            }
        }
        __syncthreads();
    }
}

// Backward substitution on the dense tail (upper triangle of D with its
// diagonal), blocks from the last one up; same structure as the forward solve.
__global__ __launch_bounds__(256) void k_dense_bwd(const double* __restrict__ D, int64_t ld, int32_t m,
                                                   double* __restrict__ y, int64_t ldy, int32_t nrhs,
                                                   int32_t* ticket, double* mail, int32_t epoch, int32_t* err) {
    __shared__ int32_t sblk;
    __shared__ double part[4][64];
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int32_t nblk = (m + 63) / 64;
    if (tid == 0) sblk = nblk - 1 - atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t blk = sblk;
    const int32_t r0 = blk * 64;
    const int32_t nr = min(64, m - r0);
    const bool rok = lane < nr;
    const int32_t row = r0 + (rok ? lane : 0);
    const uint64_t sentinel = mail_sentinel((uint32_t)epoch);
    // wave 0 holds its lane's row of the diagonal block divided by the row's
    // pivot (a unit upper triangle), computed before any wait
    double drow[NB];
    const double ddiag = rok ? D[row + (int64_t)row * ld] : 1.0;
    if (q == 0) {
#pragma unroll
        for (int c = 0; c < NB; c++) drow[c] = (rok && c < nr) ? D[row + (int64_t)(r0 + c) * ld] / ddiag : 0.0;
    }
    for (int32_t r = 0; r < nrhs; r++) {
        double* yr = y + (int64_t)r * ldy;
        double* mr = mail + (int64_t)r * m;
        double acc = 0.0;
        for (int32_t cb = nblk - 1; cb > blk; cb--) {
            const int32_t cend = min(cb * 64 + 64, m);
            double dv[16], yv[16];
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int32_t c = cb * 64 + q + 4 * i;
                dv[i] = c < cend ? D[row + (int64_t)c * ld] : 0.0;
            }
            mail_get<16>(mr, cb * 64 + q, cend, sentinel, yv, err);
#pragma unroll
            for (int i = 0; i < 16; i++) acc += dv[i] * yv[i];
        }
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0) {
            // x(j) = y(j) / U(j,j) - sum_{k > j} (U(j,k) / U(j,j)) x(k): the
            // division leaves the dependency chain, which is then a broadcast
            // and a multiply-add per step.  Branch-free: lanes past nr hold
            // x = 0 and a zero row, so their steps change nothing.
            double x = rok ? (yr[row] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane])) / ddiag : 0.0;
#pragma unroll
            for (int c = NB - 1; c > 0; c--) {
                const double xc = readlane_f64(x, c);
                const double xu = fma(-drow[c], xc, x);
                x = lane < c ? xu : x;
            }
            if (rok) {
                yr[row] = x;
                mail_put(mr, row, x);
            }
        }
        __syncthreads();
    }
}

// Tail rows of the forward solve: y(t+c) -= sum_{j < t} L(t+c, j) y(j).  The
// rows of the supply rails hold tens of thousands of entries, so each row is
// cut into chunks; one wave per chunk writes its partial sum, then one thread
// per row and right-hand side adds the row's partials in chunk order.
__global__ __launch_bounds__(256) void k_cross_part(const SolveArgs sa, int32_t t, const int32_t* __restrict__ crow,
                                                    const int64_t* __restrict__ cq0, int32_t nw,
                                                    const int64_t* __restrict__ tail_lsplit,
                                                    double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int32_t w = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (w >= nw) return;
    const int32_t c = crow[w];
    const int64_t q0 = cq0[w];
    const int64_t q1 = min(q0 + (int64_t)CROSS_CHUNK, tail_lsplit[c]);
    for (int32_t r = 0; r < sa.nrhs; r++) {
        const double* yr = sa.y + (int64_t)r * sa.n;
        double acc = 0.0;
        for (int64_t q = q0 + lane; q < q1; q += 64) acc += sa.val[sa.lrow_pos[q]] * yr[sa.lrow_col[q]];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) part[(int64_t)r * nw + w] = acc;
    }
}

__global__ __launch_bounds__(256) void k_cross_apply(const SolveArgs sa, int32_t t, int32_t m,
                                                     const int32_t* __restrict__ cptr, int32_t nw,
                                                     const double* __restrict__ part) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)m * sa.nrhs) return;
    const int32_t c = (int32_t)(x % m), r = (int32_t)(x / m);
    double acc = 0.0;
    for (int32_t w = cptr[c]; w < cptr[c + 1]; w++) acc += part[(int64_t)r * nw + w];
    sa.y[(int64_t)r * sa.n + t + c] -= acc;
}

// Backward-solve cross term of the rows before the block, y(j) -= U(j, t:n)
// x(t:n): one wave per work item (at most CROSS_CHUNK entries of one row,
// values gathered in item order) writes its partial sum; then one thread per
// row and right-hand side subtracts the row's partials in item order.
__global__ __launch_bounds__(256) void k_xpart(const double* __restrict__ xv, const int32_t* __restrict__ xc,
                                               const int64_t* __restrict__ q0, const int64_t* __restrict__ q1,
                                               int32_t nw, const double* __restrict__ y, int32_t n, int32_t nrhs,
                                               double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int32_t w = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (w >= nw) return;
    const int64_t a = q0[w], b = q1[w];
    for (int32_t r = 0; r < nrhs; r++) {
        const double* yr = y + (int64_t)r * n;
        double acc = 0.0;
        for (int64_t q = a + lane; q < b; q += 64) acc += xv[q] * yr[xc[q]];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) part[(int64_t)r * nw + w] = acc;
    }
}

__global__ __launch_bounds__(256) void k_xapply(const int32_t* __restrict__ rows, const int32_t* __restrict__ rptr,
                                                int32_t nrows, const double* __restrict__ part, int32_t nw,
                                                double* __restrict__ y, int32_t n, int32_t nrhs) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)nrows * nrhs) return;
    const int32_t c = (int32_t)(x % nrows), r = (int32_t)(x / nrows);
    double acc = 0.0;
    for (int32_t w = rptr[c]; w < rptr[c + 1]; w++) acc += part[(int64_t)r * nw + w];
    y[(int64_t)r * n + rows[c]] -= acc;
}

// Pivot check of the factored block: status[0] = the smallest column t + i
// whose pivot D(i, i) is zero or not finite.
__global__ void k_dense_pivots(const double* __restrict__ D, int64_t ld, int32_t m, int32_t t,
                               int32_t* __restrict__ status) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double d = D[i + (int64_t)i * ld];
    if (d == 0.0 || !isfinite(d)) atomicMin(&status[0], t + i);
}

// The M x M block between its FP64 home (leading dimension ld) and a packed
// FP32 copy (leading dimension M): rounded on the way in, exact on the way out.
__global__ void k_block_narrow(const double* __restrict__ D, int64_t ld, int32_t M, float* __restrict__ S) {
    const int64_t n = (int64_t)M * M;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = x / M, r = x - c * M;
        S[x] = (float)D[r + c * ld];
    }
}

__global__ void k_block_widen(const float* __restrict__ S, int32_t M, double* __restrict__ D, int64_t ld) {
    const int64_t n = (int64_t)M * M;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = x / M, r = x - c * M;
        D[r + c * ld] = (double)S[x];
    }
}

__global__ void k_reset_i32(int32_t* p, int32_t n, int32_t v) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_tail_gather(const double* val, const int64_t* asrc, const int32_t* arow, const int32_t* acol,
                              int64_t na, int32_t m, int32_t M, double* D, int64_t ld, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    if (M < m || ld < M) return hipErrorInvalidValue;
    k_tail_init<<<(unsigned)M, 256, 0, st>>>(m, M, D, ld);
    if (na > 0) k_tail_avals<<<(unsigned)((na + 255) / 256), 256, 0, st>>>(asrc, arow, acol, na, val, D, ld);
    return hipGetLastError();
}

hipError_t launch_dense_pivots(const double* D, int64_t ld, int32_t m, int32_t t, int32_t* status, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_dense_pivots<<<(m + 255) / 256, 256, 0, st>>>(D, ld, m, t, status);
    return hipGetLastError();
}

hipError_t launch_tail_scatter(const FactorArgs& a, const int64_t* tail_pos, int32_t t, int32_t m,
                               const double* D, int64_t ld, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_tail_scatter<<<m, 256, 0, st>>>(a.colptr, a.rowind, a.val, tail_pos, t, m, D, ld);
    return hipGetLastError();
}

hipError_t dense_blas_create(void** blas) {
    rocblas_handle b = nullptr;
    if (rocblas_create_handle(&b) != rocblas_status_success) return hipErrorUnknown;
    // no atomics in the library's kernels: the same inputs give the same bits
    if (rocblas_set_atomics_mode(b, rocblas_atomics_not_allowed) != rocblas_status_success) {
        (void)rocblas_destroy_handle(b);
        return hipErrorUnknown;
    }
    *blas = b;
    return hipSuccess;
}

void dense_blas_destroy(void* blas) {
    if (blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(blas));
}

hipError_t launch_dense_lu(double* D, int64_t ld, int32_t M, double* F, hipStream_t st, hipStream_t aux,
                           hipEvent_t ev_fork, hipEvent_t ev_join, void* blas) {
    if (M <= 0) return hipSuccess;
    if (M % NB != 0) return hipErrorInvalidValue;
    // Two-level blocking: outer panels of OW columns, each factored as 64-wide
    // inner panels whose updates stay inside the outer panel's columns (tall
    // region) and rows (wide region); the rest of the trailing matrix is
    // updated once per outer panel with K = OW.  That update is split: the
    // next outer panel's columns and rows go first on st (the next panel's
    // chain needs them; their tile (0,0) is its first diagonal block), and the
    // bulk beyond runs on aux at the same time as the next panel's inner
    // steps, which touch only the next panel's rows and columns.  st waits for
    // the bulk before the following outer update.  The first diagonal block
    // is factored here, every later one by the update that finishes it (or,
    // after a library strip, by its own launch).  The bulk is a plain GEMM
    // (C -= A B with K = OW): given a library handle it goes to the library's
    // DGEMM, else to k_dense_update.  Large blocks take
    // 512-wide outer panels (1024-wide from 16,384 columns): the bulk GEMMs
    // then run at K = 512 (1024), where the library's DGEMM is faster, and
    // the chain they hide grows with them; their strips go to the library's
    // DGEMM too.
    const bool big = blas && M >= 8192;
    const int32_t OW = !big ? 256 : M >= 16384 ? 1024 : 512;
    const TileRegion none = {0, 0, 0, 0};
    bool bulk_pending = false;
    k_dense_diag<<<1, 256, 0, st>>>(D, ld, F);
    for (int32_t K0 = 0; K0 < M; K0 += OW) {
        const int32_t Kend = min(K0 + OW, M);
        for (int32_t kb = K0; kb < Kend; kb += NB) {
            const int32_t rest = M - kb - NB;
            if (rest <= 0) break;
            k_dense_trsm<<<2 * (rest / NB), 256, 0, st>>>(D, ld, kb, rest / NB, F);
            const int32_t ntall = (Kend - kb - NB) / NB;
            if (ntall > 0) {
                const TileRegion tall = {kb + NB, kb + NB, rest / NB, ntall};
                const TileRegion wide = {kb + NB, Kend, ntall, (M - Kend) / NB};
                const int32_t grid = tall.ntr * tall.ntc + wide.ntr * wide.ntc;
                k_dense_update<<<grid, 256, 0, st>>>(D, ld, kb, NB, tall, wide, 1, F);
            }
        }
        if (Kend >= M) break;
        if (bulk_pending) {  // the previous panel's bulk update wrote this region
            if (hipStreamWaitEvent(st, ev_join, 0) != hipSuccess) return hipErrorUnknown;
            bulk_pending = false;
        }
        const int32_t K2 = min(Kend + OW, M);
        if (big) {
            // the strip as two library DGEMMs (aux is idle meanwhile: the
            // previous bulk has ended and the next one waits for the strip),
            // then the next panel's diagonal block
            const rocblas_handle b = static_cast<rocblas_handle>(blas);
            const double minus_one = -1.0, one = 1.0;
            if (rocblas_set_stream(b, st) != rocblas_status_success ||
                rocblas_dgemm(b, rocblas_operation_none, rocblas_operation_none, M - Kend, K2 - Kend, Kend - K0,
                              &minus_one, D + Kend + (int64_t)K0 * ld, ld, D + K0 + (int64_t)Kend * ld, ld, &one,
                              D + Kend + (int64_t)Kend * ld, ld) != rocblas_status_success ||
                (K2 < M &&
                 rocblas_dgemm(b, rocblas_operation_none, rocblas_operation_none, K2 - Kend, M - K2, Kend - K0,
                               &minus_one, D + Kend + (int64_t)K0 * ld, ld, D + K0 + (int64_t)K2 * ld, ld, &one,
                               D + Kend + (int64_t)K2 * ld, ld) != rocblas_status_success))
                return hipErrorUnknown;
            k_dense_diag<<<1, 256, 0, st>>>(D + Kend + (int64_t)Kend * ld, ld, F);
        } else {
            const TileRegion strip_c = {Kend, Kend, (M - Kend) / NB, (K2 - Kend) / NB};
            const TileRegion strip_r = {Kend, K2, (K2 - Kend) / NB, (M - K2) / NB};
            k_dense_update<<<strip_c.ntr * strip_c.ntc + strip_r.ntr * strip_r.ntc, 256, 0, st>>>(
                D, ld, K0, Kend - K0, strip_c, strip_r, 1, F);
        }
        if (K2 < M) {
            if (hipEventRecord(ev_fork, st) != hipSuccess || hipStreamWaitEvent(aux, ev_fork, 0) != hipSuccess)
                return hipErrorUnknown;
            if (blas) {
                const rocblas_handle b = static_cast<rocblas_handle>(blas);
                const double minus_one = -1.0, one = 1.0;
                if (rocblas_set_stream(b, aux) != rocblas_status_success ||
                    rocblas_dgemm(b, rocblas_operation_none, rocblas_operation_none, M - K2, M - K2, Kend - K0,
                                  &minus_one, D + K2 + (int64_t)K0 * ld, ld, D + K0 + (int64_t)K2 * ld, ld, &one,
                                  D + K2 + (int64_t)K2 * ld, ld) != rocblas_status_success)
                    return hipErrorUnknown;
            } else {
                const TileRegion bulk = {K2, K2, (M - K2) / NB, (M - K2) / NB};
                k_dense_update<<<bulk.ntr * bulk.ntc, 256, 0, aux>>>(D, ld, K0, Kend - K0, bulk, none, 0, F);
            }
            if (hipEventRecord(ev_join, aux) != hipSuccess) return hipErrorUnknown;
            bulk_pending = true;
        }
    }
    if (bulk_pending && hipStreamWaitEvent(st, ev_join, 0) != hipSuccess) return hipErrorUnknown;
    return hipGetLastError();
}

hipError_t launch_dense_lu_fp32(double* D, int64_t ld, int32_t M, float* S, void* blas, int32_t* info,
                                hipStream_t st) {
    if (M <= 0) return hipSuccess;
    if (!blas || !S || !info) return hipErrorInvalidValue;
    const unsigned grid = 4096;
    k_block_narrow<<<grid, 256, 0, st>>>(D, ld, M, S);
    const rocblas_handle b = static_cast<rocblas_handle>(blas);
    if (rocblas_set_stream(b, st) != rocblas_status_success ||
        rocsolver_sgetrf_npvt(b, M, M, S, M, reinterpret_cast<rocblas_int*>(info)) != rocblas_status_success)
        return hipErrorUnknown;
    k_block_widen<<<grid, 256, 0, st>>>(S, M, D, ld);
    return hipGetLastError();
}

hipError_t launch_tail_cross_fwd(const SolveArgs& sa, int32_t t, int32_t m, const int64_t* tail_lsplit,
                                 const int32_t* cptr, const int32_t* crow, const int64_t* cq0, int32_t nw,
                                 double* part, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    if (nw > 0) k_cross_part<<<(unsigned)((nw + 3) / 4), 256, 0, st>>>(sa, t, crow, cq0, nw, tail_lsplit, part);
    const int64_t nt = (int64_t)m * sa.nrhs;
    k_cross_apply<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(sa, t, m, cptr, nw, part);
    return hipGetLastError();
}

hipError_t launch_tail_cross_bwd(const double* xv, const int32_t* xc, const int64_t* q0, const int64_t* q1,
                                 int32_t nw, const int32_t* rows, const int32_t* rptr, int32_t nrows, double* y,
                                 int32_t n, int32_t nrhs, double* part, hipStream_t st) {
    if (nw <= 0 || nrows <= 0 || nrhs <= 0) return hipSuccess;
    k_xpart<<<(unsigned)((nw + 3) / 4), 256, 0, st>>>(xv, xc, q0, q1, nw, y, n, nrhs, part);
    const int64_t nt = (int64_t)nrows * nrhs;
    k_xapply<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(rows, rptr, nrows, part, nw, y, n, nrhs);
    return hipGetLastError();
}

hipError_t launch_dense_trsv(const double* D, int64_t ld, int32_t m, double* y, int64_t ldy, int32_t nrhs,
                             bool upper, int32_t* ticket, double* mail, int32_t epoch, int32_t* err,
                             hipStream_t st) {
    if (m <= 0 || nrhs <= 0) return hipSuccess;
    const int32_t nblk = (m + 63) / 64;
    const int64_t nm = (int64_t)m * nrhs;
    k_reset_i32<<<1, 64, 0, st>>>(ticket, 1, 0);
    k_fill_u64<<<(unsigned)((nm + 255) / 256), 256, 0, st>>>(reinterpret_cast<uint64_t*>(mail), nm,
                                                              mail_sentinel((uint32_t)epoch));
    if (upper)
        k_dense_bwd<<<nblk, 256, 0, st>>>(D, ld, m, y, ldy, nrhs, ticket, mail, epoch, err);
    else
        k_dense_fwd<<<nblk, 256, 0, st>>>(D, ld, m, y, ldy, nrhs, ticket, mail, epoch, err);
    return hipGetLastError();
}

}  // namespace glu
