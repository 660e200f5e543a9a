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

#include <cstdint>

#include "kernels.hpp"

namespace glu {

namespace {

constexpr int NB = 64;       // panel width
constexpr int SLD = NB + 1;  // padded leading dimension of 64x64 LDS blocks
constexpr int ALD = 72;      // LDS leading dimension of the GEMM's L21 tile (k-major)
constexpr int BLD = 68;      // LDS leading dimension of the GEMM's U12 tile (column-major)

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_tail_gather(const int64_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowind,
                                                     const double* __restrict__ val,
                                                     const int64_t* __restrict__ tail_pos, int32_t t,
                                                     int32_t m, int32_t M, double* __restrict__ D, int64_t ld) {
    // columns and rows m..M-1 pad the block to whole panels with the identity
    const int32_t c = blockIdx.x;
    if (c >= M) return;
    double* col = D + (int64_t)c * ld;
    for (int32_t r = threadIdx.x; r < M; r += blockDim.x) col[r] = (r == c && c >= m) ? 1.0 : 0.0;
    if (c >= m) return;
    __syncthreads();
    const int32_t k = t + c;
    for (int64_t p = tail_pos[c] + threadIdx.x; p < colptr[k + 1]; p += blockDim.x) col[rowind[p] - t] = val[p];
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

// LU without pivoting of a 64 x 64 block held by one wave, lane r holding row
// r in a[0..63].  Step c broadcasts the pivot row from lane c with v_readlane;
// lanes below the pivot divide their column-c entry by the pivot and update
// the rest of their row (the others use a zero multiplier, an exact no-op).
__device__ __forceinline__ void wave_lu(double (&a)[NB], int r) {
#pragma unroll
    for (int c = 0; c < NB - 1; c++) {
        const double piv = readlane_f64(a[c], c);
        const bool below = r > c;
        const double q = a[c] / piv;
        const double l = below ? q : 0.0;
        a[c] = below ? q : a[c];
#pragma unroll
        for (int cc = c + 1; cc < NB; cc++) a[cc] = fma(-l, readlane_f64(a[cc], c), a[cc]);
    }
}

// Store a factored diagonal block held as rows (lane r, a[0..63]) to D and to
// the side buffer the next triangular solves read with scalar loads: F row-major
// (U rows) and F + NB*NB column-major (L columns).
__device__ __forceinline__ void store_factored(const double (&a)[NB], int r, double* __restrict__ A, int64_t ld,
                                               double* __restrict__ F) {
#pragma unroll
    for (int c = 0; c < NB; c++) {
        A[r + (int64_t)c * ld] = a[c];
        F[r * NB + c] = a[c];
        F[NB * NB + c * NB + r] = a[c];
    }
}

// LU of the first 64 x 64 diagonal block in place, one wave.
__global__ __launch_bounds__(64) void k_dense_diag(double* __restrict__ D, int64_t ld, double* __restrict__ F) {
    const int r = threadIdx.x;
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; c++) a[c] = D[r + (int64_t)c * ld];
    wave_lu(a, r);
    store_factored(a, r, D, ld, F);
}

// Block rows of L21 = A21 U11^-1 (blockIdx < nrb) and block columns of
// U12 = L11^-1 A12 (blockIdx >= nrb) for the panel at kb, one wave each.  The
// wave holds the factored diagonal block too, lane c owning row c of U11 (for
// L21) or column c of L11 (for U12), read from the side buffer F, and
// broadcasts the entry each step needs with v_readlane.
// L21: lane r owns one row of the block and runs forward over the columns of
// U11.  U12: lane j owns one column (staged through LDS so the global
// accesses stay coalesced) and runs down the rows of L11.
__global__ __launch_bounds__(64) void k_dense_trsm(double* __restrict__ D, int64_t ld, int32_t kb, int32_t nrb,
                                                   const double* __restrict__ F) {
    __shared__ double T[NB * SLD];  // U12 staging: T[j * SLD + r] = A12(r, j)
    const int lane = threadIdx.x;
    double x[NB], f[NB];
    if ((int32_t)blockIdx.x < nrb) {
#pragma unroll
        for (int c = 0; c < NB; c++) f[c] = F[lane * NB + c];  // row lane of U11
        double* A21 = D + (kb + NB + (int64_t)blockIdx.x * NB + lane) + (int64_t)kb * ld;
#pragma unroll
        for (int c = 0; c < NB; c++) x[c] = A21[(int64_t)c * ld];
#pragma unroll
        for (int c = 0; c < NB; c++) {
            x[c] = x[c] / readlane_f64(f[c], c);
#pragma unroll
            for (int cc = c + 1; cc < NB; cc++) x[cc] = fma(-x[c], readlane_f64(f[cc], c), x[cc]);
        }
#pragma unroll
        for (int c = 0; c < NB; c++) A21[(int64_t)c * ld] = x[c];
    } else {
#pragma unroll
        for (int r = 0; r < NB; r++) f[r] = F[NB * NB + lane * NB + r];  // column lane of L11
        double* A12 = D + kb + (kb + NB + (int64_t)((int32_t)blockIdx.x - nrb) * NB) * ld;
        for (int j = 0; j < NB; j++) T[j * SLD + lane] = A12[lane + (int64_t)j * ld];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NB; r++) x[r] = T[lane * SLD + r];
#pragma unroll
        for (int c = 0; c < NB; c++) {
#pragma unroll
            for (int r = c + 1; r < NB; r++) x[r] = fma(-readlane_f64(f[r], c), x[c], x[r]);
        }
#pragma unroll
        for (int r = 0; r < NB; r++) T[lane * SLD + r] = x[r];
        __syncthreads();
        for (int j = 0; j < NB; j++) A12[lane + (int64_t)j * ld] = T[j * SLD + lane];
    }
}

// A22 -= L21 U12 over 64x64 output tiles; 4 waves, each a 32x32 quadrant of
// 2x2 MFMA tiles.  v_mfma_f64_16x16x4f64 takes lane l's first operand as
// P[l%16][l/16] and second as Q[l/16][l%16] and returns D[l/16 + 4v][l%16] in
// accumulator v (layout measured on gfx950).  P is U12 (16 columns x 4 k) and
// Q is L21 (4 k x 16 rows), so for each v the 16 lanes of a quarter-wave hold
// 16 consecutive rows of one column and the read-modify-write of A22 is
// coalesced.
__global__ __launch_bounds__(256) void k_dense_gemm(double* __restrict__ D, int64_t ld, int32_t m, int32_t kb,
                                                    int32_t b, int32_t ntile, double* __restrict__ F) {
    __shared__ double As[NB * ALD];  // As[k * ALD + r] = L21(r0 + r, k)
    __shared__ double Bs[NB * BLD];  // Bs[c * BLD + k] = U12(k, c0 + c)
    const int tid = threadIdx.x;
    const int32_t base = kb + b;
    const int32_t tr = blockIdx.x % ntile, tc = blockIdx.x / ntile;
    const int32_t r0 = base + tr * 64, c0 = base + tc * 64;
    const int kpad = (b + 3) & ~3;
    for (int e = tid; e < 64 * kpad; e += 256) {
        int r = e & 63, k = e >> 6;
        As[k * ALD + r] = (k < b && r0 + r < m) ? D[(r0 + r) + (int64_t)(kb + k) * ld] : 0.0;
    }
    for (int e = tid; e < 64 * kpad; e += 256) {
        int k = e % kpad, c = e / kpad;
        Bs[c * BLD + k] = (k < b && c0 + c < m) ? D[(kb + k) + (int64_t)(c0 + c) * ld] : 0.0;
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int i = lane & 15, kq = lane >> 4;
    v4d acc[2][2];
    for (int x = 0; x < 2; x++)
        for (int y = 0; y < 2; y++) acc[x][y] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int k4 = 0; k4 < kpad; k4 += 4) {
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
    if (blockIdx.x == 0) {
        // Tile (0, 0) is the next panel's diagonal block: finish its update in
        // LDS and factor it here (one wave), so the next panel starts with its
        // triangular solves.
        __syncthreads();  // every wave is done with As / Bs
        double* Tt = As;  // Tt[r * SLD + c], local row r and column c of the tile
#pragma unroll
        for (int sc = 0; sc < 2; sc++)
#pragma unroll
            for (int sr = 0; sr < 2; sr++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int rr = wr * 32 + sr * 16 + i, cc = wc * 32 + sc * 16 + kq + 4 * v;
                    const double x = (r0 + rr < m && c0 + cc < m) ? D[(r0 + rr) + (int64_t)(c0 + cc) * ld] : 0.0;
                    Tt[rr * SLD + cc] = x - acc[sc][sr][v];
                }
        __syncthreads();
        if (w == 0) {
            double a[NB];
#pragma unroll
            for (int c = 0; c < NB; c++) a[c] = Tt[lane * SLD + c];
            wave_lu(a, lane);
            store_factored(a, lane, D + base + (int64_t)base * ld, ld, F);
        }
        return;
    }
    // epilogue: all 16 loads of the C tile first, then the subtractions, then
    // all stores (the loads would otherwise wait for the preceding stores);
    // interior tiles skip the bounds checks
    double cv[2][2][4];
    const bool full = (r0 + 64 <= m) && (c0 + 64 <= m);
    if (full) {
#pragma unroll
        for (int sc = 0; sc < 2; sc++)
#pragma unroll
            for (int sr = 0; sr < 2; sr++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    cv[sc][sr][v] = D[(r0 + wr * 32 + sr * 16 + i) + (int64_t)(c0 + wc * 32 + sc * 16 + kq + 4 * v) * ld];
#pragma unroll
        for (int sc = 0; sc < 2; sc++)
#pragma unroll
            for (int sr = 0; sr < 2; sr++)
#pragma unroll
                for (int v = 0; v < 4; v++)
                    D[(r0 + wr * 32 + sr * 16 + i) + (int64_t)(c0 + wc * 32 + sc * 16 + kq + 4 * v) * ld] =
                        cv[sc][sr][v] - acc[sc][sr][v];
        return;
    }
#pragma unroll
    for (int sc = 0; sc < 2; sc++)
#pragma unroll
        for (int sr = 0; sr < 2; sr++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int32_t row = r0 + wr * 32 + sr * 16 + i;
                const int32_t col = c0 + wc * 32 + sc * 16 + kq + 4 * v;
                cv[sc][sr][v] = (row < m && col < m) ? D[row + (int64_t)col * ld] : 0.0;
            }
#pragma unroll
    for (int sc = 0; sc < 2; sc++)
#pragma unroll
        for (int sr = 0; sr < 2; sr++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int32_t row = r0 + wr * 32 + sr * 16 + i;
                const int32_t col = c0 + wc * 32 + sc * 16 + kq + 4 * v;
                if (row < m && col < m) D[row + (int64_t)col * ld] = cv[sc][sr][v] - acc[sc][sr][v];
            }
}

// ---------------------------------------------------------------- dense solves

// Bounded wait for a block flag.  Every wait ends: after kSpinLimit polls, or
// as soon as another block has reported a failed wait, the block gives up and
// flags the error (the solve then returns an error instead of hanging).
constexpr int kSpinLimit = 1 << 20;

__device__ __forceinline__ bool wait_flag(int32_t* flag, int32_t epoch, int32_t* err) {
    int it = 0;
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        if (++it > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            atomicOr(err, 2);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Forward substitution on the dense tail (unit lower triangle of D), rows in
// 64-row blocks taken in ticket order; block b first subtracts the finished
// blocks to its left (waiting on each one's flag), then solves its diagonal
// block in one wave and publishes.  y: tail part of the work vector(s).
__global__ __launch_bounds__(256) void k_dense_fwd(const double* __restrict__ D, int64_t ld, int32_t m,
                                                   double* __restrict__ y, int64_t ldy, int32_t nrhs,
                                                   int32_t* ticket, int32_t* flags, int32_t epoch, int32_t* err) {
    __shared__ int32_t sblk;
    __shared__ double part[4][64];
    __shared__ double Ld[64 * 65];  // diagonal block, column-major, padded
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    if (tid == 0) sblk = atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t blk = sblk;
    const int32_t r0 = blk * 64;
    const int32_t nr = min(64, m - r0);
    const int32_t row = r0 + lane;
    // the diagonal block does not depend on other blocks: load it before waiting
    for (int e = tid; e < nr * nr; e += 256) {
        const int rr = e % nr, cc = e / nr;
        Ld[cc * 65 + rr] = D[(r0 + rr) + (int64_t)(r0 + cc) * ld];
    }
    for (int32_t r = 0; r < nrhs; r++) {
        double* yr = y + (int64_t)r * ldy;
        double acc = 0.0;
        for (int32_t cb = 0; cb < blk; cb++) {
            if (r == 0) {
                if (tid == 0) wait_flag(&flags[cb], epoch, err);
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            if (lane < nr)
                for (int c = cb * 64 + q; c < cb * 64 + 64; c += 4) acc += D[row + (int64_t)c * ld] * yr[c];
        }
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0) {
            double x = lane < nr ? yr[row] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]) : 0.0;
            for (int c = 0; c < nr; c++) {
                const double xc = __shfl(x, c, 64);
                if (lane > c && lane < nr) x -= Ld[c * 65 + lane] * xc;
            }
            if (lane < nr) yr[row] = x;
        }
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&flags[blk], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Backward substitution on the dense tail (upper triangle of D with its
// diagonal), blocks from the last one up.
__global__ __launch_bounds__(256) void k_dense_bwd(const double* __restrict__ D, int64_t ld, int32_t m,
                                                   double* __restrict__ y, int64_t ldy, int32_t nrhs,
                                                   int32_t* ticket, int32_t* flags, int32_t epoch, int32_t* err) {
    __shared__ int32_t sblk;
    __shared__ double part[4][64];
    __shared__ double Ud[64 * 65];  // diagonal block, column-major, padded
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const int32_t nblk = (m + 63) / 64;
    if (tid == 0) sblk = nblk - 1 - atomicAdd(ticket, 1);
    __syncthreads();
    const int32_t blk = sblk;
    const int32_t r0 = blk * 64;
    const int32_t nr = min(64, m - r0);
    const int32_t row = r0 + lane;
    for (int e = tid; e < nr * nr; e += 256) {
        const int rr = e % nr, cc = e / nr;
        Ud[cc * 65 + rr] = D[(r0 + rr) + (int64_t)(r0 + cc) * ld];
    }
    for (int32_t r = 0; r < nrhs; r++) {
        double* yr = y + (int64_t)r * ldy;
        double acc = 0.0;
        for (int32_t cb = nblk - 1; cb > blk; cb--) {
            if (r == 0) {
                if (tid == 0) wait_flag(&flags[cb], epoch, err);
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            const int32_t cend = min(cb * 64 + 64, m);
            if (lane < nr)
                for (int c = cb * 64 + q; c < cend; c += 4) acc += D[row + (int64_t)c * ld] * yr[c];
        }
        part[q][lane] = acc;
        __syncthreads();
        if (q == 0) {
            double x = lane < nr ? yr[row] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]) : 0.0;
            for (int c = nr - 1; c >= 0; c--) {
                if (lane == c) x = x / Ud[c * 65 + c];
                const double xc = __shfl(x, c, 64);
                if (lane < c) x -= Ud[c * 65 + lane] * xc;
            }
            if (lane < nr) yr[row] = x;
        }
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&flags[blk], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Tail rows of the forward solve: y(i) -= sum_{j < t} L(i,j) y(j), one wave per row.
__global__ __launch_bounds__(256) void k_tail_cross_fwd(const SolveArgs sa, int32_t t, int32_t m,
                                                        const int64_t* __restrict__ tail_lsplit) {
    const int lane = threadIdx.x & 63;
    const int32_t c = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (c >= m) return;
    const int32_t i = t + c;
    const int64_t q0 = sa.lrow_ptr[i], q1 = tail_lsplit[c];
    for (int32_t r = 0; r < sa.nrhs; r++) {
        const double* yr = sa.y + (int64_t)r * sa.n;
        double acc = 0.0;
        for (int64_t q = q0 + lane; q < q1; q += 64) acc += sa.val[sa.lrow_pos[q]] * yr[sa.lrow_col[q]];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) sa.y[(int64_t)r * sa.n + i] -= acc;
    }
}

__global__ void k_reset_i32(int32_t* p, int32_t n, int32_t v) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_tail_gather(const FactorArgs& a, const int64_t* tail_pos, int32_t t, int32_t m, int32_t M,
                              double* D, int64_t ld, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_tail_gather<<<M, 256, 0, st>>>(a.colptr, a.rowind, a.val, tail_pos, t, m, M, D, ld);
    return hipGetLastError();
}

hipError_t launch_tail_scatter(const FactorArgs& a, const int64_t* tail_pos, int32_t t, int32_t m,
                               const double* D, int64_t ld, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_tail_scatter<<<m, 256, 0, st>>>(a.colptr, a.rowind, a.val, tail_pos, t, m, D, ld);
    return hipGetLastError();
}

hipError_t launch_dense_lu(double* D, int64_t ld, int32_t M, double* F, hipStream_t st) {
    if (M <= 0) return hipSuccess;
    if (M % NB != 0) return hipErrorInvalidValue;
    // the first diagonal block; every later one is factored by the previous
    // panel's trailing update (its tile (0, 0))
    k_dense_diag<<<1, 64, 0, st>>>(D, ld, F);
    for (int32_t kb = 0; kb + NB < M; kb += NB) {
        const int32_t nblk = (M - kb - NB) / NB;
        k_dense_trsm<<<2 * nblk, 64, 0, st>>>(D, ld, kb, nblk, F);
        k_dense_gemm<<<nblk * nblk, 256, 0, st>>>(D, ld, M, kb, NB, nblk, F);
    }
    return hipGetLastError();
}

hipError_t launch_tail_cross_fwd(const SolveArgs& sa, int32_t t, int32_t m, const int64_t* tail_lsplit,
                                 hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_tail_cross_fwd<<<(unsigned)((m + 3) / 4), 256, 0, st>>>(sa, t, m, tail_lsplit);
    return hipGetLastError();
}

hipError_t launch_dense_trsv(const double* D, int64_t ld, int32_t m, double* y, int64_t ldy, int32_t nrhs,
                             bool upper, int32_t* sync, int32_t epoch, int32_t* err, hipStream_t st) {
    if (m <= 0 || nrhs <= 0) return hipSuccess;
    const int32_t nblk = (m + 63) / 64;
    // sync[0] = ticket counter, sync[1..nblk] = per-block flags (epoch-stamped)
    k_reset_i32<<<1, 64, 0, st>>>(sync, 1, 0);
    if (upper)
        k_dense_bwd<<<nblk, 256, 0, st>>>(D, ld, m, y, ldy, nrhs, sync, sync + 1, epoch, err);
    else
        k_dense_fwd<<<nblk, 256, 0, st>>>(D, ld, m, y, ldy, nrhs, sync, sync + 1, epoch, err);
    return hipGetLastError();
}

}  // namespace glu
