// Relaxed dependency detection (Alg. 4) and levelization on the GPU.
//
// The host analysis computes both in a few passes over the filled pattern;
// for the largest patterns (10^9 entries) those passes take seconds, so the
// same two steps can run on the device instead (glu_options.gpu_analysis),
// with bit-identical results:
//  1. dependencies: column k depends on i < k when U(i,k) != 0 and L(:,i) has
//     an entry ("look up"), or when L(k,i) != 0 ("look left").  Every such
//     pair becomes the key k * 2^32 + i -- the look-up pairs from column k's
//     U part, the look-left pairs from every column i's L part (row k) -- and
//     a device radix sort followed by removal of repeats leaves, per column,
//     its dependencies ascending: the CSR the host builds by merging;
//  2. levels: level(k) = 0 without dependencies, else 1 + the largest level
//     of its dependencies.  Dependencies are smaller columns, so waves take
//     columns in increasing order from an atomic ticket and read the levels
//     they need from a sentinel-filled mailbox (relaxed agent-scope atomics,
//     as the triangular solves do): the earliest unfinished column has all
//     its inputs, so the sweep progresses whatever is resident; every wait is
//     bounded.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "analyze_gpu.hpp"

namespace glu {

namespace {

constexpr int kLevelSpinLimit = 1 << 22;

// look-up pairs of column j that count: U(r,j) != 0 with L(:,r) not empty
__global__ void k_dep_counts(int32_t n, const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowind,
                             const int64_t* __restrict__ diag, int64_t* __restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= n) return;
    int64_t c = 0;
    for (int64_t p = colptr[j] + lane; p < diag[j]; p += 64) {
        const int32_t r = rowind[p];
        c += diag[r] + 1 < colptr[r + 1] ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) cnt[j] = c + (colptr[j + 1] - diag[j] - 1);
}

// keys of column j at base[j]: its counted look-up pairs (j, r), then its L
// part as look-left pairs (i, j) of the later columns i
__global__ void k_dep_keys(int32_t n, const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowind,
                           const int64_t* __restrict__ diag, const int64_t* __restrict__ base,
                           uint64_t* __restrict__ keys) {
    const int lane = threadIdx.x & 63;
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= n) return;
    int64_t o = base[j];
    for (int64_t p0 = colptr[j]; p0 < diag[j]; p0 += 64) {
        const int64_t p = p0 + lane;
        int32_t r = 0;
        bool use = false;
        if (p < diag[j]) {
            r = rowind[p];
            use = diag[r] + 1 < colptr[r + 1];
        }
        const uint64_t m = __ballot(use);
        const int64_t rank = __popcll(m & ((1ull << lane) - 1));
        if (use) keys[o + rank] = ((uint64_t)j << 32) | (uint32_t)r;
        o += __popcll(m);
    }
    const int64_t b = diag[j] + 1, e = colptr[j + 1];
    for (int64_t p = b + lane; p < e; p += 64) keys[o + (p - b)] = ((uint64_t)(uint32_t)rowind[p] << 32) | (uint32_t)j;
}

// first key of each column k in the sorted, unique keys: ptr[k] = number of keys with high part < k
__global__ void k_row_starts(int64_t nkeys, const uint64_t* __restrict__ keys, int32_t n, int64_t* __restrict__ ptr) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > nkeys) return;
    const int64_t r1 = x < nkeys ? (int64_t)(keys[x] >> 32) : n;   // column of key x (n past the end)
    const int64_t r0 = x > 0 ? (int64_t)(keys[x - 1] >> 32) : -1;  // column of key x - 1
    for (int64_t r = r0 + 1; r <= r1; r++) ptr[r] = x;
}

__global__ void k_low_words(int64_t nkeys, const uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nkeys) idx[x] = (int32_t)(keys[x] & 0xffffffffu);
}

__global__ void k_level_sweep(int32_t n, const int64_t* __restrict__ dag_ptr, const int32_t* __restrict__ dag_idx,
                              int32_t* lev, int32_t* ticket, int32_t* err) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        int32_t k = 0;
        if (lane == 0) k = atomicAdd(ticket, 1);
        k = __shfl(k, 0, 64);
        if (k >= n) return;
        int32_t m = -1;
        for (int64_t e = dag_ptr[k] + lane; e < dag_ptr[k + 1]; e += 64) {
            const int32_t i = dag_idx[e];
            int32_t v = __hip_atomic_load(&lev[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int it = 0; v < 0; it++) {
                if (it > kLevelSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicOr(err, 1);
                    v = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                v = __hip_atomic_load(&lev[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            m = max(m, v);
        }
        for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
        if (lane == 0) __hip_atomic_store(&lev[k], m + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

template <class T>
struct DBuf {
    T* p = nullptr;
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc((void**)&p, std::max<size_t>(n, 1) * sizeof(T)); }
};

#define GLU_TRY(x)                          \
    do {                                    \
        hipError_t e_ = (x);                \
        if (e_ != hipSuccess) return e_;    \
    } while (0)

}  // namespace

hipError_t gpu_dag_levels(int32_t n, const std::vector<int64_t>& lu_colptr, const std::vector<int32_t>& lu_rowind,
                          const std::vector<int64_t>& diag, std::vector<int64_t>& dag_ptr,
                          std::vector<int32_t>& dag_idx, std::vector<int32_t>& level_of, int32_t* spin_err) {
    *spin_err = 0;
    dag_ptr.assign(1, 0);
    dag_idx.clear();
    level_of.clear();
    if (n <= 0) return hipSuccess;
    const int64_t nnz = (int64_t)lu_rowind.size();
    DBuf<int64_t> d_cp, d_diag, d_cnt, d_base, d_dptr;
    DBuf<int32_t> d_ri, d_didx, d_lev, d_sync;
    GLU_TRY(d_cp.alloc(n + 1));
    GLU_TRY(d_diag.alloc(n));
    GLU_TRY(d_ri.alloc(nnz));
    GLU_TRY(hipMemcpy(d_cp.p, lu_colptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    GLU_TRY(hipMemcpy(d_diag.p, diag.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    if (nnz) GLU_TRY(hipMemcpy(d_ri.p, lu_rowind.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    // 1. candidate pairs per column, their keys, sort, unique
    const unsigned gw = (unsigned)(((int64_t)n * 64 + 255) / 256);  // one wave per column
    GLU_TRY(d_cnt.alloc(n));
    k_dep_counts<<<gw, 256>>>(n, d_cp.p, d_ri.p, d_diag.p, d_cnt.p);
    GLU_TRY(hipGetLastError());
    std::vector<int64_t> base(n + 1, 0);
    GLU_TRY(hipMemcpy(base.data() + 1, d_cnt.p, n * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int32_t j = 0; j < n; j++) base[j + 1] += base[j];
    const int64_t nk = base[n];
    if (nk > INT32_MAX) return hipErrorInvalidValue;  // one device sort handles < 2^31 keys
    GLU_TRY(d_base.alloc(n + 1));
    GLU_TRY(hipMemcpy(d_base.p, base.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    DBuf<uint64_t> d_keys, d_sorted;
    GLU_TRY(d_keys.alloc(nk));
    GLU_TRY(d_sorted.alloc(nk));
    k_dep_keys<<<gw, 256>>>(n, d_cp.p, d_ri.p, d_diag.p, d_base.p, d_keys.p);
    GLU_TRY(hipGetLastError());
    int rb = 1;
    while (rb < 31 && (1 << rb) < n) rb++;
    const int end_bit = 32 + rb;
    int64_t ne = 0;
    {
        size_t tb_sort = 0, tb_uniq = 0;
        GLU_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tb_sort, d_keys.p, d_sorted.p, (int)nk, 0, end_bit));
        DBuf<int64_t> d_nsel;
        GLU_TRY(d_nsel.alloc(1));
        GLU_TRY(hipcub::DeviceSelect::Unique(nullptr, tb_uniq, d_sorted.p, d_keys.p, d_nsel.p, (int)nk));
        DBuf<uint8_t> tmp;
        GLU_TRY(tmp.alloc(std::max(tb_sort, tb_uniq)));
        GLU_TRY(hipcub::DeviceRadixSort::SortKeys(tmp.p, tb_sort, d_keys.p, d_sorted.p, (int)nk, 0, end_bit));
        GLU_TRY(hipcub::DeviceSelect::Unique(tmp.p, tb_uniq, d_sorted.p, d_keys.p, d_nsel.p, (int)nk));
        GLU_TRY(hipMemcpy(&ne, d_nsel.p, sizeof(int64_t), hipMemcpyDeviceToHost));
    }
    // unique keys are in d_keys[0, ne)
    GLU_TRY(d_dptr.alloc(n + 1));
    k_row_starts<<<(unsigned)((ne + 1 + 255) / 256), 256>>>(ne, d_keys.p, n, d_dptr.p);
    GLU_TRY(hipGetLastError());
    GLU_TRY(d_didx.alloc(ne));
    if (ne) k_low_words<<<(unsigned)((ne + 255) / 256), 256>>>(ne, d_keys.p, d_didx.p);
    GLU_TRY(hipGetLastError());
    // 2. levels: ticketed sweep over the columns with a mailbox of levels
    GLU_TRY(d_lev.alloc(n));
    GLU_TRY(d_sync.alloc(2));
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256>>>(d_lev.p, n, -1);
    k_fill_i32<<<1, 64>>>(d_sync.p, 2, 0);
    int dev = 0, ncu = 1;
    GLU_TRY(hipGetDevice(&dev));
    GLU_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    k_level_sweep<<<(unsigned)(2 * ncu), 256>>>(n, d_dptr.p, d_didx.p, d_lev.p, d_sync.p, d_sync.p + 1);
    GLU_TRY(hipGetLastError());
    dag_ptr.resize(n + 1);
    dag_idx.resize(ne);
    level_of.resize(n);
    GLU_TRY(hipMemcpy(dag_ptr.data(), d_dptr.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (ne) GLU_TRY(hipMemcpy(dag_idx.data(), d_didx.p, ne * sizeof(int32_t), hipMemcpyDeviceToHost));
    GLU_TRY(hipMemcpy(level_of.data(), d_lev.p, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    GLU_TRY(hipMemcpy(spin_err, d_sync.p + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
    return hipDeviceSynchronize();
}

}  // namespace glu
