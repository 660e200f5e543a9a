// Mailboxes: results handed from one wave to others of the same launch
// through a buffer filled beforehand with a sentinel, written with relaxed
// agent-scope atomic stores and read with relaxed agent-scope atomic loads,
// polled until the value read is not the sentinel.  Each value publishes
// itself, so no fence is needed (an agent-scope release writes back the whole
// L2 of the XCD).  The sentinel is a signalling NaN whose payload carries a
// tag unique to the call; arithmetic only ever produces quiet NaNs.  Every
// wait is bounded: after kMailSpinLimit polls, or as soon as another wave has
// reported a failed wait, the wave gives up and sets bit 2 of err.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace glu {

constexpr int kMailSpinLimit = 1 << 20;

__host__ __device__ inline uint64_t mail_sentinel(uint64_t tag) {
    return 0x7FF4000000000000ull | (tag & 0x0003FFFFFFFFFFFFull);
}

__device__ __forceinline__ void mail_put(double* mail, int64_t i, double x) {
    __hip_atomic_store(reinterpret_cast<uint64_t*>(mail) + i, (uint64_t)__double_as_longlong(x), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t mail_load(const double* mail, int64_t i) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t*>(mail) + i, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// N mailbox values mail[idx[i]] (entries with use[i] false read as 0) once
// none is the sentinel: all are loaded together, then the pending ones are
// reloaded together until none is left.
template <int N>
__device__ __forceinline__ void mail_read(const double* mail, const int64_t (&idx)[N], const bool (&use)[N],
                                          uint64_t sentinel, double (&v)[N], int32_t* err) {
    uint64_t bits[N];
#pragma unroll
    for (int i = 0; i < N; i++) bits[i] = use[i] ? mail_load(mail, idx[i]) : 0ull;
    for (int it = 0;;) {
        bool ok = true;
#pragma unroll
        for (int i = 0; i < N; i++) ok &= bits[i] != sentinel;
        if (ok) break;
        if (++it > kMailSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            atomicOr(err, 2);
#pragma unroll
            for (int i = 0; i < N; i++) bits[i] = 0ull;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int i = 0; i < N; i++)
            if (bits[i] == sentinel) bits[i] = mail_load(mail, idx[i]);
    }
#pragma unroll
    for (int i = 0; i < N; i++) v[i] = __longlong_as_double((long long)bits[i]);
}

}  // namespace glu
