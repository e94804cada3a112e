// Internal helpers shared by the gfx950 kernels of the randomized QLP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/rqlp.h"

#define RQLP_WAVE 64

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

namespace rqlp {

// ---------------------------------------------------------------------------
// host-side error plumbing
// ---------------------------------------------------------------------------
#define RQLP_HIP_TRY(expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return RQLP_E_HIP;             \
    } while (0)

// With the environment variable RQLP_TRACE set (to anything but "0"), every
// non-zero status passed up through RQLP_TRY is printed to stderr with its
// call site, so the chain from the failing call to the entry point is named.
inline bool trace_errors() {
    static const bool on = [] {
        const char* v = getenv("RQLP_TRACE");
        return v != nullptr && v[0] != '\0' && !(v[0] == '0' && v[1] == '\0');
    }();
    return on;
}

#define RQLP_TRY(expr)                                                                       \
    do {                                                                                     \
        int _s = (expr);                                                                     \
        if (_s != 0) {                                                                       \
            if (::rqlp::trace_errors())                                                      \
                fprintf(stderr, "rqlp: %s:%d: %s returned %d\n", __FILE__, __LINE__, #expr, _s); \
            return _s;                                                                       \
        }                                                                                    \
    } while (0)

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Linear carve-up of the caller's workspace (256-byte aligned pieces).
struct Arena {
    char* base;
    size_t used;
    size_t cap;
    Arena(void* b, size_t c) : base((char*)b), used(0), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        size_t bytes = align256(count * sizeof(T));
        T* p = base ? (T*)(base + used) : nullptr;
        used += bytes;
        return p;
    }
    bool ok() const { return used <= cap; }
};

// device properties cached per device (immutable after the first query, thread-safe)
struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    size_t max_lds = 0;
};
const DeviceInfo& device_info();
// Raises the dynamic LDS limit of kernel fn to `bytes` on the current device,
// once per device (thread-safe).  RQLP_E_HIP on failure.
int raise_lds_limit(const void* fn, int bytes);
// Workgroups of `block` threads with `lds` dynamic LDS bytes of kernel fn that
// the current device holds at once (occupancy x compute units), cached per
// device (thread-safe); 0 if the query fails.
int resident_capacity(const void* fn, int block, size_t lds);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, RQLP_WAVE);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, RQLP_WAVE);
    return v;
}

// 64-bit lane exchange within rows of 16 lanes by DPP (a lane whose source
// lies outside its row reads 0), and reads of one lane's 64-bit value
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}
// Maximum over the wave of a value that is already the same on the 16 lanes
// of each DPP row (all 64 lanes active): one read per row.
__device__ __forceinline__ unsigned long long rows_max_u64(unsigned long long v) {
    return umax64(umax64(readlane_u64(v, 0), readlane_u64(v, 16)), umax64(readlane_u64(v, 32), readlane_u64(v, 48)));
}
// Maximum over the wave (all 64 lanes active): DPP within rows of 16 (pairs,
// quads, half rows, rows; each level exchanges symmetric partners), then
// one read per row.  Every lane gets the result.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    v = umax64(v, dpp_u64<0xB1>(v));      // quad_perm(1, 0, 3, 2)
    v = umax64(v, dpp_u64<0x4E>(v));      // quad_perm(2, 3, 0, 1)
    v = umax64(v, dpp_u64<0x141>(v));     // row_half_mirror
    v = umax64(v, dpp_u64<0x140>(v));     // row_mirror
    return rows_max_u64(v);
}

// Order-preserving 64-bit key for a non-negative double: larger value ->
// larger key.  The low `ibits` bits carry (mask - index) so that among equal
// truncated values the smallest index wins an unsigned max.
__device__ __forceinline__ unsigned long long pivot_key(double v, unsigned idx, int ibits) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);   // v >= 0
    unsigned long long mask = (1ull << ibits) - 1ull;
    return (b & ~mask) | (mask - (unsigned long long)idx);
}
__device__ __forceinline__ unsigned key_index(unsigned long long key, int ibits) {
    unsigned long long mask = (1ull << ibits) - 1ull;
    return (unsigned)(mask - (key & mask));
}
__device__ __forceinline__ double key_value(unsigned long long key, int ibits) {
    unsigned long long mask = (1ull << ibits) - 1ull;
    return __longlong_as_double((long long)(key & ~mask));
}

// Grid-wide barrier for cooperatively launched kernels (all workgroups
// co-resident).  bar[0] counts arrivals, bar[1] is the generation.  Every
// wait is bounded: after `spin_limit` polls the barrier gives up, raises
// RQLP_INFO_BARRIER_TIMEOUT in *info and returns false; callers then leave
// the kernel, so no wave can wait forever.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned& gen,
                                             int32_t* info, unsigned long long spin_limit) {
    __shared__ int s_ok;
    // the workgroup barrier orders this workgroup's global stores before thread
    // 0's device-scope release below; thread 0's acquire plus the second
    // workgroup barrier order every thread's later loads after the other
    // workgroups' releases.
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned g = gen;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > spin_limit) {
                    ok = 0;
                    if (info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = g + 1u;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}


// Cross-workgroup exchange inside one kernel uses relaxed device-scope atomic
// loads and stores (coherent at the memory side, they bypass the per-XCD L2
// caches) plus completion waits for ordering: a workgroup's data stores are
// waited for (s_waitcnt) before it publishes a flag, and readers issue their
// loads after they observed the flag.  This avoids device-scope
// release/acquire fences, which write back and invalidate the whole L2.
__device__ __forceinline__ void st_coherent(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(const double* p) {
    return __longlong_as_double(
        (long long)__hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_coherent_u32(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_coherent_u32(const unsigned* p) {
    return __hip_atomic_load((unsigned*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// every wave waits for its outstanding memory operations, then workgroup barrier
__device__ __forceinline__ void drain_and_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4 x 32-bit counter-based generator on c with key (k0, k1).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}
// N(0, 1) by Box-Muller from the first two words of Philox4x32-10 at counter
// (c0, c1, c2, 0) with key (k0, k1).
__device__ __forceinline__ double philox_normal(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t k0, uint32_t k1) {
    uint32_t c[4] = {c0, c1, c2, 0u};
    philox4x32_10(c, k0, k1);
    const double u1 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;
    const double u2 = (double)c[1] * 2.3283064365386963e-10;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Copies from global memory straight into LDS (global_load_lds_dwordx4): the
// LDS operand is the wave's base address, lane l's 16 bytes land at base + 16 l.
#define RQLP_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))
// LDS-only barrier: the compiler's __syncthreads also waits for every
// outstanding global load (vmcnt(0)), which would drain a prefetch queue.
#define RQLP_LDS_BARRIER() asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory")

// s_waitcnt with only the vector-memory counter constrained (at most n outstanding)
template <int n>
__device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt(0x0F70 | (n & 15) | ((n >> 4) << 14));
}

}  // namespace rqlp
