// rqlp_factor without a caller workspace, for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid hipMalloc).  The workspace of rqlp_factor lives in a fixed-size
// device array of this file instead; each device the library runs on holds
// its own copy for the life of the process.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)RQLP_NOALLOC_SCRATCH_BYTES;

// The workspace: a host-side name for device memory.  Host code uses only the
// per-device address from hipGetSymbolAddress, never this name.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per device
// with that device current.
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return RQLP_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return RQLP_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return RQLP_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace

extern "C" int rqlp_factor_noalloc(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q,
                                   int d, int b, int precision, uint64_t seed, const void* Omega, int64_t ldo,
                                   void* Q, int64_t ldq, double* T, int64_t ldt, void* P, int64_t ldp,
                                   int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info, char* uplo,
                                   void* stream) {
    // argument checks of rqlp_factor (same numbering) and the workspace it needs
    RQLP_TRY(rqlp::factor_arg_status(A, lda, m, n, k, p, q, d, b, precision, Omega, ldo, Q, ldq, T, ldt, P, ldp));
    size_t need = 0;
    RQLP_TRY(rqlp_workspace_size(m, n, k, p, q, d, b, precision, &need));
    if (need > kScratchBytes) return RQLP_E_SCRATCH_LIMIT;
    void* ws = nullptr;
    RQLP_TRY(scratch_address(&ws));
    // every piece that has to start at zero (info, the CPQR key slots and
    // barrier words, Cholesky flags) is cleared by fill kernels inside the call
    return rqlp_factor(A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp, piv0, piv1,
                       lvals, info, uplo, ws, kScratchBytes, stream);
}
