// Small utility kernels: fills, copies, transposes, the L-value extraction,
// and the Gaussian test matrix (Section 2, range finder step 1).
#include <hip/hip_fp16.h>
#include <math.h>

#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_cache_mu;      // guards every per-device cache of this file
struct FnEntry {
    int device;
    const void* fn;
    int block;
    size_t lds;
    int value;
};
// never destroyed: nothing of this library runs code at process exit
std::vector<FnEntry>& fn_cache() {
    static std::vector<FnEntry>* v = new std::vector<FnEntry>();
    return *v;
}
}  // namespace

// Device properties, queried once per device (the current device of the
// calling thread); entries are written once under the lock and never change.
const DeviceInfo& device_info() {
    static DeviceInfo table[kMaxDevices];
    static const DeviceInfo none;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return none;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    DeviceInfo& di = table[dev];
    if (di.device != dev) {
        DeviceInfo n;
        n.device = dev;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) n.num_cus = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            n.max_lds = (size_t)v;
        // leave room for the kernels' static LDS
        n.max_lds = n.max_lds > 2048 ? n.max_lds - 2048 : n.max_lds;
        di = n;
    }
    return di;
}

int raise_lds_limit(const void* fn, int bytes) {
    int dev = 0;
    RQLP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (const FnEntry& e : fn_cache())
        if (e.device == dev && e.fn == fn && e.block == -1) return 0;
    RQLP_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    fn_cache().push_back(FnEntry{dev, fn, -1, (size_t)bytes, 0});
    return 0;
}

int resident_capacity(const void* fn, int block, size_t lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const int cus = device_info().num_cus;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (const FnEntry& e : fn_cache())
        if (e.device == dev && e.fn == fn && e.block == block && e.lds == lds) return e.value;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess) nb = 0;
    const int cap = nb * (cus > 0 ? cus : 0);
    fn_cache().push_back(FnEntry{dev, fn, block, lds, cap});
    return cap;
}

__global__ void fill_zero_kernel(uint32_t* p, size_t words) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

int fill_zero_bytes(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return 0;
    const size_t words = (bytes + 3) / 4;   // callers pass 4-byte multiples (Arena pieces are padded)
    unsigned blocks = (unsigned)((words + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

__global__ void copy_matrix_kernel(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y,
                                   int64_t ldy) {
    const int64_t n = rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % rows, j = idx / rows;
        Y[i + j * ldy] = X[i + j * ldx];
    }
}

int copy_matrix(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y, int64_t ldy,
                hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    int64_t blocks = ceil_div(rows * cols, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_matrix_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rows, cols, X, ldx, Y, ldy);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

__global__ void transpose_kernel(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y,
                                 int64_t ldy, int tri) {
    __shared__ double t[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        t[jj][tx] = (i < rows && j < cols) ? X[i + j * ldx] : 0.0;
    }
    __syncthreads();
    // Y(j, i) = X(i, j)
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < rows && j < cols) {
            double v = t[tx][ii];
            if (tri == 'L' && i > j) v = 0.0;      // Y(j, i) with j < i is above the diagonal
            if (tri == 'U' && i < j) v = 0.0;
            Y[j + i * ldy] = v;
        }
    }
}

int transpose_matrix(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     int tri, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    dim3 grid((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(cols, 32));
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, rows, cols, X, ldx, Y, ldy, tri);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

__global__ void set_identity_kernel(int64_t n, double* Y, int64_t ldy) {
    const int64_t total = n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        Y[i + j * ldy] = (i == j) ? 1.0 : 0.0;
    }
}

int set_identity(int64_t n, double* Y, int64_t ldy, hipStream_t s) {
    if (n <= 0) return 0;
    int64_t blocks = ceil_div(n * n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(set_identity_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, Y, ldy);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

__global__ void finish_lvals_kernel(int64_t l, const double* T, int64_t ldt, double* lvals, int32_t* info) {
    // one wave per column: lvals = diag(T), any NaN / Inf in T flagged
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= l) return;
    int bad = 0;
    for (int64_t i = lane; i < l; i += 64) {
        const double x = T[i + j * ldt];
        if (!(x == x) || x > 1.7e308 || x < -1.7e308) bad = 1;
    }
    if (lane == 0 && lvals) lvals[j] = T[j + j * ldt];
    if (__any(bad) && lane == 0 && info) atomicOr(info, RQLP_INFO_NONFINITE);
}

int finish_lvals(int64_t l, const double* T, int64_t ldt, double* lvals, int32_t* info, hipStream_t s) {
    if (l <= 0) return 0;
    hipLaunchKernelGGL(finish_lvals_kernel, dim3((unsigned)ceil_div(l, 4)), dim3(256), 0, s, l, T, ldt, lvals, info);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

__global__ void copy_i64_kernel(int64_t n, const int64_t* src, int64_t* dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] : i;
}

int copy_i64(int64_t n, const int64_t* src, int64_t* dst, hipStream_t s) {
    if (n <= 0 || dst == nullptr) return 0;
    hipLaunchKernelGGL(copy_i64_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (philox4x32_10, common.hpp) + Box-Muller (1958).
// Element (i, j): counter (i, j, 0, 0), key (lo32(seed), hi32(seed)).
__device__ __forceinline__ float round_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(b);
}

__global__ void omega_kernel(int64_t n, int64_t l, uint32_t k0, uint32_t k1, int precision, void* Omega,
                             int64_t ldo) {
    const int64_t total = n * l;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n, j = idx / n;
        uint32_t c[4] = {(uint32_t)i, (uint32_t)j, 0u, 0u};
        philox4x32_10(c, k0, k1);
        const double u1 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;
        const double u2 = (double)c[1] * 2.3283064365386963e-10;
        const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        if (precision == RQLP_F64) {
            ((double*)Omega)[i + j * ldo] = g;
        } else {
            float f = (float)g;
            if (precision == RQLP_MIXED_BF16 || precision == RQLP_MIXED_BF16X3) f = round_bf16(f);
            else if (precision == RQLP_MIXED_FP16) f = (float)(__half)f;
            ((float*)Omega)[i + j * ldo] = f;
        }
    }
}

int generate_omega(int64_t n, int64_t l, uint64_t seed, int precision, void* Omega, int64_t ldo,
                   hipStream_t s) {
    if (n <= 0 || l <= 0) return 0;
    int64_t blocks = ceil_div(n * l, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(omega_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, l, (uint32_t)(seed & 0xFFFFFFFFu),
                       (uint32_t)(seed >> 32), precision, Omega, ldo);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}


// Orthonormal completion of a basis whose input columns were numerically zero
// (exactly zero columns of R0^T after a rank stop of the first CPQR, or a
// sketch of a zero matrix): after a shifted CholeskyQR pass such a column is
// still (close to) zero and no later pass can normalise it, so it is replaced
// by a Gaussian vector, which the following passes orthonormalise against the
// earlier columns.  Zeroing L(j, j) of the pass's factor keeps X_in = X L^T
// exact for a zero input column (its row and column of L are zero apart from
// the diagonal), so the triangular factor R of the whole CholeskyQR gets a zero
// row j.  One workgroup per column.
__global__ __launch_bounds__(256) void complete_columns_kernel(int64_t rows, int64_t c, double* X, int64_t ldx,
                                                               double* L, int64_t ldl, double tau2,
                                                               const int32_t* gate, int64_t col0) {
    if (*gate == 0) return;
    __shared__ double s_red[4];
    const int64_t j = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* x = X + j * ldx;
    double ss = 0.0;
    for (int64_t i = tid; i < rows; i += 256) ss += x[i] * x[i];
    ss = wave_sum(ss);
    if (lane == 0) s_red[wave] = ss;
    __syncthreads();
    const double nrm2 = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    if (!(nrm2 <= tau2)) return;                      // also keeps NaN columns as they are
    const double scale = 1.0 / sqrt((double)rows);
    for (int64_t i = tid; i < rows; i += 256) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(col0 + j), 1u, 0u};
        philox4x32_10(ctr, 0x5EED1234u, 0x0C0FFEE5u);
        const double u1 = ((double)ctr[0] + 1.0) * 2.3283064365386963e-10;
        const double u2 = (double)ctr[1] * 2.3283064365386963e-10;
        x[i] = scale * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
    if (L && tid == 0) L[j + j * ldl] = 0.0;
}

int complete_columns(int64_t rows, int64_t c, double* X, int64_t ldx, double* L, int64_t ldl, double tau2,
                     const int32_t* gate, hipStream_t s, int64_t col0) {
    if (rows <= 0 || c <= 0) return 0;
    hipLaunchKernelGGL(complete_columns_kernel, dim3((unsigned)c), dim3(256), 0, s, rows, c, X, ldx, L, ldl, tau2,
                       gate, col0);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

}  // namespace rqlp
