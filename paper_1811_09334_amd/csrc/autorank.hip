// Kernels of auto-rank (fixed-accuracy) RQLP (Section 6): the error indicator
// ||E||_F^2 = ||A||_F^2 - ||B||_F^2 (the identity (fixedrank) of Section 2)
// after every block of B, and the first block where it reaches the tolerance.
// B comes from the blocked range finder over all lmax columns; its leading
// block rows are those the block-by-block loop would have produced (the
// triangular block orthonormalisation keeps every prefix of blocks), so the
// indicator of each prefix is a prefix sum of the blocks' ||B_j||_F^2.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {
namespace {

constexpr int AR_T = 256;

// ||A||_F^2 partials: workgroup g sums the columns g, g + G, ... (FP64 sums)
template <typename T>
__global__ __launch_bounds__(AR_T) void frob2_kernel(int64_t m, int64_t n, const T* __restrict__ A, int64_t lda,
                                                     double* __restrict__ part) {
    __shared__ double s_red[AR_T / 64];
    double s = 0.0;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        const T* a = A + j * lda;
        for (int64_t i = threadIdx.x; i < m; i += AR_T) {
            const double v = (double)a[i];
            s += v * v;
        }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// ||B_j||_F^2 partials of the block rows of B (l x n, ldb): thread = column,
// workgroup g writes part[g * nblk + j] for every block j
__global__ __launch_bounds__(AR_T) void block_rownorm_kernel(int64_t l, int64_t n, const double* __restrict__ B,
                                                             int64_t ldb, int64_t bs, int nblk,
                                                             double* __restrict__ part) {
    __shared__ double s_red[AR_T / 64];
    const int64_t c = (int64_t)blockIdx.x * AR_T + threadIdx.x;
    const double* col = B + c * ldb;
    for (int j = 0; j < nblk; ++j) {
        const int64_t r0 = (int64_t)j * bs, r1 = (r0 + bs < l) ? r0 + bs : l;
        double s = 0.0;
        if (c < n)
            for (int64_t r = r0; r < r1; ++r) s += col[r] * col[r];
        s = wave_sum(s);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nblk + j] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

// One workgroup: ||A||_F^2 and the ||B_j||_F^2 from their partials (fixed
// order), then the first block J (1-based) with ||A||^2 - sum_{i <= J} ||B_i||^2
// <= eps, or nblk when none; out = {J, ||E||_F^2 at J, ||A||_F^2}.
__global__ __launch_bounds__(AR_T) void autorank_decide_kernel(const double* __restrict__ apart, int na,
                                                               const double* __restrict__ bpart, int nb_wg,
                                                               int nblk, double eps, double* __restrict__ bnorm,
                                                               double* __restrict__ out) {
    for (int j = threadIdx.x; j < nblk; j += AR_T) {
        double s = 0.0;
        for (int g = 0; g < nb_wg; ++g) s += bpart[(int64_t)g * nblk + j];
        bnorm[j] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a2 = 0.0;
        for (int g = 0; g < na; ++g) a2 += apart[g];
        double b2 = 0.0, e2 = a2;
        int J = nblk;
        for (int j = 0; j < nblk; ++j) {
            b2 += bnorm[j];
            e2 = a2 - b2;
            if (e2 <= eps) {
                J = j + 1;
                break;
            }
        }
        out[0] = (double)J;
        out[1] = e2;
        out[2] = a2;
    }
}

template <typename T>
__global__ void fill_cols_kernel(int64_t rows, int64_t c0, int64_t c1, T* __restrict__ X, int64_t ldx) {
    const int64_t total = rows * (c1 - c0);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        X[t % rows + (c0 + t / rows) * ldx] = (T)0;
}

__global__ void or_flag_kernel(int32_t* info, int32_t bit) { atomicOr(info, bit); }

__global__ void fill_i64_kernel(int64_t n, int64_t* __restrict__ p, int64_t v) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

inline dim3 grid_of(int64_t total) {
    int64_t b = ceil_div(total, 256);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

}  // namespace

size_t autorank_scratch_doubles(int64_t n, int64_t l, int64_t bs) {
    const int64_t nblk = ceil_div(l, bs > 0 ? bs : l);
    return (size_t)AR_FROB_PARTS + (size_t)ceil_div(n, AR_T) * nblk + (size_t)nblk + 4;
}

template <typename T>
int autorank_indicator(const T* A, int64_t lda, int64_t m, int64_t n, const double* B, int64_t ldb, int64_t l,
                       int64_t bs, double eps, double* scratch, double* out3, hipStream_t s) {
    const int64_t bsz = bs > 0 ? bs : l;
    const int nblk = (int)ceil_div(l, bsz);
    const int nbw = (int)ceil_div(n, AR_T);
    const int na = (int)(n < AR_FROB_PARTS ? n : AR_FROB_PARTS);
    double* apart = scratch;
    double* bpart = apart + AR_FROB_PARTS;
    double* bnorm = bpart + (size_t)nbw * nblk;
    hipLaunchKernelGGL(frob2_kernel<T>, dim3((unsigned)na), dim3(AR_T), 0, s, m, n, A, lda, apart);
    hipLaunchKernelGGL(block_rownorm_kernel, dim3((unsigned)nbw), dim3(AR_T), 0, s, l, n, B, ldb, bsz, nblk, bpart);
    hipLaunchKernelGGL(autorank_decide_kernel, dim3(1), dim3(AR_T), 0, s, apart, na, bpart, nbw, nblk, eps, bnorm,
                       out3);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template int autorank_indicator<double>(const double*, int64_t, int64_t, int64_t, const double*, int64_t, int64_t,
                                        int64_t, double, double*, double*, hipStream_t);
template int autorank_indicator<float>(const float*, int64_t, int64_t, int64_t, const double*, int64_t, int64_t,
                                       int64_t, double, double*, double*, hipStream_t);

template <typename T>
int zero_cols(int64_t rows, int64_t c0, int64_t c1, T* X, int64_t ldx, hipStream_t s) {
    if (rows <= 0 || c1 <= c0) return 0;
    hipLaunchKernelGGL(fill_cols_kernel<T>, grid_of(rows * (c1 - c0)), dim3(256), 0, s, rows, c0, c1, X, ldx);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}
template int zero_cols<double>(int64_t, int64_t, int64_t, double*, int64_t, hipStream_t);
template int zero_cols<float>(int64_t, int64_t, int64_t, float*, int64_t, hipStream_t);

int set_info_flag(int32_t* info, int32_t bit, hipStream_t s) {
    hipLaunchKernelGGL(or_flag_kernel, dim3(1), dim3(1), 0, s, info, bit);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

int fill_i64(int64_t n, int64_t* p, int64_t v, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_i64_kernel, grid_of(n), dim3(256), 0, s, n, p, v);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

}  // namespace rqlp
