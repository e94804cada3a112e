// Cholesky factor and its inverse for CholeskyQR (the "[V, ~] = qr(Y)" step of
// the range finder, Algorithm 2.1 step 3, and the inner QR steps of
// Algorithm 2.2, realised as CholeskyQR2: Fukaya, Nakatsukasa, Yanagisawa,
// Yamamoto 2014; shifted retry per Fukaya, Kannan, Nakatsukasa, Zhang,
// Yamamoto 2020).
//
// One workgroup of 512 threads factors the c x c Gram matrix G = L L^T with a
// right-looking blocked algorithm (32-column blocks) and, fused into the same
// sweep, solves L X = I for X = L^{-1} (right-looking block forward
// substitution sharing the panel).  The 32 x 32 diagonal blocks are factored
// by one wave in registers (lane i holds row i, columns broadcast by
// shuffles).  The current panel L(J0:c, K0:K0+32) and block row X(K0:K0+32,
// 0:J0) are cached in LDS (up to 256 rows / columns, the rest is read from
// the L2-resident scratch copies), and the trailing updates run as 4 x 4
// register tiles.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

constexpr int CH_NB = 32;
constexpr int CH_T = 512;
constexpr int CH_PMAX = 256;
constexpr int CH_XMAX = 256;
constexpr int CH_PS = CH_NB + 1;

static inline int ch_prows(int64_t c) { return (int)(c < CH_PMAX ? c : CH_PMAX); }
static inline int ch_xcols(int64_t c) { return (int)(c < CH_XMAX ? c : CH_XMAX); }

size_t chol_inv_lds_bytes(int64_t c) {
    return sizeof(double) * (size_t)(2 * CH_NB * CH_PS + ch_prows(c) * CH_PS + CH_NB * (ch_xcols(c) + 1));
}

__global__ __launch_bounds__(CH_T) void chol_inv_kernel(int c, const double* __restrict__ G, int64_t ldg,
                                                        double* __restrict__ R, int64_t ldr,
                                                        double* __restrict__ Rinv, int64_t ldri,
                                                        double shift_scale, double* __restrict__ W,
                                                        double* __restrict__ X, int64_t ldw, int32_t* info,
                                                        int prows, int xcols) {
    extern __shared__ double lds[];
    double* D = lds;                           // [32][33]
    double* Dinv = D + CH_NB * CH_PS;          // [32][33]
    double* P = Dinv + CH_NB * CH_PS;          // [prows][33]
    double* XK = P + (size_t)prows * CH_PS;    // [32][xcols + 1]
    const int xs = xcols + 1;
    __shared__ int s_bad;
    __shared__ double s_red[CH_T / 64];
    __shared__ double s_trace;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // trace(G) for the shift
    {
        double t = 0.0;
        for (int i = tid; i < c; i += CH_T) t += G[i + i * ldg];
        t = wave_sum(t);
        if (lane == 0) s_red[wave] = t;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < CH_T / 64; ++w) s += s_red[w];
            s_trace = s;
        }
        __syncthreads();
    }

    for (int attempt = 0; attempt < 2; ++attempt) {
        const double shift = attempt == 0 ? 0.0 : shift_scale * s_trace;
        for (int64_t idx = tid; idx < (int64_t)c * c; idx += CH_T) {
            const int i = (int)(idx % c), j = (int)(idx / c);
            if (i >= j) W[i + j * ldw] = G[i + j * ldg] + (i == j ? shift : 0.0);
            X[i + j * ldw] = (i == j) ? 1.0 : 0.0;
        }
        if (tid == 0) s_bad = 0;
        __syncthreads();

        for (int K0 = 0; K0 < c; K0 += CH_NB) {
            const int kb = (c - K0) < CH_NB ? (c - K0) : CH_NB;
            const int J0 = K0 + kb;
            // (1) diagonal block -> D
            for (int idx = tid; idx < CH_NB * CH_NB; idx += CH_T) {
                const int i = idx % CH_NB, j = idx / CH_NB;
                D[i * CH_PS + j] = (i < kb && j < kb && i >= j) ? W[(K0 + i) + (int64_t)(K0 + j) * ldw] : 0.0;
            }
            __syncthreads();
            // (2) one wave factors D in registers (lane i = row i)
            if (wave == 0) {
                double d[CH_NB];
#pragma unroll
                for (int j = 0; j < CH_NB; ++j) d[j] = (lane < CH_NB) ? D[lane * CH_PS + j] : 0.0;
                int bad = 0;
#pragma unroll
                for (int j = 0; j < CH_NB; ++j) {
                    if (j < kb) {
                        const double pj = __shfl(d[j], j);
                        const bool ok = (pj > 0.0) && (pj < 1.0e308);
                        if (!ok) bad = 1;
                        const double sj = ok ? sqrt(pj) : 1.0;
                        if (lane == j) d[j] = sj;
                        else if (lane > j) d[j] = d[j] / sj;
#pragma unroll
                        for (int jj = j + 1; jj < CH_NB; ++jj) {
                            const double cj = __shfl(d[j], jj);
                            if (lane >= jj) d[jj] -= d[j] * cj;
                        }
                    }
                }
                if (lane < CH_NB) {
#pragma unroll
                    for (int j = 0; j < CH_NB; ++j) D[lane * CH_PS + j] = (j <= lane) ? d[j] : 0.0;
                }
                if (lane == 0 && bad) s_bad = 1;
            }
            __syncthreads();
            if (s_bad) break;
            // (3) Dinv = D^{-1} (lower); thread j < 32 solves column j in place in LDS
            if (tid < CH_NB) {
                const int j = tid;
                for (int i = 0; i < CH_NB; ++i) {
                    double s = (i == j) ? 1.0 : 0.0;
                    for (int t = j; t < i; ++t) s -= D[i * CH_PS + t] * Dinv[t * CH_PS + j];
                    Dinv[i * CH_PS + j] = (i >= j && i < kb) ? s / D[i * CH_PS + i] : 0.0;
                }
            }
            for (int idx = tid; idx < kb * kb; idx += CH_T) {
                const int i = idx % kb, j = idx / kb;
                if (i >= j) W[(K0 + i) + (int64_t)(K0 + j) * ldw] = D[i * CH_PS + j];
            }
            __syncthreads();
            // (4) panel rows i >= J0: L(i, K0:J0) = W(i, K0:J0) Dinv^T
            for (int i = J0 + tid; i < c; i += CH_T) {
                double w[CH_NB];
#pragma unroll
                for (int t = 0; t < CH_NB; ++t) w[t] = (t < kb) ? W[i + (int64_t)(K0 + t) * ldw] : 0.0;
                for (int s = 0; s < kb; ++s) {
                    double y = 0.0;
#pragma unroll
                    for (int t = 0; t < CH_NB; ++t) y += (t <= s) ? w[t] * Dinv[s * CH_PS + t] : 0.0;
                    W[i + (int64_t)(K0 + s) * ldw] = y;
                    if (i - J0 < prows) P[(i - J0) * CH_PS + s] = y;
                }
            }
            // (5) block row of the inverse: X(K0:J0, 0:J0) = Dinv X(K0:J0, 0:J0)
            for (int j = tid; j < J0; j += CH_T) {
                double xc[CH_NB];
#pragma unroll
                for (int t = 0; t < CH_NB; ++t) xc[t] = (t < kb) ? X[(K0 + t) + (int64_t)j * ldw] : 0.0;
                for (int s = 0; s < kb; ++s) {
                    double y = 0.0;
#pragma unroll
                    for (int t = 0; t < CH_NB; ++t) y += (t <= s) ? Dinv[s * CH_PS + t] * xc[t] : 0.0;
                    X[(K0 + s) + (int64_t)j * ldw] = y;
                    if (j < xcols) XK[s * xs + j] = y;
                }
            }
            __syncthreads();
            if (J0 >= c) break;
            // (6a) trailing update W(i, j) -= L(i, K) L(j, K)^T, J0 <= j <= i < c
            {
                const int nt = (c - J0 + 3) / 4;
                const int64_t T = (int64_t)nt * (nt + 1) / 2;
                for (int64_t idx = tid; idx < T; idx += CH_T) {
                    int ti = (int)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
                    while ((int64_t)ti * (ti + 1) / 2 > idx) --ti;
                    while ((int64_t)(ti + 1) * (ti + 2) / 2 <= idx) ++ti;
                    const int tj = (int)(idx - (int64_t)ti * (ti + 1) / 2);
                    const int i0 = J0 + 4 * ti, j0 = J0 + 4 * tj;
                    double acc[4][4] = {};
                    for (int s = 0; s < kb; ++s) {
                        double a[4], b[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = i0 + r, j = j0 + r;
                            a[r] = (i < c) ? ((i - J0 < prows) ? P[(i - J0) * CH_PS + s]
                                                               : W[i + (int64_t)(K0 + s) * ldw])
                                           : 0.0;
                            b[r] = (j < c) ? ((j - J0 < prows) ? P[(j - J0) * CH_PS + s]
                                                               : W[j + (int64_t)(K0 + s) * ldw])
                                           : 0.0;
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * b[q];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = i0 + r, j = j0 + q;
                            if (i < c && j < c && i >= j) W[i + (int64_t)j * ldw] -= acc[r][q];
                        }
                }
            }
            // (6b) inverse update X(i, j) -= L(i, K) X(K, j), i >= J0, j < J0
            {
                const int nti = (c - J0 + 3) / 4, ntj = (J0 + 3) / 4;
                const int64_t T = (int64_t)nti * ntj;
                for (int64_t idx = tid; idx < T; idx += CH_T) {
                    const int ti = (int)(idx / ntj), tj = (int)(idx % ntj);
                    const int i0 = J0 + 4 * ti, j0 = 4 * tj;
                    double acc[4][4] = {};
                    for (int s = 0; s < kb; ++s) {
                        double a[4], b[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = i0 + r, j = j0 + r;
                            a[r] = (i < c) ? ((i - J0 < prows) ? P[(i - J0) * CH_PS + s]
                                                               : W[i + (int64_t)(K0 + s) * ldw])
                                           : 0.0;
                            b[r] = (j < J0) ? ((j < xcols) ? XK[s * xs + j] : X[(K0 + s) + (int64_t)j * ldw])
                                            : 0.0;
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * b[q];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = i0 + r, j = j0 + q;
                            if (i < c && j < J0) X[i + (int64_t)j * ldw] -= acc[r][q];
                        }
                }
            }
            __syncthreads();
        }
        if (!s_bad) break;
        if (tid == 0 && info) atomicOr(info, attempt == 0 ? RQLP_INFO_CHOLQR_SHIFTED : RQLP_INFO_CHOL_FAILED);
        __syncthreads();
        if (attempt == 1) break;
    }
    __syncthreads();
    // outputs: R = L^T, Rinv = X^T (upper triangular, zero below)
    for (int64_t idx = tid; idx < (int64_t)c * c; idx += CH_T) {
        const int i = (int)(idx % c), j = (int)(idx / c);   // output element (i, j)
        if (R) R[i + j * ldr] = (i <= j) ? W[j + (int64_t)i * ldw] : 0.0;
        if (Rinv) Rinv[i + j * ldri] = (i <= j) ? X[j + (int64_t)i * ldw] : 0.0;
    }
}

int chol_inv(int64_t c, const double* G, int64_t ldg, double* R, int64_t ldr, double* Rinv, int64_t ldri,
             double shift_scale, double* W1, double* W2, int32_t* info, hipStream_t s) {
    if (c <= 0) return 0;
    const size_t lds = chol_inv_lds_bytes(c);
    static bool attr_set = false;
    if (!attr_set) {
        RQLP_HIP_TRY(hipFuncSetAttribute((const void*)chol_inv_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)chol_inv_lds_bytes(1 << 20)));
        attr_set = true;
    }
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(CH_T), lds, s, (int)c, G, ldg, R, ldr, Rinv, ldri,
                       shift_scale, W1, W2, c, info, ch_prows(c), ch_xcols(c));
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

}  // namespace rqlp
