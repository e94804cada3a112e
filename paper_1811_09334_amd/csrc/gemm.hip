// Skinny dense products of the range finder and the projection:
//   Y = A * X          (sketch, Algorithm 2.1 step 2; subspace iteration)
//   Z = A^T * V        (subspace iteration; B^T = A^T V, Algorithm 2.1 step 4)
//   G = X^T * X        (Gram matrix of CholeskyQR)
//   Y = X * L^{-T}     (CholeskyQR update, B transposed), Q = V Q_B (assembly)
// in FP64 or FP32 on the gfx950 matrix cores (v_mfma_f64_16x16x4f64 /
// v_mfma_f32_16x16x4f32), FP accumulation in the input precision.
//
// Tiling: a workgroup of 4 waves owns a (64*MB) x (16*NB) block of C; the
// four waves are stacked along M, each computing (16*MB) x (16*NB) with
// MB*NB 16x16 accumulators.  N (= the sketch width l, at most a few hundred)
// is covered by one or two column tiles, so A streams through HBM once per
// column tile.  K is split across blockIdx.z when the M x N tile grid alone
// cannot fill the 256 CUs; partial sums then go to a workspace and a second
// kernel adds them in a fixed order (bitwise reproducible results).
//
// LDS layouts (chosen for conflict-free fragment reads on 64 banks):
//   A, op(A) = A   : [k][i], row stride BM + 16   (global loads run along i)
//   A, op(A) = A^T : [i][k], row stride BK + 2    (global loads run along k)
//   B              : [j][k], row stride BK + 2    (global loads run along k)
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

template <typename T>
struct Mfma;

// Operand layouts (both types): lane l holds A(l % 16, k0 + l / 16) and
// B(k0 + l / 16, l % 16).  Accumulator element r of lane l holds
//   f64: C((l / 16) + 4 r, l % 16)      f32: C(4 (l / 16) + r, l % 16).
template <>
struct Mfma<double> {
    typedef double4_t acc_t;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
    typedef float4_t acc_t;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int GEMM_BK = 32;
constexpr int GEMM_THREADS = 256;

template <typename T, bool TA, bool TB, int MB, int NB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_skinny_kernel(
    int64_t M, int64_t N, int64_t K, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc, int64_t split_stride,
    int64_t kchunk) {
    constexpr int BK = GEMM_BK;
    constexpr int BM = 64 * MB;
    constexpr int BN = 16 * NB;
    constexpr int SA = TA ? (BK + 2) : (BM + 16);
    constexpr int A_ELEMS = TA ? BM * SA : BK * SA;
    constexpr int SB = BK + 2;
    constexpr int A_PER_T = BM * BK / GEMM_THREADS;     // 8 * MB
    constexpr int B_PER_T = BN * BK / GEMM_THREADS;     // 2 * NB
    typedef typename Mfma<T>::acc_t acc_t;

    __shared__ T As[A_ELEMS];
    __shared__ T Bs[BN * SB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * BM;
    const int64_t n0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

    acc_t acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    T ra[A_PER_T];
    T rb[B_PER_T];

    // ---- global -> registers for the tile starting at kt ----
    auto load_tile = [&](int64_t kt) {
        if (!TA) {
            // i = tid % 64 + 64 r, k = tid / 64 + 4 c
#pragma unroll
            for (int r = 0; r < MB; ++r)
#pragma unroll
                for (int c = 0; c < BK / 4; ++c) {
                    int64_t i = m0 + (tid & 63) + 64 * r;
                    int64_t k = kt + (tid >> 6) + 4 * c;
                    ra[r * (BK / 4) + c] = (i < M && k < kend) ? A[i + k * lda] : T(0);
                }
        } else {
            // k = tid % 32, i = tid / 32 + 8 r
#pragma unroll
            for (int r = 0; r < A_PER_T; ++r) {
                int64_t k = kt + (tid & 31);
                int64_t i = m0 + (tid >> 5) + 8 * r;
                ra[r] = (i < M && k < kend) ? A[k + i * lda] : T(0);
            }
        }
        if (!TB) {
            // op(B) = B (K x N): k = tid % 32, j = tid / 32 + 8 r
#pragma unroll
            for (int r = 0; r < B_PER_T; ++r) {
                int64_t k = kt + (tid & 31);
                int64_t j = n0 + (tid >> 5) + 8 * r;
                rb[r] = (j < N && k < kend) ? B[k + j * ldb] : T(0);
            }
        } else {
            // op(B) = B^T, B stored N x K: consecutive threads run along j
#pragma unroll
            for (int r = 0; r < B_PER_T; ++r) {
                const int e = tid + GEMM_THREADS * r;
                int64_t j = n0 + e % BN;
                int64_t k = kt + e / BN;
                rb[r] = (j < N && k < kend) ? B[j + k * ldb] : T(0);
            }
        }
    };
    auto store_tile = [&]() {
        if (!TA) {
#pragma unroll
            for (int r = 0; r < MB; ++r)
#pragma unroll
                for (int c = 0; c < BK / 4; ++c)
                    As[((tid >> 6) + 4 * c) * SA + (tid & 63) + 64 * r] = ra[r * (BK / 4) + c];
        } else {
#pragma unroll
            for (int r = 0; r < A_PER_T; ++r) As[((tid >> 5) + 8 * r) * SA + (tid & 31)] = ra[r];
        }
        if (!TB) {
#pragma unroll
            for (int r = 0; r < B_PER_T; ++r) Bs[((tid >> 5) + 8 * r) * SB + (tid & 31)] = rb[r];
        } else {
#pragma unroll
            for (int r = 0; r < B_PER_T; ++r) {
                const int e = tid + GEMM_THREADS * r;
                Bs[(e % BN) * SB + e / BN] = rb[r];
            }
        }
    };

    if (kbeg < kend) load_tile(kbeg);
    for (int64_t kt = kbeg; kt < kend; kt += BK) {
        __syncthreads();
        store_tile();
        __syncthreads();
        if (kt + BK < kend) load_tile(kt + BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            T af[MB], bf[NB];
#pragma unroll
            for (int a = 0; a < MB; ++a) {
                const int i = wave * 16 * MB + a * 16 + (lane & 15);
                af[a] = TA ? As[i * SA + kk] : As[kk * SA + i];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) bf[b] = Bs[(b * 16 + (lane & 15)) * SB + kk];
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = Mfma<T>::op(af[a], bf[b], acc[a][b]);
        }
    }

    // ---- write C (or this split's partial) ----
    T* Cs = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t j = n0 + b * 16 + (lane & 15);
            if (j >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wave * 16 * MB + a * 16 + Mfma<T>::row(lane, r);
                if (i < M) Cs[i + j * ldc] = acc[a][b][r];
            }
        }
}

// C (M x N, or its transpose when trans_out) = alpha * sum_s W_s + beta * C,
// summed in the fixed order s = 0, 1, ...
template <typename T, bool TRANS_OUT>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int64_t M, int64_t N, const T* __restrict__ W,
                                                            int64_t ldw, int64_t split_stride, int S,
                                                            T alpha, T beta, T* __restrict__ C,
                                                            int64_t ldc) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        T v = T(0);
        if (i < M && j < N) {
            for (int s = 0; s < S; ++s) v += W[s * split_stride + i + j * ldw];
            v *= alpha;
            if (!TRANS_OUT) {
                if (beta != T(0)) v += beta * C[i + j * ldc];
                C[i + j * ldc] = v;
            }
        }
        if (TRANS_OUT) tile[jj][tx] = v;
    }
    if (!TRANS_OUT) return;
    __syncthreads();
    // C is N x M: element (j, i) at C[j + i * ldc]
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < M && j < N) {
            T v = tile[tx][ii];
            if (beta != T(0)) v += beta * C[j + i * ldc];
            C[j + i * ldc] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
struct GemmPlan {
    int nb;          // 16-column blocks per workgroup tile
    int64_t tm, tn;  // tile grid
    int64_t S;       // K splits
    int64_t kchunk;
};

GemmPlan plan_gemm(int64_t M, int64_t N, int64_t K) {
    GemmPlan p;
    int64_t nblk = ceil_div(N, 16);
    int64_t ntiles = ceil_div(nblk, 16);
    p.nb = (int)ceil_div(nblk, ntiles);
    p.tm = ceil_div(M, 64);
    p.tn = ceil_div(N, 16 * p.nb);
    const int cus = device_info().num_cus > 0 ? device_info().num_cus : 256;
    int64_t want = 2 * cus;
    int64_t S = ceil_div(want, p.tm * p.tn);
    int64_t smax = ceil_div(K, 4 * GEMM_BK);
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    if (K <= 0) {
        p.S = 1;
        p.kchunk = GEMM_BK;
        return p;
    }
    p.kchunk = ceil_div(ceil_div(K, S), GEMM_BK) * GEMM_BK;
    p.S = ceil_div(K, p.kchunk);
    if (p.S < 1) p.S = 1;
    return p;
}

template <typename T, bool TA, bool TB, int NB>
void launch_nb(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda,
               const T* B, int64_t ldb, T* C, int64_t ldc, int64_t split_stride, hipStream_t s) {
    dim3 grid((unsigned)p.tm, (unsigned)p.tn, (unsigned)p.S);
    hipLaunchKernelGGL((gemm_skinny_kernel<T, TA, TB, 1, NB>), grid, dim3(GEMM_THREADS), 0, s, M, N, K, A,
                       lda, B, ldb, C, ldc, split_stride, p.kchunk);
}

template <typename T, bool TA, bool TB>
void launch_dispatch(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda,
                     const T* B, int64_t ldb, T* C, int64_t ldc, int64_t split_stride, hipStream_t s) {
    switch (p.nb) {
#define RQLP_NB_CASE(X) \
    case X: launch_nb<T, TA, TB, X>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, s); break;
        RQLP_NB_CASE(1) RQLP_NB_CASE(2) RQLP_NB_CASE(3) RQLP_NB_CASE(4)
        RQLP_NB_CASE(5) RQLP_NB_CASE(6) RQLP_NB_CASE(7) RQLP_NB_CASE(8)
        RQLP_NB_CASE(9) RQLP_NB_CASE(10) RQLP_NB_CASE(11) RQLP_NB_CASE(12)
        RQLP_NB_CASE(13) RQLP_NB_CASE(14) RQLP_NB_CASE(15) RQLP_NB_CASE(16)
#undef RQLP_NB_CASE
        default: break;
    }
}
}  // namespace

size_t gemm_workspace_elems(int64_t M, int64_t N, int64_t K) {
    GemmPlan p = plan_gemm(M, N, K);
    return (size_t)(p.S * M * N);
}

template <typename T>
static void launch_any(bool ta, bool tb, const GemmPlan& p, int64_t M, int64_t N, int64_t K, const T* A,
                       int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc, int64_t split_stride,
                       hipStream_t s) {
    if (ta && tb) return;   // not needed by the method
    if (ta) launch_dispatch<T, true, false>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, s);
    else if (tb) launch_dispatch<T, false, true>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, s);
    else launch_dispatch<T, false, false>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, s);
}

template <typename T>
int gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B, int64_t ldb,
         T* C, int64_t ldc, bool trans_out, T alpha, T beta, T* ws, size_t ws_elems, hipStream_t s) {
    if (ta && tb) return RQLP_E_UNSUPPORTED;
    if (M <= 0 || N <= 0) return 0;
    GemmPlan p = plan_gemm(M, N, K);
    const bool direct = (p.S == 1 && !trans_out && alpha == T(1) && beta == T(0));
    if (direct) {
        launch_any<T>(ta, tb, p, M, N, K, A, lda, B, ldb, C, ldc, 0, s);
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    }
    if ((size_t)(p.S * M * N) > ws_elems || ws == nullptr) return RQLP_E_WORKSPACE;
    launch_any<T>(ta, tb, p, M, N, K, A, lda, B, ldb, ws, M, M * N, s);
    dim3 grid((unsigned)ceil_div(M, 32), (unsigned)ceil_div(N, 32));
    if (trans_out)
        hipLaunchKernelGGL((splitk_reduce_kernel<T, true>), grid, dim3(256), 0, s, M, N, ws, M, M * N,
                           (int)p.S, alpha, beta, C, ldc);
    else
        hipLaunchKernelGGL((splitk_reduce_kernel<T, false>), grid, dim3(256), 0, s, M, N, ws, M, M * N,
                           (int)p.S, alpha, beta, C, ldc);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template int gemm<double>(bool, bool, int64_t, int64_t, int64_t, const double*, int64_t, const double*, int64_t,
                          double*, int64_t, bool, double, double, double*, size_t, hipStream_t);
template int gemm<float>(bool, bool, int64_t, int64_t, int64_t, const float*, int64_t, const float*, int64_t,
                         float*, int64_t, bool, float, float, float*, size_t, hipStream_t);

}  // namespace rqlp
