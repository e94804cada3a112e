// Skinny dense products of the range finder and the projection:
//   Y = A * X          (sketch of Algorithm 2.1; subspace iteration)
//   Z = A^T * V        (subspace iteration; the projection B^T = A^T V of Algorithm 2.1)
//   G = X^T * X        (Gram matrix of CholeskyQR)
//   Y = X * L^{-T}     (CholeskyQR update, B transposed), Q = V Q_B (assembly)
// in FP64 or FP32 on the gfx950 matrix cores (v_mfma_f64_16x16x4f64 /
// v_mfma_f32_16x16x4f32), FP accumulation in the input precision.
//
// Tiling: a workgroup of 4 waves owns a 64 x (16*NB) block of C (NB <= 7);
// the four waves are stacked along M, each computing 16 x (16*NB) with NB
// 16x16 accumulators.  K advances in stages of 16 through two LDS buffers
// (the next stage is fetched into registers and stored while the current one
// feeds the MFMAs; one barrier per stage), which keeps a workgroup at ~53 KB
// of LDS so that three are resident per CU and hide each other's latencies
// (measured: 1 resident workgroup with 224-column tiles ran at ~33 TFLOP/s,
// 3 resident with 112-column tiles at ~50 TFLOP/s on the 20000 x 10000 x 210
// products).  K is split across the grid's third dimension (the split count
// fills whole rounds of the resident workgroups), and the tiles are dealt to
// the XCDs in contiguous ranges (gemm_tile); partial sums go to a workspace and a second kernel adds them in a fixed
// order (bitwise reproducible results).
//
// LDS layouts (chosen for conflict-free fragment reads on 64 banks):
//   A, op(A) = A   : [k][i], row stride BM + 16   (global loads run along i)
//   A, op(A) = A^T : [i][k], row stride BK + 2    (global loads run along k)
//   B              : [j][k], row stride BK + 2    (global loads run along k)
#include <type_traits>

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

constexpr int GEMM_BK = 16;        // K depth of one LDS stage (two stages resident), FP64
// FP32 stages are twice as deep: the next stage's loads are issued one stage
// ahead, and a 16-deep FP32 stage computes for less than a memory round trip
template <typename T>
constexpr int gemm_bk() { return sizeof(T) == 4 ? 2 * GEMM_BK : GEMM_BK; }
constexpr int pow2_floor(int x) {
    int p = 1;
    while (2 * p <= x) p *= 2;
    return p;
}
constexpr int GEMM_MAX_NB = 7;     // at most 7 blocks of 16 columns per tile: 3 workgroups per CU
constexpr int GEMM_THREADS = 256;

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin
// (linear id L to XCD L % 8), so tile P = (first tile of XCD L % 8) + L / 8
// gives every XCD a contiguous range of tiles; in that order the N tiles run
// fastest, then the M tiles, then the K chunks, so that the tiles reading the
// same rows of op(A) (and, within a K chunk, of op(B)) run at the same time on
// one XCD and share its L2.  The map is a bijection for any grid.
__device__ __forceinline__ void gemm_tile(int64_t& bx, int64_t& by, int64_t& bz) {
    const uint32_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    const uint32_t n = gx * gy * gz;
    const uint32_t L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const uint32_t x8 = L & 7u, q = n >> 3, r = n & 7u;
    const uint32_t P = x8 * q + (x8 < r ? x8 : r) + (L >> 3);
    by = P % gy;
    bx = (P / gy) % gx;
    bz = P / (gx * gy);
}

// Zero words that the product kernels load in place of elements outside
// op(A) / op(B) (never written; not const, so that the load stays a load and
// needs no select after it, which would make the prefetch wait at once).
__device__ double g_gemm_zero[2];

// T: arithmetic (MFMA) type; TI: element type of A and B (converted to T when
// stored to LDS); TC: element type of C / of the split-K partials.
template <typename T, bool TA, bool TB, int MB, int NB, int BK, typename TI, typename TC, bool AB>
__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(std::is_same<T, TI>::value ? 1 : 3))) void gemm_skinny_kernel(
    int64_t M, int64_t N, int64_t K, const TI* __restrict__ A, int64_t lda,
    const TI* __restrict__ B, int64_t ldb, TC* __restrict__ C, int64_t ldc, int64_t split_stride,
    int64_t kchunk, const int32_t* __restrict__ gate, int gate_copy, int tri, T alpha, T beta) {
    constexpr int BM = 64 * MB;
    constexpr int BN = 16 * NB;
    constexpr int SA = TA ? (BK + 2) : (BM + 16);
    constexpr int A_ELEMS = TA ? BM * SA : BK * SA;
    constexpr int SB = BK + 2;
    constexpr int B_ELEMS = BN * SB;
    constexpr int A_PER_T = BM * BK / GEMM_THREADS;
    constexpr int B_PER_T = BN * BK / GEMM_THREADS;
    constexpr int KSTEP = GEMM_THREADS / BK;             // rows covered per pass of a k-contiguous load
    // op(B) = B^T (B stored N x K, j contiguous): thread t < TBP BN takes
    // column t % BN of the tile and k = t / BN + TBP e, e < TBE, so that its
    // loads step through B with one stride and consecutive threads read
    // consecutive columns
    constexpr int TBP = pow2_floor(GEMM_THREADS / BN);
    constexpr int TBE = BK / TBP;
    constexpr int RB = TB ? TBE : B_PER_T;                // B elements staged per thread
    static_assert(TBP * TBE == BK && TBP * BN <= GEMM_THREADS, "B^T staging must cover the stage once");
    static_assert(GEMM_THREADS % BK == 0 && BK % 4 == 0, "BK must divide the workgroup size");
    typedef typename Mfma<T>::acc_t acc_t;

    // two LDS buffers: the tile for step t+1 is stored while step t computes
    __shared__ T As[2][A_ELEMS];
    __shared__ T Bs[2][B_ELEMS];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int64_t bx, by, bz;
    gemm_tile(bx, by, bz);
    const int64_t m0 = bx * BM;
    const int64_t n0 = by * BN;
    // conditional product: when *gate is 0 nothing is computed; with gate_copy
    // the tile of op(A) is copied to C instead (the product with an identity)
    if (gate != nullptr && *gate == 0) {
        if (gate_copy && !TA)
            for (int idx = tid; idx < BM * BN; idx += GEMM_THREADS) {
                const int64_t i = m0 + idx % BM, j = n0 + idx / BM;
                if (i < M && j < N) C[i + j * ldc] = (TC)A[i + j * lda];
            }
        return;
    }
    // tri 1: only the lower triangle of C is wanted (Gram matrix): tiles wholly
    // above the diagonal are skipped.  tri 2: op(B)(k, j) = 0 for k > j (B^T of a
    // lower triangular B), so the K range of a tile ends at its last column.
    if (tri == 1 && m0 + BM <= n0) return;
    const int64_t kbeg = bz * kchunk;
    int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    if (tri == 2 && kend > n0 + BN) kend = n0 + BN;

    acc_t acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    TI ra[A_PER_T];
    TI rb[RB];
    const TI* zp = reinterpret_cast<const TI*>(g_gemm_zero);

    // ---- global -> registers for the tile starting at kt ----
    // Per-thread element pointers at k = 0 are formed once; a K stage of a
    // tile that lies wholly inside op(A) (op(B)) loads without bounds checks,
    // otherwise every element is checked, and one outside the matrix is read
    // from a zero word instead (an address select, not a branch per element).
    const bool a_inside = m0 + BM <= M;
    const bool b_inside = n0 + BN <= N;
    const TI* pa;
    const TI* pb;
    if (!TA) pa = A + (m0 + (tid & 63)) + (int64_t)(tid >> 6) * lda;       // + 64 r + (kt + 4 c) lda
    else     pa = A + (tid % BK) + (m0 + tid / BK) * lda;                 // + kt + KSTEP r lda
    if (!TB) pb = B + (tid % BK) + (n0 + tid / BK) * ldb;                 // + kt + KSTEP r ldb
    else     pb = B + (n0 + tid % BN) + (int64_t)(tid / BN) * ldb;         // + (kt + TBP e) ldb
    const bool tb_act = tid < TBP * BN;
    auto load_tile = [&](int64_t kt) {
        const bool kfull = kt + BK <= kend;
        if (!TA) {
            const TI* p = pa + kt * lda;
            if (a_inside && kfull) {
#pragma unroll
                for (int r = 0; r < MB; ++r)
#pragma unroll
                    for (int c = 0; c < BK / 4; ++c) ra[r * (BK / 4) + c] = p[64 * r + (int64_t)(4 * c) * lda];
            } else {
#pragma unroll
                for (int r = 0; r < MB; ++r)
#pragma unroll
                    for (int c = 0; c < BK / 4; ++c) {
                        const bool ok = (m0 + (tid & 63) + 64 * r < M) && (kt + (tid >> 6) + 4 * c < kend);
                        ra[r * (BK / 4) + c] = *(ok ? p + 64 * r + (int64_t)(4 * c) * lda : zp);
                    }
            }
        } else {
            const TI* p = pa + kt;
            if (a_inside && kfull) {
#pragma unroll
                for (int r = 0; r < A_PER_T; ++r) ra[r] = p[(int64_t)(KSTEP * r) * lda];
            } else {
                const bool kok = kt + (tid % BK) < kend;
#pragma unroll
                for (int r = 0; r < A_PER_T; ++r) {
                    const bool ok = kok && (m0 + (tid / BK) + KSTEP * r < M);
                    ra[r] = *(ok ? p + (int64_t)(KSTEP * r) * lda : zp);
                }
            }
        }
        if (!TB) {
            const TI* p = pb + kt;
            if (b_inside && kfull) {
#pragma unroll
                for (int r = 0; r < B_PER_T; ++r) rb[r] = p[(int64_t)(KSTEP * r) * ldb];
            } else {
                const bool kok = kt + (tid % BK) < kend;
#pragma unroll
                for (int r = 0; r < B_PER_T; ++r) {
                    const bool ok = kok && (n0 + (tid / BK) + KSTEP * r < N);
                    rb[r] = *(ok ? p + (int64_t)(KSTEP * r) * ldb : zp);
                }
            }
        } else {
            const TI* p = pb + kt * ldb;
            if (b_inside && kfull) {
                if (tb_act) {
#pragma unroll
                    for (int e = 0; e < TBE; ++e) rb[e] = p[(int64_t)(TBP * e) * ldb];
                }
            } else {
                const bool jok = tb_act && n0 + tid % BN < N;
#pragma unroll
                for (int e = 0; e < TBE; ++e) {
                    const bool ok = jok && (kt + tid / BN + TBP * e < kend);
                    rb[e] = *(ok ? p + (int64_t)(TBP * e) * ldb : zp);
                }
            }
        }
    };
    auto store_tile = [&](int buf) {
        T* as = As[buf];
        T* bs = Bs[buf];
        if (!TA) {
#pragma unroll
            for (int r = 0; r < MB; ++r)
#pragma unroll
                for (int c = 0; c < BK / 4; ++c)
                    as[((tid >> 6) + 4 * c) * SA + (tid & 63) + 64 * r] = (T)ra[r * (BK / 4) + c];
        } else {
#pragma unroll
            for (int r = 0; r < A_PER_T; ++r) as[((tid / BK) + KSTEP * r) * SA + (tid % BK)] = (T)ra[r];
        }
        if (!TB) {
#pragma unroll
            for (int r = 0; r < B_PER_T; ++r) bs[((tid / BK) + KSTEP * r) * SB + (tid % BK)] = (T)rb[r];
        } else if (tb_act) {
#pragma unroll
            for (int e = 0; e < TBE; ++e) bs[(tid % BN) * SB + tid / BN + TBP * e] = (T)rb[e];
        }
    };

    if (kbeg < kend) {
        load_tile(kbeg);
        store_tile(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t kt = kbeg; kt < kend; kt += BK) {
        const bool more = kt + BK < kend;
        if (more) load_tile(kt + BK);
        const T* as = As[buf];
        const T* bs = Bs[buf];
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            T af[MB], bf[NB];
#pragma unroll
            for (int a = 0; a < MB; ++a) {
                const int i = wave * 16 * MB + a * 16 + (lane & 15);
                af[a] = TA ? as[i * SA + kk] : as[kk * SA + i];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) bf[b] = bs[(b * 16 + (lane & 15)) * SB + kk];
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = Mfma<T>::op(af[a], bf[b], acc[a][b]);
        }
        if (more) store_tile(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // ---- write C (or this split's partial); AB: C = alpha op(A) op(B) + beta C
    // for a product in one K split (C read only when beta != 0) ----
    TC* Cs = C + bz * split_stride;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t j = n0 + b * 16 + (lane & 15);
            if (j >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wave * 16 * MB + a * 16 + Mfma<T>::row(lane, r);
                if (i < M) {
                    if constexpr (AB) {
                        T v = alpha * acc[a][b][r];
                        if (beta != T(0)) v += beta * (T)Cs[i + j * ldc];
                        Cs[i + j * ldc] = (TC)v;
                    } else {
                        Cs[i + j * ldc] = (TC)acc[a][b][r];
                    }
                }
            }
        }
}

// C (M x N) = alpha * sum_s W_s + beta * C, one output element per thread,
// summed in the fixed order s = 0, 1, ...
template <typename T, typename TO>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int64_t M, int64_t N, const T* __restrict__ W,
                                                            int64_t ldw, int64_t split_stride, int S, T alpha,
                                                            T beta, TO* __restrict__ C, int64_t ldc,
                                                            const int32_t* __restrict__ gate, int tri) {
    if (gate != nullptr && *gate == 0) return;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx % M, j = idx / M;
    if (tri == 1 && j > i) return;                   // partials of skipped tiles were never written
    const T* w = W + i + j * ldw;
    T v0 = T(0), v1 = T(0);
    int s = 0;
    for (; s + 1 < S; s += 2) {
        v0 += w[s * split_stride];
        v1 += w[(s + 1) * split_stride];
    }
    if (s < S) v0 += w[s * split_stride];
    T v = alpha * (v0 + v1);
    if (beta != T(0)) v += beta * (T)C[i + j * ldc];
    C[i + j * ldc] = (TO)v;
}

// C (N x M) = (alpha * sum_s W_s + beta * C^T)^T through 32 x 32 LDS tiles.
template <typename T, typename TO>
__global__ __launch_bounds__(256) void splitk_reduce_t_kernel(int64_t M, int64_t N, const T* __restrict__ W,
                                                              int64_t ldw, int64_t split_stride, int S, T alpha,
                                                              T beta, TO* __restrict__ C, int64_t ldc,
                                                              const int32_t* __restrict__ gate) {
    if (gate != nullptr && *gate == 0) return;
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        T v = T(0);
        if (i < M && j < N) {
            for (int s = 0; s < S; ++s) v += W[s * split_stride + i + j * ldw];
            v *= alpha;
        }
        tile[jj][tx] = v;
    }
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < M && j < N) {
            T v = tile[tx][ii];
            if (beta != T(0)) v += beta * (T)C[j + i * ldc];
            C[j + i * ldc] = (TO)v;
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

// 16-column blocks per workgroup tile (at most GEMM_MAX_NB, the column
// tiles as even as possible)
int plan_nb(int64_t N) {
    const int64_t nblk = ceil_div(N, 16);
    const int64_t ntiles = ceil_div(nblk, GEMM_MAX_NB);
    return (int)ceil_div(nblk, ntiles);
}

// The largest number of K splits: K chunks of at least 256, and partial sums
// (S M N) of at most a quarter of the operands' volume K (M + N).
int64_t split_limit(int64_t M, int64_t N, int64_t K) {
    int64_t smax = ceil_div(K, 256);
    const int64_t straffic = (K * (M + N)) / (4 * M * N);
    if (smax > straffic) smax = straffic > 1 ? straffic : 1;
    return smax < 1 ? 1 : smax;
}

// cap: the product kernel's resident workgroups on the device (0: three per
// CU).  The number of K splits is the one whose workgroups fill whole rounds
// of the resident slots best: a last round a fraction full leaves the rest of
// the device idle for a whole workgroup's time (FP64 20000 x 10000 x 210: 626
// tiles fill 768 slots to 82% with any split count up to 5, to 98% with 6).
// A larger count is taken only for at least 2% more fill (each split adds
// partial sums to write and reduce).
GemmPlan plan_gemm(int64_t M, int64_t N, int64_t K, int bk = GEMM_BK, int64_t cap = 0) {
    GemmPlan p;
    p.nb = plan_nb(N);
    p.tm = ceil_div(M, 64);
    p.tn = ceil_div(N, 16 * p.nb);
    if (K <= 0) {
        p.S = 1;
        p.kchunk = bk;
        return p;
    }
    const int cus = device_info().num_cus > 0 ? device_info().num_cus : 256;
    if (cap <= 0) cap = 3 * (int64_t)cus;
    const int64_t T = p.tm * p.tn, smax = split_limit(M, N, K);
    int64_t best_kc = ceil_div(K, bk) * bk;
    double best_fill = -1.0;
    for (int64_t s = 1; s <= smax; ++s) {
        const int64_t kc = ceil_div(ceil_div(K, s), bk) * bk;
        const int64_t w = T * ceil_div(K, kc);                 // workgroups
        const double fill = (double)w / (double)(ceil_div(w, cap) * cap);
        if (fill > best_fill + 0.02) {
            best_fill = fill;
            best_kc = kc;
        }
    }
    p.kchunk = best_kc;
    p.S = ceil_div(K, p.kchunk);
    return p;
}

// resident workgroups of the split-K product kernel that a product with these
// operand forms and column blocks launches (0 when unknown)
template <typename T, typename TI, bool TA, bool TB>
int64_t kernel_capacity(int nb) {
    const void* f = nullptr;
    switch (nb) {
#define RQLP_CAP_CASE(X)                                                                               \
    case X:                                                                                             \
        f = (const void*)gemm_skinny_kernel<T, TA, TB, 1, X, gemm_bk<T>(), TI, T, false>;              \
        break;
        RQLP_CAP_CASE(1) RQLP_CAP_CASE(2) RQLP_CAP_CASE(3) RQLP_CAP_CASE(4)
        RQLP_CAP_CASE(5) RQLP_CAP_CASE(6) RQLP_CAP_CASE(7)
#undef RQLP_CAP_CASE
        default: break;
    }
    return f ? (int64_t)resident_capacity(f, GEMM_THREADS, 0) : 0;
}

template <typename T, typename TI>
int64_t product_capacity(bool ta, bool tb, int64_t N) {
    const int nb = plan_nb(N);
    if (ta) return kernel_capacity<T, TI, true, false>(nb);
    if (tb) return kernel_capacity<T, TI, false, true>(nb);
    return kernel_capacity<T, TI, false, false>(nb);
}

template <typename T, typename TI, typename TC, bool TA, bool TB, int NB>
void launch_nb(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const TI* A, int64_t lda,
               const TI* B, int64_t ldb, TC* C, int64_t ldc, int64_t split_stride, const int32_t* gate, int gate_copy,
               int tri, T alpha, T beta, hipStream_t s) {
    dim3 grid((unsigned)p.tm, (unsigned)p.tn, (unsigned)p.S);
    // (the alpha / beta epilogue is a variant of its own: keeping it out of the
    // plain product leaves that kernel's register count, hence its occupancy, alone)
    if (alpha == T(1) && beta == T(0))
        hipLaunchKernelGGL((gemm_skinny_kernel<T, TA, TB, 1, NB, gemm_bk<T>(), TI, TC, false>), grid, dim3(GEMM_THREADS),
                           0, s, M, N, K, A, lda, B, ldb, C, ldc, split_stride, p.kchunk, gate, gate_copy, tri, alpha,
                           beta);
    else
        hipLaunchKernelGGL((gemm_skinny_kernel<T, TA, TB, 1, NB, gemm_bk<T>(), TI, TC, true>), grid, dim3(GEMM_THREADS),
                           0, s, M, N, K, A, lda, B, ldb, C, ldc, split_stride, p.kchunk, gate, gate_copy, tri, alpha,
                           beta);
}

template <typename T, typename TI, typename TC, bool TA, bool TB>
void launch_dispatch(const GemmPlan& p, int64_t M, int64_t N, int64_t K, const TI* A, int64_t lda,
                     const TI* B, int64_t ldb, TC* C, int64_t ldc, int64_t split_stride, const int32_t* gate,
                     int gate_copy, int tri, T alpha, T beta, hipStream_t s) {
    switch (p.nb) {
#define RQLP_NB_CASE(X)                                                                                           \
    case X:                                                                                                       \
        launch_nb<T, TI, TC, TA, TB, X>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, gate, gate_copy, tri,   \
                                        alpha, beta, s);                                                          \
        break;
        RQLP_NB_CASE(1) RQLP_NB_CASE(2) RQLP_NB_CASE(3) RQLP_NB_CASE(4)
        RQLP_NB_CASE(5) RQLP_NB_CASE(6) RQLP_NB_CASE(7)
#undef RQLP_NB_CASE
        default: break;
    }
}
}  // namespace

size_t gemm_workspace_elems(int64_t M, int64_t N, int64_t K) {
    // (every plan splits K at most split_limit times)
    size_t e = (size_t)(split_limit(M, N, K) * M * N);
    if (M == N) {                                    // a Gram matrix may take the CholeskyQR kernel
        const size_t g = gram_workspace_elems(K, M);
        if (g > e) e = g;
    }
    return e;
}

template <typename T, typename TI, typename TC>
static void launch_any(bool ta, bool tb, const GemmPlan& p, int64_t M, int64_t N, int64_t K, const TI* A,
                       int64_t lda, const TI* B, int64_t ldb, TC* C, int64_t ldc, int64_t split_stride,
                       const int32_t* gate, int gate_copy, int tri, T alpha, T beta, hipStream_t s) {
    if (ta && tb) return;   // not needed by the method
    if (ta)
        launch_dispatch<T, TI, TC, true, false>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, gate, gate_copy, tri,
                                                alpha, beta, s);
    else if (tb)
        launch_dispatch<T, TI, TC, false, true>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, gate, gate_copy, tri,
                                                alpha, beta, s);
    else
        launch_dispatch<T, TI, TC, false, false>(p, M, N, K, A, lda, B, ldb, C, ldc, split_stride, gate, gate_copy,
                                                 tri, alpha, beta, s);
}

// T: arithmetic and split-K partial type; TI: A, B; TC: C.
template <typename T, typename TI, typename TC>
static int gemm_impl(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const TI* A, int64_t lda, const TI* B,
                     int64_t ldb, TC* C, int64_t ldc, bool trans_out, T alpha, T beta, T* ws, size_t ws_elems,
                     hipStream_t s, const int32_t* gate, int gate_mode, int tri = 0) {
    if (ta && tb) return RQLP_E_UNSUPPORTED;
    if (M <= 0 || N <= 0) return 0;
    if ((tri == 1 && (trans_out || beta != T(0))) || (tri == 2 && !tb)) return RQLP_E_UNSUPPORTED;
    if constexpr (std::is_same<T, TI>::value && std::is_same<T, TC>::value) {
        // the two products of a CholeskyQR pass have kernels of their own
        if (alpha == T(1) && beta == T(0) && !trans_out) {
            if (tri == 1 && ta && M == N && (const void*)A == (const void*)B && lda == ldb && gate_mode != 2 &&
                gram_fits<T>(K, M, A, lda, ws, ws_elems))
                return gram<T>(K, M, A, lda, C, ldc, ws, ws_elems, s, gate);
            if (tri == 2 && !ta && N == K && ldb >= N && ldb <= (1 << 20) && trmm_fits<T>(M, N, A, lda, C, ldc))
                return trmm_lt<T>(M, N, A, lda, B, ldb, C, ldc, s, gate, gate_mode);
        }
    }
    // the general kernels read A and B while other workgroups write C: no aliasing
    if ((const void*)C == (const void*)A || (const void*)C == (const void*)B) return RQLP_E_UNSUPPORTED;
    GemmPlan p = plan_gemm(M, N, K, gemm_bk<T>(), product_capacity<T, TI>(ta, tb, N));
    // one K split: the product kernel applies alpha and beta itself
    const bool direct = (p.S == 1 && !trans_out);
    // the gated copy (gate_mode 2) writes op(A) straight into C: only for a
    // direct product C = op(A) op(B) with op(A) = A of the output's shape
    if (gate_mode == 2 && (!direct || ta || K != N || alpha != T(1) || beta != T(0))) return RQLP_E_UNSUPPORTED;
    const int gate_copy = gate_mode == 2 ? 1 : 0;
    if (direct) {
        launch_any<T, TI, TC>(ta, tb, p, M, N, K, A, lda, B, ldb, C, ldc, 0, gate, gate_copy, tri, alpha, beta, s);
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    }
    if ((size_t)(p.S * M * N) > ws_elems || ws == nullptr) return RQLP_E_WORKSPACE;
    launch_any<T, TI, T>(ta, tb, p, M, N, K, A, lda, B, ldb, ws, M, M * N, gate, 0, tri, T(1), T(0), s);
    if (trans_out) {
        dim3 grid((unsigned)ceil_div(M, 32), (unsigned)ceil_div(N, 32));
        hipLaunchKernelGGL((splitk_reduce_t_kernel<T, TC>), grid, dim3(256), 0, s, M, N, ws, M, M * N, (int)p.S,
                           alpha, beta, C, ldc, gate);
    } else {
        hipLaunchKernelGGL((splitk_reduce_kernel<T, TC>), dim3((unsigned)ceil_div(M * N, 256)), dim3(256), 0, s, M,
                           N, ws, M, M * N, (int)p.S, alpha, beta, C, ldc, gate, tri);
    }
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template <typename T>
int gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B, int64_t ldb,
         T* C, int64_t ldc, bool trans_out, T alpha, T beta, T* ws, size_t ws_elems, hipStream_t s,
         const int32_t* gate, int gate_mode, int tri) {
    return gemm_impl<T, T, T>(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, trans_out, alpha, beta, ws, ws_elems, s, gate,
                              gate_mode, tri);
}

int gemm_f32_acc64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                   int64_t ldb, float* C, int64_t ldc, bool trans_out, double alpha, double beta, double* ws,
                   size_t ws_elems, hipStream_t s, const int32_t* gate, int gate_mode) {
    return gemm_impl<double, float, float>(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, trans_out, alpha, beta, ws,
                                           ws_elems, s, gate, gate_mode);
}

template int gemm<double>(bool, bool, int64_t, int64_t, int64_t, const double*, int64_t, const double*, int64_t,
                          double*, int64_t, bool, double, double, double*, size_t, hipStream_t, const int32_t*, int,
                          int);
template int gemm<float>(bool, bool, int64_t, int64_t, int64_t, const float*, int64_t, const float*, int64_t,
                         float*, int64_t, bool, float, float, float*, size_t, hipStream_t, const int32_t*, int, int);

}  // namespace rqlp
