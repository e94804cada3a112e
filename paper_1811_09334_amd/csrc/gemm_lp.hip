// 16-bit skinny products of the mixed-precision range finder and projection:
//   Y = A W   and   Z = A^T V   (Algorithm 2.1 steps 2 and 4, and the
// subspace iterations), with A, W, V rounded to bfloat16 or IEEE half and
// FP32 accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16 /
// _f16).  The split form ("bf16x3") keeps x = hi + lo in two bfloat16 parts
// and accumulates hi*hi + hi*lo + lo*hi (Henry, Tang, Heinecke, ARITH 2019).
//
// The kernel computes C(i, j) = sum_k P(k + i * ldp) * Q(k + j * ldq): both
// operands are "k-contiguous", which is what the 16x16x32 MFMA wants (a lane
// feeds 8 consecutive k of one row or column).  A W uses a row-major 16-bit
// copy of A, A^T V the column-major one; W and V are column-major.
//
// Tiling: 4 waves, each 32 rows x (16 NB) columns (2 x NB accumulators of
// 16x16); a workgroup covers 128 rows and all (or a share) of the l columns,
// so A streams from HBM about once per product.  K advances in stages of 32
// through two LDS buffers (rows padded to 40 elements so that the 16-byte
// fragment reads of a wave spread over all banks); split-K partial sums are
// added in a fixed order by a separate reduce, so results are reproducible.
//
// IEEE half has too little exponent range for typical matrix entries, so
// the FP16 form stores A D^{-1} with D = diag(2^e_j) chosen per column
// (max |A(:, j)| 2^-e_j in [2^14, 2^15)); A W = (A D^{-1}) (D W) with D W
// stored as 2^-g D W (g = max e_j) and the 2^g put back in the epilogue, and
// A^T V = D (A D^{-1})^T V with the row scale applied in the epilogue.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

constexpr int LP_BM = 128;
constexpr int LP_BK = 32;
constexpr int LP_SK = LP_BK + 8;     // LDS row stride in 16-bit elements (80 bytes)
constexpr int LP_THREADS = 256;

template <int KIND>
__device__ __forceinline__ float4_t mfma_lp(u16x8_t a, u16x8_t b, float4_t c) {
    if constexpr (KIND == RQLP_MIXED_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// X3: operands come in (hi, lo) pairs at the same offsets of P / Plo and Q / Qlo.
// VEC: every 8-element k-chunk is 16-byte aligned and lies wholly inside or
// outside [0, K) (K, ldp, ldq multiples of 8, aligned bases), so tiles load
// with plain 16-byte loads; otherwise element loads with bounds checks.
template <int KIND, int NB, bool X3, bool VEC>
__global__ __launch_bounds__(LP_THREADS) void gemm_lp_kernel(
    int64_t M, int64_t N, int64_t K, const unsigned short* __restrict__ P, const unsigned short* __restrict__ Plo,
    int64_t ldp, const unsigned short* __restrict__ Q, const unsigned short* __restrict__ Qlo, int64_t ldq,
    float* __restrict__ C, int64_t ldc, int64_t split_stride, int64_t kchunk) {
    constexpr int NP = X3 ? 2 : 1;                                  // operand parts
    constexpr int BN = 16 * NB;
    constexpr int A_CH = LP_BM * LP_BK / 8 / LP_THREADS;            // 16-byte chunks per thread: 2
    constexpr int B_CH = (BN * LP_BK / 8 + LP_THREADS - 1) / LP_THREADS;
    __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][LP_BM * LP_SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][BN * LP_SK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * LP_BM;
    const int64_t n0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

    float4_t acc[2][NB];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};

    u16x8_t ra[NP][A_CH], rb[NP][B_CH];
    // 16-byte chunk ch of a tile row: k = 8 (ch % 4) .. +7 of row ch / 4
    auto load8 = [&](const unsigned short* base, int64_t ld, int64_t row, int64_t rows, int64_t k) {
        u16x8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (VEC) {
            if (row < rows && k < kend) v = *(const u16x8_t*)(base + k + row * ld);
        } else if (row < rows) {
            const unsigned short* p = base + k + row * ld;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (k + e < kend) ? p[e] : (unsigned short)0;
        }
        return v;
    };
    auto load_tile = [&](int64_t kt) {
#pragma unroll
        for (int c = 0; c < A_CH; ++c) {
            const int ch = tid + LP_THREADS * c;
            ra[0][c] = load8(P, ldp, m0 + (ch >> 2), M, kt + 8 * (ch & 3));
            if constexpr (X3) ra[NP - 1][c] = load8(Plo, ldp, m0 + (ch >> 2), M, kt + 8 * (ch & 3));
        }
#pragma unroll
        for (int c = 0; c < B_CH; ++c) {
            const int ch = tid + LP_THREADS * c;
            if (ch < BN * 4) {
                rb[0][c] = load8(Q, ldq, n0 + (ch >> 2), N, kt + 8 * (ch & 3));
                if constexpr (X3) rb[NP - 1][c] = load8(Qlo, ldq, n0 + (ch >> 2), N, kt + 8 * (ch & 3));
            }
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int h = 0; h < NP; ++h) {
#pragma unroll
            for (int c = 0; c < A_CH; ++c) {
                const int ch = tid + LP_THREADS * c;
                *(u16x8_t*)&As[buf][h][(ch >> 2) * LP_SK + 8 * (ch & 3)] = ra[h][c];
            }
#pragma unroll
            for (int c = 0; c < B_CH; ++c) {
                const int ch = tid + LP_THREADS * c;
                if (ch < BN * 4) *(u16x8_t*)&Bs[buf][h][(ch >> 2) * LP_SK + 8 * (ch & 3)] = rb[h][c];
            }
        }
    };

    if (kbeg < kend) {
        load_tile(kbeg);
        store_tile(0);
    }
    __syncthreads();
    int buf = 0;
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    for (int64_t kt = kbeg; kt < kend; kt += LP_BK) {
        const bool more = kt + LP_BK < kend;
        if (more) load_tile(kt + LP_BK);
        u16x8_t af[NP][2];
#pragma unroll
        for (int h = 0; h < NP; ++h)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                af[h][a] = *(const u16x8_t*)&As[buf][h][(wave * 32 + a * 16 + fr) * LP_SK + fk];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const u16x8_t bf = *(const u16x8_t*)&Bs[buf][0][(b * 16 + fr) * LP_SK + fk];
            if constexpr (X3) {
                const u16x8_t bl = *(const u16x8_t*)&Bs[buf][NP - 1][(b * 16 + fr) * LP_SK + fk];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    acc[a][b] = mfma_lp<KIND>(af[NP - 1][a], bf, acc[a][b]);
                    acc[a][b] = mfma_lp<KIND>(af[0][a], bl, acc[a][b]);
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) acc[a][b] = mfma_lp<KIND>(af[0][a], bf, acc[a][b]);
        }
        if (more) store_tile(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // accumulator element r of lane l holds C(4 (l / 16) + r, l % 16)
    float* Cs = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = m0 + wave * 32 + a * 16 + 4 * (lane >> 4) + r;
            if (i >= M) continue;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int64_t j = n0 + b * 16 + fr;
                if (j < N) Cs[i + j * ldc] = acc[a][b][r];
            }
        }
}

// C = 2^(gexp + rexp[i]) sum_s W_s (M x N FP32 partials, fixed order; the
// exponents only for the IEEE half form, else NULL), converted to TO, written
// as C (M x N) or, transposed, as C^T (N x M) through 32 x 32 LDS tiles.
template <typename TO, bool TRANS>
__global__ __launch_bounds__(256) void lp_reduce_kernel(int64_t M, int64_t N, const float* __restrict__ W,
                                                        int64_t split_stride, int S, TO* __restrict__ C,
                                                        int64_t ldc, const int* __restrict__ rexp,
                                                        const int* __restrict__ gexp) {
    __shared__ float tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int g = gexp ? *gexp : 0;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        float v0 = 0.f, v1 = 0.f;
        if (i < M && j < N) {
            const float* w = W + i + j * M;
            int s = 0;
            for (; s + 1 < S; s += 2) {
                v0 += w[s * split_stride];
                v1 += w[(s + 1) * split_stride];
            }
            if (s < S) v0 += w[s * split_stride];
            const int e = g + (rexp ? rexp[i] : 0);
            v0 = e ? ldexpf(v0 + v1, e) : v0 + v1;
            if (!TRANS) C[i + j * ldc] = (TO)v0;
        }
        if (TRANS) tile[jj][tx] = v0;
    }
    if (!TRANS) return;
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < M && j < N) C[j + i * ldc] = (TO)tile[tx][ii];
    }
}

// ---------------------------------------------------------------------------
namespace {
constexpr int LP_NBS[] = {1, 2, 3, 4, 6, 8, 9, 12, 17, 18};

struct LpPlan {
    int nb;
    int64_t tm, tn, S, kchunk;
};

LpPlan plan_lp(int64_t M, int64_t N, int64_t K) {
    LpPlan p;
    const int64_t nblk = ceil_div(N, 16);
    const int64_t ntiles = ceil_div(nblk, 18);
    const int64_t want_nb = ceil_div(nblk, ntiles);
    p.nb = 18;
    for (int v : LP_NBS)
        if (v >= want_nb) {
            p.nb = v;
            break;
        }
    p.tm = ceil_div(M, LP_BM);
    p.tn = ceil_div(N, 16 * p.nb);
    const int cus = device_info().num_cus > 0 ? device_info().num_cus : 256;
    int64_t S = ceil_div(4 * cus, p.tm * p.tn);
    int64_t smax = ceil_div(K, 512);
    // keep the partial-sum traffic S M N below a quarter of the operand traffic K (M + N)
    const int64_t straffic = (K * (M + N)) / (4 * M * N);
    if (smax > straffic) smax = straffic > 1 ? straffic : 1;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    p.kchunk = K <= 0 ? LP_BK : ceil_div(ceil_div(K, S), LP_BK) * LP_BK;
    p.S = K <= 0 ? 1 : ceil_div(K, p.kchunk);
    return p;
}

template <int KIND, int NB, bool X3>
void launch_lp(const LpPlan& p, int64_t M, int64_t N, int64_t K, const unsigned short* P, const unsigned short* Plo,
               int64_t ldp, const unsigned short* Q, const unsigned short* Qlo, int64_t ldq, float* C, int64_t ldc,
               int64_t ss, hipStream_t s) {
    auto al16 = [](const void* q) { return q == nullptr || (((uintptr_t)q) & 15) == 0; };
    const bool vec = (K % 8 == 0) && (ldp % 8 == 0) && (ldq % 8 == 0) && al16(P) && al16(Plo) && al16(Q) && al16(Qlo);
    const dim3 grid((unsigned)p.tm, (unsigned)p.tn, (unsigned)p.S);
    if (vec)
        hipLaunchKernelGGL((gemm_lp_kernel<KIND, NB, X3, true>), grid, dim3(LP_THREADS), 0, s, M, N, K, P, Plo, ldp, Q,
                           Qlo, ldq, C, ldc, ss, p.kchunk);
    else
        hipLaunchKernelGGL((gemm_lp_kernel<KIND, NB, X3, false>), grid, dim3(LP_THREADS), 0, s, M, N, K, P, Plo, ldp,
                           Q, Qlo, ldq, C, ldc, ss, p.kchunk);
}

template <int KIND, bool X3>
void dispatch_lp(const LpPlan& p, int64_t M, int64_t N, int64_t K, const unsigned short* P,
                 const unsigned short* Plo, int64_t ldp, const unsigned short* Q, const unsigned short* Qlo,
                 int64_t ldq, float* C, int64_t ldc, int64_t ss, hipStream_t s) {
    switch (p.nb) {
#define RQLP_LP_CASE(X)                                                                                      \
    case X:                                                                                                  \
        launch_lp<KIND, X, X3>(p, M, N, K, P, Plo, ldp, Q, Qlo, ldq, C, ldc, ss, s);                        \
        break;
        RQLP_LP_CASE(1) RQLP_LP_CASE(2) RQLP_LP_CASE(3) RQLP_LP_CASE(4) RQLP_LP_CASE(6)
        RQLP_LP_CASE(8) RQLP_LP_CASE(9) RQLP_LP_CASE(12) RQLP_LP_CASE(17) RQLP_LP_CASE(18)
#undef RQLP_LP_CASE
        default: break;
    }
}
}  // namespace

size_t gemm_lp_workspace_elems(int64_t M, int64_t N, int64_t K) {
    LpPlan p = plan_lp(M, N, K);
    return (size_t)(p.S * M * N);
}

template <typename TO>
int gemm_lp(int kind, int64_t M, int64_t N, int64_t K, const unsigned short* P, const unsigned short* Plo,
            int64_t ldp, const unsigned short* Q, const unsigned short* Qlo, int64_t ldq, TO* C, int64_t ldc,
            bool trans_out, const int* rexp, const int* gexp, float* ws, size_t ws_elems, hipStream_t s) {
    if (M <= 0 || N <= 0) return 0;
    const bool x3 = (Plo != nullptr && Qlo != nullptr);
    if (x3 != (kind == RQLP_MIXED_BF16X3)) return RQLP_E_UNSUPPORTED;
    LpPlan p = plan_lp(M, N, K);
    const bool scaled = rexp != nullptr || gexp != nullptr;
    const bool direct = (p.S == 1 && !trans_out && !scaled && sizeof(TO) == sizeof(float));
    float* dst = direct ? (float*)C : ws;
    const int64_t ld = direct ? ldc : M;
    if (!direct && ((size_t)(p.S * M * N) > ws_elems || ws == nullptr)) return RQLP_E_WORKSPACE;
    if (kind == RQLP_MIXED_FP16)
        dispatch_lp<RQLP_MIXED_FP16, false>(p, M, N, K, P, Plo, ldp, Q, Qlo, ldq, dst, ld, M * N, s);
    else if (x3)
        dispatch_lp<RQLP_MIXED_BF16, true>(p, M, N, K, P, Plo, ldp, Q, Qlo, ldq, dst, ld, M * N, s);
    else
        dispatch_lp<RQLP_MIXED_BF16, false>(p, M, N, K, P, Plo, ldp, Q, Qlo, ldq, dst, ld, M * N, s);
    if (hipGetLastError() != hipSuccess) return RQLP_E_HIP;
    if (direct) return 0;
    dim3 grid((unsigned)ceil_div(M, 32), (unsigned)ceil_div(N, 32));
    if (trans_out)
        hipLaunchKernelGGL((lp_reduce_kernel<TO, true>), grid, dim3(256), 0, s, M, N, ws, M * N, (int)p.S, C, ldc, rexp,
                           gexp);
    else
        hipLaunchKernelGGL((lp_reduce_kernel<TO, false>), grid, dim3(256), 0, s, M, N, ws, M * N, (int)p.S, C, ldc,
                           rexp, gexp);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template int gemm_lp<float>(int, int64_t, int64_t, int64_t, const unsigned short*, const unsigned short*, int64_t,
                            const unsigned short*, const unsigned short*, int64_t, float*, int64_t, bool, const int*,
                            const int*, float*, size_t, hipStream_t);
template int gemm_lp<double>(int, int64_t, int64_t, int64_t, const unsigned short*, const unsigned short*, int64_t,
                             const unsigned short*, const unsigned short*, int64_t, double*, int64_t, bool,
                             const int*, const int*, float*, size_t, hipStream_t);

// ---------------------------------------------------------------------------
// FP32 -> 16-bit conversions, round to nearest even.
__device__ __forceinline__ unsigned short f32_to_bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u) return (unsigned short)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (unsigned short)(b >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ unsigned short f32_to_f16_bits(float x) {
    return __builtin_bit_cast(unsigned short, (_Float16)x);
}

// dst (16-bit) = 2^(rexp[i] - cexp[j] - gexp) src(i, j) for the rows x cols
// FP32 matrix src (absent exponents count as 0); with transpose the
// destination holds the cols x rows matrix src^T.  dlo (bf16x3 only) gets
// the rounded remainder x - hi.  32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void cast_lp_kernel(int64_t rows, int64_t cols, const float* __restrict__ src,
                                                      int64_t lds_, unsigned short* __restrict__ dst,
                                                      unsigned short* __restrict__ dlo, int64_t ldd, int kind,
                                                      int transpose, const int* __restrict__ rexp,
                                                      const int* __restrict__ cexp, const int* __restrict__ gexp) {
    __shared__ unsigned short t[2][32][34];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int g = gexp ? *gexp : 0;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        unsigned short v = 0, vl = 0;
        if (i < rows && j < cols) {
            float x = src[i + j * lds_];
            const int e = (rexp ? rexp[i] : 0) - (cexp ? cexp[j] : 0) - g;
            if (e) x = ldexpf(x, e);
            if (kind == RQLP_MIXED_FP16) {
                v = f32_to_f16_bits(x);
            } else {
                v = f32_to_bf16_bits(x);
                if (dlo) vl = f32_to_bf16_bits(x - bf16_bits_to_f32(v));
            }
            if (!transpose) {
                dst[i + j * ldd] = v;
                if (dlo) dlo[i + j * ldd] = vl;
            }
        }
        t[0][jj][tx] = v;
        t[1][jj][tx] = vl;
    }
    if (!transpose) return;
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < rows && j < cols) {
            dst[j + i * ldd] = t[0][tx][ii];
            if (dlo) dlo[j + i * ldd] = t[1][tx][ii];
        }
    }
}

// Both 16-bit layouts of the m x n FP32 matrix A in one pass over A:
// Ac (m x n, column-major, ldc) and Ar (= A^T, n x m, ldr), with the bf16x3
// remainders (Aclo / Arlo) and the FP16 column exponents (cexp) as in
// cast_lp_kernel.  64 x 64 tiles: 16-byte reads of A, 8-byte writes of Ac,
// the transpose through LDS and 16-byte writes of Ar.  Needs m, lda, ldc
// multiples of 4, ldr a multiple of 8 and 16-byte aligned bases.
__global__ __launch_bounds__(256) void encode_both_kernel(int64_t m, int64_t n, const float* __restrict__ A,
                                                          int64_t lda, unsigned short* __restrict__ Ac,
                                                          unsigned short* __restrict__ Aclo, int64_t ldc,
                                                          unsigned short* __restrict__ Ar,
                                                          unsigned short* __restrict__ Arlo, int64_t ldr, int kind,
                                                          const int* __restrict__ cexp) {
    typedef unsigned short u16x4_t __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) unsigned short t[2][64][64 + 8];   // [part][column][row]
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
    const bool split = Aclo != nullptr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = tid + 256 * e;
        const int cj = idx >> 4, ri = (idx & 15) * 4;
        const int64_t i = i0 + ri, j = j0 + cj;
        u16x4_t v = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
        if (j < n && i < m) {
            const float4_t x = *(const float4_t*)(A + i + j * lda);     // m % 4 == 0: whole chunk inside
            const int ex = cexp ? -cexp[j] : 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float y = ex ? ldexpf(x[q], ex) : x[q];
                if (kind == RQLP_MIXED_FP16) {
                    v[q] = f32_to_f16_bits(y);
                } else {
                    v[q] = f32_to_bf16_bits(y);
                    if (split) vl[q] = f32_to_bf16_bits(y - bf16_bits_to_f32(v[q]));
                }
            }
            *(u16x4_t*)(Ac + i + j * ldc) = v;
            if (split) *(u16x4_t*)(Aclo + i + j * ldc) = vl;
        }
        *(u16x4_t*)&t[0][cj][ri] = v;
        *(u16x4_t*)&t[1][cj][ri] = vl;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int idx = tid + 256 * e;
        const int ri = idx >> 3, cc = (idx & 7) * 8;
        const int64_t i = i0 + ri, j = j0 + cc;
        if (i >= m || j >= n) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            unsigned short* D = h ? Arlo : Ar;
            if (!D) continue;
            u16x8_t v;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = t[h][cc + q][ri];
            if (j + 8 <= n) {
                *(u16x8_t*)(D + j + i * ldr) = v;
            } else {
                for (int q = 0; q < 8; ++q)
                    if (j + q < n) D[j + q + i * ldr] = v[q];
            }
        }
    }
}

int encode_both(int kind, int64_t m, int64_t n, const float* A, int64_t lda, unsigned short* Ac, unsigned short* Aclo,
                int64_t ldc, unsigned short* Ar, unsigned short* Arlo, int64_t ldr, const int* cexp, hipStream_t s) {
    if (m <= 0 || n <= 0) return 0;
    if ((kind == RQLP_MIXED_BF16X3) != (Aclo != nullptr) || (Aclo != nullptr) != (Arlo != nullptr))
        return RQLP_E_UNSUPPORTED;
    auto al16 = [](const void* q) { return q == nullptr || (((uintptr_t)q) & 15) == 0; };
    const bool fast = m % 4 == 0 && lda % 4 == 0 && ldc % 4 == 0 && ldr % 8 == 0 && al16(A) && al16(Ac) &&
                      al16(Aclo) && al16(Ar) && al16(Arlo);
    if (!fast) {
        RQLP_TRY(cast_to_lp(kind, m, n, A, lda, Ac, Aclo, ldc, false, nullptr, cexp, nullptr, s));
        return cast_to_lp(kind, m, n, A, lda, Ar, Arlo, ldr, true, nullptr, cexp, nullptr, s);
    }
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(n, 64));
    hipLaunchKernelGGL(encode_both_kernel, grid, dim3(256), 0, s, m, n, A, lda, Ac, Aclo, ldc, Ar, Arlo, ldr, kind,
                       cexp);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

int cast_to_lp(int kind, int64_t rows, int64_t cols, const float* src, int64_t lds_, unsigned short* dst,
               unsigned short* dlo, int64_t ldd, bool transpose, const int* rexp, const int* cexp, const int* gexp,
               hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    if ((kind == RQLP_MIXED_BF16X3) != (dlo != nullptr)) return RQLP_E_UNSUPPORTED;
    dim3 grid((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(cols, 32));
    hipLaunchKernelGGL(cast_lp_kernel, grid, dim3(256), 0, s, rows, cols, src, lds_, dst, dlo, ldd, kind,
                       transpose ? 1 : 0, rexp, cexp, gexp);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

// colexp[j] = e with max_i |A(i, j)| 2^-e in [2^14, 2^15) (0 for a zero or
// non-finite column); one workgroup per column.
__global__ __launch_bounds__(256) void colexp_kernel(int64_t rows, const float* __restrict__ A, int64_t lda,
                                                     int* __restrict__ colexp) {
    __shared__ float red[4];
    const int64_t j = blockIdx.x;
    float mx = 0.f;
    for (int64_t i = threadIdx.x; i < rows; i += 256) mx = fmaxf(mx, fabsf(A[i + j * lda]));
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        colexp[j] = (mx > 0.f && mx <= 3.4e38f) ? ilogbf(mx) - 14 : 0;
    }
}

// *gexp = max_j colexp[j]; one workgroup.
__global__ __launch_bounds__(256) void gexp_kernel(int64_t n, const int* __restrict__ colexp, int* __restrict__ gexp) {
    __shared__ int red[4];
    int mx = -1 << 30;
    for (int64_t j = threadIdx.x; j < n; j += 256) mx = max(mx, colexp[j]);
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) *gexp = max(max(red[0], red[1]), max(red[2], red[3]));
}

int column_exponents(int64_t rows, int64_t cols, const float* A, int64_t lda, int* colexp, int* gexp,
                     hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    hipLaunchKernelGGL(colexp_kernel, dim3((unsigned)cols), dim3(256), 0, s, rows, A, lda, colexp);
    hipLaunchKernelGGL(gexp_kernel, dim3(1), dim3(256), 0, s, cols, colexp, gexp);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template <typename S, typename D>
__global__ void cast_kernel(int64_t rows, int64_t cols, const S* __restrict__ src, int64_t lds_, D* __restrict__ dst,
                            int64_t ldd) {
    const int64_t n = rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % rows, j = idx / rows;
        dst[i + j * ldd] = (D)src[i + j * lds_];
    }
}

template <typename S, typename D>
int cast_matrix(int64_t rows, int64_t cols, const S* src, int64_t lds_, D* dst, int64_t ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    int64_t blocks = ceil_div(rows * cols, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((cast_kernel<S, D>), dim3((unsigned)blocks), dim3(256), 0, s, rows, cols, src, lds_, dst, ldd);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}
template int cast_matrix<float, double>(int64_t, int64_t, const float*, int64_t, double*, int64_t, hipStream_t);
template int cast_matrix<double, float>(int64_t, int64_t, const double*, int64_t, float*, int64_t, hipStream_t);
template int cast_matrix<float, float>(int64_t, int64_t, const float*, int64_t, float*, int64_t, hipStream_t);

}  // namespace rqlp
