// 16-bit skinny products of the mixed-precision range finder and projection:
//   Y = A W   and   Z = A^T V   (the sketch and the projection of Algorithm 2.1, and the
// subspace iterations), with A, W, V rounded to bfloat16 or IEEE half and
// FP32 accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16 /
// _f16).  The split form ("bf16x3") keeps x = hi + lo in two bfloat16 parts
// and accumulates lo*hi + hi*lo + hi*hi (Henry, Tang, Heinecke, ARITH 2019).
//
// Operand format ("fragment tiles").  Every product here is
// C(i, j) = sum_k X(i, k) Y(j, k) with both operands k-contiguous, which is
// what the 16x16x32 MFMA consumes: lane t of a wave feeds row t % 16 and the
// eight k values 8 (t / 16) .. +7.  The 16-bit copies are therefore stored as
// 1 KB blocks of 16 rows x 32 k in exactly that lane order (block (rb, kb) at
// element (rb * nkb + kb) * 512, lane t at + 8 t), zero-padded to whole
// blocks.  A wave then reads a fragment as one contiguous 1 KB, every block
// row is one sequential stream through HBM, and ragged edges need no bounds
// checks (the padding multiplies as zero).  A row-major or column-major
// 16-bit copy instead makes every 16-byte fragment load touch a different
// DRAM row, which held these products to about a third of the HBM rate.
//
// Kernel: 8 waves per workgroup, each 32 rows x (16 NB) columns (2 x NB
// accumulator tiles); the workgroup covers 256 rows of X and NB column blocks
// of Y.  X fragments go straight from HBM into registers (each wave owns its
// rows), NBUF stages ahead; the Y blocks, shared by all waves, are copied
// into LDS by the load unit itself (global_load_lds_dwordx4, no registers)
// in the same fragment order, so the MFMA reads them with conflict-free
// 16-byte LDS loads.  The barrier between stages waits only for the copies of
// the stage about to be used (explicit vmcnt), keeping NBUF - 1 stages of
// both operands in flight.  K is split over workgroups (fixed-order
// reduction in a second kernel, so results are reproducible), and the
// workgroups sharing one K range of Y are placed on one XCD (blocks are
// dealt round-robin to the 8 XCDs), so that slice of Y stays in that XCD's L2;
// with several column tiles (l above 272) those of one row block run side by
// side on one XCD, so that X is fetched from HBM about once, not once per
// column tile.
//
// IEEE half has too little exponent range for typical matrix entries, so
// the FP16 form stores A D^{-1} with D = diag(2^e_j) chosen per column
// (max |A(:, j)| 2^-e_j in [2^14, 2^15)); A W = (A D^{-1}) (D W) with D W
// stored as 2^-g D W (g = max e_j) and the 2^g put back in the reduction, and
// A^T V = D (A D^{-1})^T V with the row scale applied in the reduction.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

constexpr int LP_WAVES = 8;
constexpr int LP_THREADS = 64 * LP_WAVES;
constexpr int LP_BM = 32 * LP_WAVES;     // rows of X per workgroup
constexpr int LP_BLK = 512;              // elements of one 16 x 32 fragment block

template <int KIND>
__device__ __forceinline__ float4_t mfma_lp(u16x8_t a, u16x8_t b, float4_t c) {
    if constexpr (KIND == RQLP_MIXED_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

struct LpGrid {
    int64_t tm, tn, S;      // row tiles, column tiles, K splits
    int64_t per_xcd, T;     // tiles per XCD, total tiles
    int64_t kcb;            // K blocks (of 32) per split
};

// C(i, j) (+ split z * split_stride) = sum over the z-th K range of X(i, k) Y(j, k),
// for rows i < mstore (all of a 4-row group stored at once) and columns j < N.
// X: tiled M x K (P, lo part Plo), Y: tiled N x K (Q, Qlo); nkb = ceil(K / 32).
template <int KIND, int NB, bool X3>
__global__ __launch_bounds__(LP_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm_lp_kernel(
    int64_t M, int64_t N, int64_t nkb, const unsigned short* __restrict__ P, const unsigned short* __restrict__ Plo,
    const unsigned short* __restrict__ Q, const unsigned short* __restrict__ Qlo, float* __restrict__ C, int64_t ldc,
    int64_t mstore, int64_t split_stride, LpGrid g) {
    constexpr int NP = X3 ? 2 : 1;                    // operand parts
    constexpr int NBUF = X3 ? (NB > 9 ? 2 : 3) : 4;   // LDS stages (register budget of the split form)
    constexpr int NBW = (NB + LP_WAVES - 1) / LP_WAVES;
    constexpr int OPS = NP * (NBW + 2);               // vector-memory instructions per wave and stage
    constexpr int STAGE = NP * NB * LP_BLK;
    __shared__ __attribute__((aligned(16))) unsigned short Ls[NBUF * STAGE + LP_BLK];   // + a sink kilobyte

    // tile of this workgroup: consecutive tiles on one XCD, the column tiles of
    // one row block adjacent (they read the same rows of X, which the XCD's L2
    // then serves to all but the first), then the row blocks, then the K ranges
    const int64_t L = blockIdx.x, slot = L >> 3;
    const int64_t t = (L & 7) * g.per_xcd + slot;
    if (slot >= g.per_xcd || t >= g.T) return;
    const int64_t by = t % g.tn, bx = (t / g.tn) % g.tm, bz = t / (g.tm * g.tn);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nrb = (M + 15) >> 4, ncb = (N + 15) >> 4;
    const int64_t kb0 = bz * g.kcb;
    const int64_t kb1 = (kb0 + g.kcb < nkb) ? kb0 + g.kcb : nkb;
    const int64_t nst = kb1 > kb0 ? kb1 - kb0 : 0;
    const u16x8_t* sink = (const u16x8_t*)(Q + lane * 8);

    float4_t acc[2][NB];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};

    // Y blocks this wave copies (b = wave, wave + 8, ...); slots past NB copy a
    // fixed chunk into the sink kilobyte so that every wave issues OPS copies.
    const unsigned short* qb[NP][NBW];
    int lofs[NP][NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
        const int b = wave + LP_WAVES * i;
        int64_t cb = by * NB + b;
        if (cb > ncb - 1) cb = ncb - 1;
#pragma unroll
        for (int h = 0; h < NP; ++h) {
            const unsigned short* base = h ? Qlo : Q;
            qb[h][i] = b < NB ? base + cb * nkb * LP_BLK + lane * 8 : nullptr;
            lofs[h][i] = b < NB ? (h * NB + b) * LP_BLK : NBUF * STAGE;
        }
    }
    // X block rows of this wave (clamped into the matrix; the extra rows are never stored)
    const unsigned short* pa[NP][2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        int64_t rb = bx * (2 * LP_WAVES) + wave * 2 + a;
        if (rb > nrb - 1) rb = nrb - 1;
#pragma unroll
        for (int h = 0; h < NP; ++h) pa[h][a] = (h ? Plo : P) + rb * nkb * LP_BLK + lane * 8;
    }
    u16x8_t ar[NBUF][NP][2];

    auto issue = [&](int s, int64_t kb) {
        if (kb > nkb - 1) kb = nkb - 1;               // stages past the range re-read the last block
        const int64_t ko = kb * LP_BLK;
#pragma unroll
        for (int h = 0; h < NP; ++h)
#pragma unroll
            for (int i = 0; i < NBW; ++i) {
                const void* src = qb[h][i] ? (const void*)(qb[h][i] + ko) : (const void*)sink;
                const int lo = lofs[h][i] < NBUF * STAGE ? s * STAGE + lofs[h][i] : NBUF * STAGE;
                __builtin_amdgcn_global_load_lds(src, RQLP_LDS_PTR(&Ls[lo]), 16, 0, 0);
            }
#pragma unroll
        for (int h = 0; h < NP; ++h)
#pragma unroll
            for (int a = 0; a < 2; ++a) ar[s][h][a] = *(const u16x8_t*)(pa[h][a] + ko);
    };
    auto step = [&](int u, int64_t j) {
        wait_vm<(NBUF - 2) * OPS>();                  // this wave's copies of stage j have landed
        RQLP_LDS_BARRIER();                           // ... and every wave's; stage j - 1 is free
        issue((u + NBUF - 1) % NBUF, kb0 + j + NBUF - 1);
        const unsigned short* Ly = &Ls[u * STAGE + lane * 8];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const u16x8_t bf = *(const u16x8_t*)(Ly + b * LP_BLK);
            if constexpr (X3) {
                const u16x8_t bl = *(const u16x8_t*)(Ly + (NB + b) * LP_BLK);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    acc[a][b] = mfma_lp<KIND>(ar[u][1][a], bf, acc[a][b]);
                    acc[a][b] = mfma_lp<KIND>(ar[u][0][a], bl, acc[a][b]);
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) acc[a][b] = mfma_lp<KIND>(ar[u][0][a], bf, acc[a][b]);
        }
    };

#pragma unroll
    for (int s = 0; s < NBUF - 1; ++s) issue(s, kb0 + s);
    int64_t j0 = 0;
    for (; j0 + NBUF <= nst; j0 += NBUF) {
#pragma unroll
        for (int u = 0; u < NBUF; ++u) step(u, j0 + u);
    }
#pragma unroll
    for (int u = 0; u < NBUF; ++u)
        if (j0 + u < nst) step(u, j0 + u);
    wait_vm<0>();                                     // no copy into LDS may outlive the workgroup

    // accumulator element r of lane l holds C(4 (l / 16) + r, l % 16): one 16-byte store per tile
    float* Cs = C + bz * split_stride;
    const int64_t m0 = bx * LP_BM + wave * 32 + 4 * (lane >> 4), n0 = by * 16 * NB + (lane & 15);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t i = m0 + a * 16;
        if (i >= mstore) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t j = n0 + b * 16;
            if (j < N) *(float4_t*)&Cs[i + j * ldc] = acc[a][b];
        }
    }
}

// C = 2^(gexp + rexp[i]) sum_s W_s (M x N FP32 partials with leading dimension
// ldw, fixed order; the exponents only for the IEEE half form, else NULL),
// converted to TO, written as C (M x N) or, transposed, as C^T (N x M) through
// 32 x 32 LDS tiles.  S = 0 writes zeros.
template <typename TO, bool TRANS>
__global__ __launch_bounds__(256) void lp_reduce_kernel(int64_t M, int64_t N, const float* __restrict__ W, int64_t ldw,
                                                        int64_t split_stride, int S, TO* __restrict__ C, int64_t ldc,
                                                        const int* __restrict__ rexp, const int* __restrict__ gexp) {
    __shared__ float tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int g = gexp ? *gexp : 0;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        float v0 = 0.f, v1 = 0.f;
        if (i < M && j < N) {
            const float* w = W + i + j * ldw;
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
constexpr int LP_NBS[] = {1, 2, 4, 6, 9, 12, 17};

struct LpPlan {
    int nb;
    LpGrid g;
};

LpPlan plan_lp(int64_t M, int64_t N, int64_t K) {
    LpPlan p;
    const int64_t nblk = ceil_div(N, 16);
    const int64_t ntiles = ceil_div(nblk, 17);
    const int64_t want_nb = ceil_div(nblk, ntiles);
    p.nb = 17;
    for (int v : LP_NBS)
        if (v >= want_nb) {
            p.nb = v;
            break;
        }
    LpGrid& g = p.g;
    g.tm = ceil_div(M, LP_BM);
    g.tn = ceil_div(N, 16 * p.nb);
    const int64_t nkb = ceil_div(K, 32);
    const int cus = device_info().num_cus > 0 ? device_info().num_cus : 256;
    // about one workgroup per CU (one is resident at a time: a second round only
    // doubled the partial sums written and read back, 6.68 -> 6.39 ms on the
    // 32768 x 16384 x 272 factorisation), at least 16 K blocks per split, and the
    // partial-sum traffic S M N below a quarter of the operand traffic K (M + N)
    int64_t S = ceil_div(cus, g.tm * g.tn);
    int64_t smax = ceil_div(nkb, 16);
    const int64_t straffic = (K * (M + N)) / (4 * M * N);
    if (smax > straffic) smax = straffic > 1 ? straffic : 1;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    g.kcb = nkb > 0 ? ceil_div(nkb, S) : 1;
    g.S = nkb > 0 ? ceil_div(nkb, g.kcb) : 1;
    g.T = g.tm * g.tn * g.S;
    g.per_xcd = ceil_div(g.T, 8);
    return p;
}

template <int KIND, bool X3>
void dispatch_lp(const LpPlan& p, int64_t M, int64_t N, int64_t nkb, const unsigned short* P,
                 const unsigned short* Plo, const unsigned short* Q, const unsigned short* Qlo, float* C, int64_t ldc,
                 int64_t mstore, int64_t ss, hipStream_t s) {
    const dim3 grid((unsigned)(8 * p.g.per_xcd));
    switch (p.nb) {
#define RQLP_LP_CASE(X)                                                                                         \
    case X:                                                                                                     \
        hipLaunchKernelGGL((gemm_lp_kernel<KIND, X, X3>), grid, dim3(LP_THREADS), 0, s, M, N, nkb, P, Plo, Q, Qlo, \
                           C, ldc, mstore, ss, p.g);                                                            \
        break;
        RQLP_LP_CASE(1) RQLP_LP_CASE(2) RQLP_LP_CASE(4) RQLP_LP_CASE(6) RQLP_LP_CASE(9) RQLP_LP_CASE(12)
        RQLP_LP_CASE(17)
#undef RQLP_LP_CASE
        default: break;
    }
}
}  // namespace

size_t lp_tiled_elems(int64_t rows, int64_t K) {
    if (rows <= 0 || K <= 0) return 0;
    return (size_t)(ceil_div(rows, 16) * 16) * (size_t)(ceil_div(K, 32) * 32);
}

size_t gemm_lp_workspace_elems(int64_t M, int64_t N, int64_t K) {
    LpPlan p = plan_lp(M, N, K);
    return (size_t)(p.g.S * ceil_div(M, 16) * 16 * N);
}

template <typename TO>
int gemm_lp(int kind, int64_t M, int64_t N, int64_t K, const unsigned short* P, const unsigned short* Plo,
            const unsigned short* Q, const unsigned short* Qlo, TO* C, int64_t ldc, bool trans_out, const int* rexp,
            const int* gexp, float* ws, size_t ws_elems, hipStream_t s) {
    if (M <= 0 || N <= 0) return 0;
    const bool x3 = (Plo != nullptr && Qlo != nullptr);
    if (x3 != (kind == RQLP_MIXED_BF16X3)) return RQLP_E_UNSUPPORTED;
    const dim3 rgrid((unsigned)ceil_div(M, 32), (unsigned)ceil_div(N, 32));
    auto reduce = [&](const float* W, int64_t ldw, int S) {
        if (trans_out)
            hipLaunchKernelGGL((lp_reduce_kernel<TO, true>), rgrid, dim3(256), 0, s, M, N, W, ldw, ldw * N, S, C, ldc,
                               rexp, gexp);
        else
            hipLaunchKernelGGL((lp_reduce_kernel<TO, false>), rgrid, dim3(256), 0, s, M, N, W, ldw, ldw * N, S, C, ldc,
                               rexp, gexp);
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    };
    if (K <= 0) return reduce(nullptr, M, 0);          // empty sum: zeros
    LpPlan p = plan_lp(M, N, K);
    const int64_t Mp = ceil_div(M, 16) * 16;
    const bool scaled = rexp != nullptr || gexp != nullptr;
    const bool direct = p.g.S == 1 && !trans_out && !scaled && sizeof(TO) == sizeof(float) && M % 4 == 0 &&
                        ldc % 4 == 0 && (((uintptr_t)C) & 15) == 0;
    float* dst = direct ? (float*)C : ws;
    const int64_t ld = direct ? ldc : Mp;
    if (!direct && ((size_t)(p.g.S * Mp * N) > ws_elems || ws == nullptr)) return RQLP_E_WORKSPACE;
    const int64_t nkb = ceil_div(K, 32), mstore = direct ? M : Mp;
    if (kind == RQLP_MIXED_FP16)
        dispatch_lp<RQLP_MIXED_FP16, false>(p, M, N, nkb, P, Plo, Q, Qlo, dst, ld, mstore, Mp * N, s);
    else if (x3)
        dispatch_lp<RQLP_MIXED_BF16, true>(p, M, N, nkb, P, Plo, Q, Qlo, dst, ld, mstore, Mp * N, s);
    else
        dispatch_lp<RQLP_MIXED_BF16, false>(p, M, N, nkb, P, Plo, Q, Qlo, dst, ld, mstore, Mp * N, s);
    if (hipGetLastError() != hipSuccess) return RQLP_E_HIP;
    return direct ? 0 : reduce(ws, Mp, (int)p.g.S);
}

template int gemm_lp<float>(int, int64_t, int64_t, int64_t, const unsigned short*, const unsigned short*,
                            const unsigned short*, const unsigned short*, float*, int64_t, bool, const int*,
                            const int*, float*, size_t, hipStream_t);
template int gemm_lp<double>(int, int64_t, int64_t, int64_t, const unsigned short*, const unsigned short*,
                             const unsigned short*, const unsigned short*, double*, int64_t, bool, const int*,
                             const int*, float*, size_t, hipStream_t);

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
// x -> (hi, lo) 16-bit patterns for `kind` (lo only for the split form)
__device__ __forceinline__ void encode16(int kind, bool split, float x, unsigned short& hi, unsigned short& lo) {
    if (kind == RQLP_MIXED_FP16) {
        hi = f32_to_f16_bits(x);
        lo = 0;
    } else {
        hi = f32_to_bf16_bits(x);
        lo = split ? f32_to_bf16_bits(x - bf16_bits_to_f32(hi)) : (unsigned short)0;
    }
}

// Fragment-tiled 16-bit copies of the m x n FP32 matrix A in one pass over A:
//   Tc: X = A^T (rows = columns of A, k = row index; the operand of A^T V),
//   Tr: X = A   (rows = rows of A,    k = column index; the operand of A W),
// each optional, with the split remainders (Tclo / Trlo, bf16x3) and the FP16
// column scaling 2^-cexp[j].  64 x 64 tiles of A through LDS; vec: 16-byte
// reads allowed (lda % 4 == 0, A 16-byte aligned).
__global__ __launch_bounds__(256) void encode_tiled_kernel(int64_t m, int64_t n, const float* __restrict__ A,
                                                           int64_t lda, int vec, unsigned short* __restrict__ Tc,
                                                           unsigned short* __restrict__ Tclo,
                                                           unsigned short* __restrict__ Tr,
                                                           unsigned short* __restrict__ Trlo, int kind,
                                                           const int* __restrict__ cexp) {
    typedef unsigned short u16x4_t __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) unsigned short t[2][64][64 + 8];   // [part][column j][row i]
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
    const bool split = Tclo != nullptr || Trlo != nullptr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = tid + 256 * e;
        const int cj = idx >> 4, ri = (idx & 15) * 4;
        const int64_t i = i0 + ri, j = j0 + cj;
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        if (j < n) {
            const float* a = A + i + j * lda;
            if (vec && i + 3 < m) {
                const float4_t v = *(const float4_t*)a;
                x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (i + q < m) x[q] = a[q];
            }
        }
        const int ex = (cexp && j < n) ? -cexp[j] : 0;
        u16x4_t hv, lv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float y = ex ? ldexpf(x[q], ex) : x[q];
            unsigned short h, l;
            encode16(kind, split, y, h, l);
            hv[q] = h;
            lv[q] = l;
        }
        *(u16x4_t*)&t[0][cj][ri] = hv;
        *(u16x4_t*)&t[1][cj][ri] = lv;
    }
    __syncthreads();
    // Tc blocks in this tile: 4 column groups (rows of X) x 2 row groups of 32 (k)
    if (Tc) {
        const int64_t nkb = (m + 31) >> 5, nrb = (n + 15) >> 4;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + 256 * e, blk = idx >> 6, ln = idx & 63;
            const int jb = blk & 3, ib = blk >> 2;
            const int64_t rb = (j0 >> 4) + jb, kb = (i0 >> 5) + ib;
            if (rb >= nrb || kb >= nkb) continue;
            const int jl = jb * 16 + (ln & 15), il = ib * 32 + 8 * (ln >> 4);
            const int64_t o = (rb * nkb + kb) * LP_BLK + ln * 8;
            *(u16x8_t*)(Tc + o) = *(const u16x8_t*)&t[0][jl][il];
            if (Tclo) *(u16x8_t*)(Tclo + o) = *(const u16x8_t*)&t[1][jl][il];
        }
    }
    // Tr blocks: 4 row groups of 16 (rows of X) x 2 column groups of 32 (k)
    if (Tr) {
        const int64_t nkb = (n + 31) >> 5, nrb = (m + 15) >> 4;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + 256 * e, blk = idx >> 6, ln = idx & 63;
            const int ib = blk & 3, jb = blk >> 2;
            const int64_t rb = (i0 >> 4) + ib, kb = (j0 >> 5) + jb;
            if (rb >= nrb || kb >= nkb) continue;
            const int il = ib * 16 + (ln & 15), jl = jb * 32 + 8 * (ln >> 4);
            const int64_t o = (rb * nkb + kb) * LP_BLK + ln * 8;
            u16x8_t v, vl;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                v[q] = t[0][jl + q][il];
                vl[q] = t[1][jl + q][il];
            }
            *(u16x8_t*)(Tr + o) = v;
            if (Trlo) *(u16x8_t*)(Trlo + o) = vl;
        }
    }
}

int encode_tiled(int kind, int64_t m, int64_t n, const float* A, int64_t lda, unsigned short* Tc,
                 unsigned short* Tclo, unsigned short* Tr, unsigned short* Trlo, const int* cexp, hipStream_t s) {
    if (m <= 0 || n <= 0) return 0;
    const bool x3 = kind == RQLP_MIXED_BF16X3;
    if ((Tc && x3 != (Tclo != nullptr)) || (Tr && x3 != (Trlo != nullptr))) return RQLP_E_UNSUPPORTED;
    const int vec = (lda % 4 == 0) && ((((uintptr_t)A) & 15) == 0);
    const dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(n, 64));
    hipLaunchKernelGGL(encode_tiled_kernel, grid, dim3(256), 0, s, m, n, A, lda, vec, Tc, Tc ? Tclo : nullptr, Tr,
                       Tr ? Trlo : nullptr, kind, cexp);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

// Fragment-tiled 16-bit copy of a panel operand X (R x K) with
// X(r, k) = 2^(kexp[k] - gexp) src(k + r ld) (src: column r of a K x R FP32
// panel; absent exponents count as 0); dlo: split remainders.  One thread per
// 16-byte chunk (8 consecutive k of one row).
__global__ __launch_bounds__(256) void cast_panel_kernel(int64_t R, int64_t K, const float* __restrict__ src,
                                                         int64_t ld, unsigned short* __restrict__ dst,
                                                         unsigned short* __restrict__ dlo, int kind,
                                                         const int* __restrict__ kexp,
                                                         const int* __restrict__ gexp, int vec) {
    const int64_t nkb = (K + 31) >> 5, nrb = (R + 15) >> 4;
    const int64_t chunks = nrb * nkb * 64;
    const int g = gexp ? *gexp : 0;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < chunks; idx += (int64_t)gridDim.x * 256) {
        const int64_t blk = idx >> 6;
        const int ln = (int)(idx & 63);
        const int64_t rb = blk / nkb, kb = blk - rb * nkb;
        const int64_t r = rb * 16 + (ln & 15), k0 = kb * 32 + 8 * (ln >> 4);
        u16x8_t v = {0, 0, 0, 0, 0, 0, 0, 0}, vl = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r < R) {
            const float* p = src + r * ld;
            float xs[8];
            if (vec && k0 + 8 <= K) {                    // two 16-byte loads
                const float4_t a = *(const float4_t*)(p + k0), b = *(const float4_t*)(p + k0 + 4);
                xs[0] = a[0]; xs[1] = a[1]; xs[2] = a[2]; xs[3] = a[3];
                xs[4] = b[0]; xs[5] = b[1]; xs[6] = b[2]; xs[7] = b[3];
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) xs[q] = (k0 + q < K) ? p[k0 + q] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t k = k0 + q;
                if (k < K) {
                    float x = xs[q];
                    const int e = (kexp ? kexp[k] : 0) - g;
                    if (e) x = ldexpf(x, e);
                    unsigned short h, l;
                    encode16(kind, dlo != nullptr, x, h, l);
                    v[q] = h;
                    vl[q] = l;
                }
            }
        }
        *(u16x8_t*)(dst + blk * LP_BLK + ln * 8) = v;
        if (dlo) *(u16x8_t*)(dlo + blk * LP_BLK + ln * 8) = vl;
    }
}

int cast_panel(int kind, int64_t R, int64_t K, const float* src, int64_t ld, unsigned short* dst, unsigned short* dlo,
               const int* kexp, const int* gexp, hipStream_t s) {
    if (R <= 0 || K <= 0) return 0;
    if ((kind == RQLP_MIXED_BF16X3) != (dlo != nullptr)) return RQLP_E_UNSUPPORTED;
    int64_t blocks = ceil_div(ceil_div(R, 16) * ceil_div(K, 32) * 64, 256);
    if (blocks > 16384) blocks = 16384;
    const int vec = (ld % 4 == 0) && ((((uintptr_t)src) & 15) == 0);
    hipLaunchKernelGGL(cast_panel_kernel, dim3((unsigned)blocks), dim3(256), 0, s, R, K, src, ld, dst, dlo, kind,
                       kexp, gexp, vec);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

// colexp[j] = e with max_i |A(i, j)| 2^-e in [2^14, 2^15) (0 for a zero or
// non-finite column); one workgroup per column, 16-byte loads when the
// columns are 16-byte aligned (vec).
__global__ __launch_bounds__(256) void colexp_kernel(int64_t rows, const float* __restrict__ A, int64_t lda,
                                                     int vec, int* __restrict__ colexp) {
    __shared__ float red[4];
    const int64_t j = blockIdx.x;
    const float* col = A + j * lda;
    float mx = 0.f;
    int64_t i = threadIdx.x;
    if (vec) {
        const int64_t r4 = rows >> 2;
        for (int64_t q = threadIdx.x; q < r4; q += 256) {
            const float4_t v = *(const float4_t*)(col + 4 * q);
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
        }
        i = 4 * r4 + threadIdx.x;
    }
    for (; i < rows; i += 256) mx = fmaxf(mx, fabsf(col[i]));
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
    int mx = -(1 << 30);
    for (int64_t j = threadIdx.x; j < n; j += 256) mx = max(mx, colexp[j]);
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) *gexp = max(max(red[0], red[1]), max(red[2], red[3]));
}

int column_exponents(int64_t rows, int64_t cols, const float* A, int64_t lda, int* colexp, int* gexp,
                     hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    const int vec = (lda % 4 == 0) && ((((uintptr_t)A) & 15) == 0);
    hipLaunchKernelGGL(colexp_kernel, dim3((unsigned)cols), dim3(256), 0, s, rows, A, lda, vec, colexp);
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
