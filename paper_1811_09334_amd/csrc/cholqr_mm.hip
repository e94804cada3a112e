// The two products of one CholeskyQR pass on a tall panel X (R x c,
// column-major, c <= 512), the orthonormalisation of the range finder
// (Algorithm 2.1, and the inner QR steps of Algorithm 2.2):
//   G = X^T X       Gram matrix, lower triangle only
//   Y = X L^{-T}    update with the inverse Cholesky factor (L^{-1} lower
//                   triangular, so Y(i, j) = sum_{k <= j} X(i, k) L^{-1}(j, k))
// in FP32 or FP64 on the gfx950 matrix cores (v_mfma_f32_16x16x4f32 /
// v_mfma_f64_16x16x4f64), accumulation in the input precision.
//
// Both kernels read X with 16-byte loads along its columns.  An MFMA operand
// lane holds one row index and one k index, so consecutive rows of a column
// normally sit in different lanes; here each lane instead loads VEC = 16 /
// sizeof(T) consecutive rows and feeds them to VEC MFMAs:
//   Gram: the contraction index is the row of X.  MFMA t of a 4 VEC-row
//     fragment takes rows VEC kappa + t (kappa = lane / 16), the same for
//     both operands, so the VEC MFMAs together sum over all rows of the
//     fragment.
//   Update: the row of X is the output row.  MFMA t takes the 16 rows
//     i0 + VEC rho + t (rho = lane % 16); the accumulators then hold VEC
//     consecutive rows of one output column per lane, stored as one 16-byte
//     vector.
//
// Gram kernel: a workgroup of 8 waves owns a range of row fragments (K split
// over workgroups, partial sums reduced in a fixed order by a second kernel
// that also adds the last R mod 4 VEC rows) and a set of lower 16 x 16 blocks
// of G (gr_bpw per wave).  Fragments of all needed column blocks are copied
// into LDS by the load unit (global_load_lds_dwordx4) GR_NBUF - 1 stages
// ahead, in the layout the MFMA reads with one conflict-free 16-byte load.
//
// Update kernel: a workgroup of 8 waves (two per SIMD: at c = 512 its LDS
// slice leaves room for one workgroup per CU, and a single wave per SIMD
// issued its MFMAs at half the peak rate) owns 16 VEC rows of Y; the rows of
// X (all 16 ceil(c / 16) columns) are copied into LDS once, then each wave
// sweeps k for its column blocks (every eighth block, highest first, so that
// the triangular work is spread over the waves; odd workgroups mirror the
// assignment so that consecutive workgroups load the SIMDs evenly),
// with the L^{-1} values of the next 16 k prefetched into registers.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

typedef double double2_t __attribute__((ext_vector_type(2)));

template <typename T>
struct CqMfma;

// Operand layouts: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16);
// accumulator element r of lane l holds D(row(l, r), l % 16).
template <>
struct CqMfma<float> {
    typedef float4_t acc_t;
    typedef float4_t vec_t;
    static constexpr int VEC = 4;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct CqMfma<double> {
    typedef double4_t acc_t;
    typedef double2_t vec_t;
    static constexpr int VEC = 2;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int GR_WAVES = 8;
constexpr int GR_THREADS = 64 * GR_WAVES;
constexpr int GR_NBUF = 4;          // LDS stages
// lower 16 x 16 blocks of G per wave: 10, or for wide FP32 panels 17 (as
// many as the registers of two waves per SIMD hold: every group of
// workgroups re-reads the panel, and at c = 512 the 528 blocks make 4
// groups instead of 7); narrower panels keep 10, which splits their blocks
// evenly over the groups (at c = 272: 80 + 73 rather than 136 + 17)
template <typename T>
inline int gr_bpw(int64_t c) { return (sizeof(T) == 4 && c > 384) ? 17 : 10; }
constexpr int GR_FRAG = 1024;       // bytes of one fragment (64 lanes x 16 bytes)
constexpr int CQ_MAXC = 512;

// lower block pair p = bi (bi + 1) / 2 + bj, bj <= bi (row-major order)
__host__ __device__ inline void cq_pair(int p, int& bi, int& bj) {
    int i = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    while (i * (i + 1) / 2 > p) --i;
    bi = i;
    bj = p - i * (i + 1) / 2;
}

// Partial Gram blocks of the row fragments [f0, f1) of this workgroup:
// ws[(split P + p) 256 + 4 lane + r] = accumulator r of lane l for pair p.
template <typename T, int OPS, int GR_BPW>
__global__ __launch_bounds__(GR_THREADS) void gram_kernel(int c, const T* __restrict__ X, int64_t ldx, int64_t nfrag,
                                                          int64_t fper, int P, T* __restrict__ ws,
                                                          const int32_t* __restrict__ gate) {
    typedef CqMfma<T> Mm;
    typedef typename Mm::acc_t acc_t;
    typedef typename Mm::vec_t vec_t;
    constexpr int VEC = Mm::VEC;
    constexpr int KF = 4 * VEC;                              // rows of one fragment
    constexpr int STAGE = GR_WAVES * OPS * GR_FRAG;
    __shared__ __attribute__((aligned(16))) char Ls[GR_NBUF * STAGE + GR_FRAG];   // + a sink fragment
    if (gate != nullptr && *gate == 0) return;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t f0 = (int64_t)blockIdx.x * fper;
    const int64_t f1 = (f0 + fper < nfrag) ? f0 + fper : nfrag;
    const int64_t nst = f1 - f0;
    const int pg0 = (int)blockIdx.y * GR_WAVES * GR_BPW;     // first pair of this workgroup
    const int pw0 = pg0 + wave * GR_BPW;                     // ... of this wave
    // column blocks this workgroup needs: 0 .. block row of its last pair
    int plast = pg0 + GR_WAVES * GR_BPW - 1;
    if (plast > P - 1) plast = P - 1;
    int bil = 0, bjl = 0;
    cq_pair(plast, bil, bjl);
    const int nbl = bil + 1;                                // column blocks 0 .. bil (bjl <= bil)

    // copy slots: block b = wave + 8 i; slots past nbl copy into the sink
    const char* src[OPS];
    int lofs[OPS];
#pragma unroll
    for (int i = 0; i < OPS; ++i) {
        const int b = wave + GR_WAVES * i;
        int col = 16 * b + (lane & 15);
        if (col > c - 1) col = c - 1;
        src[i] = (const char*)(X + (int64_t)col * ldx + VEC * (lane >> 4));
        lofs[i] = b < nbl ? b * GR_FRAG : GR_NBUF * STAGE;
    }
    // LDS byte offsets of the two operand fragments of each pair; slots past
    // the last pair compute block (0, 0) again and are not stored
    int oa[GR_BPW], ob[GR_BPW];
#pragma unroll
    for (int s = 0; s < GR_BPW; ++s) {
        const int p = pw0 + s;
        int bi = 0, bj = 0;
        if (p < P) cq_pair(p, bi, bj);
        oa[s] = bi * GR_FRAG;
        ob[s] = bj * GR_FRAG;
    }
    acc_t acc[GR_BPW];
#pragma unroll
    for (int s = 0; s < GR_BPW; ++s) acc[s] = acc_t{0, 0, 0, 0};

    auto issue = [&](int st, int64_t f) {
        if (f > f1 - 1) f = f1 - 1;                          // stages past the range re-read the last fragment
        const int64_t off = f * KF * (int64_t)sizeof(T);
#pragma unroll
        for (int i = 0; i < OPS; ++i) {
            const int lo = lofs[i] < GR_NBUF * STAGE ? st * STAGE + lofs[i] : GR_NBUF * STAGE;
            __builtin_amdgcn_global_load_lds((const void*)(src[i] + off), RQLP_LDS_PTR(Ls + lo), 16, 0, 0);
        }
    };
    auto step = [&](int u, int64_t j) {
        wait_vm<(GR_NBUF - 2) * OPS>();                      // this wave's copies of stage j have landed
        RQLP_LDS_BARRIER();                                  // ... and every wave's; stage j - 1 is free
        issue((u + GR_NBUF - 1) % GR_NBUF, f0 + j + GR_NBUF - 1);
        const char* Lb = Ls + u * STAGE + 16 * lane;
        vec_t a[GR_BPW], b[GR_BPW];
#pragma unroll
        for (int s = 0; s < GR_BPW; ++s) {
            a[s] = *(const vec_t*)(Lb + oa[s]);
            b[s] = *(const vec_t*)(Lb + ob[s]);
        }
        // t outer: consecutive MFMAs update different accumulators
#pragma unroll
        for (int t = 0; t < VEC; ++t)
#pragma unroll
            for (int s = 0; s < GR_BPW; ++s) acc[s] = Mm::op(a[s][t], b[s][t], acc[s]);
    };

#pragma unroll
    for (int s = 0; s < GR_NBUF - 1; ++s) issue(s, f0 + s);
    int64_t j0 = 0;
    for (; j0 + GR_NBUF <= nst; j0 += GR_NBUF) {
#pragma unroll
        for (int u = 0; u < GR_NBUF; ++u) step(u, j0 + u);
    }
#pragma unroll
    for (int u = 0; u < GR_NBUF; ++u)
        if (j0 + u < nst) step(u, j0 + u);
    wait_vm<0>();                                            // no copy into LDS may outlive the workgroup

    T* W = ws + (int64_t)blockIdx.x * P * 256 + 4 * lane;
#pragma unroll
    for (int s = 0; s < GR_BPW; ++s)
        if (pw0 + s < P) *(acc_t*)(W + (int64_t)(pw0 + s) * 256) = acc[s];
}

// G(i, j) for i >= j: the S partial sums of its pair, plus the rows R0 .. R-1
// that fill no whole fragment.  A workgroup takes 64 entries of one pair;
// wave h adds the splits s = h mod 4 in four interleaved chains, and the
// four wave sums are combined in a fixed order (reproducible results).
template <typename T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(int c, int P, int S, const T* __restrict__ ws, int64_t R0,
                                                          int64_t R, const T* __restrict__ X, int64_t ldx,
                                                          T* __restrict__ G, int64_t ldg,
                                                          const int32_t* __restrict__ gate) {
    if (gate != nullptr && *gate == 0) return;
    __shared__ T part[4][64];
    const int p = blockIdx.x >> 2, el = threadIdx.x & 63, h = threadIdx.x >> 6;
    const int e = (blockIdx.x & 3) * 64 + el;
    const T* w = ws + (int64_t)p * 256 + e;
    const int64_t stride = (int64_t)P * 256;
    T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
    int s = h;
    for (; s + 12 < S; s += 16) {
        v0 += w[s * stride];
        v1 += w[(s + 4) * stride];
        v2 += w[(s + 8) * stride];
        v3 += w[(s + 12) * stride];
    }
    for (; s < S; s += 4) v0 += w[s * stride];
    part[h][el] = (v0 + v1) + (v2 + v3);
    __syncthreads();
    if (h != 0) return;
    int bi, bj;
    cq_pair(p, bi, bj);
    const int lane = e >> 2, r = e & 3;
    const int ii = CqMfma<T>::row(lane, r), jj = lane & 15;
    if (bi == bj && jj > ii) return;
    const int i = 16 * bi + ii, j = 16 * bj + jj;
    if (i >= c) return;                                      // j <= i
    T v = (part[0][el] + part[1][el]) + (part[2][el] + part[3][el]);
    const T* xi = X + (int64_t)i * ldx;
    const T* xj = X + (int64_t)j * ldx;
    for (int64_t k = R0; k < R; ++k) v += xi[k] * xj[k];
    G[i + (int64_t)j * ldg] = v;
}

constexpr int TR_WAVES = 8;        // two waves per SIMD: one workgroup per CU fills the LDS
constexpr int TR_THREADS = 64 * TR_WAVES;

// Y = X L^{-T} for the 16 VEC rows of this workgroup; Li = L^{-1} (c x c lower
// triangular, its strict upper part is not read).  gate: when *gate is 0
// nothing is computed, or with gate_copy the rows of X are copied to Y.
template <typename T, int MAXB>
__global__ __launch_bounds__(TR_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void trmm_kernel(
    int64_t R, int c, const T* X, int64_t ldx, const T* __restrict__ Li, int64_t ldl,
    T* Y, int64_t ldy, const int32_t* __restrict__ gate, int gate_copy) {
    typedef CqMfma<T> Mm;
    typedef typename Mm::acc_t acc_t;
    typedef typename Mm::vec_t vec_t;
    constexpr int VEC = Mm::VEC;
    constexpr int RT = 16 * VEC;                             // rows per workgroup: one 256-byte column slice
    extern __shared__ __attribute__((aligned(16))) char Xs[];   // column k of the slice at 256 k bytes

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t i0 = (int64_t)blockIdx.x * RT;
    if (gate != nullptr && *gate == 0) {
        if (gate_copy) {
            constexpr int NV = RT / VEC;
            for (int idx = tid; idx < c * NV; idx += TR_THREADS) {
                const int64_t col = idx / NV, row = i0 + VEC * (idx % NV);
                if (row < R) *(vec_t*)(Y + col * ldy + row) = *(const vec_t*)(X + col * ldx + row);
            }
        }
        return;
    }
    const int nb = (c + 15) >> 4;
    // rows of X into LDS, 4 columns per copy; columns past c repeat column c - 1
    // (their L^{-1} factors are zero) and rows past R repeat the last vector
    // (those outputs are not stored)
    {
        int64_t row = i0 + VEC * (lane & 15);
        if (row > R - VEC) row = R - VEC;
        for (int q = wave; q < 4 * nb; q += TR_WAVES) {
            int col = 4 * q + (lane >> 4);
            if (col > c - 1) col = c - 1;
            __builtin_amdgcn_global_load_lds((const void*)(X + (int64_t)col * ldx + row), RQLP_LDS_PTR(Xs + q * 1024),
                                             16, 0, 0);
        }
    }
    // column blocks of this wave: b_q = bmax - TR_WAVES q
    const int wsel = (blockIdx.x & 1) ? TR_WAVES - 1 - wave : wave;
    const int bmax = nb - 1 - wsel;
    const int kend = (16 * bmax + 16 < c) ? 16 * bmax + 16 : c;
    const int ng = bmax >= 0 ? (kend + 15) >> 4 : 0;         // groups of 16 k

    acc_t acc[MAXB][VEC];
#pragma unroll
    for (int q = 0; q < MAXB; ++q)
#pragma unroll
        for (int t = 0; t < VEC; ++t) acc[q][t] = acc_t{0, 0, 0, 0};
    T b0[MAXB][4], b1[MAXB][4];
    // L^{-1}(j, k) for k = 16 g + 4 (lane / 16) + s, j = 16 b_q + lane % 16,
    // loaded raw from clamped addresses (32-bit offsets: c <= 512) so that the
    // loads stay in flight; the diagonal group masks k > j at use (k >= c only
    // occurs there), and columns j >= c are computed but never stored
    const int ldl32 = (int)ldl;
    auto load_b = [&](T (&bq)[MAXB][4], int g) {
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int b = bmax - TR_WAVES * q;
            const int j = 16 * b + (lane & 15);
            const int jc = j < 0 ? 0 : (j < c ? j : c - 1);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * g + 4 * (lane >> 4) + s;
                const int kc = k < c ? k : c - 1;
                bq[q][s] = Li[jc + kc * ldl32];
            }
        }
    };
    auto step = [&](const T (&bq)[MAXB][4], int g) {
        vec_t a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            a[s] = *(const vec_t*)(Xs + (16 * g + 4 * (lane >> 4) + s) * 256 + 16 * (lane & 15));
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int b = bmax - TR_WAVES * q;
            if (b < g) continue;                             // block done: k past its last column
            const bool diag = b == g;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * g + 4 * (lane >> 4) + s;
                const T bv = (!diag || k <= 16 * b + (lane & 15)) ? bq[q][s] : T(0);
#pragma unroll
                for (int t = 0; t < VEC; ++t) acc[q][t] = Mm::op(a[s][t], bv, acc[q][t]);
            }
        }
    };
    if (ng > 0) load_b(b0, 0);
    __syncthreads();                                         // X rows in LDS (waits for every copy)
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) load_b(b1, g + 1);
        step(b0, g);
        if (g + 1 >= ng) break;
        if (g + 2 < ng) load_b(b0, g + 2);
        step(b1, g + 1);
    }

    // lane l holds rows i0 + VEC row(l, r) + t (t < VEC) of column 16 b_q + l % 16
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int b = bmax - TR_WAVES * q;
        const int j = 16 * b + (lane & 15);
        if (b < 0 || j >= c) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = i0 + VEC * Mm::row(lane, r);
            if (row >= R) continue;
            vec_t v;
#pragma unroll
            for (int t = 0; t < VEC; ++t) v[t] = acc[q][t][r];
            *(vec_t*)(Y + (int64_t)j * ldy + row) = v;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
struct GramPlan {
    int nb, P, groups, ops;
    int64_t nfrag, fper, S;
};

GramPlan plan_gram(int64_t R, int64_t c, int kf, int bpw) {
    GramPlan p;
    p.nb = (int)((c + 15) / 16);
    p.P = p.nb * (p.nb + 1) / 2;
    p.groups = (int)ceil_div(p.P, GR_WAVES * bpw);
    p.ops = (int)ceil_div(p.nb, GR_WAVES);
    p.nfrag = R > 0 ? R / kf : 0;
    const int cus = device_info().num_cus > 0 ? device_info().num_cus : 256;
    int64_t want = cus / p.groups;                           // one workgroup per CU
    if (want < 1) want = 1;
    p.S = p.nfrag < want ? p.nfrag : want;
    p.fper = 0;
    if (p.S > 0) {
        p.fper = ceil_div(p.nfrag, p.S);
        p.S = ceil_div(p.nfrag, p.fper);
    }
    return p;
}

template <typename T, int OPS, int BPW>
void launch_gram(const GramPlan& p, int64_t c, const T* X, int64_t ldx, T* ws, const int32_t* gate, hipStream_t s) {
    hipLaunchKernelGGL((gram_kernel<T, OPS, BPW>), dim3((unsigned)p.S, (unsigned)p.groups), dim3(GR_THREADS), 0, s,
                       (int)c, X, ldx, p.nfrag, p.fper, p.P, ws, gate);
}

template <typename T, int MAXB>
int launch_trmm(int64_t R, int64_t c, const T* X, int64_t ldx, const T* Li, int64_t ldl, T* Y, int64_t ldy,
                const int32_t* gate, int gate_copy, hipStream_t s) {
    RQLP_TRY(raise_lds_limit((const void*)trmm_kernel<T, MAXB>, 4096 * (CQ_MAXC / 16)));
    constexpr int RT = 16 * CqMfma<T>::VEC;
    const size_t lds = 4096 * (size_t)ceil_div(c, 16);
    hipLaunchKernelGGL((trmm_kernel<T, MAXB>), dim3((unsigned)ceil_div(R, RT)), dim3(TR_THREADS), lds, s, R, (int)c,
                       X, ldx, Li, ldl, Y, ldy, gate, gate_copy);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
}  // namespace

size_t gram_workspace_elems(int64_t R, int64_t c) {
    if (c <= 0 || c > CQ_MAXC) return 0;
    // the larger of the FP64 and FP32 plans
    const GramPlan p64 = plan_gram(R, c, 8, gr_bpw<double>(c)), p32 = plan_gram(R, c, 16, gr_bpw<float>(c));
    const size_t e64 = (size_t)(p64.S * p64.P * 256), e32 = (size_t)(p32.S * p32.P * 256);
    return e64 > e32 ? e64 : e32;
}

template <typename T>
bool gram_fits(int64_t R, int64_t c, const T* X, int64_t ldx, const T* ws, size_t ws_elems) {
    constexpr int VEC = CqMfma<T>::VEC;
    if (c <= 0 || c > CQ_MAXC || R < 0 || !aligned16(X) || ldx % VEC != 0) return false;
    const GramPlan p = plan_gram(R, c, 4 * VEC, gr_bpw<T>(c));
    return p.S == 0 || (ws != nullptr && (size_t)(p.S * p.P * 256) <= ws_elems);
}

template <typename T>
int gram(int64_t R, int64_t c, const T* X, int64_t ldx, T* G, int64_t ldg, T* ws, size_t ws_elems, hipStream_t s,
         const int32_t* gate) {
    if (c <= 0) return 0;
    if (!gram_fits<T>(R, c, X, ldx, ws, ws_elems)) return RQLP_E_UNSUPPORTED;
    constexpr int KF = 4 * CqMfma<T>::VEC;
    const int bpw = gr_bpw<T>(c);
    const GramPlan p = plan_gram(R, c, KF, bpw);
    if (p.S > 0) {
        if (bpw == 17) {
            // (c > 384: four copy slots per wave)
            if constexpr (sizeof(T) == 4) launch_gram<T, 4, 17>(p, c, X, ldx, ws, gate, s);
        } else {
            switch (p.ops) {
                case 1: launch_gram<T, 1, 10>(p, c, X, ldx, ws, gate, s); break;
                case 2: launch_gram<T, 2, 10>(p, c, X, ldx, ws, gate, s); break;
                case 3: launch_gram<T, 3, 10>(p, c, X, ldx, ws, gate, s); break;
                default: launch_gram<T, 4, 10>(p, c, X, ldx, ws, gate, s); break;
            }
        }
    }
    hipLaunchKernelGGL((gram_reduce_kernel<T>), dim3((unsigned)(4 * p.P)), dim3(256), 0, s, (int)c, p.P, (int)p.S, ws,
                       p.nfrag * KF, R, X, ldx, G, ldg, gate);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

template <typename T>
bool trmm_fits(int64_t R, int64_t c, const T* X, int64_t ldx, const T* Y, int64_t ldy) {
    constexpr int VEC = CqMfma<T>::VEC;
    const int64_t cmax = CQ_MAXC;
    // a workgroup per 16 VEC rows: below 16 workgroups the general product is faster
    // (Y may be X itself: a workgroup reads all of its rows into LDS, waits
    // for every copy, and only then writes those same rows)
    return c >= 1 && c <= cmax && R >= 16 * 16 * VEC && R % VEC == 0 && ldx % VEC == 0 && ldy % VEC == 0 &&
           aligned16(X) && aligned16(Y) && (X != Y || ldx == ldy);
}

template <typename T>
int trmm_lt(int64_t R, int64_t c, const T* X, int64_t ldx, const T* Li, int64_t ldl, T* Y, int64_t ldy,
            hipStream_t s, const int32_t* gate, int gate_mode) {
    if (R <= 0 || c <= 0) return 0;
    if (!trmm_fits<T>(R, c, X, ldx, Y, ldy) || ldl < c || ldl > (1 << 20)) return RQLP_E_UNSUPPORTED;
    const int gc = gate_mode == 2 ? 1 : 0;
    switch ((int)ceil_div(ceil_div(c, 16), TR_WAVES)) {
        case 1: return launch_trmm<T, 1>(R, c, X, ldx, Li, ldl, Y, ldy, gate, gc, s);
        case 2: return launch_trmm<T, 2>(R, c, X, ldx, Li, ldl, Y, ldy, gate, gc, s);
        case 3: return launch_trmm<T, 3>(R, c, X, ldx, Li, ldl, Y, ldy, gate, gc, s);
        default: return launch_trmm<T, 4>(R, c, X, ldx, Li, ldl, Y, ldy, gate, gc, s);
    }
}

template bool gram_fits<float>(int64_t, int64_t, const float*, int64_t, const float*, size_t);
template bool gram_fits<double>(int64_t, int64_t, const double*, int64_t, const double*, size_t);
template int gram<float>(int64_t, int64_t, const float*, int64_t, float*, int64_t, float*, size_t, hipStream_t,
                         const int32_t*);
template int gram<double>(int64_t, int64_t, const double*, int64_t, double*, int64_t, double*, size_t, hipStream_t,
                          const int32_t*);
template bool trmm_fits<float>(int64_t, int64_t, const float*, int64_t, const float*, int64_t);
template bool trmm_fits<double>(int64_t, int64_t, const double*, int64_t, const double*, int64_t);
template int trmm_lt<float>(int64_t, int64_t, const float*, int64_t, const float*, int64_t, float*, int64_t,
                            hipStream_t, const int32_t*, int);
template int trmm_lt<double>(int64_t, int64_t, const double*, int64_t, const double*, int64_t, double*, int64_t,
                             hipStream_t, const int32_t*, int);

}  // namespace rqlp
