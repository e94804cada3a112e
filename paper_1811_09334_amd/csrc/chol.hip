// Cholesky factor and its inverse for CholeskyQR (the orthonormalisation of
// the range finder in Algorithm 2.1, and the inner QR steps of
// Algorithm 2.2, realised as CholeskyQR2: Fukaya, Nakatsukasa, Yanagisawa,
// Yamamoto 2014; shifted retry per Fukaya, Kannan, Nakatsukasa, Zhang,
// Yamamoto 2020).
//
// One workgroup of 512 threads factors the c x c Gram matrix G = L L^T with a
// right-looking blocked algorithm (16-column blocks) and, fused into the same
// sweep, solves L X = I for X = L^{-1} (right-looking block forward
// substitution sharing the panel).  Per block step:
//   (1) the 16 x 16 diagonal block is factored and inverted by one wave in
//       LDS (unblocked, wave-synchronous: no workgroup barrier per column);
//   (3) the panel L(J0:c, K) = W(J0:c, K) L_KK^{-T} and the block row
//       X(K, 0:J0) = L_KK^{-1} X(K, 0:J0), and
//   (4) the trailing updates W -= L(:,K) L(:,K)^T and X -= L(:,K) X(K,:),
//       all as 16 x 16 FP64 MFMA tiles distributed over the 8 waves, the
//       panel and the block row read from LDS (up to 256 rows / columns
//       cached; beyond that from the L2-resident scratch).
// Loops are kept compact on purpose: fully unrolled triangular loops here
// overflow the instruction cache and run several times slower.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

// Orders LDS traffic between the lanes of one wave: DS instructions of a wave
// execute in order, so only the compiler must be kept from reordering.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int CH_NB = 16;                 // block size (multiple of 16: one MFMA tile)
constexpr int CH_NBT = CH_NB / 16;
constexpr int CH_T = 512;
constexpr int CH_PMAX = 256;
constexpr int CH_XMAX = 256;
constexpr int CH_PS = CH_NB + 1;

static inline int ch_prows(int64_t c) { return (int)(c < CH_PMAX ? c : CH_PMAX); }
static inline int ch_xcols(int64_t c) { return (int)(c < CH_XMAX ? c : CH_XMAX); }

// at least one block of panel rows is allocated
static inline int ch_prows_alloc(int64_t c) { return ch_prows(c) > CH_NB ? ch_prows(c) : CH_NB; }

size_t chol_inv_lds_bytes(int64_t c) {
    return sizeof(double) *
           (size_t)(2 * CH_NB * CH_PS + ch_prows_alloc(c) * CH_PS + CH_NB * (ch_xcols(c) + 1));
}

template <typename TG>
__global__ __launch_bounds__(CH_T) void chol_inv_kernel(int c, const TG* __restrict__ G, int64_t ldg,
                                                        double shift_scale, double* __restrict__ W,
                                                        double* __restrict__ X, float* __restrict__ Xf,
                                                        int64_t ldw, int32_t* info, int prows, int xcols,
                                                        const int32_t* __restrict__ run_flag,
                                                        int32_t* __restrict__ shifted_out, int shifted_mode,
                                                        double pivot_rel) {
    extern __shared__ double lds[];
    double* D = lds;                           // [NB][NB+1] factored diagonal block
    double* Dinv = D + CH_NB * CH_PS;          // [NB][NB+1] its inverse
    double* P = Dinv + CH_NB * CH_PS;          // [prows][33] panel rows J0..
    double* XK = P + (size_t)(prows > CH_NB ? prows : CH_NB) * CH_PS;   // [NB][xcols + 1] block row of X
    const int xs = xcols + 1;
    __shared__ int s_bad;
    __shared__ double s_red[CH_T / 64];
    __shared__ double s_trace;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NWAVE = CH_T / 64;

    // conditional pass: when *run_flag is 0 the factor is the identity
    if (run_flag && *run_flag == 0) {
        for (int j = wave; j < c; j += NWAVE)
            for (int i = lane; i < c; i += 64) {
                const double v = (i == j) ? 1.0 : 0.0;
                W[i + (int64_t)j * ldw] = v;
                X[i + (int64_t)j * ldw] = v;
                if (Xf) Xf[i + (int64_t)j * ldw] = (float)v;
            }
        return;
    }

    // trace(G) for the shift
    {
        double t = 0.0;
        for (int i = tid; i < c; i += CH_T) t += (double)G[i + i * ldg];
        t = wave_sum(t);
        if (lane == 0) s_red[wave] = t;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NWAVE; ++w) s += s_red[w];
            s_trace = s;
        }
        __syncthreads();
    }

    int attempt = 0;
    for (; attempt < 2; ++attempt) {
        // a zero Gram matrix (X = 0) gets a unit shift: its factor is then I
        const double shift = attempt == 0 ? 0.0 : (s_trace == 0.0 ? 1.0 : shift_scale * s_trace);
        for (int j = wave; j < c; j += NWAVE) {
            for (int i = lane; i < c; i += 64) {
                if (i >= j) W[i + (int64_t)j * ldw] = (double)G[i + (int64_t)j * ldg] + (i == j ? shift : 0.0);
                X[i + (int64_t)j * ldw] = (i == j) ? 1.0 : 0.0;
            }
        }
        if (tid == 0) s_bad = 0;
        __syncthreads();

        for (int K0 = 0; K0 < c; K0 += CH_NB) {
            const int kb = (c - K0) < CH_NB ? (c - K0) : CH_NB;
            const int J0 = K0 + kb;
            // ---- (1) diagonal block factor and inverse: one wave, LDS-resident,
            // wave-synchronous (DS operations of one wave complete in order) ----
            for (int idx = tid; idx < CH_NB * CH_NB; idx += CH_T) {
                const int i = idx % CH_NB, j = idx / CH_NB;
                D[i * CH_PS + j] = (i < kb && j < kb && i >= j) ? W[(K0 + i) + (int64_t)(K0 + j) * ldw] : 0.0;
                Dinv[i * CH_PS + j] = (i == j && i < kb) ? 1.0 : 0.0;
            }
            __syncthreads();
            if (wave == 0) {
                int bad = 0;
                for (int j = 0; j < kb; ++j) {
                    const double pj = D[j * CH_PS + j];
                    // plain attempt: a pivot below pivot_rel times the column's
                    // squared norm marks a numerically dependent column
                    const double thr = attempt == 0 ? pivot_rel * (double)G[(K0 + j) + (int64_t)(K0 + j) * ldg] : 0.0;
                    const bool ok = (pj > thr) && (pj > 0.0) && (pj < 1.0e308);
                    bad |= !ok;
                    const double sj = ok ? sqrt(pj) : 1.0;
                    wave_sync();
                    if (lane == j) D[j * CH_PS + j] = sj;
                    else if (lane > j && lane < kb) D[lane * CH_PS + j] /= sj;
                    wave_sync();
                    // all loads first, then the stores (loads may not pass stores)
                    double u[CH_NB * CH_NB / 64];
#pragma unroll
                    for (int e = 0; e < CH_NB * CH_NB / 64; ++e) {
                        const int idx = lane + 64 * e;
                        const int i = idx % CH_NB, jj = idx / CH_NB;
                        u[e] = D[i * CH_PS + jj] - D[i * CH_PS + j] * D[jj * CH_PS + j];
                    }
#pragma unroll
                    for (int e = 0; e < CH_NB * CH_NB / 64; ++e) {
                        const int idx = lane + 64 * e;
                        const int i = idx % CH_NB, jj = idx / CH_NB;
                        if (jj > j && i >= jj && i < kb) D[i * CH_PS + jj] = u[e];
                    }
                    wave_sync();
                }
                for (int t = 0; t < kb; ++t) {
                    const double rt = 1.0 / D[t * CH_PS + t];
                    wave_sync();
                    if (lane <= t) Dinv[t * CH_PS + lane] *= rt;
                    wave_sync();
                    double u[CH_NB * CH_NB / 64];
#pragma unroll
                    for (int e = 0; e < CH_NB * CH_NB / 64; ++e) {
                        const int idx = lane + 64 * e;
                        const int i = idx % CH_NB, jj = idx / CH_NB;
                        u[e] = Dinv[i * CH_PS + jj] - D[i * CH_PS + t] * Dinv[t * CH_PS + jj];
                    }
#pragma unroll
                    for (int e = 0; e < CH_NB * CH_NB / 64; ++e) {
                        const int idx = lane + 64 * e;
                        const int i = idx % CH_NB, jj = idx / CH_NB;
                        if (i > t && i < kb && jj <= t) Dinv[i * CH_PS + jj] = u[e];
                    }
                    wave_sync();
                }
                if (lane == 0) s_bad = bad;
            }
            __syncthreads();
            if (s_bad) break;
            // L_KK into W
            for (int idx = tid; idx < CH_NB * CH_NB; idx += CH_T) {
                const int i = idx % CH_NB, j = idx / CH_NB;
                if (i < kb && j < kb && i >= j) W[(K0 + i) + (int64_t)(K0 + j) * ldw] = D[i * CH_PS + j];
            }
            __syncthreads();
            // MFMA fragment helpers (v_mfma_f64_16x16x4f64): lane l holds
            // A(l % 16, k) and B(k, l % 16) with k = 4 ks + l / 16; accumulator
            // element r of lane l is C(l / 16 + 4 r, l % 16).
            const int fr = lane & 15, fk = lane >> 4;
            // L(i, K0 + k) for i >= J0: from the LDS panel (zero-padded past c
            // and kb) when all rows are cached, else from the scratch copy
            const bool all_cached = (c - J0) <= prows - 16;
            auto panel = [&](int i, int k) -> double {
                double v = 0.0;
                if (all_cached || (i < c && k < kb && i - J0 < prows)) {
                    v = P[(i - J0) * CH_PS + k];
                } else if (i < c && k < kb) {
                    v = W[i + (int64_t)(K0 + k) * ldw];
                }
                return v;
            };
            // ---- (3a) panel L(J0:c, K) = W(J0:c, K) Dinv^T ----
            {
                const int nti = (c - J0 + 15) >> 4;
                for (int tile = wave; tile < nti * CH_NBT; tile += NWAVE) {
                    const int i0 = J0 + 16 * (tile / CH_NBT), s0 = 16 * (tile % CH_NBT);
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < CH_NB / 4; ++ks) {
                        const int i = i0 + fr, k = 4 * ks + fk;
                        const double a = (i < c && k < kb) ? W[i + (int64_t)(K0 + k) * ldw] : 0.0;
                        const double bb = Dinv[(s0 + fr) * CH_PS + k];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
                    }
                    // all loads of W(i, K) by this wave are done before it writes L(i, K)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + fk + 4 * r, sx = s0 + fr;
                        if (i < c && sx < kb) W[i + (int64_t)(K0 + sx) * ldw] = acc[r];
                        if (i - J0 < prows) P[(i - J0) * CH_PS + sx] = (i < c && sx < kb) ? acc[r] : 0.0;
                    }
                }
            }
            // ---- (3b) block row of the inverse: X(K, 0:J0) = Dinv X(K, 0:J0) ----
            {
                const int ntj = (J0 + 15) >> 4;
                for (int tile = wave; tile < ntj * CH_NBT; tile += NWAVE) {
                    const int s0 = 16 * (tile % CH_NBT), j0 = 16 * (tile / CH_NBT);
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < CH_NB / 4; ++ks) {
                        const int k = 4 * ks + fk, j = j0 + fr;
                        const double a = Dinv[(s0 + fr) * CH_PS + k];
                        const double bb = (j < J0 && k < kb) ? X[(K0 + k) + (int64_t)j * ldw] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int sx = s0 + fk + 4 * r, j = j0 + fr;
                        if (sx < kb && j < J0) X[(K0 + sx) + (int64_t)j * ldw] = acc[r];
                        if (j < xcols) XK[sx * xs + j] = (sx < kb && j < J0) ? acc[r] : 0.0;
                    }
                }
            }
            __syncthreads();
            if (J0 >= c) break;
            // ---- (4a) trailing update W(i, j) -= L(i, K) L(j, K)^T, J0 <= j <= i < c ----
            {
                const int nt = (c - J0 + 15) >> 4;
                const int T = nt * (nt + 1) / 2;
                for (int idx = wave; idx < T; idx += NWAVE) {
                    int ti = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
                    while (ti * (ti + 1) / 2 > idx) --ti;
                    while ((ti + 1) * (ti + 2) / 2 <= idx) ++ti;
                    const int tj = idx - ti * (ti + 1) / 2;
                    const int i0 = J0 + 16 * ti, j0 = J0 + 16 * tj;
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < CH_NB / 4; ++ks) {
                        const int k = 4 * ks + fk;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(panel(i0 + fr, k), panel(j0 + fr, k), acc,
                                                                   0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + fk + 4 * r, j = j0 + fr;
                        if (i < c && j < c && i >= j) W[i + (int64_t)j * ldw] -= acc[r];
                    }
                }
            }
            // ---- (4b) inverse update X(i, j) -= L(i, K) X(K, j), i >= J0, j < J0 ----
            {
                const int nti = (c - J0 + 15) >> 4, ntj = (J0 + 15) >> 4;
                for (int idx = wave; idx < nti * ntj; idx += NWAVE) {
                    const int ti = idx / ntj, tj = idx - (idx / ntj) * ntj;
                    const int i0 = J0 + 16 * ti, j0 = 16 * tj;
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < CH_NB / 4; ++ks) {
                        const int k = 4 * ks + fk, j = j0 + fr;
                        double bb = 0.0;
                        if (j < J0 && k < kb) {
                            if (j < xcols) bb = XK[k * xs + j];
                            else bb = X[(K0 + k) + (int64_t)j * ldw];
                        }
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(panel(i0 + fr, k), bb, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + fk + 4 * r, j = j0 + fr;
                        if (i < c && j < J0) X[i + (int64_t)j * ldw] -= acc[r];
                    }
                }
            }
            __syncthreads();
        }
        if (!s_bad) break;
        if (tid == 0 && info) atomicOr(info, attempt == 0 ? RQLP_INFO_CHOLQR_SHIFTED : RQLP_INFO_CHOL_FAILED);
        __syncthreads();
    }
    __syncthreads();
    // outputs are the working buffers themselves: W holds L (lower), X holds
    // L^{-1} (lower; its strictly upper part is zero); zero W's upper part.
    for (int j = wave; j < c; j += NWAVE)
        for (int i = lane; i < j; i += 64) W[i + (int64_t)j * ldw] = 0.0;
    if (shifted_out && tid == 0 && (shifted_mode == 1 || attempt > 0)) *shifted_out = attempt > 0 ? 1 : 0;
    // optional FP32 copy of L^{-1} for FP32 panel updates
    if (Xf)
        for (int j = wave; j < c; j += NWAVE)
            for (int i = lane; i < c; i += 64) Xf[i + (int64_t)j * ldw] = (float)X[i + (int64_t)j * ldw];
}

// ---------------------------------------------------------------------------
// Near-identity form.  The second pass of CholeskyQR2 (and the CholeskyQR
// after the second projection of block Gram-Schmidt) sees G = I + E with
// ||E||_F around 1e-6 for FP32 panels and 1e-13 for FP64 ones.  Then
// L = I + Phi(E) and L^{-1} = I - Phi(E), where Phi(E) is the strict lower
// triangle of E plus half its diagonal, are exact to about 2 ||E||_F^2:
// L L^T = I + E + Phi(E) Phi(E)^T, and (I + Phi(E)) (I - Phi(E)) =
// I - Phi(E)^2.  The first kernel writes both and one partial sum of
// ||E||_F^2 per 32 x 32 tile; the second sums the partials in a fixed order
// and keeps the result when ||E||_F <= tau (2 tau^2 at most 1/16 of the unit
// roundoff of G's arithmetic), else it sets the flag on which the full
// factorisation then runs and overwrites every output.
constexpr int NI_T = 256;

template <typename TG>
__global__ __launch_bounds__(NI_T) void nearid_kernel(int c, const TG* __restrict__ G, int64_t ldg,
                                                      double* __restrict__ L, double* __restrict__ Linv,
                                                      float* __restrict__ Linv32, int64_t ld,
                                                      double* __restrict__ part) {
    __shared__ double red[NI_T / 64];
    const int nt = (c + 31) >> 5;
    const int ti = (int)blockIdx.x % nt, tj = (int)blockIdx.x / nt;
    double ss = 0.0;
    for (int q = threadIdx.x; q < 1024; q += NI_T) {
        const int i = 32 * ti + (q & 31), j = 32 * tj + (q >> 5);
        if (i >= c || j >= c) continue;
        double phi = 0.0;
        if (i >= j) {                                   // (lower triangle of G read)
            const double e = (double)G[i + (int64_t)j * ldg] - (i == j ? 1.0 : 0.0);
            ss += (i == j) ? e * e : 2.0 * e * e;
            phi = (i == j) ? 0.5 * e : e;
        }
        const double d = (i == j) ? 1.0 : 0.0;
        const double li = d - phi;
        L[i + (int64_t)j * ld] = d + phi;
        Linv[i + (int64_t)j * ld] = li;
        if (Linv32) Linv32[i + (int64_t)j * ld] = (float)li;
    }
    ss = wave_sum(ss);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void nearid_decide_kernel(int nparts, const double* __restrict__ part, double tau2,
                                                           int32_t* need_full, int32_t* shifted_out,
                                                           int shifted_mode) {
    double t = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 64) t += part[k];
    t = wave_sum(t);
    if (threadIdx.x == 0) {
        const bool ok = t <= tau2;                      // (NaN: the full factorisation)
        *need_full = ok ? 0 : 1;
        // the pass used no shift (the full factorisation writes the word itself)
        if (ok && shifted_out && shifted_mode == 1) *shifted_out = 0;
    }
}

template <typename TG>
int chol_inv(int64_t c, const TG* G, int64_t ldg, double* L, double* Linv, float* Linv32, int64_t ld,
             double shift_scale, int32_t* info, hipStream_t s, const int32_t* run_flag, int32_t* shifted_out,
             unsigned* sync, int shifted_mode, double pivot_rel, bool near_identity) {
    if (c <= 0) return 0;
    if (near_identity && sync && c <= CHOL_MW_MAXC && run_flag == nullptr) {
        // tau: FP32 4e-5 (2 tau^2 = 3.2e-9 < 6e-8 / 16), FP64 1e-9 (2e-18 < 1.1e-16 / 16)
        const double tau = sizeof(TG) == 4 ? 4e-5 : 1e-9;
        const int nt = (int)((c + 31) / 32);
        double* part = (double*)(sync + NEARID_PART_WORD);
        int32_t* need = (int32_t*)(sync + NEARID_FLAG_WORD);
        hipLaunchKernelGGL((nearid_kernel<TG>), dim3((unsigned)(nt * nt)), dim3(NI_T), 0, s, (int)c, G, ldg, L, Linv,
                           Linv32, ld, part);
        hipLaunchKernelGGL(nearid_decide_kernel, dim3(1), dim3(64), 0, s, nt * nt, (const double*)part, tau * tau,
                           need, shifted_out, shifted_mode);
        RQLP_HIP_TRY(hipGetLastError());
        return chol_mw<TG>(c, G, ldg, L, Linv, Linv32, ld, shift_scale, info, sync, s, need, shifted_out,
                           shifted_mode, pivot_rel, 2);
    }
    if (sync && c <= CHOL_MW_MAXC)
        return chol_mw<TG>(c, G, ldg, L, Linv, Linv32, ld, shift_scale, info, sync, s, run_flag, shifted_out,
                           shifted_mode, pivot_rel);
    const size_t lds = chol_inv_lds_bytes(c);
    RQLP_TRY(raise_lds_limit((const void*)chol_inv_kernel<TG>, (int)chol_inv_lds_bytes(1 << 20)));
    hipLaunchKernelGGL((chol_inv_kernel<TG>), dim3(1), dim3(CH_T), lds, s, (int)c, G, ldg, shift_scale, L, Linv,
                       Linv32, ld, info, ch_prows(c), ch_xcols(c), run_flag, shifted_out, shifted_mode, pivot_rel);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}
template int chol_inv<double>(int64_t, const double*, int64_t, double*, double*, float*, int64_t, double, int32_t*,
                              hipStream_t, const int32_t*, int32_t*, unsigned*, int, double, bool);
template int chol_inv<float>(int64_t, const float*, int64_t, double*, double*, float*, int64_t, double, int32_t*,
                             hipStream_t, const int32_t*, int32_t*, unsigned*, int, double, bool);

}  // namespace rqlp
