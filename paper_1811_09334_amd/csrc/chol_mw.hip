// Cholesky factor and inverse of a c x c Gram matrix (c <= 512) on many
// workgroups: the Cholesky step of CholeskyQR (the orthonormalisation of the
// range finder in Algorithm 2.1, and the inner QR steps of Algorithm 2.2).
//
// Workgroup J owns block column J (16 columns) of both the factor L and of
// X = L^{-1}, rows 16 J .. c-1, in LDS for the whole factorisation.  The
// right-looking block algorithm runs as a pipeline of point-to-point flags
// instead of grid barriers:
//   step K (owner K): factor the 16 x 16 diagonal block, L_KK and its
//     inverse D_K = L_KK^{-1} (one wave, LDS-resident), solve the panel
//     L(i, K) = W(i, K) D_K^T for the rows below, publish L(:, K) and D_K in
//     the output arrays and raise flag K;
//   workgroup J > K, on flag K: W(:, J) -= L(:, K) L(J, K)^T  (16 x 16 FP64
//     MFMA tiles);
//   workgroup J < K, on flag K: X(K, J) <- D_K X(K, J), then
//     X(i, J) -= L(i, K) X(K, J) for the block rows i below K (block forward
//     substitution of L X = I fused into the same sweep).
// A workgroup waits only for the flags it needs, so the critical path is
// one flag hand-off, one rank-16 update and one diagonal factorisation per
// block step.  Flags carry a per-launch epoch, so no reset is needed.
//
// Breakdown (a non-positive or non-finite pivot) in the plain attempt sets
// RQLP_INFO_CHOLQR_SHIFTED and the device word *retry; the same launch then
// factors G + shift_scale trace(G) I (Fukaya et al. 2020) and flags
// RQLP_INFO_CHOL_FAILED if that breaks too.
// Cross-workgroup data uses relaxed device-scope atomic loads / stores.
#include <time.h>
#include <unistd.h>

#include <atomic>

#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

constexpr int MW_T = 256;
constexpr int MW_NW = MW_T / 64;
constexpr int MW_S = 17;                               // LDS row stride in doubles
constexpr unsigned long long MW_SPIN_LIMIT = 1ull << 22;
constexpr unsigned MW_EARLY = 0x80000000u;
constexpr int MW_MAXB = CHOL_MW_MAXC / 16;               // flag words per attempt               // early-flag marker (epochs are odd, < 2^31 apart)
constexpr int MW_MAXT = CHOL_MW_MAXC / 16 / MW_NW;       // row tiles per wave (at most)

__device__ __forceinline__ double mw_readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One wave: lane (i = lane % 16, g = lane / 16) holds d[e] = D(i, 4 g + e)
// of the 16 x 16 block (lower triangle read).  On return d holds the
// Cholesky factor L (zero above the diagonal) and x its inverse X = L^{-1}
// (zero above the diagonal).  Returns true when a pivot was non-positive or
// not finite (it is then replaced by 1).  Each column step broadcasts the
// pivot with a read-lane; the lanes holding column j of L write it to the
// LDS scratch sc (16 doubles), the lanes holding row j of X write that row
// (sc + 16, 16 doubles), and every lane reads back L(i, j), L(4 g .. 4 g + 3,
// j) and X(j, 4 g .. 4 g + 3): one LDS round trip per step (the LDS
// operations of one wave complete in order, so the reads see the writes and
// the next step's writes come after this step's reads).  The row sweep of
// L X = I runs in the same loop: its step j needs only L(i, j) and
// 1 / L(j, j) from the factor's step j, so the two dependency chains overlap.
__device__ bool mw_factor_diag(double d[4], double x[4], double thr, int lane, double* sc) {
    const int i = lane & 15, g = lane >> 4;
    bool bad = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = (i == 4 * g + e) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int gj = j >> 2, ej = j & 3;
        const double piv = mw_readlane(d[ej], j + 16 * gj);
        const bool ok = (piv > mw_readlane(thr, j)) && (piv > 0.0) && (piv < 1.0e308);
        bad |= !ok;
        // 1 / sqrt(piv) from the hardware estimate and one Newton step
        // (relative error ~1e-16), then sqrt(piv) = piv / sqrt(piv)
        const double p = ok ? piv : 1.0;
        double rinv = __builtin_amdgcn_rsq(p);
        rinv = rinv * (1.5 - 0.5 * p * rinv * rinv);
        const double lj = p * rinv;
        if (g == gj) {
            d[ej] = (i == j) ? lj : (i > j ? d[ej] * rinv : 0.0);
            sc[i] = d[ej];                                   // L(i, j)
        }
        // row sweep of L X = I: X(j, :) /= L(j, j), then X(i, :) -= L(i, j) X(j, :) below
        if (i == j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[e] *= rinv;
                sc[16 + 4 * g + e] = x[e];                   // X(j, 4 g + e)
            }
        }
        __builtin_amdgcn_wave_barrier();
        const double lij = sc[i];
        double lkj[4], xt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            lkj[e] = sc[4 * g + e];
            xt[e] = sc[16 + 4 * g + e];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * g + e > j) d[e] -= lij * lkj[e];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (i > j) x[e] -= lij * xt[e];
    }
    return bad;
}

// The diagonal-block factorisation of one wave as a function of its own: D
// from W (LDS, row stride MW_S) is replaced by its factor L, and L^{-1} goes
// to Dv.  Row i's pivot threshold is pivot_rel G(i, i) (gd: the diagonal of
// G, rows past nvalid: 0) when use_thr is set, else 0.  Not inlined: inside
// the kernel the column loop shared the kernel's scalar registers and
// reloaded spilled ones at every step.
__device__ __noinline__ int mw_factor_block(double* W, double* Dv, double* sc, const double* gd, int use_thr,
                                            double pivot_rel, int nvalid) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    double d[4], x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = W[i * MW_S + 4 * g + e];
    const double thr = (use_thr && i < nvalid) ? pivot_rel * gd[i] : 0.0;
    const bool bad = mw_factor_diag(d, x, thr, lane, sc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        W[i * MW_S + 4 * g + e] = d[e];
        Dv[i * MW_S + 4 * g + e] = x[e];
    }
    return bad ? 1 : 0;
}

// gate_mode: 0 always run; 1 when *gate == 0 write identities and return
// (conditional extra CholeskyQR pass).  The shifted retry runs in the same
// launch: at the end of the plain attempt every workgroup has waited for
// every other block's flag, and a breakdown sets *retry before its owner
// raises its flag, so all workgroups read the same *retry and either finish
// or start the shifted attempt together (flags0 + MW_MAXB, epoch0 + 2).
template <typename TG>
__global__ __launch_bounds__(MW_T) void chol_mw_kernel(int c, const TG* __restrict__ G, int64_t ldg,
                                                       double shift_scale, double* __restrict__ Lo,
                                                       double* __restrict__ Xo, float* __restrict__ Xf, int64_t ld,
                                                       int32_t* info, unsigned* flags0, unsigned epoch0,
                                                       int32_t* retry, const int32_t* gate, int gate_mode,
                                                       int32_t* shifted_out, int shifted_mode, double pivot_rel) {
    extern __shared__ double lds[];
    const int J = blockIdx.x, NB = gridDim.x;
    const int j0 = 16 * J;
    const int kb = (c - j0) < 16 ? (c - j0) : 16;
    const int nrt = (c - j0 + 15) >> 4;                 // row tiles of this block column
    double* Wc = lds;                                   // [16 nrt][MW_S]: W, then L (rows j0..)
    double* Xc = Wc + (size_t)nrt * 16 * MW_S;          // [16 nrt][MW_S]: X = L^{-1} (rows j0..)
    double* Dv = Xc + (size_t)nrt * 16 * MW_S;          // [16][MW_S]
    __shared__ double s_red[MW_NW];
    __shared__ __attribute__((aligned(16))) double s_fd[32];   // column / row exchange of the diagonal factor
    __shared__ double s_gd[16];                                // G(j0 + t, j0 + t): pivot thresholds
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int fr = lane & 15, fk = lane >> 4;

    if (gate_mode != 0 && *gate == 0) {
        if (gate_mode == 1) {
            for (int idx = tid; idx < c * 16; idx += MW_T) {
                const int i = idx % c, t = idx / c;
                if (t >= kb) continue;
                const int64_t col = j0 + t;
                const double v = (i == col) ? 1.0 : 0.0;
                Lo[i + col * ld] = v;
                Xo[i + col * ld] = v;
                if (Xf) Xf[i + col * ld] = (float)v;
            }
            if (J == 0 && tid == 0) {
                if (retry) *retry = 0;
                if (shifted_out && shifted_mode == 1) *shifted_out = 0;
            }
        }
        return;
    }

    __shared__ int s_again;
    unsigned* flags = flags0;
    unsigned epoch = epoch0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        flags = flags0 + attempt * MW_MAXB;
        epoch = epoch0 + 2u * (unsigned)attempt;
        double shift = 0.0;
        if (attempt) {
            double t = 0.0;
            for (int i = tid; i < c; i += MW_T) t += (double)G[i + (int64_t)i * ldg];
            t = wave_sum(t);
            if (lane == 0) s_red[wave] = t;
            __syncthreads();
            double tr = 0.0;
            for (int w = 0; w < MW_NW; ++w) tr += s_red[w];
            shift = tr == 0.0 ? 1.0 : shift_scale * tr;     // a zero Gram matrix: factor I
        }
        for (int idx = tid; idx < nrt * 16 * 16; idx += MW_T) {
            const int r = idx >> 4, t = idx & 15;
            const int i = j0 + r;
            double w = 0.0;
            if (t < kb && i < c && r >= t) w = (double)G[i + (int64_t)(j0 + t) * ldg] + (r == t ? shift : 0.0);
            if (r == t) s_gd[t] = (t < kb && i < c) ? (double)G[i + (int64_t)(j0 + t) * ldg] : 0.0;
            if (t >= kb && r == t) w = 1.0;                 // identity padding of a ragged last block
            Wc[r * MW_S + t] = w;
            Xc[r * MW_S + t] = (r == t) ? 1.0 : 0.0;
        }
        if (J == 0 && tid == 0) {
            if (attempt == 0 && retry) __hip_atomic_store(retry, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // shifted_mode 1: *shifted_out = "this factorisation used the shift";
            // 2: only ever set (accumulates over several factorisations)
            if (shifted_out && (shifted_mode == 1 || attempt == 1)) *shifted_out = attempt;
        }
        __syncthreads();

        // The diagonal block, factored by wave 0: D = L_JJ^{-1} into Dv, L_JJ into
        // tile 0 of Wc, breakdown into s_bad.
        auto factor_diag = [&]() {
            if (wave == 0) {
                // plain attempt: a pivot below pivot_rel times the column's squared
                // norm marks a numerically dependent column (lane i: column j0 + i)
                // (G's diagonal was kept in LDS when the block column was loaded:
                // a global load here would sit on the critical path of every step)
                const int bad = mw_factor_block(Wc, Dv, s_fd, s_gd, attempt == 0, pivot_rel, c - j0);
                if (lane == 0) s_bad = bad;
            }
        };
        // W(r0.., J) -= A B^T for one 16-row tile: a = L(rows, K), b = L(J, K)^T
        auto update_tile = [&](int r0, const double (&a)[4], const double (&b)[4]) {
            const bool in = j0 + r0 + fr < c;
            double4_t acc;
    #pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = Wc[(r0 + fk + 4 * r) * MW_S + fr];
    #pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? -a[ks] : 0.0, b[ks], acc, 0, 0, 0);
    #pragma unroll
            for (int r = 0; r < 4; ++r) Wc[(r0 + fk + 4 * r) * MW_S + fr] = acc[r];
        };
        // Flag words: owner K first stores MW_EARLY ^ epoch once the rows of block
        // K + 1 of L(:, K) are published (all that owner K + 1 needs to update and
        // factor its diagonal block), then epoch once all of L(:, K) and D_K are.
        auto wait_flag = [&](int K, bool early_ok) {
            if (tid == 0) {
                unsigned long long spins = 0;
                for (;;) {
                    const unsigned f = ld_coherent_u32(flags + K);
                    if (f == epoch || (early_ok && f == (epoch ^ MW_EARLY))) break;
                    if (++spins > MW_SPIN_LIMIT) {
                        if (info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
        };

        for (int K = 0; K < NB; ++K) {
            const int64_t kc = 16 * (int64_t)K;
            const bool ahead = K == J - 1;                  // the panel just before this workgroup's own step
            if (K != J) wait_flag(K, ahead);
            if (K < J) {
                // W(:, J) -= L(:, K) L(J, K)^T over the rows j0.. of this block column
                // b = L(J, K)^T is the same for every tile of this workgroup
                double b[4];
                {
                    const int jt = j0 + fr;
                    const int jc = jt < c ? jt : c - 1;
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) b[ks] = ld_coherent(Lo + jc + (kc + 4 * ks + fk) * ld);
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) b[ks] = jt < c ? b[ks] : 0.0;
                }
                if (ahead) {
                    // look-ahead: wave 0 updates the diagonal tile (its panel rows are
                    // b, out with the early flag) and factors it, while the other waves
                    // wait for the whole panel and update the remaining tiles
                    if (wave == 0) {
                        update_tile(0, b, b);
                        __builtin_amdgcn_wave_barrier();
                        factor_diag();
                    } else {
                        if (lane == 0) {
                            unsigned long long spins = 0;
                            while (ld_coherent_u32(flags + K) != epoch) {
                                if (++spins > MW_SPIN_LIMIT) {
                                    if (info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                        }
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        constexpr int NW1 = MW_NW - 1;
                        for (int q0 = 0; 1 + (wave - 1) + NW1 * q0 < nrt; q0 += MW_MAXT) {
                            double a[MW_MAXT][4];
    #pragma unroll
                            for (int q = 0; q < MW_MAXT; ++q) {
                                const int tile = 1 + (wave - 1) + NW1 * (q0 + q);
                                const int i = j0 + 16 * tile + fr;
                                const int ic = (tile < nrt && i < c) ? i : c - 1;
    #pragma unroll
                                for (int ks = 0; ks < 4; ++ks)
                                    a[q][ks] = ld_coherent(Lo + ic + (kc + 4 * ks + fk) * ld);
                            }
    #pragma unroll
                            for (int q = 0; q < MW_MAXT; ++q) {
                                const int tile = 1 + (wave - 1) + NW1 * (q0 + q);
                                if (tile >= nrt) break;
                                update_tile(16 * tile, a[q], b);
                            }
                        }
                    }
                    __syncthreads();
                } else {
                    // all panel loads of this wave's tiles are issued before the first use
                    double a[MW_MAXT][4];
    #pragma unroll
                    for (int q = 0; q < MW_MAXT; ++q) {
                        const int tile = wave + MW_NW * q;
                        const int i = j0 + 16 * tile + fr;
                        const int ic = (tile < nrt && i < c) ? i : c - 1;
    #pragma unroll
                        for (int ks = 0; ks < 4; ++ks) a[q][ks] = ld_coherent(Lo + ic + (kc + 4 * ks + fk) * ld);
                    }
    #pragma unroll
                    for (int q = 0; q < MW_MAXT; ++q) {
                        const int tile = wave + MW_NW * q;
                        if (tile >= nrt) break;
                        update_tile(16 * tile, a[q], b);
                    }
                    __syncthreads();
                }
            } else if (K == J) {
                // ---- own step: diagonal factor (unless done ahead), panel, publication ----
                if (J == 0) {
                    factor_diag();
                    __syncthreads();
                }
                if (s_bad && tid == 0) {
                    if (attempt == 0) {
                        if (info) atomicOr(info, RQLP_INFO_CHOLQR_SHIFTED);
                        if (retry) __hip_atomic_store(retry, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else if (info) {
                        atomicOr(info, RQLP_INFO_CHOL_FAILED);
                    }
                }
                // panel rows below the diagonal block: L(i, J) = W(i, J) D^T.  Tile 1
                // (the rows of block J + 1) first, by wave 0, published at once
                for (int tile = 1 + wave; tile < nrt; tile += MW_NW) {
                    const int r0 = 16 * tile;
                    double a[4], b[4];
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int k = 4 * ks + fk;
                        a[ks] = Wc[(r0 + fr) * MW_S + k];
                        b[ks] = Dv[fr * MW_S + k];
                    }
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
    #pragma unroll
                    for (int r = 0; r < 4; ++r) Wc[(r0 + fk + 4 * r) * MW_S + fr] = acc[r];
                    if (tile == 1) {
                        // accumulator r holds L(j0 + 16 + fk + 4 r, j0 + fr)
                        if (fr < kb) {
    #pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int i = j0 + 16 + fk + 4 * r;
                                if (i < c) st_coherent(Lo + i + (int64_t)(j0 + fr) * ld, acc[r]);
                            }
                        }
                        __builtin_amdgcn_s_waitcnt(0);
                        if (lane == 0) st_coherent_u32(flags + J, epoch ^ MW_EARLY);
                    }
                }
                // X(J, J) = D
                for (int idx = tid; idx < 256; idx += MW_T) {
                    const int r = idx >> 4, t = idx & 15;
                    Xc[r * MW_S + t] = (r >= t) ? Dv[r * MW_S + t] : 0.0;
                }
                __syncthreads();
                // publish the rest of L(j0.., J) and D into the outputs, then raise flag J
                for (int idx = tid; idx < nrt * 16 * 16; idx += MW_T) {
                    const int r = idx >> 4, t = idx & 15;
                    const int i = j0 + r;
                    if (i >= c || t >= kb || (r >= 16 && r < 32)) continue;
                    const int64_t col = j0 + t;
                    st_coherent(Lo + i + col * ld, r >= t ? Wc[r * MW_S + t] : 0.0);
                    if (r < 16) st_coherent(Xo + i + col * ld, r >= t ? Dv[r * MW_S + t] : 0.0);
                }
                drain_and_sync();
                if (tid == 0) st_coherent_u32(flags + J, epoch);
                // X(i, J) -= L(i, J) X(J, J) for the rows below, from LDS
                for (int tile = 1 + wave; tile < nrt; tile += MW_NW) {
                    const int r0 = 16 * tile;
                    double a[4], b[4];
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int k = 4 * ks + fk;
                        a[ks] = -Wc[(r0 + fr) * MW_S + k];
                        b[ks] = Xc[k * MW_S + fr];
                    }
                    double4_t acc;
    #pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = Xc[(r0 + fk + 4 * r) * MW_S + fr];
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
    #pragma unroll
                    for (int r = 0; r < 4; ++r) Xc[(r0 + fk + 4 * r) * MW_S + fr] = acc[r];
                }
                __syncthreads();
            } else {
                // ---- K > J: X(K, J) <- D_K X(K, J); X(i, J) -= L(i, K) X(K, J) below ----
                const int rK = (int)(kc - j0);
                if (wave == 0) {
                    double a[4], b[4];
                    const int64_t s_ = kc + fr;
                    const int64_t sc_ = s_ < c ? s_ : c - 1;
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int64_t kk = kc + 4 * ks + fk;
                        a[ks] = ld_coherent(Xo + sc_ + (kk < c ? kk : c - 1) * ld);
                    }
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int k = 4 * ks + fk;
                        const int64_t kk = kc + k;
                        a[ks] = (s_ < c && kk < c && kk <= s_) ? a[ks] : 0.0;
                        b[ks] = Xc[(rK + k) * MW_S + fr];
                    }
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    #pragma unroll
                    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
    #pragma unroll
                    for (int r = 0; r < 4; ++r) Xc[(rK + fk + 4 * r) * MW_S + fr] = acc[r];
                }
                __syncthreads();
                {
                    const int t0 = (rK >> 4) + 1;
                    double a[MW_MAXT][4];
    #pragma unroll
                    for (int q = 0; q < MW_MAXT; ++q) {
                        const int tile = t0 + wave + MW_NW * q;
                        const int i = j0 + 16 * tile + fr;
                        const int ic = (tile < nrt && i < c) ? i : c - 1;
    #pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const int64_t kk = kc + 4 * ks + fk;
                            a[q][ks] = ld_coherent(Lo + ic + (kk < c ? kk : c - 1) * ld);
                        }
                    }
    #pragma unroll
                    for (int q = 0; q < MW_MAXT; ++q) {
                        const int tile = t0 + wave + MW_NW * q;
                        if (tile >= nrt) break;
                        const int r0 = 16 * tile;
                        const bool in = j0 + r0 + fr < c;
                        double b[4];
    #pragma unroll
                        for (int ks = 0; ks < 4; ++ks) b[ks] = Xc[(rK + 4 * ks + fk) * MW_S + fr];
                        double4_t acc;
    #pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r] = Xc[(r0 + fk + 4 * r) * MW_S + fr];
    #pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const bool kin = kc + 4 * ks + fk < c;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(in && kin ? -a[q][ks] : 0.0, b[ks], acc, 0, 0, 0);
                        }
    #pragma unroll
                        for (int r = 0; r < 4; ++r) Xc[(r0 + fk + 4 * r) * MW_S + fr] = acc[r];
                    }
                }
                __syncthreads();
            }
        }
        if (attempt == 0) {
            if (tid == 0) s_again = (retry && ld_coherent_u32((const unsigned*)retry) != 0u) ? 1 : 0;
            __syncthreads();
            if (s_again) continue;                          // the same decision in every workgroup
        }
        // outputs of this block column: zeros above row j0, X (and its FP32 copy) below
        for (int idx = tid; idx < c * 16; idx += MW_T) {
            const int i = idx % c, t = idx / c;
            if (t >= kb) continue;
            const int64_t col = j0 + t;
            if (i < j0) {
                Lo[i + col * ld] = 0.0;
                Xo[i + col * ld] = 0.0;
                if (Xf) Xf[i + col * ld] = 0.0f;
            } else {
                const double x = Xc[(i - j0) * MW_S + t];
                if (i - j0 >= 16) Xo[i + col * ld] = x;
                if (Xf) Xf[i + col * ld] = (float)x;
            }
        }
        break;
    }
}

size_t chol_mw_lds_bytes(int64_t c) {
    const int64_t nrt = (c + 15) / 16;
    return sizeof(double) * (size_t)((2 * nrt * 16 + 16) * MW_S);
}

template <typename TG>
int chol_mw(int64_t c, const TG* G, int64_t ldg, double* L, double* Linv, float* Linv32, int64_t ld,
            double shift_scale, int32_t* info, unsigned* sync, hipStream_t s, const int32_t* run_flag,
            int32_t* shifted_out, int shifted_mode, double pivot_rel, int gate_mode) {
    // per-process start value, so that flag words left in reused memory by
    // another process are unlikely to match
    static std::atomic<unsigned> epoch_counter{(unsigned)(getpid() * 2654435761u) ^ (unsigned)time(nullptr)};
    RQLP_TRY(raise_lds_limit((const void*)chol_mw_kernel<TG>, (int)chol_mw_lds_bytes(CHOL_MW_MAXC)));
    const int NB = (int)((c + 15) / 16);
    if (device_info().num_cus > 0 && NB > device_info().num_cus) return RQLP_E_UNSUPPORTED;
    const size_t lds = chol_mw_lds_bytes(c);
    // epochs: odd and distinct per launch (a zeroed flag word never matches)
    const unsigned e0 = 2u * epoch_counter.fetch_add(2) + 1u;
    int32_t* retry = (int32_t*)(sync + 2 * MW_MAXB);   // after the two attempts' flag words
    // A plain launch: the NB <= 32 workgroups (one per block column, at most
    // one per CU by their LDS) all fit on the device at once, and every wait
    // is bounded.  (A cooperative launch gave the same residency but cost
    // ~15 us of idle device time before and ~10 us after each launch.)
    hipLaunchKernelGGL((chol_mw_kernel<TG>), dim3(NB), dim3(MW_T), (unsigned)lds, s, (int)c, G, ldg, shift_scale, L,
                       Linv, Linv32, ld, info, sync, e0, retry, run_flag,
                       run_flag ? (gate_mode >= 0 ? gate_mode : 1) : 0, shifted_out, shifted_mode, pivot_rel);
    RQLP_HIP_TRY(hipGetLastError());
    return 0;
}

template int chol_mw<double>(int64_t, const double*, int64_t, double*, double*, float*, int64_t, double, int32_t*,
                             unsigned*, hipStream_t, const int32_t*, int32_t*, int, double, int);
template int chol_mw<float>(int64_t, const float*, int64_t, double*, double*, float*, int64_t, double, int32_t*,
                            unsigned*, hipStream_t, const int32_t*, int32_t*, int, double, int);

}  // namespace rqlp
