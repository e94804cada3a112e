// Batched pivoted QLP of the block rows of B for block RQLP (Algorithm 4.1:
// every block row B_j = V_j^T A, j = 1..h, gets its own pivoted QLP
// B_j = Q_B^(j) L_j P_B^(j)^T, independently of the others; T = blkdiag(L_j)).
// All h blocks go through the same few launches:
//   1. bcpqr_kernel: the first CPQR B_j Pi0_j = Q0_j R0_j of every block row
//      (bj <= 64 rows, all n columns) at once.  One column per thread, held
//      in registers for the whole factorisation; the n columns of a block are
//      spread over G workgroups (gridDim.x) and the blocks over gridDim.y.
//      Each pivot step is one agreement among the G workgroups of a block:
//      every workgroup publishes its best column (largest residual norm, ties
//      -> smallest index) and a key in its own slot, the block's last
//      workgroup polls the slots, decides and publishes the winner in the
//      block's result word, which the others poll.  Every workgroup forms the
//      Householder reflector of the winner itself (bitwise identical) and
//      applies it to its active columns, whose residual norms are then
//      recomputed exactly (the step's barriers are LDS-only except the drain
//      before a key slot is published).  Output: R0_j^T in original column order, the
//      reflectors and the numerical rank of every block.  Columns of R0_j^T
//      past the rank (exactly zero rows of R0_j) are replaced by Gaussian
//      vectors, so the next step sees a full-rank panel; their rows of the
//      triangular factor are zeroed afterwards (orthonormal completion: the
//      factorisation is triangular, so the leading columns are unaffected).
//   2. block-diagonal CholeskyQR2 of R0^T (n x l): R0_j^T = Qt_j Rt_j for
//      every block (Gram partials, Cholesky and inverse per block,
//      X_j <- X_j L_j^{-T}), twice, and twice more for the blocks whose
//      Cholesky needed the shifted retry (a shifted CholeskyQR3 is not always
//      orthonormal for numerically dependent columns, four passes are).
//   3. bqlp_small_kernel, one wave per block: the pivoted QR of the bj x bj
//      factor Rt_j, Rt_j Pi1_j = Qhat_j L_j^T.  A pivoted QR is unchanged by
//      an orthogonal factor on the left, so Pi1_j and L_j are those of the
//      pivoted QR of R0_j^T (the second factorisation of Algorithm 2.1); the
//      kernel writes L_j into T, forms Qhat_j, and Q_B^(j) = Q0_j Pi1_j from
//      the reflectors of stage 1.
//   4. bd_rmul_kernel: P_j = Qt_j Qhat_j and Q_j = V_j Q_B^(j) (the assembly
//      of Algorithm 4.1).
// Pivot rule, sign convention (diag(R) >= 0, Parlett's form of the reflector)
// and numerical-rank stop (largest residual <= max(rows, cols) eps ||M||_F)
// are those of the single-matrix CPQR.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

namespace {

constexpr int BQ_T = 256;                             // columns (threads) per workgroup of the first CPQR
constexpr int BQ_MAXG = 256;                          // workgroups per block: n <= 65536
constexpr int BQ_MAXB = 64;                           // largest block
constexpr int BQ_LD = 64;                             // leading dimension of the per-block 64 x 64 factors
constexpr size_t BQ_SQ = (size_t)BQ_LD * BQ_LD;       // elements of one per-block factor
constexpr int BG_ROWS = 256;                          // panel rows per workgroup (Gram, update, products)
constexpr unsigned long long BQ_SPIN = 1ull << 20;    // ~1 s of polling
constexpr double kEpsD = 2.220446049250313e-16;
constexpr unsigned long long kTag = 1ull << 63;       // "slot written" mark (never set in a finite key)

// Householder reflector of x = (x0, x_{j+1}, ...) in Parlett's form: H x =
// mu e_j with mu = ||x|| >= 0; v = (1, x_{j+1} / v0, ...), beta = 2 v0^2 /
// (sigma + v0^2).  rv0 = 1 / v0 (0 when sigma == 0).
__device__ __forceinline__ void reflector(double x0, double sigma, double& mu, double& beta, double& rv0) {
    mu = sqrt(x0 * x0 + sigma);
    double v0;
    if (sigma == 0.0) {
        v0 = 1.0;
        beta = (x0 >= 0.0) ? 0.0 : 2.0;
    } else {
        v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma / (x0 + mu));
        beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    }
    rv0 = (sigma == 0.0) ? 0.0 : 1.0 / v0;
}

// ---------------------------------------------------------------------------
// 1. first CPQR of every block row.  RB: register rows (>= block size).
// Scratch per block: key slots (bs steps x G x 2 words, zero on entry), the
// workgroups' partial ||B_j||_F^2 (G), the candidate columns (2 x G x RB,
// double-buffered by step parity) and the result word (one 128-byte line,
// zero on entry).
template <int RB>
__global__ __launch_bounds__(BQ_T, 3) void bcpqr_kernel(
    const double* __restrict__ B, int64_t ldb, int n, int l, int bs, int ibits, unsigned long long* keys,
    double* frop, double* candcol, unsigned long long* gwords, int64_t* piv0, double* Vh0, double* beta0,
    double* Rt, int64_t ldrt, int* rank_out, int32_t* info, unsigned long long spin_limit) {
    __shared__ double vsh[RB];                           // the step's scaled reflector
    __shared__ double colsh[RB];                         // this workgroup's candidate column
    __shared__ double s_red[BQ_T / 64];
    __shared__ unsigned long long s_kred[2][BQ_T / 64];
    __shared__ double s_beta, s_mu, s_tol2;
    __shared__ int s_ok, s_stop, s_rank;
    __shared__ unsigned s_pay;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x, g = blockIdx.x, blk = blockIdx.y;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    const int c = g * BQ_T + tid;
    const bool have = c < n;
    unsigned long long* gw = gwords + 16 * (size_t)blk;
    unsigned gen = 0;

    double x[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) x[r] = (have && r < bj) ? B[s0 + r + (int64_t)c * ldb] : 0.0;
    int act = have ? -1 : -2;                            // -1 active, >= 0 pivot step, -2 no column
    double nrm2 = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r) nrm2 += x[r] * x[r];
    {
        // this workgroup's part of ||B_j||_F^2 (the decider sums them at step 0)
        const double f = wave_sum(have ? nrm2 : 0.0);
        if (lane == 0) s_red[wave] = f;
        __syncthreads();
        if (tid == 0) {
            st_coherent(frop + (size_t)blk * G + g, (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
            s_stop = 0;
            s_rank = bj;
        }
    }
    __syncthreads();

    for (int j = 0; j < bj; ++j) {
        const int stopped = s_stop;
        // ---- candidates of this workgroup: by norm (k0) and by smallest index (k1) ----
        unsigned long long k0 = 0, k1 = 0;
        if (act == -1) {
            k0 = pivot_key(stopped ? 0.0 : nrm2, (unsigned)c, ibits);
            k1 = pivot_key(0.0, (unsigned)c, ibits);
        }
        k0 = wave_max_u64(k0);
        k1 = wave_max_u64(k1);
        if (lane == 0) {
            s_kred[0][wave] = k0;
            s_kred[1][wave] = k1;
        }
        RQLP_LDS_BARRIER();
        unsigned long long lk0 = 0, lk1 = 0;
#pragma unroll
        for (int w = 0; w < BQ_T / 64; ++w) {
            lk0 = s_kred[0][w] > lk0 ? s_kred[0][w] : lk0;
            lk1 = s_kred[1][w] > lk1 ? s_kred[1][w] : lk1;
        }
        // ---- publish the best column, then the keys; the last workgroup decides.
        // The owner thread hands its column to LDS; wave 0 stores it with one
        // coalesced store (lane r: row r), waits for it and stores the keys,
        // so only that wave waits for the memory round trip ----
        const bool pub = lk0 != 0 && !stopped;           // the same in every thread
        if (pub) {
            if (c == (int)key_index(lk0, ibits)) {
#pragma unroll
                for (int r = 0; r < RB; ++r) colsh[r] = x[r];
            }
            RQLP_LDS_BARRIER();
        }
        unsigned long long* ks = keys + ((size_t)blk * bs + j) * G * 2;
        if (wave == 0) {
            if (pub) {
                double* dst = candcol + (((size_t)blk * 2 + (j & 1)) * G + g) * RB;
                if (lane < RB && lane >= j && lane < bj) st_coherent(dst + lane, colsh[lane]);
                __builtin_amdgcn_s_waitcnt(0);           // the column store is complete
            }
            if (lane == 0) {
                __hip_atomic_store(ks + 2 * g, lk0 | kTag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(ks + 2 * g + 1, lk1 | kTag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (g == G - 1) {
            if (wave == 0) {
                unsigned long long m0 = 0, m1 = 0;
                int ok = 1;
                for (int h0 = 0; h0 < G && ok; h0 += 64) {
                    const int h = h0 + lane;
                    unsigned long long spins = 0;
                    while (true) {
                        unsigned long long a = kTag, b = kTag;
                        if (h < G) {
                            a = __hip_atomic_load(ks + 2 * h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            b = __hip_atomic_load(ks + 2 * h + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        if (__all((int)((a & b) >> 63))) {
                            const unsigned long long ka = a & ~kTag, kb = b & ~kTag;
                            m0 = ka > m0 ? ka : m0;
                            m1 = kb > m1 ? kb : m1;
                            break;
                        }
                        if (++spins > spin_limit) {
                            ok = 0;
                            if (lane == 0 && info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                m0 = wave_max_u64(m0);
                m1 = wave_max_u64(m1);
                if (lane == 0) {
                    unsigned pay = 0;
                    if (ok) {
                        if (j == 0) {
                            // ||B_j||_F^2 in workgroup order (each part was stored
                            // before its workgroup's step-0 key slot)
                            double f = 0.0;
                            for (int h = 0; h < G; ++h) f += ld_coherent(frop + (size_t)blk * G + h);
                            const double tol = (double)(bj > n ? bj : n) * kEpsD;
                            s_tol2 = tol * tol * f;
                        }
                        unsigned stopnow = 0;
                        if (!stopped) {
                            const double kv = key_value(m0, ibits);
                            if (!(kv > s_tol2) && kv == kv) stopnow = 1;   // NaN norms never stop
                        }
                        const unsigned win = (stopped || stopnow) ? key_index(m1, ibits) : key_index(m0, ibits);
                        pay = win | (stopnow << 31);
                        __hip_atomic_store(gw, ((unsigned long long)(gen + 1u) << 32) | pay, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                    s_pay = pay;
                    s_ok = ok;
                }
            }
        } else if (tid == 0) {
            int ok = 1;
            unsigned pay = 0;
            unsigned long long spins = 0;
            while (true) {
                const unsigned long long w = __hip_atomic_load(gw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(w >> 32) != gen) {
                    pay = (unsigned)w;
                    break;
                }
                if (++spins > spin_limit) {
                    ok = 0;
                    if (info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            s_pay = pay;
            s_ok = ok;
        }
        RQLP_LDS_BARRIER();
        gen += 1u;
        if (!s_ok) return;
        const unsigned pay = s_pay;
        const int now_stopped = stopped | (int)(pay >> 31);
        const int gidx = (int)(pay & 0x7FFFFFFFu);
        const int owner = gidx / BQ_T;
        // ---- reflector of the winning column, formed by wave 0 of every workgroup ----
        if (!now_stopped) {
            if (wave == 0) {
                const double* src = candcol + (((size_t)blk * 2 + (j & 1)) * G + owner) * RB;
                const double xv = (lane >= j && lane < bj) ? ld_coherent(src + lane) : 0.0;
                const double sigma = __shfl(wave_sum(lane > j ? xv * xv : 0.0), 0, RQLP_WAVE);
                const double x0 = __shfl(xv, j, RQLP_WAVE);
                double mu, bb, rv0;
                reflector(x0, sigma, mu, bb, rv0);
                if (lane < RB) vsh[lane] = (lane > j) ? xv * rv0 : (lane == j ? 1.0 : 0.0);
                if (lane == 0) {
                    s_beta = bb;
                    s_mu = mu;
                }
            }
        } else if (tid == 0) {
            s_beta = 0.0;
            s_mu = 0.0;
            if (!stopped) {
                s_stop = 1;
                s_rank = j;
            }
        }
        RQLP_LDS_BARRIER();
        const double b = s_beta;
        // ---- bookkeeping (first workgroup of the block) ----
        if (g == 0) {
            if (tid == 0) {
                piv0[s0 + j] = gidx;
                beta0[s0 + j] = b;
            }
            if (tid < bj)
                Vh0[(size_t)blk * bs * bs + tid + (size_t)j * bs] = now_stopped ? (tid == j ? 1.0 : 0.0) : vsh[tid];
        }
        if (c == gidx) {
            act = j;
            if (!now_stopped) {
                const double mu = s_mu;
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r >= j) x[r] = (r == j) ? mu : 0.0;
            }
        } else if (!now_stopped && act == -1) {
            // ---- apply H = I - b v v^T (v = 0 above row j), exact residual norm ----
            // (chunks of 8 rows wholly above row j are skipped: a uniform
            // branch; the reflector is read from LDS again for the update: an
            // opaque zero offset keeps the compiler from holding all RB entries
            // in registers next to the column)
            double dot = 0.0;
#pragma unroll
            for (int r0 = 0; r0 < RB; r0 += 8)
                if (r0 + 8 > j) {
#pragma unroll
                    for (int r = r0; r < r0 + 8; ++r) dot += vsh[r] * x[r];
                }
            const double w = b * dot;
            int off = 0;
            asm volatile("" : "+v"(off));
            double sn = 0.0;
#pragma unroll
            for (int r0 = 0; r0 < RB; r0 += 8)
                if (r0 + 8 > j) {
#pragma unroll
                    for (int r = r0; r < r0 + 8; ++r) {
                        x[r] -= w * vsh[r + off];
                        sn += (r > j) ? x[r] * x[r] : 0.0;
                    }
                }
            nrm2 = sn;
        }
        RQLP_LDS_BARRIER();
    }

    // ---- R0_j^T in original column order; rows past the rank: completion ----
    const int rank = s_rank;
    if (g == 0 && tid == 0) {
        rank_out[blk] = rank;
        if (rank < bj && info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
    }
    if (have) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (r < rank) Rt[c + (int64_t)(s0 + r) * ldrt] = x[r];
        for (int r = rank; r < bj; ++r)
            Rt[c + (int64_t)(s0 + r) * ldrt] =
                philox_normal((uint32_t)c, (uint32_t)(s0 + r), 2u, 0x5EED1234u, 0x0C0FFEE5u);
    }
}

// ---------------------------------------------------------------------------
// 2. block-diagonal CholeskyQR of the rows x l panel Z (blocks of bs columns).
// Gram partials: workgroup (ch, blk) sums Z_j^T Z_j over rows
// [ch * BG_ROWS, (ch + 1) * BG_ROWS) into part[blk][ch] (64 x 64, FP64 MFMA);
// gate (per block, optional): skip the blocks whose word is 0.
__global__ __launch_bounds__(256) void bd_gram_kernel(const double* __restrict__ Z, int64_t ldz, int rows, int l,
                                                      int bs, double* __restrict__ part,
                                                      const int32_t* __restrict__ gate) {
    const int ch = blockIdx.x, blk = blockIdx.y, nch = gridDim.x;
    if (gate && gate[blk] == 0) return;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    __shared__ double tile[64][64 + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double4_t acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = double4_t{0.0, 0.0, 0.0, 0.0};
    for (int sub = 0; sub < BG_ROWS / 64; ++sub) {
        const int r0 = ch * BG_ROWS + sub * 64;
        if (r0 >= rows) break;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + 256 * e;
            const int rr = idx & 63, cc = idx >> 6;
            const int row = r0 + rr;
            tile[rr][cc] = (row < rows && cc < bj) ? Z[row + (int64_t)(s0 + cc) * ldz] : 0.0;
        }
        __syncthreads();
        // G(i, j) += sum_k Z(k, i) Z(k, j): wave w owns rows 16 w .. 16 w + 15 of G
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int k = k0 + (lane >> 4);
            const double a = tile[k][16 * wave + (lane & 15)];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, tile[k][16 * nb + (lane & 15)], acc[nb], 0, 0, 0);
        }
    }
    double* P = part + ((size_t)blk * nch + ch) * BQ_SQ;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * wave + (lane >> 4) + 4 * r, jj = 16 * nb + (lane & 15);
            P[i + BQ_LD * jj] = acc[nb][r];
        }
}

// Cholesky G_j = L_j L_j^T of every block's Gram matrix (sum of the nch
// partials) and L_j^{-1}, one workgroup per block.  On breakdown (a pivot
// <= pivot_rel * G(i, i), or not positive) the factorisation restarts from
// G_j + shift_scale tr(G_j) I (shifted[blk] set, RQLP_INFO_CHOLQR_SHIFTED;
// shifted_mode 1 writes the word, 2 only sets it).  rt_mode 1: RT_j = Lprev_j
// L_j; rt_mode 2: RT_j <- RT_j Lprev_j L_j; the rows of RT_j at and past
// rank[blk] are zeroed (the completed columns).  Outputs per block (64 x 64):
// Lout column-major, Linv row-major.
constexpr int BDC_T = 512;
__global__ __launch_bounds__(BDC_T) void bd_chol_kernel(const double* __restrict__ part, int nch, int l, int bs,
                                                      double shift_scale, double pivot_rel, double* Lout,
                                                      double* Linv, const double* Lprev, double* RT, int rt_mode,
                                                      const int* rank, int32_t* shifted, int shifted_mode,
                                                      const int32_t* gate, int32_t* info) {
    const int blk = blockIdx.x, tid = threadIdx.x;
    if (gate && gate[blk] == 0) return;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    constexpr int LA = 65;
    __shared__ double a[64 * LA];        // a[i * LA + k] = L(i, k)
    __shared__ double w[64 * LA];        // inverse, then products
    __shared__ double s_shift;
    const double* Pb = part + (size_t)blk * nch * BQ_SQ;
    // Thread (q = tid / 8, r = tid % 8) holds rows i = 8 r + e (e < 8) of
    // column q of the matrix being reduced (x) and of X = L^{-1} (y), in
    // registers.  Step j: the owner group of column j puts it (unscaled) in
    // LDS, one barrier, then every thread applies the trailing update
    // A(i, q) -= c_i c_q / d (q > j, c = column j, d = c_j) and the
    // Gauss-Jordan step of L X = I: X(j, :) /= sqrt(d), X(i, :) -= (c_i / d)
    // X(j, :) for i > j (row j of X comes from the same group by a shuffle).
    // Row and column conditions are multipliers, not selects.  The columns
    // of L are scaled by 1 / sqrt of their pivots at the end.
    __shared__ double col[2][64];        // column of the step, by step parity
    __shared__ double gdiag[64];         // diagonal of G (pivot test, trace)
    const int q = tid >> 3, r = tid & 7, i0 = 8 * r;
    double x[8], y[8];
    double dq = 1.0;                     // pivot of step q
    int used_shift = 0;
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
        // G_j from the partials, summed in chunk order (eight chunks in
        // flight): element (i, k) = (tid % 64, tid / 64 + 8 f) so that a wave
        // reads one contiguous column per load, then through LDS into the
        // register layout
        {
            double g[8];
#pragma unroll
            for (int f = 0; f < 8; ++f) g[f] = 0.0;
            const int gi = tid & 63, gk0 = tid >> 6;
            for (int ch = 0; ch < nch; ch += 8) {
                double t[8][8];
#pragma unroll
                for (int c = 0; c < 8; ++c)
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const int gk = gk0 + 8 * f;
                        t[c][f] = (ch + c < nch && gk <= gi)
                                      ? Pb[(size_t)(ch + c) * BQ_SQ + gi + BQ_LD * gk] : 0.0;
                    }
#pragma unroll
                for (int c = 0; c < 8; ++c)
#pragma unroll
                    for (int f = 0; f < 8; ++f) g[f] += t[c][f];
            }
#pragma unroll
            for (int f = 0; f < 8; ++f) a[gi * LA + gk0 + 8 * f] = g[f];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = a[(i0 + e) * LA + q];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int i = i0 + e;
            if (i >= bj || q >= bj) x[e] = (i == q) ? 1.0 : 0.0;
            else if (i < q) x[e] = 0.0;
            if (i == q) gdiag[q] = x[e];
            y[e] = (i == q) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (tid == 0) {
            double tr = 0.0;
            for (int i = 0; i < bj; ++i) tr += gdiag[i];
            s_shift = shift_scale * tr;
        }
        __syncthreads();
        if (attempt == 1 && q < bj) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (i0 + e == q) x[e] += s_shift;
        }
        const double prel = attempt == 0 ? pivot_rel : 0.0;
        bool fail = false;
        for (int jj = 0; jj < 8; ++jj) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = 8 * jj + u;
                if (fail) continue;                          // (uniform: every thread read the same d)
                double* cb = col[j & 1];
                if (q == j) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) cb[i0 + e] = x[e];
                }
                RQLP_LDS_BARRIER();
                const double d = cb[j];
                if (!(d > prel * gdiag[j]) || !(d > 0.0)) {
                    fail = true;
                    continue;
                }
                // 1 / sqrt(d): hardware estimate and two Newton steps; 1 / d = its square
                double rs = __builtin_amdgcn_rsq(d);
                rs = rs * (1.5 - 0.5 * d * rs * rs);
                rs = rs * (1.5 - 0.5 * d * rs * rs);
                const double rd = rs * rs;
                if (q == j) dq = d;
                const double cq = (q > j) ? cb[q] * rd : 0.0;         // trailing columns only
                const double xj = __shfl(y[u], (tid & ~7) + jj, RQLP_WAVE);   // X(j, q)
                const double xr = xj * rd;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double c = cb[i0 + e];
                    x[e] -= c * cq;
                    y[e] -= (c * ((i0 + e > j) ? xr : 0.0));
                }
                if (r == jj) y[u] = xj * rs;                  // row j of X
            }
        }
        if (!fail) {
            ok = true;
        } else if (attempt == 0) {
            used_shift = 1;
        } else if (tid == 0 && info) {
            atomicOr(info, RQLP_INFO_CHOL_FAILED);
        }
        __syncthreads();
    }
    if (tid == 0 && shifted) {
        if (shifted_mode == 1) shifted[blk] = used_shift;
        else if (used_shift) shifted[blk] = 1;
        if (used_shift && info) atomicOr(info, RQLP_INFO_CHOLQR_SHIFTED);
    }
    // L (column q scaled by 1 / sqrt(pivot q), zero above the diagonal) and
    // L^{-1} into LDS for the outputs and the products below
    {
        double rsq = __builtin_amdgcn_rsq(dq);
        rsq = rsq * (1.5 - 0.5 * dq * rsq * rsq);
        rsq = rsq * (1.5 - 0.5 * dq * rsq * rsq);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int i = i0 + e;
            a[i * LA + q] = (i >= q) ? x[e] * rsq : 0.0;
            w[i * LA + q] = y[e];
        }
    }
    __syncthreads();
    double* Lo = Lout + (size_t)blk * BQ_SQ;
    double* Li = Linv + (size_t)blk * BQ_SQ;
    for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
        const int i = idx & 63, k = idx >> 6;
        Lo[i + BQ_LD * k] = a[i * LA + k];
        Li[i * BQ_LD + k] = w[i * LA + k];               // row-major (uniform reads of the update)
    }
    if (rt_mode == 0) return;
    // M = Lprev L (lower) into w, then RT = M or RT <- RT M; the global
    // operand of each product is staged in LDS (stg) first
    __shared__ double stg[64 * LA];
    const double* Lp = Lprev + (size_t)blk * BQ_SQ;
    for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
        const int i = idx & 63, t = idx >> 6;
        stg[i * LA + t] = Lp[i + BQ_LD * t];
    }
    __syncthreads();
    for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
        const int i = idx & 63, k = idx >> 6;
        double v = 0.0;
        for (int t = k; t <= i; ++t) v += stg[i * LA + t] * a[t * LA + k];
        w[i * LA + k] = (k <= i) ? v : 0.0;
    }
    __syncthreads();
    double* R = RT + (size_t)blk * BQ_SQ;
    const int rk = rank[blk];
    if (rt_mode == 2) {
        for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
            const int i = idx & 63, t = idx >> 6;
            stg[i * LA + t] = R[i + BQ_LD * t];
        }
        __syncthreads();
        for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
            const int i = idx & 63, k = idx >> 6;
            double v = 0.0;
            for (int t = k; t <= i; ++t) v += stg[i * LA + t] * w[t * LA + k];
            a[i * LA + k] = (k <= i) ? v : 0.0;
        }
        __syncthreads();
        for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
            const int i = idx & 63, k = idx >> 6;
            R[i + BQ_LD * k] = (i >= rk || i >= bj || k >= bj) ? 0.0 : a[i * LA + k];
        }
    } else {
        for (int idx = tid; idx < 64 * 64; idx += BDC_T) {
            const int i = idx & 63, k = idx >> 6;
            R[i + BQ_LD * k] = (i >= rk || i >= bj || k >= bj) ? 0.0 : w[i * LA + k];
        }
    }
}

// X_j <- X_j L_j^{-T} for every block, one row of the panel per thread, in
// place.  LinvR: per block 64 x 64 row-major L_j^{-1} (LinvR[k * 64 + i] =
// Linv(k, i)); its entries are the same for every thread, read with uniform
// addresses (scalar loads).
template <int RB>
__global__ __launch_bounds__(256) void bd_trmm_kernel(double* __restrict__ Z, int64_t ldz, int rows, int l, int bs,
                                                      const double* __restrict__ LinvR,
                                                      const int32_t* __restrict__ gate) {
    const int blk = blockIdx.y;
    if (gate && gate[blk] == 0) return;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    const double* Lb = LinvR + (size_t)blk * BQ_SQ;
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= rows) return;
    double x[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) x[i] = (i < bj) ? Z[row + (int64_t)(s0 + i) * ldz] : 0.0;
    // y_k = sum_{i <= k} Linv(k, i) x_i, from the last column down (x_k is last read for y_k);
    // rows and columns of Linv past bj are those of the identity
#pragma unroll
    for (int k = RB - 1; k >= 0; --k) {
        double y = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) y += Lb[k * BQ_LD + i] * x[i];
        x[k] = y;
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
        if (i < bj) Z[row + (int64_t)(s0 + i) * ldz] = x[i];
}

// ---------------------------------------------------------------------------
// 3. pivoted QR of every block's bj x bj factor Rt_j = RT_j^T, one wave per
// block; lane c holds column c.  Writes L_j = R^T into T (its diagonal block,
// zeros above the diagonal), the pivots (0-based within the block), Qhat_j =
// H_0 ... H_{bj-1} and Q_B^(j) = Q0_j Pi1_j (Q0_j from the reflectors Vh0 /
// beta0 of the first CPQR).
// sum_r v[r] x[r] over 64 rows as four interleaved partial sums (one wave
// per block: a single 64-long chain of dependent FMAs would set the pace)
__device__ __forceinline__ double dot64(const double* v, const double (&x)[64]) {
    double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 64; ++r) d[r & 3] += v[r] * x[r];
    return (d[0] + d[1]) + (d[2] + d[3]);
}

__global__ __launch_bounds__(64) void bqlp_small_kernel(const double* __restrict__ RT, int l, int bs,
                                                        const double* __restrict__ Vh0,
                                                        const double* __restrict__ beta0, double* T, int64_t ldt,
                                                        int64_t* piv1, double* Qhat, double* QB, int32_t* info) {
    constexpr int LV = 65;
    __shared__ double V[64 * LV];                        // reflector j at V[j * LV + r]
    __shared__ double vcol[64];
    __shared__ double sbeta[64];
    __shared__ int spiv[64];
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    int ibits = 1;
    while ((1 << ibits) <= bj) ++ibits;
    const double* R = RT + (size_t)blk * BQ_SQ;
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) x[r] = (lane < bj && r < bj) ? R[lane + BQ_LD * r] : 0.0;
    int act = lane < bj ? -1 : -2;
    double nrm2 = 0.0;
#pragma unroll
    for (int r = 0; r < 64; ++r) nrm2 += x[r] * x[r];
    const double fro = __shfl(wave_sum(act == -1 ? nrm2 : 0.0), 0, RQLP_WAVE);
    const double tol = (double)bj * kEpsD;
    const double tol2 = tol * tol * fro;
    int stopped = 0, rank = bj;
    for (int j = 0; j < bj; ++j) {
        unsigned long long k0 = 0, k1 = 0;
        if (act == -1) {
            k0 = pivot_key(stopped ? 0.0 : nrm2, (unsigned)lane, ibits);
            k1 = pivot_key(0.0, (unsigned)lane, ibits);
        }
        k0 = wave_max_u64(k0);
        k1 = wave_max_u64(k1);
        int stopnow = 0;
        if (!stopped) {
            const double kv = key_value(k0, ibits);
            if (!(kv > tol2) && kv == kv) stopnow = 1;
        }
        const int win = (int)((stopped || stopnow) ? key_index(k1, ibits) : key_index(k0, ibits));
        const int now_stopped = stopped | stopnow;
        if (stopnow) {
            stopped = 1;
            rank = j;
        }
        double b = 0.0;
        if (!now_stopped) {
            if (lane == win) {
#pragma unroll
                for (int r = 0; r < 64; ++r) vcol[r] = (r >= j) ? x[r] : 0.0;
            }
            __syncthreads();
            // sigma: lane r squares row r, one wave reduction (rows past bj are 0)
            const double vl = vcol[lane];
            const double sigma = wave_sum(lane > j ? vl * vl : 0.0);
            double mu, rv0;
            reflector(vcol[j], sigma, mu, b, rv0);
            V[j * LV + lane] = (lane > j) ? vcol[lane] * rv0 : (lane == j ? 1.0 : 0.0);
            __syncthreads();
            if (lane == win) {
                act = j;
#pragma unroll
                for (int r = 0; r < 64; ++r)
                    if (r >= j) x[r] = (r == j) ? mu : 0.0;
            } else if (act == -1) {
                const double wv = b * dot64(&V[j * LV], x);
                double sn = 0.0;
#pragma unroll
                for (int r = 0; r < 64; ++r) {
                    x[r] -= wv * V[j * LV + r];
                    sn += (r > j) ? x[r] * x[r] : 0.0;
                }
                nrm2 = sn;
            }
        } else {
            V[j * LV + lane] = (lane == j) ? 1.0 : 0.0;
            if (lane == win) act = j;
        }
        if (lane == 0) sbeta[j] = b;
        __syncthreads();
    }
    if (rank < bj && lane == 0 && info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
    // L_j = R^T: row `act` of L_j is column `act` of R
    if (act >= 0) {
        spiv[act] = lane;
        piv1[s0 + act] = lane;
#pragma unroll
        for (int i = 0; i < 64; ++i)
            if (i < bj) T[(s0 + act) + (int64_t)(s0 + i) * ldt] = (i <= act && i < rank) ? x[i] : 0.0;
    }
    __syncthreads();
    // Qhat = H_0 ... H_{bj-1}, column `lane`
    double y[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) y[r] = (r == lane) ? 1.0 : 0.0;
    for (int j = bj - 1; j >= 0; --j) {
        const double wv = sbeta[j] * dot64(&V[j * LV], y);
#pragma unroll
        for (int r = 0; r < 64; ++r) y[r] -= wv * V[j * LV + r];
    }
    if (lane < bj) {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < bj) Qhat[(size_t)blk * BQ_SQ + r + BQ_LD * lane] = y[r];
    }
    __syncthreads();
    // Q_B = Q0 Pi1: the first CPQR's reflectors applied to e_{piv1(lane)}
    const double* Vb = Vh0 + (size_t)blk * bs * bs;
    for (int j = 0; j < bj; ++j) V[j * LV + lane] = (lane < bj) ? Vb[lane + (size_t)j * bs] : 0.0;
    if (lane < bj) sbeta[lane] = beta0[s0 + lane];
    __syncthreads();
    const int u = lane < bj ? spiv[lane] : -1;
#pragma unroll
    for (int r = 0; r < 64; ++r) y[r] = (r == u) ? 1.0 : 0.0;
    for (int j = bj - 1; j >= 0; --j) {
        const double wv = sbeta[j] * dot64(&V[j * LV], y);
#pragma unroll
        for (int r = 0; r < 64; ++r) y[r] -= wv * V[j * LV + r];
    }
    if (lane < bj) {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < bj) QB[(size_t)blk * BQ_SQ + r + BQ_LD * lane] = y[r];
    }
}

// ---------------------------------------------------------------------------
// 4. Y_j = X_j M_j for every block (M per block 64 x 64, FP64, applied in the
// arithmetic of Y); one row of the panel per thread.
template <typename TX, typename TY, int RB>
__global__ __launch_bounds__(256) void bd_rmul_kernel(const TX* __restrict__ X, int64_t ldx, int rows, int l, int bs,
                                                      const double* __restrict__ M, TY* __restrict__ Y,
                                                      int64_t ldy) {
    const int blk = blockIdx.y;
    const int s0 = blk * bs;
    const int bj = (l - s0) < bs ? (l - s0) : bs;
    __shared__ TY Ms[RB * RB];                           // Ms[c * RB + i] = M(i, c)
    const double* Mb = M + (size_t)blk * BQ_SQ;
    for (int idx = threadIdx.x; idx < RB * RB; idx += 256) {
        const int i = idx % RB, c = idx / RB;
        Ms[idx] = (i < bj && c < bj) ? (TY)Mb[i + BQ_LD * c] : (TY)0;
    }
    __syncthreads();
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= rows) return;
    TY x[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) x[i] = (i < bj) ? (TY)X[row + (int64_t)(s0 + i) * ldx] : (TY)0;
#pragma unroll
    for (int c = 0; c < RB; ++c) {
        if (c >= bj) break;
        TY acc = 0;
#pragma unroll
        for (int i = 0; i < RB; ++i) acc += Ms[c * RB + i] * x[i];
        Y[row + (int64_t)(s0 + c) * ldy] = acc;
    }
}

int index_bits_of(int64_t cols) {
    int b = 1;
    while ((1ll << b) <= cols) ++b;
    return b;
}

int rows_class(int64_t bs) { return bs <= 16 ? 16 : (bs <= 32 ? 32 : 64); }

template <int RB>
int bcpqr_capacity() {
    return resident_capacity((const void*)bcpqr_kernel<RB>, BQ_T, 0);
}

}  // namespace

bool bqlp_supported(int64_t n, int64_t l, int64_t bs) {
    if (bs <= 0 || bs > BQ_MAXB || bs >= l) return false;
    const int64_t G = ceil_div(n, BQ_T);
    if (G > BQ_MAXG) return false;
    const int64_t total = G * ceil_div(l, bs);
    int cap = 0;
    switch (rows_class(bs)) {
        case 16: cap = bcpqr_capacity<16>(); break;
        case 32: cap = bcpqr_capacity<32>(); break;
        default: cap = bcpqr_capacity<64>(); break;
    }
    return total <= cap;
}

void bqlp_carve(Arena& ar, int64_t n, int64_t l, int64_t bs, BqlpScratch* sc) {
    const int64_t nb = ceil_div(l, bs > 0 ? bs : 1);
    const int64_t G = ceil_div(n, BQ_T);
    const int64_t nch = ceil_div(n, BG_ROWS);
    sc->keys = ar.take<unsigned long long>((size_t)nb * bs * G * 2);
    sc->gw = ar.take<unsigned long long>((size_t)nb * 16);
    sc->frop = ar.take<double>((size_t)nb * G);
    sc->candcol = ar.take<double>((size_t)nb * 2 * G * BQ_MAXB);
    sc->Vh0 = ar.take<double>((size_t)nb * bs * bs);
    sc->beta0 = ar.take<double>((size_t)l);
    sc->rank = ar.take<int>((size_t)nb);
    sc->shifted = ar.take<int32_t>((size_t)nb);
    sc->part = ar.take<double>((size_t)nb * nch * BQ_SQ);
    sc->Ls = ar.take<double>((size_t)4 * nb * BQ_SQ);
    sc->Linv = ar.take<double>((size_t)nb * BQ_SQ);
    sc->RT = ar.take<double>((size_t)nb * BQ_SQ);
    sc->Qhat = ar.take<double>((size_t)nb * BQ_SQ);
    sc->QB = ar.take<double>((size_t)nb * BQ_SQ);
}

template <typename TV>
int bqlp(const double* B, int64_t ldb, int64_t n, int64_t l, int64_t bs, const BqlpScratch& sc, double* Z,
         const TV* V, int64_t ldv, int64_t m, TV* Q, int64_t ldq, double* Pd, int64_t ldpd, double* T, int64_t ldt,
         int64_t* piv0, int64_t* piv1, int32_t* info, hipStream_t s) {
    const int nb = (int)ceil_div(l, bs);
    const int G = (int)ceil_div(n, BQ_T);
    const int nch = (int)ceil_div(n, BG_ROWS);
    const int rc = rows_class(bs);
    const int n_i = (int)n, l_i = (int)l, bs_i = (int)bs;
    RQLP_TRY(fill_zero_bytes(sc.keys, sizeof(unsigned long long) * (size_t)nb * bs * G * 2, s));
    RQLP_TRY(fill_zero_bytes(sc.gw, sizeof(unsigned long long) * (size_t)nb * 16, s));
    RQLP_TRY(set_identity(l, T, ldt, s));
    const int ibits = index_bits_of(n);
    // 1. first CPQR of every block row (plain launch: the grid fits on the device
    // at once, checked by bqlp_supported; every wait is bounded)
#define RQLP_BCPQR(R)                                                                                            \
    hipLaunchKernelGGL(bcpqr_kernel<R>, dim3(G, nb), dim3(BQ_T), 0, s, B, ldb, n_i, l_i, bs_i, ibits, sc.keys, \
                       sc.frop, sc.candcol, sc.gw, piv0, sc.Vh0, sc.beta0, Z, n, sc.rank, info, BQ_SPIN)
    if (rc == 16) RQLP_BCPQR(16);
    else if (rc == 32) RQLP_BCPQR(32);
    else RQLP_BCPQR(64);
#undef RQLP_BCPQR
    RQLP_HIP_TRY(hipGetLastError());
    // 2. block-diagonal CholeskyQR2 of R0^T (+ two passes for shifted blocks)
    const double shift = 11.0 * ((double)n * bs + (double)bs * (bs + 1)) * kEpsD;
    const dim3 pgrid(nch, nb);
    for (int pass = 0; pass < 4; ++pass) {
        const int32_t* gate = pass >= 2 ? sc.shifted : nullptr;
        hipLaunchKernelGGL(bd_gram_kernel, pgrid, dim3(256), 0, s, Z, n, n_i, l_i, bs_i, sc.part, gate);
        double* Lp = sc.Ls + (size_t)pass * nb * BQ_SQ;
        const double* Lprev = (pass == 1) ? sc.Ls : (pass == 3 ? sc.Ls + (size_t)2 * nb * BQ_SQ : nullptr);
        const int rt_mode = pass == 1 ? 1 : (pass == 3 ? 2 : 0);
        hipLaunchKernelGGL(bd_chol_kernel, dim3(nb), dim3(BDC_T), 0, s, sc.part, nch, l_i, bs_i, shift,
                           pass == 0 ? 1e-12 : 0.0, Lp, sc.Linv, Lprev, sc.RT, rt_mode, sc.rank, sc.shifted,
                           pass == 0 ? 1 : 2, gate, info);
        if (rc == 16) hipLaunchKernelGGL(bd_trmm_kernel<16>, pgrid, dim3(256), 0, s, Z, n, n_i, l_i, bs_i, sc.Linv, gate);
        else if (rc == 32) hipLaunchKernelGGL(bd_trmm_kernel<32>, pgrid, dim3(256), 0, s, Z, n, n_i, l_i, bs_i, sc.Linv, gate);
        else hipLaunchKernelGGL(bd_trmm_kernel<64>, pgrid, dim3(256), 0, s, Z, n, n_i, l_i, bs_i, sc.Linv, gate);
        RQLP_HIP_TRY(hipGetLastError());
    }
    // 3. second pivoted factorisation of every block, Qhat_j, Q_B^(j)
    hipLaunchKernelGGL(bqlp_small_kernel, dim3(nb), dim3(64), 0, s, sc.RT, l_i, bs_i, sc.Vh0, sc.beta0, T, ldt, piv1,
                       sc.Qhat, sc.QB, info);
    RQLP_HIP_TRY(hipGetLastError());
    // 4. P_j = Qt_j Qhat_j, Q_j = V_j Q_B^(j)
    const dim3 ngrid((unsigned)ceil_div(n, 256), nb), mgrid((unsigned)ceil_div(m, 256), nb);
    const int m_i = (int)m;
#define RQLP_RMUL(R)                                                                                                  \
    do {                                                                                                              \
        hipLaunchKernelGGL((bd_rmul_kernel<double, double, R>), ngrid, dim3(256), 0, s, (const double*)Z, n, n_i, l_i, \
                           bs_i, sc.Qhat, Pd, ldpd);                                                                  \
        hipLaunchKernelGGL((bd_rmul_kernel<TV, TV, R>), mgrid, dim3(256), 0, s, V, ldv, m_i, l_i, bs_i, sc.QB, Q, ldq); \
    } while (0)
    if (rc == 16) RQLP_RMUL(16);
    else if (rc == 32) RQLP_RMUL(32);
    else RQLP_RMUL(64);
#undef RQLP_RMUL
    RQLP_HIP_TRY(hipGetLastError());
    return 0;
}

template int bqlp<double>(const double*, int64_t, int64_t, int64_t, int64_t, const BqlpScratch&, double*,
                          const double*, int64_t, int64_t, double*, int64_t, double*, int64_t, double*, int64_t,
                          int64_t*, int64_t*, int32_t*, hipStream_t);
template int bqlp<float>(const double*, int64_t, int64_t, int64_t, int64_t, const BqlpScratch&, double*,
                         const float*, int64_t, int64_t, float*, int64_t, double*, int64_t, double*, int64_t,
                         int64_t*, int64_t*, int32_t*, hipStream_t);

}  // namespace rqlp
