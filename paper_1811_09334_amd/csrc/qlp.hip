// Deterministic truncated pivoted QLP (Stewart's QLP, eq. (1.2) of Section 1;
// the QLP comparison method of Section 5): kt steps of column-pivoted
// Householder QR of A itself (A Pi0 = Qhat R, R kept as its first kt rows),
// then the pivoted QR of R^T, as in the second stage of RQLP.
//
// The first CPQR streams the m x n working copy of A through the device once
// per pivot step (one launch per step): each wave owns a few columns, holds
// one column in registers at a time, applies the previous step's reflector
// to it, recomputes its residual norm exactly (rows below the step) and
// keeps the best key; every workgroup publishes its best key in its own slot
// and counts itself in with a device-scope atomic; the last workgroup to
// arrive picks the next pivot (largest residual norm, ties -> smallest index;
// numerical-rank stop as in the other CPQRs) and stores it, which the next
// launch reads.  Every workgroup of the next launch builds the reflector of
// the winning column itself from the column in memory (bitwise identical in
// all of them) and nobody writes that column in that launch, so no column
// data crosses workgroups inside a launch.  The pivoted column's entry of R
// (mu = ||x|| >= 0 on the diagonal, zeros below) is formed at extraction;
// the reflectors are kept for Q.
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {
namespace {

constexpr int QS_T = 256;                             // threads per workgroup (4 waves)
constexpr double kEpsQ = 2.220446049250313e-16;

// One launch of the streamed first CPQR.  t: the step whose reflector is
// applied (-1 for the first launch, which only computes norms and ||A||_F^2);
// the launch then decides step t + 1 when t + 1 < kt.
// state: [0] stopped, [1] rank (int32); dstate: [0] tol^2 (double).
// slots: per workgroup 4 words (norm key, index key, ||.||_F^2 part, unused).
// colstep: per column the step it was pivoted at (-1 active), initialised by
// the first launch.
template <int RPL>
__global__ __launch_bounds__(QS_T) void qlp_step_kernel(double* __restrict__ M, int64_t ldm, int m, int n, int kt,
                                                        int t, int ibits, double* __restrict__ Vh, int64_t ldv,
                                                        double* __restrict__ beta_out, double* __restrict__ mu_out,
                                                        int64_t* __restrict__ piv, int* __restrict__ colstep,
                                                        unsigned long long* slots,
                                                        unsigned* counter, int* state, double* dstate,
                                                        int32_t* info) {
    __shared__ double v[RPL * 64];
    __shared__ double s_red[QS_T / 64];
    __shared__ unsigned long long s_k[2][QS_T / 64];
    __shared__ double s_beta, s_mu;
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x, g = blockIdx.x;
    const int stopped = (t >= 0) ? state[0] : 0;
    const int p = (t >= 0) ? (int)piv[t] : -1;
    // ---- reflector of step t from column p, rows t..m-1 (every workgroup) ----
    double b = 0.0;
    if (t >= 0 && !stopped) {
        const double* col = M + (int64_t)p * ldm;
        double sg = 0.0;
        for (int i = tid; i < RPL * 64; i += QS_T) {
            const double x = (i >= t && i < m) ? col[i] : 0.0;
            v[i] = x;
            if (i > t) sg += x * x;
        }
        sg = wave_sum(sg);
        if (lane == 0) s_red[wave] = sg;
        __syncthreads();
        if (tid == 0) {
            const double sigma = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
            const double x0 = v[t];
            const double mu = sqrt(x0 * x0 + sigma);
            double v0, bb;
            if (sigma == 0.0) {
                v0 = 1.0;
                bb = (x0 >= 0.0) ? 0.0 : 2.0;
            } else {
                v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma / (x0 + mu));
                bb = 2.0 * v0 * v0 / (sigma + v0 * v0);
            }
            s_beta = bb;
            s_mu = mu;
            s_red[0] = (sigma == 0.0) ? 0.0 : 1.0 / v0;
        }
        __syncthreads();
        const double rv0 = s_red[0];
        for (int i = t + 1 + tid; i < m; i += QS_T) v[i] *= rv0;
        __syncthreads();
        if (tid == 0) v[t] = 1.0;
        __syncthreads();
        b = s_beta;
        if (g == 0) {
            for (int i = tid; i < m; i += QS_T) Vh[i + (int64_t)t * ldv] = (i < t) ? 0.0 : v[i];
            if (tid == 0) {
                beta_out[t] = b;
                mu_out[t] = s_mu;
            }
        }
    } else if (t >= 0) {
        if (g == 0) {
            for (int i = tid; i < m; i += QS_T) Vh[i + (int64_t)t * ldv] = (i == t) ? 1.0 : 0.0;
            if (tid == 0) {
                beta_out[t] = 0.0;
                mu_out[t] = 0.0;
            }
        }
    }
    // ---- apply to this workgroup's columns, residual norms, best keys ----
    unsigned long long k0 = 0, k1 = 0;
    double fro = 0.0;
    const int nw = G * (QS_T / 64);
    for (int c = g * (QS_T / 64) + wave; c < n; c += nw) {
        double* col = M + (int64_t)c * ldm;
        int cs;
        if (t < 0) {
            cs = -1;
            if (lane == 0) colstep[c] = -1;
        } else {
            cs = colstep[c];
        }
        if (c == p) {
            // the pivot column: every workgroup reads it in this launch to form
            // the reflector, so it is left as it is; its column of R (mu on the
            // diagonal, zeros below) is formed when R is extracted
            if (lane == 0) colstep[c] = t;
            continue;
        }
        if (cs >= 0) continue;                            // pivoted at an earlier step
        double x[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            x[r] = (i < m) ? col[i] : 0.0;
        }
        const int i0 = t + 1;                             // rows of the residual after step t
        if (t >= 0 && !stopped) {
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) d += v[lane + 64 * r] * x[r];
            d = wave_sum(d);
            const double w = b * d;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i >= t && i < m) {
                    x[r] -= w * v[i];
                    col[i] = x[r];
                }
            }
        }
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            s += (i >= i0) ? x[r] * x[r] : 0.0;
        }
        s = wave_sum(s);
        if (t < 0) fro += s;
        const unsigned long long a = pivot_key(stopped ? 0.0 : s, (unsigned)c, ibits);
        const unsigned long long bk = pivot_key(0.0, (unsigned)c, ibits);
        k0 = a > k0 ? a : k0;
        k1 = bk > k1 ? bk : k1;
    }
    if (t + 1 >= kt) return;                              // nothing left to decide
    // ---- this workgroup's best keys, then the last workgroup decides step t + 1 ----
    if (lane == 0) {
        s_k[0][wave] = k0;
        s_k[1][wave] = k1;
        s_red[wave] = fro;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long a = 0, c = 0;
        for (int w = 0; w < QS_T / 64; ++w) {
            a = s_k[0][w] > a ? s_k[0][w] : a;
            c = s_k[1][w] > c ? s_k[1][w] : c;
        }
        unsigned long long* sl = slots + 4 * (size_t)g;
        __hip_atomic_store(sl, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sl + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < 0) {
            const double f = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
            __hip_atomic_store(sl + 2, (unsigned long long)__double_as_longlong(f), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned arrived = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (arrived == (unsigned)G - 1u);
    }
    __syncthreads();
    if (!s_last || tid != 0) return;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long a = 0, c = 0;
    double f = 0.0;
    for (int h = 0; h < G; ++h) {
        const unsigned long long* sl = slots + 4 * (size_t)h;
        const unsigned long long ka = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long kc = __hip_atomic_load(sl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a = ka > a ? ka : a;
        c = kc > c ? kc : c;
        if (t < 0)
            f += __longlong_as_double((long long)__hip_atomic_load(sl + 2, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT));
    }
    int st = stopped, rank = (t < 0) ? kt : state[1];
    if (t < 0) {
        const double tol = (double)(m > n ? m : n) * kEpsQ;
        dstate[0] = tol * tol * f;
    }
    const double tol2 = dstate[0];
    if (!st) {
        const double kv = key_value(a, ibits);
        if (!(kv > tol2) && kv == kv) {                  // NaN norms never stop
            st = 1;
            rank = t + 1;
            if (info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
        }
    }
    piv[t + 1] = (int64_t)(st ? key_index(c, ibits) : key_index(a, ibits));
    state[0] = st;
    state[1] = rank;
}

// R^T (n x kt, original column order) of the first CPQR: a column pivoted at
// step s has R(s, c) = mu_s and zeros below; rows of R at and past the
// numerical rank are zero.
__global__ void qlp_extract_kernel(const double* __restrict__ M, int64_t ldm, int n, int kt,
                                   const int* __restrict__ colstep, const double* __restrict__ mu, const int* state,
                                   double* __restrict__ Z, int64_t ldz) {
    const int rank = state[1];
    const int64_t total = (int64_t)n * kt;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx % n, i = idx / n;
        const int cs = colstep[c];
        double r = 0.0;
        if (i < rank) {
            if (cs < 0 || i < cs) r = M[i + c * ldm];
            else if (i == cs) r = mu[cs];
        }
        Z[c + i * ldz] = r;
    }
}

// Y(:, c) = H_0 H_1 ... H_{k-1} e_{unit[c]} (e_c when unit is NULL; rows x
// ncols; H_j = I - beta_j v_j v_j^T, v_j = Vh(:, j)), one workgroup per
// column, the column in LDS.
__global__ __launch_bounds__(256) void householder_tall_kernel(int rows, int k, const double* __restrict__ Vh,
                                                               int64_t ldv, const double* __restrict__ beta,
                                                               const int64_t* __restrict__ unit,
                                                               double* __restrict__ Y, int64_t ldy) {
    extern __shared__ double y[];
    __shared__ double s_red[4];
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t u = unit ? unit[c] : (int64_t)c;
    for (int i = tid; i < rows; i += 256) y[i] = (i == u) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
        const double* vj = Vh + (int64_t)j * ldv;
        double d = 0.0;
        for (int i = j + tid; i < rows; i += 256) d += vj[i] * y[i];
        d = wave_sum(d);
        if (lane == 0) s_red[wave] = d;
        __syncthreads();
        const double w = beta[j] * ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
        for (int i = j + tid; i < rows; i += 256) y[i] -= w * vj[i];
        __syncthreads();
    }
    for (int i = tid; i < rows; i += 256) Y[i + (int64_t)c * ldy] = y[i];
}

int rpl_class(int64_t m) {
    static const int opts[] = {4, 8, 16, 32, 48, 64, 96};
    for (int o : opts)
        if ((int64_t)64 * o >= m) return o;
    return 0;
}

}  // namespace

int qlp_max_rows() { return 96 * 64; }

int qlp_grid(int64_t n) {
    int64_t g = ceil_div(n, QS_T / 64);
    const int cap = 2 * (device_info().num_cus > 0 ? device_info().num_cus : 256);
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

int qlp_first_cpqr(double* M, int64_t ldm, int64_t m, int64_t n, int64_t kt, double* Vh, int64_t ldv, double* beta,
                   double* mu, int64_t* piv, int* colstep, unsigned long long* slots, unsigned* counter, int* state,
                   double* dstate, int32_t* info, hipStream_t s) {
    const int rpl = rpl_class(m);
    if (rpl == 0) return RQLP_E_UNSUPPORTED;
    const int G = qlp_grid(n);
    int ibits = 1;
    while ((1ll << ibits) <= n) ++ibits;
    RQLP_TRY(fill_zero_bytes(counter, sizeof(unsigned), s));
    RQLP_TRY(fill_zero_bytes(state, 2 * sizeof(int), s));
    const int m_i = (int)m, n_i = (int)n, kt_i = (int)kt;
    for (int t = -1; t < kt_i; ++t) {
#define RQLP_QS(R)                                                                                               \
    hipLaunchKernelGGL(qlp_step_kernel<R>, dim3(G), dim3(QS_T), 0, s, M, ldm, m_i, n_i, kt_i, t, ibits, Vh, ldv, \
                       beta, mu, piv, colstep, slots, counter, state, dstate, info)
        switch (rpl) {
            case 4: RQLP_QS(4); break;
            case 8: RQLP_QS(8); break;
            case 16: RQLP_QS(16); break;
            case 32: RQLP_QS(32); break;
            case 48: RQLP_QS(48); break;
            case 64: RQLP_QS(64); break;
            default: RQLP_QS(96); break;
        }
#undef RQLP_QS
        RQLP_HIP_TRY(hipGetLastError());
    }
    return 0;
}

int qlp_extract_rt(const double* M, int64_t ldm, int64_t n, int64_t kt, const int* colstep, const double* mu,
                   const int* state, double* Z, int64_t ldz, hipStream_t s) {
    int64_t blocks = ceil_div(n * kt, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(qlp_extract_kernel, dim3((unsigned)blocks), dim3(256), 0, s, M, ldm, (int)n, (int)kt, colstep,
                       mu, state, Z, ldz);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

int householder_tall(int64_t rows, int64_t k, const double* Vh, int64_t ldv, const double* beta, const int64_t* unit,
                     int64_t ncols, double* Y, int64_t ldy, hipStream_t s) {
    if (rows <= 0 || ncols <= 0) return 0;
    const size_t lds = sizeof(double) * (size_t)rows;
    RQLP_TRY(raise_lds_limit((const void*)householder_tall_kernel, (int)(device_info().max_lds > 0
                                                                             ? device_info().max_lds : 65536)));
    if (device_info().max_lds > 0 && lds > device_info().max_lds) return RQLP_E_UNSUPPORTED;
    hipLaunchKernelGGL(householder_tall_kernel, dim3((unsigned)ncols), dim3(256), lds, s, (int)rows, (int)k, Vh, ldv,
                       beta, unit, Y, ldy);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

}  // namespace rqlp
