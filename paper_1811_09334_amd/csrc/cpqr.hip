// Column-pivoted Householder QR of the reduced matrix (the first CPQR of
// Algorithms 2.1 and 2.2; CPQR as defined in Section 1) and of the small l x l
// factor of the second stage (the pivoted second factorisation of Algorithm 2.1).
//
// Design: the matrix is distributed by columns over G co-resident workgroups
// (a grid no larger than the device holds at once), each holding its columns in LDS for the whole
// factorisation, so the matrix never returns to HBM until the end.  Every
// pivot step needs one grid-wide agreement on the winning column:
//   1. each workgroup finds its best active column (largest residual norm,
//      ties -> smallest index) and publishes it: a 64-bit key (norm^2 with the
//      low mantissa bits replaced by the complemented column index) goes into
//      an atomic max of its group of 16 workgroups (forwarded to a top slot by
//      the group's last arriver), and the column itself into a
//      double-buffered exchange slot;
//   2. one two-level grid barrier (relaxed device-scope atomics only, see
//      below), whose last arriver reads the winning key and publishes the
//      decision inside the barrier's generation word;
//   3. every workgroup reads the winning column, builds the same
//      Householder reflector redundantly (bitwise identical, fixed reduction
//      order), applies it to its own active columns and recomputes their
//      residual norms exactly from LDS.
// The reflector keeps R(j, j) = ||x|| >= 0 (Parlett's form of the
// Householder vector; Golub & Van Loan, Alg. 5.1.1).  Columns whose norms
// agree to 2^-(52 - index bits) may be taken in either order.
// Numerical-rank stop: when the largest residual norm is <= max(rows, cols)
// * eps * ||M||_F, the remaining steps take the smallest-index active columns,
// apply no reflection, and the trailing rows of R are zero.
// With G = 1 the exchange goes through LDS only.  The register-resident
// kernel (cpqr_reg_kernel, below) agrees through per-workgroup key slots
// instead of the counters of step 2 (slot_agree).
#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {

constexpr int CP_T = 256;
constexpr unsigned long long CP_SPIN_LIMIT = 1ull << 20;   // ~1 s of polling

// Cross-workgroup traffic of the CPQR uses only relaxed device-scope atomic
// loads and stores (st_coherent / ld_coherent) plus completion waits for
// ordering (drain_and_sync).

// Two-level grid barrier: workgroups arrive on the counter of their group of
// 16 (each counter on its own 128-byte line), the last of a group forwards
// the group's pivot keys to the top slot and arrives on the top counter, and
// the very last arriver evaluates `decide()` and publishes its 32-bit result
// together with the new generation in one 64-bit word, which the others poll.
// Every wait is bounded by spin_limit polls (RQLP_INFO_BARRIER_TIMEOUT,
// returns false).
constexpr int CP_GROUP = 16;
__host__ __device__ constexpr int cp_bar_words(int G) { return 32 * ((G + CP_GROUP - 1) / CP_GROUP + 2); }
// Key slots of one step: (groups + 1) slots of 16 u64 (one 128-byte line
// each); slot[0] is the max-by-norm key, slot[1] the max-by-index key.
__host__ __device__ constexpr int cp_key_words(int G) { return 16 * ((G + CP_GROUP - 1) / CP_GROUP + 1); }

template <typename F>
__device__ __forceinline__ bool grid_sync_decide(unsigned* bar, int G, unsigned& gen, unsigned& payload,
                                                 int32_t* info, unsigned long long spin_limit,
                                                 unsigned long long* kslots, unsigned long long lk0,
                                                 unsigned long long lk1, F decide) {
    __shared__ int s_ok;
    __shared__ unsigned s_pay;
    drain_and_sync();
    if (threadIdx.x == 0) {
        const int ng = (G + CP_GROUP - 1) / CP_GROUP;
        const int grp = (int)blockIdx.x / CP_GROUP;
        const int gsz = (G - grp * CP_GROUP) < CP_GROUP ? (G - grp * CP_GROUP) : CP_GROUP;
        unsigned* cnt = bar + 32 * grp;
        unsigned* top = bar + 32 * ng;
        unsigned long long* gw = (unsigned long long*)(bar + 32 * (ng + 1));
        const unsigned g = gen;
        int ok = 1;
        unsigned pay = 0;
        bool last = false;
        if (kslots && lk0 != 0) {
            atomicMax(kslots + 16 * grp, lk0);
            atomicMax(kslots + 16 * grp + 1, lk1);
            __builtin_amdgcn_s_waitcnt(0);
        }
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)gsz - 1u) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (kslots) {
                // forward this group's maxima to the top slot
                const unsigned long long g0 =
                    __hip_atomic_load(kslots + 16 * grp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long g1 =
                    __hip_atomic_load(kslots + 16 * grp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (g0 != 0) {
                    atomicMax(kslots + 16 * ng, g0);
                    atomicMax(kslots + 16 * ng + 1, g1);
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
            if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)ng - 1u) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (last) {
            pay = decide();
            __builtin_amdgcn_s_waitcnt(0);
            __hip_atomic_store(gw, ((unsigned long long)(g + 1u) << 32) | pay, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (true) {
                const unsigned long long w = __hip_atomic_load(gw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(w >> 32) != g) {
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
        }
        __builtin_amdgcn_s_waitcnt(0);
        gen = g + 1u;
        s_ok = ok;
        s_pay = pay;
    }
    __syncthreads();
    payload = s_pay;
    return s_ok != 0;
}

// Grid barrier of the register-resident kernel (once per factorisation, for
// the Frobenius norm): arrival counters of groups of GRP workgroups that grow
// monotonically (no resets); a group's last arriver forwards its arrival to
// the top counter, and the very last arriver publishes the new generation in
// the 64-bit word gw (the result word of slot_agree), which the others poll.
// Bounded waits as in grid_sync_decide.
template <int GRP>
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned long long* gw, int G, unsigned& gen,
                                             int32_t* info, unsigned long long spin_limit) {
    __shared__ int s_ok;
    const int ng = (G + GRP - 1) / GRP;
    const int grp = (int)blockIdx.x / GRP;
    const unsigned gsz = (unsigned)((G - grp * GRP) < GRP ? (G - grp * GRP) : GRP);
    unsigned* cnt = bar + 32 * grp;
    unsigned* top = bar + 32 * ng;
    const unsigned g = gen;
    drain_and_sync();                                    // this workgroup's stores are done
    if (threadIdx.x == 0) {
        int ok = 1;
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsz * (g + 1u) - 1u &&
            __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)ng * (g + 1u) - 1u) {
            __hip_atomic_store(gw, (unsigned long long)(g + 1u) << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while ((unsigned)(__hip_atomic_load(gw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) == g) {
                if (++spins > spin_limit) {
                    ok = 0;
                    if (info) atomicOr(info, RQLP_INFO_BARRIER_TIMEOUT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    gen = g + 1u;
    return s_ok != 0;
}

// Pivot agreement of the register-resident kernel through one key slot per
// workgroup and step instead of arrival counters (atomics on one address are
// serialised, about 20 ns each): once its column stores are complete, every
// workgroup stores its two keys, tagged with bit 63, into its own slot of the
// step (the slots are zero-filled before the launch); the last workgroup polls
// all slots with one wave, decides, and publishes the result with the new
// generation in the 64-bit word gw, which the others poll.  Keys of finite
// norms never have bit 63 set (norms are >= 0, the index key has only index
// bits), so the tag changes no comparison (a NaN norm loses its sign bit and
// still ranks above every finite one).  Bounded waits as in grid_sync_decide.
template <typename F>
__device__ __forceinline__ bool slot_agree(unsigned long long* slots, unsigned long long* gw, int G, unsigned& gen,
                                           unsigned& payload, int32_t* info, unsigned long long spin_limit,
                                           unsigned long long lk0, unsigned long long lk1, F decide) {
    constexpr unsigned long long TAG = 1ull << 63;
    __shared__ int s_ok;
    __shared__ unsigned s_pay;
    const unsigned g = gen;
    drain_and_sync();                                    // this workgroup's column stores are complete
    if (threadIdx.x == 0) {
        __hip_atomic_store(slots + 2 * blockIdx.x, lk0 | TAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(slots + 2 * blockIdx.x + 1, lk1 | TAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if ((int)blockIdx.x == G - 1) {
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            unsigned long long m0 = 0, m1 = 0;
            int ok = 1;
            // slots h0 + lane + 64 u, all loads of a poll in flight together
            for (int h0 = 0; h0 < G && ok; h0 += 256) {
                unsigned long long spins = 0;
                while (true) {
                    unsigned long long a[4], c[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int h = h0 + lane + 64 * u;
                        a[u] = TAG;
                        c[u] = TAG;
                        if (h < G) {
                            a[u] = __hip_atomic_load(slots + 2 * h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            c[u] = __hip_atomic_load(slots + 2 * h + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                    int here = 1;
#pragma unroll
                    for (int u = 0; u < 4; ++u) here &= (int)((a[u] & c[u]) >> 63);
                    if (__all(here)) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const unsigned long long ka = a[u] & ~TAG, kc = c[u] & ~TAG;
                            m0 = ka > m0 ? ka : m0;
                            m1 = kc > m1 ? kc : m1;
                        }
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
                    pay = decide(m0, m1);
                    __hip_atomic_store(gw, ((unsigned long long)(g + 1u) << 32) | pay, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
                s_pay = pay;
                s_ok = ok;
            }
        }
    } else if (threadIdx.x == 0) {
        int ok = 1;
        unsigned pay = 0;
        unsigned long long spins = 0;
        while (true) {
            const unsigned long long w = __hip_atomic_load(gw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)(w >> 32) != g) {
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
    RQLP_LDS_BARRIER();                                  // (the result word's store need not complete here)
    gen = g + 1u;
    payload = s_pay;
    return s_ok != 0;
}

template <bool SINGLE>
__global__ __launch_bounds__(CP_T) void cpqr_kernel(
    const double* __restrict__ M, int64_t ldm, int rows, int cols, int cpw, int kmax, int ibits,
    unsigned long long* keys, double* candcol, double* partial, unsigned* bar, int64_t* piv,
    double* Vh, int64_t ldv, double* beta_out, double* Rpiv, int64_t ldr, double* Rt, int64_t ldrt,
    int32_t* info, unsigned long long spin_limit) {
    extern __shared__ double lds[];
    const int ldl = rows | 1;
    double* colv = lds;                                  // cpw x ldl
    double* nrm2 = colv + (size_t)cpw * ldl;             // cpw
    double* v = nrm2 + cpw;                              // rows
    int* act = (int*)(v + rows);                         // cpw: -1 active, else pivot step

    __shared__ double s_red[CP_T / 64];
    __shared__ unsigned long long s_kred[2][CP_T / 64];
    __shared__ unsigned long long s_key[2];
    __shared__ double s_beta, s_mu, s_tol2;
    __shared__ int s_stop, s_rank;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x, g = blockIdx.x;
    const int c0 = g * cpw;
    const int ncol = (cols - c0) < cpw ? ((cols - c0) > 0 ? cols - c0 : 0) : cpw;
    unsigned gen = 0;

    for (int idx = tid; idx < ncol * rows; idx += CP_T) {
        const int c = idx / rows, i = idx % rows;
        colv[c * ldl + i] = M[i + (int64_t)(c0 + c) * ldm];
    }
    for (int c = tid; c < ncol; c += CP_T) act[c] = -1;
    __syncthreads();

    // exact column norms (4 threads per column) and ||M||_F^2
    for (int c = tid >> 2; c < ncol; c += CP_T / 4) {
        const int qd = tid & 3;
        double s = 0.0;
        for (int i = qd; i < rows; i += 4) s += colv[c * ldl + i] * colv[c * ldl + i];
        s += __shfl_xor(s, 1, RQLP_WAVE);
        s += __shfl_xor(s, 2, RQLP_WAVE);
        if (qd == 0) nrm2[c] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double f = 0.0;
        for (int c = 0; c < ncol; ++c) f += nrm2[c];
        if (!SINGLE) st_coherent(partial + g, f);
        s_tol2 = f;
    }
    if (!SINGLE) {
        unsigned pay;
        if (!grid_sync_decide(bar, G, gen, pay, info, spin_limit, nullptr, 0ull, 0ull, []() { return 0u; }))
            return;
        if (tid == 0) {
            double f = 0.0;
            for (int h = 0; h < G; ++h) f += ld_coherent(partial + h);
            s_tol2 = f;
        }
    }
    if (tid == 0) {
        const double tol = (double)(rows > cols ? rows : cols) * 2.220446049250313e-16;
        s_tol2 = tol * tol * s_tol2;
        s_stop = 0;
        s_rank = kmax;
    }
    // threads per column in the update: a power of two up to 16
    int tpc = 1;
    while (tpc < 16 && tpc * 2 * cpw <= CP_T) tpc *= 2;
    __syncthreads();

    for (int j = 0; j < kmax; ++j) {
        const int stopped = s_stop;
        // ---- 1. local candidates: by norm (k0) and by smallest index (k1) ----
        unsigned long long k0 = 0, k1 = 0;
        for (int c = tid; c < ncol; c += CP_T) {
            if (act[c] < 0) {
                const unsigned long long a = pivot_key(stopped ? 0.0 : nrm2[c], (unsigned)(c0 + c), ibits);
                const unsigned long long b = pivot_key(0.0, (unsigned)(c0 + c), ibits);
                k0 = a > k0 ? a : k0;
                k1 = b > k1 ? b : k1;
            }
        }
        k0 = wave_max_u64(k0);
        k1 = wave_max_u64(k1);
        if (lane == 0) {
            s_kred[0][wave] = k0;
            s_kred[1][wave] = k1;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long a = 0, b = 0;
            for (int w = 0; w < CP_T / 64; ++w) {
                a = s_kred[0][w] > a ? s_kred[0][w] : a;
                b = s_kred[1][w] > b ? s_kred[1][w] : b;
            }
            s_key[0] = a;
            s_key[1] = b;
        }
        __syncthreads();
        // ---- 2. agree on the pivot (the last arriver decides) ----
        unsigned pay = 0;
        {
            const unsigned long long lk0 = s_key[0], lk1 = s_key[1];
            const double tol2 = s_tol2;
            auto decide = [&](unsigned long long k0g, unsigned long long k1g) -> unsigned {
                unsigned stopnow = 0;
                if (!stopped) {
                    const double kv = key_value(k0g, ibits);
                    if (!(kv > tol2) && kv == kv) stopnow = 1;   // NaN norms never trigger the stop
                }
                const unsigned win = (stopped || stopnow) ? key_index(k1g, ibits) : key_index(k0g, ibits);
                return win | (stopnow << 31);
            };
            if (SINGLE) {
                if (tid == 0) s_red[0] = __longlong_as_double((long long)decide(lk0, lk1));
                __syncthreads();
                pay = (unsigned)__double_as_longlong(s_red[0]);
                __syncthreads();
            } else {
                if (lk0 != 0 && !stopped) {
                    const int bc = (int)key_index(lk0, ibits) - c0;
                    double* slot = candcol + ((size_t)(j & 1) * G + g) * rows;
                    for (int i = j + tid; i < rows; i += CP_T) st_coherent(slot + i, colv[bc * ldl + i]);
                }
                unsigned long long* ks = keys + (size_t)j * cp_key_words(G);
                unsigned long long* top = ks + 16 * ((G + CP_GROUP - 1) / CP_GROUP);
                if (!grid_sync_decide(bar, G, gen, pay, info, spin_limit, ks, lk0, lk1, [&]() {
                        return decide(__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                      __hip_atomic_load(top + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    }))
                    return;
            }
        }
        const int now_stopped = stopped | (int)(pay >> 31);
        const int gidx = (int)(pay & 0x7FFFFFFFu);
        const int owner = gidx / cpw;
        // ---- 3. reflector (Parlett's form, R(j, j) = ||x|| >= 0) ----
        if (!now_stopped) {
            const double* src = SINGLE ? (colv + (gidx - c0) * ldl)
                                       : (candcol + ((size_t)(j & 1) * G + owner) * rows);
            double sg = 0.0;
            for (int i = j + tid; i < rows; i += CP_T) {
                const double x = SINGLE ? src[i] : ld_coherent(src + i);
                v[i] = x;
                if (i > j) sg += x * x;
            }
            sg = wave_sum(sg);
            if (lane == 0) s_red[wave] = sg;
            __syncthreads();
            if (tid == 0) {
                double sigma = 0.0;
                for (int w = 0; w < CP_T / 64; ++w) sigma += s_red[w];
                const double x0 = v[j];
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
            for (int i = j + 1 + tid; i < rows; i += CP_T) v[i] *= rv0;
            if (tid == 0) v[j] = 1.0;
        } else {
            if (tid == 0) {
                s_beta = 0.0;
                s_mu = 0.0;
                if (!stopped) {
                    s_stop = 1;
                    s_rank = j;
                }
            }
        }
        __syncthreads();
        const double b = s_beta;
        // ---- 4. bookkeeping ----
        if (g == 0) {
            if (tid == 0) {
                if (piv) piv[j] = gidx;
                if (beta_out) beta_out[j] = b;
            }
            if (Vh) {
                for (int i = tid; i < rows; i += CP_T)
                    Vh[i + (int64_t)j * ldv] = (i < j || now_stopped) ? ((i == j) ? 1.0 : 0.0) : v[i];
            }
        }
        if (owner == g) {
            const int lc = gidx - c0;
            if (tid == 0) act[lc] = j;
            if (!now_stopped) {
                for (int i = j + tid; i < rows; i += CP_T) colv[lc * ldl + i] = (i == j) ? s_mu : 0.0;
            }
        }
        __syncthreads();
        // ---- 5. apply H = I - b v v^T to the active local columns, exact norms ----
        if (!now_stopped) {
            const int qd = tid & (tpc - 1);
            for (int c = tid / tpc; c < ncol; c += CP_T / tpc) {
                if (act[c] >= 0) continue;   // whole group of tpc lanes skips together
                double* col = colv + c * ldl;
                double d0 = 0.0, d1 = 0.0;
                int i = j + qd;
                for (; i + tpc < rows; i += 2 * tpc) {
                    d0 += v[i] * col[i];
                    d1 += v[i + tpc] * col[i + tpc];
                }
                if (i < rows) d0 += v[i] * col[i];
                double dot = d0 + d1;
                for (int off = tpc >> 1; off > 0; off >>= 1) dot += __shfl_xor(dot, off, RQLP_WAVE);
                const double w = b * dot;
                double s0 = 0.0, s1 = 0.0;
                i = j + qd;
                for (; i + tpc < rows; i += 2 * tpc) {
                    const double x = col[i] - w * v[i];
                    const double y = col[i + tpc] - w * v[i + tpc];
                    col[i] = x;
                    col[i + tpc] = y;
                    s0 += (i > j) ? x * x : 0.0;
                    s1 += y * y;
                }
                if (i < rows) {
                    const double x = col[i] - w * v[i];
                    col[i] = x;
                    s0 += (i > j) ? x * x : 0.0;
                }
                double sn = s0 + s1;
                for (int off = tpc >> 1; off > 0; off >>= 1) sn += __shfl_xor(sn, off, RQLP_WAVE);
                if (qd == 0) nrm2[c] = sn;
            }
        }
        __syncthreads();
    }

    // ---- write back: R^T in original column order, pivoted columns of R ----
    const int rank = s_rank;
    if (rank < kmax && g == 0 && tid == 0 && info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
    if (Rt) {
        for (int idx = tid; idx < ncol * rows; idx += CP_T) {
            const int c = idx % ncol, i = idx / ncol;
            Rt[(c0 + c) + (int64_t)i * ldrt] = (i >= rank) ? 0.0 : colv[c * ldl + i];
        }
    }
    if (Rpiv) {
        for (int c = 0; c < ncol; ++c) {
            const int js = act[c];
            if (js < 0) continue;
            for (int i = tid; i < rows; i += CP_T)
                Rpiv[i + (int64_t)js * ldr] = (i >= rank || i > js) ? 0.0 : colv[c * ldl + i];
        }
    }
}

// ---------------------------------------------------------------------------
// The same factorisation with the columns held in registers instead of LDS.
// 64 columns per workgroup, 16 per wave; lane l of a wave owns the RPT
// consecutive rows 16-group (l % 16) of the 4 columns 4 t + l / 16 (t < 4)
// of its wave.  Per pivot step: the 16 lanes of the workgroup's best column
// store its rows >= j and sigma (its squared norm below row j) straight from
// registers; slot_agree decides the pivot; every thread then reads the
// winner's sigma and x(j), forms the same reflector (Parlett's form, as in
// cpqr_kernel) and scales the published rows into v in LDS; the workgroup
// owning the pivot column writes the pivot, beta and the Householder vector.
// The dot products and norms reduce over the 16 lanes of a column with DPP;
// the update is branch-free (row masks are multipliers).  Inside the step
// loop only the drain before a key slot is published waits for this
// workgroup's global stores (the candidate column must be visible to the
// others first); the other barriers guard LDS data.
// lane permutation of a double within DPP rows of 16 lanes
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int CPR_RG = 16;                   // row groups (lanes per column)
constexpr int CPR_CT = 4;                    // columns per lane
constexpr int CPR_CPW = 64;                  // columns per workgroup
#ifndef CPR_GROUP
#define CPR_GROUP 16                         // workgroups per arrival counter
#endif
// scratch words: key slots of one step (slot_agree), counters + generation word (grid_barrier<CPR_GROUP>)
__host__ __device__ constexpr int cpr_key_words(int G) { return 2 * G; }
__host__ __device__ constexpr int cpr_bar_words(int G) { return 32 * ((G + CPR_GROUP - 1) / CPR_GROUP + 2); }

template <int RPT>
__global__ __launch_bounds__(CP_T) void cpqr_reg_kernel(
    const double* __restrict__ M, int64_t ldm, int rows, int cols, int kmax, int ibits, unsigned long long* keys,
    double* candcol, double* partial, unsigned* bar, int64_t* piv, double* Vh, int64_t ldv, double* beta_out,
    double* Rpiv, int64_t ldr, double* Rt, int64_t ldrt, int32_t* info, unsigned long long spin_limit) {
    __shared__ double v[CPR_RG * RPT];
    __shared__ double s_red[CP_T / 64];
    __shared__ unsigned long long s_kred[2][2][CP_T / 64];   // [step parity][k0, k1][wave]
    __shared__ double s_tol2;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x, g = blockIdx.x;
    const int c0 = g * CPR_CPW;
    const int qd = lane % CPR_RG, cs = lane / CPR_RG;
    const int r0 = qd * RPT;                             // first row held by this lane
    int col[CPR_CT], act[CPR_CT];                        // act: -1 active, >= 0 pivot step, -2 no column
    unsigned gen = 0;
    // generation word of grid_barrier<CPR_GROUP>, also the result word of slot_agree
    unsigned long long* gw = (unsigned long long*)(bar + 32 * ((G + CPR_GROUP - 1) / CPR_GROUP + 1));

    double x[CPR_CT][RPT];
#pragma unroll
    for (int t = 0; t < CPR_CT; ++t) {
        col[t] = c0 + 16 * wave + 4 * t + cs;
        const bool have = col[t] < cols;
        act[t] = have ? -1 : -2;
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            x[t][r] = (have && r0 + r < rows) ? M[r0 + r + (int64_t)col[t] * ldm] : 0.0;
    }
    for (int i = rows + tid; i < CPR_RG * RPT; i += CP_T) v[i] = 0.0;   // rows past the end reflect as zero

    // sum over the 16 lanes of a column (one DPP row): pair sums within quads,
    // then across the quads of each half row and across the two halves;
    // every lane ends with the same value (each level adds symmetric pairs)
    auto colsum = [](double s) {
        s += dpp_f64<0xB1>(s);     // quad_perm(1, 0, 3, 2)
        s += dpp_f64<0x4E>(s);     // quad_perm(2, 3, 0, 1)
        s += dpp_f64<0x141>(s);    // row_half_mirror
        s += dpp_f64<0x140>(s);    // row_mirror
        return s;
    };
    // exact column norms and ||M||_F^2
    double nrm2[CPR_CT];
    double fro = 0.0;
#pragma unroll
    for (int t = 0; t < CPR_CT; ++t) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) s += x[t][r] * x[t][r];
        nrm2[t] = colsum(s);
        fro += (qd == 0 && act[t] == -1) ? nrm2[t] : 0.0;
    }
    fro = wave_sum(fro);
    if (lane == 0) s_red[wave] = fro;
    __syncthreads();
    if (tid == 0) {
        double f = 0.0;
        for (int w = 0; w < CP_T / 64; ++w) f += s_red[w];
        st_coherent(partial + g, f);
    }
    if (!grid_barrier<CPR_GROUP>(bar, gw, G, gen, info, spin_limit)) return;
    if (tid == 0) {
        double f = 0.0;
        for (int h = 0; h < G; ++h) f += ld_coherent(partial + h);
        const double tol = (double)(rows > cols ? rows : cols) * 2.220446049250313e-16;
        s_tol2 = tol * tol * f;
    }
    __syncthreads();
    const double tol2 = s_tol2;
    const int64_t cstride = (int64_t)rows + 1;           // published column: rows values, then sigma
    int stopped = 0, rank = kmax;

    for (int j = 0; j < kmax; ++j) {
        // ---- 1. local candidates: by norm (k0) and by smallest index (k1) ----
        // (col, act and nrm2 are the same on the 16 lanes of a column, so the
        // wave maximum needs only one read per lane group)
        unsigned long long k0 = 0, k1 = 0;
#pragma unroll
        for (int t = 0; t < CPR_CT; ++t) {
            if (act[t] == -1) {
                const unsigned long long a = pivot_key(stopped ? 0.0 : nrm2[t], (unsigned)col[t], ibits);
                const unsigned long long b = pivot_key(0.0, (unsigned)col[t], ibits);
                k0 = a > k0 ? a : k0;
                k1 = b > k1 ? b : k1;
            }
        }
        k0 = rows_max_u64(k0);
        k1 = rows_max_u64(k1);
        // (double-buffered by step parity: nothing else separates this
        // step's reads from the next step's writes)
        unsigned long long(*kr)[CP_T / 64] = s_kred[j & 1];
        if (lane == 0) {
            kr[0][wave] = k0;
            kr[1][wave] = k1;
        }
        RQLP_LDS_BARRIER();
        unsigned long long lk0 = 0, lk1 = 0;
#pragma unroll
        for (int w = 0; w < CP_T / 64; ++w) {
            lk0 = kr[0][w] > lk0 ? kr[0][w] : lk0;
            lk1 = kr[1][w] > lk1 ? kr[1][w] : lk1;
        }
        // ---- 2. publish the local best column (rows >= j) and sigma, its
        // squared norm below row j, straight from the 16 lanes that hold it;
        // slot_agree makes these stores complete before the keys ----
        if (lk0 != 0 && !stopped) {
            const int bc = (int)key_index(lk0, ibits);
            double* dst = candcol + ((size_t)(j & 1) * G + g) * cstride;
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) {
                if (col[t] == bc) {
                    double sq = 0.0;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int i = r0 + r;
                        if (i >= j && i < rows) st_coherent(dst + i, x[t][r]);
                        const double xm = x[t][r] * ((i > j) ? 1.0 : 0.0);
                        sq += xm * xm;
                    }
                    sq = colsum(sq);
                    if (qd == 0) st_coherent(dst + rows, sq);
                }
            }
        }
        unsigned pay = 0;
        {
            auto decide = [&](unsigned long long k0g, unsigned long long k1g) -> unsigned {
                unsigned stopnow = 0;
                if (!stopped) {
                    const double kv = key_value(k0g, ibits);
                    if (!(kv > tol2) && kv == kv) stopnow = 1;   // NaN norms never trigger the stop
                }
                const unsigned win = (stopped || stopnow) ? key_index(k1g, ibits) : key_index(k0g, ibits);
                return win | (stopnow << 31);
            };
            unsigned long long* ks = keys + (size_t)j * cpr_key_words(G);
            if (!slot_agree(ks, gw, G, gen, pay, info, spin_limit, lk0, lk1, decide)) return;
        }
        const int stopnow = (int)(pay >> 31);
        const int now_stopped = stopped | stopnow;
        if (stopnow) {
            stopped = 1;
            rank = j;
        }
        const int gidx = (int)(pay & 0x7FFFFFFFu);
        const int owner = gidx / CPR_CPW;
        // ---- 3. reflector (Parlett's form, R(j, j) = ||x|| >= 0), formed by
        // every thread from the published sigma and x(j) ----
        double b = 0.0, mu = 0.0;
        if (!now_stopped) {
            const double* src = candcol + ((size_t)(j & 1) * G + owner) * cstride;
            constexpr int NLD = (CPR_RG * RPT + CP_T - 1) / CP_T;
            double xs[NLD];
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                const int i = j + 1 + tid + u * CP_T;
                xs[u] = (i < rows) ? ld_coherent(src + i) : 0.0;
            }
            const double sg = ld_coherent(src + rows), x0 = ld_coherent(src + j);
            mu = sqrt(x0 * x0 + sg);
            double v0;
            if (sg == 0.0) {
                v0 = 1.0;
                b = (x0 >= 0.0) ? 0.0 : 2.0;
            } else {
                v0 = (x0 <= 0.0) ? (x0 - mu) : (-sg / (x0 + mu));
                b = 2.0 * v0 * v0 / (sg + v0 * v0);
            }
            const double rv0 = (sg == 0.0) ? 0.0 : 1.0 / v0;
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                const int i = j + 1 + tid + u * CP_T;
                if (i < rows) v[i] = xs[u] * rv0;
            }
            if (tid == 0) {
                v[j] = 1.0;
                if (j > 0) v[j - 1] = 0.0;               // v(i) = 0 for every i < j
            }
            RQLP_LDS_BARRIER();
        }
        // ---- 4. bookkeeping, by the workgroup of the pivot column ----
        if (owner == g) {
            if (tid == 0) {
                if (piv) piv[j] = gidx;
                if (beta_out) beta_out[j] = b;
            }
            if (Vh) {
                for (int i = tid; i < rows; i += CP_T)
                    Vh[i + (int64_t)j * ldv] = (i < j || now_stopped) ? ((i == j) ? 1.0 : 0.0) : v[i];
            }
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) {
                if (col[t] != gidx) continue;
                act[t] = j;
                if (!now_stopped) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int i = r0 + r;
                        if (i >= j) x[t][r] = (i == j) ? mu : 0.0;
                    }
                }
            }
        }
        // ---- 5. apply H = I - b v v^T to the active columns, exact norms ----
        // (v is zero above row j and past the last row, so the sums run over
        // all rows; the row mask i > j is a multiplier, not a select)
        if (!now_stopped) {
            double vr[RPT], msk[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                vr[r] = v[r0 + r];
                msk[r] = (r0 + r > j) ? 1.0 : 0.0;
            }
            double dot[CPR_CT];
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) {
                double sd = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) sd += vr[r] * x[t][r];
                dot[t] = sd;
            }
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) dot[t] = colsum(dot[t]);
            double sn[CPR_CT];
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) {
                const double w = (act[t] == -1) ? b * dot[t] : 0.0;
                double ss = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    x[t][r] -= w * vr[r];
                    const double xm = x[t][r] * msk[r];
                    ss += xm * x[t][r];
                }
                sn[t] = ss;
            }
#pragma unroll
            for (int t = 0; t < CPR_CT; ++t) {
                const double sv = colsum(sn[t]);
                if (act[t] == -1) nrm2[t] = sv;
            }
        }
        // (v and the key buffers are written again only after the next
        // step's slot_agree, whose workgroup barrier every thread reaches
        // after its reads here)
    }

    // ---- write back: R^T in original column order, pivoted columns of R ----
    if (rank < kmax && g == 0 && tid == 0 && info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
#pragma unroll
    for (int t = 0; t < CPR_CT; ++t) {
        if (act[t] == -2) continue;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = r0 + r;
            if (i >= rows) continue;
            if (Rt) Rt[col[t] + (int64_t)i * ldrt] = (i >= rank) ? 0.0 : x[t][r];
            if (Rpiv && act[t] >= 0) Rpiv[i + (int64_t)act[t] * ldr] = (i >= rank || i > act[t]) ? 0.0 : x[t][r];
        }
    }
}

// ---------------------------------------------------------------------------
// Small matrices (rows <= 16 RPT, cols <= 32 CT) held whole in the registers of
// one workgroup of 512 threads: 16 lanes per column (one DPP row), lane group
// s (32 of them) holds the columns s + 32 t (t < CT), its lane qd the rows
// qd RPT .. qd RPT + RPT - 1.  No grid agreement: every thread combines the
// 8 waves' best keys itself and takes the same decision; two workgroup
// barriers per pivot step (the keys, then the winning column in LDS, from
// which every thread forms the same reflector), LDS-only ones: the step's
// global stores (pivot, beta, reflector) are never read back inside the
// kernel, and a full __syncthreads would wait for them.
// Pivot rule, reflector, rank stop and outputs as in cpqr_kernel.
constexpr int CPW_T = 512;
template <int RPT, int CT>
__global__ __launch_bounds__(CPW_T) void cpqr_wg_kernel(const double* __restrict__ M, int64_t ldm, int rows, int cols,
                                                        int kmax, int ibits, int64_t* piv, double* Vh, int64_t ldv,
                                                        double* beta_out, double* Rpiv, int64_t ldr, double* Rt,
                                                        int64_t ldrt, int32_t* info) {
    __shared__ double vcol[16 * RPT];
    __shared__ unsigned long long s_k[2][2][CPW_T / 64];   // [step parity][k0, k1][wave]
    __shared__ double s_part[CPW_T / 64];
    __shared__ double s_sig;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qd = lane & 15;
    const int slot = wave * 4 + (lane >> 4);
    const int r0 = qd * RPT;
    int col[CT], act[CT];
    double x[CT][RPT], nrm2[CT];
    auto colsum = [](double v) {
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        v += dpp_f64<0x141>(v);
        v += dpp_f64<0x140>(v);
        return v;
    };
    double fro = 0.0;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        col[t] = slot + 32 * t;
        const bool have = col[t] < cols;
        act[t] = have ? -1 : -2;
        double sq = 0.0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            x[t][r] = (have && r0 + r < rows) ? M[r0 + r + (int64_t)col[t] * ldm] : 0.0;
            sq += x[t][r] * x[t][r];
        }
        nrm2[t] = colsum(sq);
        fro += (qd == 0 && have) ? nrm2[t] : 0.0;
    }
    fro = wave_sum(fro);
    if (lane == 0) s_part[wave] = fro;
    __syncthreads();
    double tol2;
    {
        double f = 0.0;
        for (int w = 0; w < CPW_T / 64; ++w) f += s_part[w];
        const double tol = (double)(rows > cols ? rows : cols) * 2.220446049250313e-16;
        tol2 = tol * tol * f;
    }
    int stopped = 0, rank = kmax;
    for (int j = 0; j < kmax; ++j) {
        // ---- best keys: by norm (k0) and by smallest index (k1) ----
        // (col, act and nrm2 are the same on the 16 lanes of a column, so the
        // wave maximum needs only one read per lane group)
        unsigned long long k0 = 0, k1 = 0;
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            if (act[t] == -1) {
                const unsigned long long a = pivot_key(stopped ? 0.0 : nrm2[t], (unsigned)col[t], ibits);
                const unsigned long long b = pivot_key(0.0, (unsigned)col[t], ibits);
                k0 = a > k0 ? a : k0;
                k1 = b > k1 ? b : k1;
            }
        }
        k0 = rows_max_u64(k0);
        k1 = rows_max_u64(k1);
        // (double-buffered by step parity: after the rank stop a step has no
        // second barrier, and a fast wave's next keys must not overwrite
        // slots a slow wave is still reading)
        unsigned long long(*sk)[CPW_T / 64] = s_k[j & 1];
        if (lane == 0) {
            sk[0][wave] = k0;
            sk[1][wave] = k1;
        }
        RQLP_LDS_BARRIER();
        k0 = 0;
        k1 = 0;
#pragma unroll
        for (int w = 0; w < CPW_T / 64; ++w) {
            k0 = sk[0][w] > k0 ? sk[0][w] : k0;
            k1 = sk[1][w] > k1 ? sk[1][w] : k1;
        }
        int stopnow = 0;
        if (!stopped) {
            const double kv = key_value(k0, ibits);
            if (!(kv > tol2) && kv == kv) stopnow = 1;    // NaN norms never stop
        }
        const int win = (int)((stopped || stopnow) ? key_index(k1, ibits) : key_index(k0, ibits));
        const int now_stopped = stopped | stopnow;
        if (stopnow) {
            stopped = 1;
            rank = j;
        }
        if (!now_stopped) {
            // ---- the owner group stages the winning column (rows >= j) in
            // LDS with sigma = its squared norm below row j; every thread
            // then forms the same reflector (no third barrier) ----
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                if (col[t] == win) {
                    double sq = 0.0;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int i = r0 + r;
                        const double xv = x[t][r];
                        vcol[i] = (i >= j) ? xv : 0.0;
                        sq += (i > j) ? xv * xv : 0.0;
                    }
                    sq = colsum(sq);
                    if (qd == 0) s_sig = sq;
                }
            }
            RQLP_LDS_BARRIER();
            const double sg = s_sig, x0 = vcol[j];
            const double mu = sqrt(x0 * x0 + sg);
            double v0, b;
            if (sg == 0.0) {
                v0 = 1.0;
                b = (x0 >= 0.0) ? 0.0 : 2.0;
            } else {
                v0 = (x0 <= 0.0) ? (x0 - mu) : (-sg / (x0 + mu));
                b = 2.0 * v0 * v0 / (sg + v0 * v0);
            }
            const double rv0 = (sg == 0.0) ? 0.0 : 1.0 / v0;
            // the reflector rows of this lane and the row mask i > j, in
            // arithmetic form (v(i) = x(i) / v0 below row j, 1 at row j, 0
            // above: vcol is zero above row j): a select here compiles to a
            // divergent branch per row
            double vr[RPT], msk[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = r0 + r;
                msk[r] = (i > j) ? 1.0 : 0.0;
                vr[r] = vcol[i] * (rv0 * msk[r]) + ((i == j) ? 1.0 : 0.0);
            }
            if (tid == 0) {
                if (piv) piv[j] = win;
                if (beta_out) beta_out[j] = b;
            }
            if (Vh && tid < rows) Vh[tid + (int64_t)j * ldv] = (tid > j) ? vcol[tid] * rv0 : (tid == j ? 1.0 : 0.0);
            double dot[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                double sdot = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) sdot += vr[r] * x[t][r];
                dot[t] = sdot;
            }
#pragma unroll
            for (int t = 0; t < CT; ++t) dot[t] = colsum(dot[t]);
            // the pivot column becomes column j of R and leaves the active set
            // (its update below is then the identity)
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                if (col[t] == win) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int i = r0 + r;
                        if (i >= j) x[t][r] = (i == j) ? mu : 0.0;
                    }
                    act[t] = j;
                }
            }
            double sn[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const double w = (act[t] == -1) ? b * dot[t] : 0.0;
                double ss = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    x[t][r] -= w * vr[r];
                    const double xm = x[t][r] * msk[r];
                    ss += xm * x[t][r];
                }
                sn[t] = ss;
            }
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const double v = colsum(sn[t]);
                if (act[t] == -1) nrm2[t] = v;
            }
        } else {
            if (tid == 0) {
                if (piv) piv[j] = win;
                if (beta_out) beta_out[j] = 0.0;
            }
            if (Vh && tid < rows) Vh[tid + (int64_t)j * ldv] = (tid == j) ? 1.0 : 0.0;
#pragma unroll
            for (int t = 0; t < CT; ++t)
                if (col[t] == win) act[t] = j;
        }
        // vcol and s_sig are written again only after the next step's key barrier
    }
    if (rank < kmax && tid == 0 && info) atomicOr(info, RQLP_INFO_RANK_DEFICIENT);
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        if (act[t] == -2) continue;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = r0 + r;
            if (i >= rows) continue;
            if (Rt) Rt[col[t] + (int64_t)i * ldrt] = (i >= rank) ? 0.0 : x[t][r];
            if (Rpiv && act[t] >= 0) Rpiv[i + (int64_t)act[t] * ldr] = (i >= rank || i > act[t]) ? 0.0 : x[t][r];
        }
    }
}

// rows per lane (16 lanes per column) and column groups of the one-workgroup
// register kernel, 0 when the matrix does not fit
static int cpqr_wg_rpt(int64_t rows) {
    static const int opts[] = {2, 4, 6, 9, 12};
    for (int o : opts)
        if (16 * (int64_t)o >= rows) return o;
    return 0;
}
static int cpqr_wg_ct(int64_t cols) {
    static const int opts[] = {2, 4, 6};               // (one group spills: the compiler keeps more live)
    for (int o : opts)
        if (32 * (int64_t)o >= cols) return o;
    return 0;
}

// ---------------------------------------------------------------------------
static int index_bits(int64_t cols) {
    int b = 1;
    while ((1ll << b) <= cols) ++b;
    return b;
}

static size_t cpqr_lds(int64_t rows, int cpw) {
    const int ldl = (int)(rows | 1);
    return sizeof(double) * ((size_t)cpw * ldl + cpw + rows) + sizeof(int) * (size_t)cpw;
}

// rows held per thread by the register-resident kernel (0: rows too large)
static int cpqr_rpt(int64_t rows) {
    static const int opts[] = {2, 4, 6, 9, 12, 14, 17, 18, 24};
    for (int o : opts)
        if (CPR_RG * (int64_t)o >= rows) return o;
    return 0;
}

template <int RPT>
static int cpqr_reg_capacity() {
    return resident_capacity((const void*)cpqr_reg_kernel<RPT>, CP_T, 0);
}

static int cpqr_reg_cap(int rpt) {
    switch (rpt) {
        case 2: return cpqr_reg_capacity<2>();
        case 4: return cpqr_reg_capacity<4>();
        case 6: return cpqr_reg_capacity<6>();
        case 9: return cpqr_reg_capacity<9>();
        case 12: return cpqr_reg_capacity<12>();
        case 14: return cpqr_reg_capacity<14>();
        case 17: return cpqr_reg_capacity<17>();
        case 18: return cpqr_reg_capacity<18>();
        case 24: return cpqr_reg_capacity<24>();
        default: return 0;
    }
}

int cpqr_plan(int64_t rows, int64_t cols, CpqrPlan* plan) {
    const DeviceInfo& di = device_info();
    const size_t budget = di.max_lds > 0 ? di.max_lds : 65536;
    const int cus = di.num_cus > 0 ? di.num_cus : 1;
    plan->rpt = 0;
    plan->wg_rpt = 0;
    plan->wg_ct = 0;
    // one workgroup, everything in registers
    if (cpqr_wg_rpt(rows) > 0 && cpqr_wg_ct(cols) > 0) {
        plan->G = 1;
        plan->cpw = (int)cols;
        plan->lds = 0;
        plan->single = true;
        plan->wg_rpt = cpqr_wg_rpt(rows);
        plan->wg_ct = cpqr_wg_ct(cols);
        return 0;
    }
    // single workgroup when everything fits
    if (cpqr_lds(rows, (int)cols) <= budget && cols <= 512) {
        plan->G = 1;
        plan->cpw = (int)cols;
        plan->lds = cpqr_lds(rows, (int)cols);
        plan->single = true;
        return 0;
    }
    // columns in registers, 64 per workgroup, when the rows fit and the grid is co-resident
    const int rpt = cpqr_rpt(rows);
    if (rpt > 0) {
        const int64_t G = ceil_div(cols, CPR_CPW);
        if (G <= cpqr_reg_cap(rpt)) {
            plan->G = (int)G;
            plan->cpw = CPR_CPW;
            plan->lds = 0;
            plan->single = false;
            plan->rpt = rpt;
            return 0;
        }
    }
    int cpw = (int)ceil_div(cols, cus);
    if (cpw < 1) cpw = 1;
    while (cpqr_lds(rows, cpw) > budget && cpw > 1) --cpw;
    if (cpqr_lds(rows, cpw) > budget) return RQLP_E_UNSUPPORTED;
    const int64_t G = ceil_div(cols, cpw);
    if (G > cus) return RQLP_E_UNSUPPORTED;   // would not be co-resident (one workgroup per CU)
    plan->G = (int)G;
    plan->cpw = cpw;
    plan->lds = cpqr_lds(rows, cpw);
    plan->single = (G == 1);
    return 0;
}

size_t cpqr_scratch_bytes(int64_t rows, int64_t cols) {
    Arena ar(nullptr, 0);
    CpqrScratch sc;
    cpqr_carve(ar, rows, cols, &sc);
    return ar.used;
}

void cpqr_carve(Arena& ar, int64_t rows, int64_t cols, CpqrScratch* sc) {
    // sized for the larger of the two multi-workgroup grids (one per CU, or 64 columns each)
    int gm = device_info().num_cus > 0 ? device_info().num_cus : 256;
    if (ceil_div(cols, CPR_CPW) > gm) gm = (int)ceil_div(cols, CPR_CPW);
    const int64_t kmax = rows < cols ? rows : cols;
    const int kw = cp_key_words(gm) > cpr_key_words(gm) ? cp_key_words(gm) : cpr_key_words(gm);
    const int bw = cp_bar_words(gm) > cpr_bar_words(gm) ? cp_bar_words(gm) : cpr_bar_words(gm);
    sc->keys = ar.take<unsigned long long>((size_t)kmax * kw);
    sc->candcol = ar.take<double>((size_t)2 * gm * (rows + 1));   // a column and its sigma per slot
    sc->partial = ar.take<double>(gm);
    sc->bar = ar.take<unsigned>(bw);
}

int cpqr(const double* M, int64_t ldm, int64_t rows, int64_t cols, const CpqrScratch& sc, int64_t* piv,
         double* Vh, int64_t ldv, double* beta, double* Rpiv, int64_t ldr, double* Rt, int64_t ldrt,
         int32_t* info, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    CpqrPlan plan;
    RQLP_TRY(cpqr_plan(rows, cols, &plan));
    const int64_t kmax = rows < cols ? rows : cols;
    int ibits = index_bits(cols);
    int rows_i = (int)rows, cols_i = (int)cols, cpw = plan.cpw, kmax_i = (int)kmax;
    unsigned long long spin = CP_SPIN_LIMIT;
    {
        const int mx = (int)(device_info().max_lds > 0 ? device_info().max_lds : 65536);
        RQLP_TRY(raise_lds_limit((const void*)cpqr_kernel<true>, mx));
        RQLP_TRY(raise_lds_limit((const void*)cpqr_kernel<false>, mx));
    }
    if (plan.wg_rpt > 0) {
#define RQLP_CPW(R, C)                                                                                          \
    hipLaunchKernelGGL((cpqr_wg_kernel<R, C>), dim3(1), dim3(CPW_T), 0, s, M, ldm, rows_i, cols_i, kmax_i, ibits, piv, \
                       Vh, ldv, beta, Rpiv, ldr, Rt, ldrt, info)
#define RQLP_CPW_C(R)                        \
    switch (plan.wg_ct) {                    \
        case 2: RQLP_CPW(R, 2); break;       \
        case 4: RQLP_CPW(R, 4); break;       \
        default: RQLP_CPW(R, 6); break;      \
    }
        switch (plan.wg_rpt) {
            case 2: RQLP_CPW_C(2); break;
            case 4: RQLP_CPW_C(4); break;
            case 6: RQLP_CPW_C(6); break;
            case 9: RQLP_CPW_C(9); break;
            default: RQLP_CPW_C(12); break;
        }
#undef RQLP_CPW_C
#undef RQLP_CPW
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    }
    if (plan.single) {
        hipLaunchKernelGGL(cpqr_kernel<true>, dim3(1), dim3(CP_T), plan.lds, s, M, ldm, rows_i, cols_i, cpw,
                           kmax_i, ibits, sc.keys, sc.candcol, sc.partial, sc.bar, piv, Vh, ldv, beta, Rpiv,
                           ldr, Rt, ldrt, info, spin);
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    }
    const size_t kw = plan.rpt > 0 ? (size_t)cpr_key_words(plan.G) : (size_t)cp_key_words(plan.G);
    const size_t bw = plan.rpt > 0 ? (size_t)cpr_bar_words(plan.G) : (size_t)cp_bar_words(plan.G);
    RQLP_TRY(fill_zero_bytes(sc.keys, sizeof(unsigned long long) * (size_t)kmax * kw, s));
    RQLP_TRY(fill_zero_bytes(sc.bar, sizeof(unsigned) * bw, s));
    // Plain launches: the grid is at most the number of workgroups the device
    // holds at once (checked against the occupancy), so every workgroup is
    // resident once the previous kernel of the stream has drained, and every
    // wait inside is bounded (RQLP_INFO_BARRIER_TIMEOUT).  A cooperative
    // launch gives the same residency at the cost of idle device time around
    // the launch.
    if (plan.rpt > 0) {
#define RQLP_CPR(R)                                                                                             \
    hipLaunchKernelGGL(cpqr_reg_kernel<R>, dim3(plan.G), dim3(CP_T), 0, s, M, ldm, rows_i, cols_i, kmax_i, ibits, \
                       sc.keys, sc.candcol, sc.partial, sc.bar, piv, Vh, ldv, beta, Rpiv, ldr, Rt, ldrt, info, spin)
        switch (plan.rpt) {
            case 2: RQLP_CPR(2); break;
            case 4: RQLP_CPR(4); break;
            case 6: RQLP_CPR(6); break;
            case 9: RQLP_CPR(9); break;
            case 12: RQLP_CPR(12); break;
            case 14: RQLP_CPR(14); break;
            case 17: RQLP_CPR(17); break;
            case 18: RQLP_CPR(18); break;
            default: RQLP_CPR(24); break;
        }
#undef RQLP_CPR
        return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
    }
    if ((int64_t)resident_capacity((const void*)cpqr_kernel<false>, CP_T, plan.lds) < plan.G)
        return RQLP_E_UNSUPPORTED;
    hipLaunchKernelGGL(cpqr_kernel<false>, dim3(plan.G), dim3(CP_T), plan.lds, s, M, ldm, rows_i, cols_i, cpw,
                       kmax_i, ibits, sc.keys, sc.candcol, sc.partial, sc.bar, piv, Vh, ldv, beta, Rpiv, ldr, Rt,
                       ldrt, info, spin);
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

// ---------------------------------------------------------------------------
// Y = H_0 H_1 ... H_{k-1} X, one wave per column, the column held in registers
// (RPL rows per lane), the next reflectors prefetched while the current one is
// applied.
template <int RPL>
__global__ __launch_bounds__(256) void apply_householder_kernel(int rows, int k, const double* __restrict__ Vh,
                                                                int64_t ldv, const double* __restrict__ beta,
                                                                const double* __restrict__ X, int64_t ldx,
                                                                const int64_t* __restrict__ unit, int ncols,
                                                                double* __restrict__ Y, int64_t ldy) {
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= ncols) return;
    double x[RPL];
    const int64_t u = unit ? unit[col] : (int64_t)col;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        x[r] = (i < rows) ? (X ? X[i + (int64_t)col * ldx] : (i == u ? 1.0 : 0.0)) : 0.0;
    }
    if (k > 0) {
        // D reflectors in flight in a ring of registers (the loop is unrolled
        // by D, so no register is copied while its load is outstanding); the
        // loads are unconditional from clamped rows (no branches that would
        // make the compiler wait for all of them), rows past the end are
        // masked where they are used
        constexpr int D = 4;
        int ic[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            ic[r] = i < rows ? i : rows - 1;
        }
        double vb[D][RPL];
        auto load = [&](double (&v)[RPL], int j) {
            const double* p = Vh + (int64_t)(j > 0 ? j : 0) * ldv;
#pragma unroll
            for (int r = 0; r < RPL; ++r) v[r] = p[ic[r]];
        };
        auto apply = [&](const double (&v)[RPL], int j) {
            const double bj = beta[j];
            double dot = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                dot += (i >= j && i < rows) ? v[r] * x[r] : 0.0;
            }
            dot = wave_sum(dot);
            const double w = bj * dot;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i >= j && i < rows) x[r] -= w * v[r];
            }
        };
#pragma unroll
        for (int d = 0; d < D; ++d) load(vb[d], k - 1 - d);
        int j = k - 1;
        for (; j >= D - 1; j -= D) {                  // vb[d] holds reflector j - d
#pragma unroll
            for (int d = 0; d < D; ++d) {
                apply(vb[d], j - d);
                load(vb[d], j - d - D);
            }
        }
#pragma unroll
        for (int d = 0; d < D - 1; ++d)
            if (d <= j) apply(vb[d], j - d);          // the last j + 1 reflectors
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < rows) Y[i + (int64_t)col * ldy] = x[r];
    }
}

int apply_householder(int64_t rows, int64_t k, const double* Vh, int64_t ldv, const double* beta,
                      const double* X, int64_t ldx, const int64_t* unit, int64_t ncols, double* Y,
                      int64_t ldy, hipStream_t s) {
    if (rows <= 0 || ncols <= 0) return 0;
    dim3 grid((unsigned)ceil_div(ncols, 4));
    const int rpl = (int)ceil_div(rows, 64);
#define RQLP_AH(R)                                                                                       \
    hipLaunchKernelGGL(apply_householder_kernel<R>, grid, dim3(256), 0, s, (int)rows, (int)k, Vh, ldv, beta, \
                       X, ldx, unit, (int)ncols, Y, ldy)
    if (rpl <= 1) RQLP_AH(1);
    else if (rpl <= 2) RQLP_AH(2);
    else if (rpl <= 4) RQLP_AH(4);
    else if (rpl <= 5) RQLP_AH(5);
    else if (rpl <= 8) RQLP_AH(8);
    else if (rpl <= 17) RQLP_AH(17);
    else return RQLP_E_UNSUPPORTED;
#undef RQLP_AH
    return hipGetLastError() == hipSuccess ? 0 : RQLP_E_HIP;
}

}  // namespace rqlp
