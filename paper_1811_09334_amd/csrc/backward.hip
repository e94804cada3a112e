// Adjoint of the randomized QLP pipeline with frozen pivots: dA for a
// cotangent dT on the triangular factor T (Algorithm 2.1 with d = 0; the
// range finder with q subspace iterations).
//
// The forward is recomputed from A and Omega (nothing is stored between the
// calls): Y0 = A Omega, V0 = orth(Y0), W_i = orth(A^T V_{i-1}), V_i = orth(A W_i),
// B = V_q^T A, then with the frozen pivots X1 = B(:, piv0) = Q0 R01 (square
// QR), R0^T = B^T Q0 (original column order) and R0^T(:, piv1) = Q1 L^T.
// Every QR is CholeskyQR (two FP64 passes, or FP32 shifted CholeskyQR3 for
// FP32 panels), which also yields R^T and R^{-T} as products of the Cholesky
// factors and of their inverses.
//
// Reverse sweep, with the thin-QR adjoint of X = QR (rows >= cols):
//     dX = (dQ + Q sym(M)) R^{-T},  M = R dR^T - dQ^T Q,
//     sym(M) = tril(M) + tril(M, -1)^T;
// the wide QR of B Pi0 splits into the square QR of the pivot columns and
// R02 = Q0^T X2 (dX2 = Q0 dR02, dQ0 += X2 dR02^T); B = V^T A gives
// dV = A dB^T and dA += V dB; each product of the range finder contributes
// one rank-l term to dA.  All terms are gathered into one product
//     dA = [V_q, dY_q, V_{q-1}, dY_{q-1}, ..., V_0, dY_0]
//          [dB^T, W_q, dZ_q, W_{q-1}, dZ_{q-1}, ..., dZ_1, Omega]^T
// with inner dimension (2q + 2) l, so the m x n output is written once.
// The passes over A run in the panels' precision (FP32 or FP64); the l x l
// and n x l algebra of the small stage is FP64.
#include <array>

#include "common.hpp"
#include "kernels.hpp"

namespace rqlp {
namespace {

// ---------------------------------------------------------------------------
// small kernels

inline dim3 grid_for(int64_t total) {
    int64_t b = ceil_div(total, 256);
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// Y(:, j) = X(:, idx[j]) (gather) or Y(:, idx[j]) = X(:, j) (scatter); indices
// outside [0, limit) are skipped (they are reported by check_pivots_kernel).
template <typename T>
__global__ void permute_cols_kernel(int64_t rows, int64_t nc, const T* __restrict__ X, int64_t ldx,
                                    const int64_t* __restrict__ idx, int64_t limit, T* __restrict__ Y, int64_t ldy,
                                    int scatter) {
    const int64_t total = rows * nc;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % rows, j = t / rows;
        const int64_t c = idx[j];
        if (c < 0 || c >= limit) continue;
        if (scatter) Y[i + c * ldy] = X[i + j * ldx];
        else Y[i + j * ldy] = X[i + c * ldx];
    }
}

// Y(:, idx[j]) = 0
__global__ void zero_cols_kernel(int64_t rows, int64_t nc, const int64_t* __restrict__ idx, int64_t limit,
                                 double* __restrict__ Y, int64_t ldy) {
    const int64_t total = rows * nc;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % rows, j = t / rows;
        const int64_t c = idx[j];
        if (c >= 0 && c < limit) Y[i + c * ldy] = 0.0;
    }
}

// S = sym(M) with M(a, b) = P(b, a) - D(a, b) on the lower triangle (a >= b);
// P and D optional; written as TO.
template <typename TO>
__global__ void sym_lower_kernel(int64_t c, const double* __restrict__ P, int64_t ldp, const double* __restrict__ D,
                                 int64_t ldd, TO* __restrict__ S, int64_t lds) {
    const int64_t total = c * c;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % c, j = t / c;
        const int64_t a = i >= j ? i : j, b = i >= j ? j : i;
        double v = 0.0;
        if (P) v += P[b + a * ldp];
        if (D) v -= D[a + b * ldd];
        S[i + j * lds] = (TO)v;
    }
}

// U = triu(X) (flip == 0) or U(i, j) = X(j, i) for i <= j (flip == 1); zero below
__global__ void triu_kernel(int64_t c, const double* __restrict__ X, int64_t ldx, double* __restrict__ U, int64_t ldu,
                            int flip) {
    const int64_t total = c * c;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % c, j = t / c;
        U[i + j * ldu] = (i <= j) ? (flip ? X[j + i * ldx] : X[i + j * ldx]) : 0.0;
    }
}

// Y (cols x rows, TO) = X^T (X: rows x cols, double), 32 x 32 LDS tiles
template <typename TO>
__global__ void transpose_cast_kernel(int64_t rows, int64_t cols, const double* __restrict__ X, int64_t ldx,
                                      TO* __restrict__ Y, int64_t ldy) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    for (int jj = ty; jj < 32; jj += 8) {
        const int64_t i = i0 + tx, j = j0 + jj;
        tile[jj][tx] = (i < rows && j < cols) ? X[i + j * ldx] : 0.0;
    }
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int64_t j = j0 + tx, i = i0 + ii;
        if (i < rows && j < cols) Y[j + i * ldy] = (TO)tile[tx][ii];
    }
}

// piv0: l distinct indices in [0, n); piv1: a permutation of [0, l).  Sets
// RQLP_INFO_BAD_PIVOTS otherwise.  One workgroup; a bit per index in LDS.
__global__ __launch_bounds__(256) void check_pivots_kernel(int64_t l, int64_t n, const int64_t* __restrict__ piv0,
                                                           const int64_t* __restrict__ piv1, int32_t* info) {
    extern __shared__ unsigned bits[];                 // ceil(n / 32) + ceil(l / 32) words
    const int64_t w0 = (n + 31) / 32, w1 = (l + 31) / 32;
    for (int64_t t = threadIdx.x; t < w0 + w1; t += blockDim.x) bits[t] = 0u;
    __syncthreads();
    int bad = 0;
    for (int64_t j = threadIdx.x; j < l; j += blockDim.x) {
        const int64_t a = piv0[j], b = piv1[j];
        if (a < 0 || a >= n) {
            bad = 1;
        } else {
            const unsigned mask = 1u << (a & 31);
            if (atomicOr(bits + (a >> 5), mask) & mask) bad = 1;
        }
        if (b < 0 || b >= l) {
            bad = 1;
        } else {
            const unsigned mask = 1u << (b & 31);
            if (atomicOr(bits + w0 + (b >> 5), mask) & mask) bad = 1;
        }
    }
    if (bad && info) atomicOr(info, RQLP_INFO_BAD_PIVOTS);
}

template <typename T>
int copy_panel(int64_t rows, int64_t cols, const T* X, int64_t ldx, T* Y, int64_t ldy, hipStream_t s) {
    if constexpr (sizeof(T) == sizeof(double)) return copy_matrix(rows, cols, (const double*)X, ldx, (double*)Y, ldy, s);
    else return cast_matrix<float, float>(rows, cols, (const float*)X, ldx, (float*)Y, ldy, s);
}

template <typename TO>
int from_double(int64_t rows, int64_t cols, const double* X, int64_t ldx, TO* Y, int64_t ldy, hipStream_t s) {
    if constexpr (sizeof(TO) == sizeof(double)) return copy_matrix(rows, cols, X, ldx, (double*)Y, ldy, s);
    else return cast_matrix<double, float>(rows, cols, X, ldx, (float*)Y, ldy, s);
}

// ---------------------------------------------------------------------------
// workspace of one backward call (T: element type of A and of the panels)
template <typename T>
struct BwdBufs {
    T* Left;        // m x K
    T* Right;       // n x K
    T* Ya;          // max(m, n) x l working panels
    T* Yb;
    T* tmp;
    T* tmp2;
    double* ws;     // split-K partials of the panel products (FP64 accumulation)
    size_t ws_elems;
    double* dws;    // split-K partials of the FP64 products
    size_t dws_elems;
    double* RinvV;  // (q + 1) blocks of l x l: R^{-T} of V_0 .. V_q
    double* RinvW;  // q blocks: R^{-T} of W_1 .. W_q
    double* B;      // l x n
    float* B32;     // l x n (FP32 panels)
    double* C1;     // l x l
    double* C1b;
    double* RT01;   // R01^T
    double* Rinv01;
    double* R0t;    // n x l
    double* Mm;     // n x l
    double* Mm2;
    double* RTL;    // L = (L^T)^T, the R^T of the second QR
    double* RinvL;
    double* dLt;
    double* dM;     // n x l
    double* dR0t;   // n x l
    double* dR0o;   // l x n
    double* dR01;
    double* dB;     // l x n
    double* dQ0;
    double* dX1;
    double* Md;     // l x l scratch
    double* Pd;
    double* Ld;     // FP64 Cholesky factor of a pass
    double* Lid;    // its inverse
    double* Rtmp;
    double* X1;     // l x l scratch of the square-QR adjoint
    double* X2;
    double* X3;
    T* Gt;          // l x l Gram in T
    T* St;          // l x l
    T* RinvT_T;     // l x l
    float* Li32;    // l x l (FP32 panels)
    unsigned* sync;
    int32_t* shifted;
    int32_t* info;
};

template <typename T>
void carve_bwd(Arena& ar, int64_t m, int64_t n, int64_t l, int q, bool need_omega, BwdBufs<T>* b) {
    const int64_t K = (2 * q + 2) * l;
    const int64_t mx = m > n ? m : n;
    (void)need_omega;          // Omega lives in the last block of Right
    b->Left = ar.take<T>(m * K);
    b->Right = ar.take<T>(n * K);
    b->Ya = ar.take<T>(mx * l);
    b->Yb = ar.take<T>(mx * l);
    b->tmp = ar.take<T>(mx * l);
    b->tmp2 = ar.take<T>(mx * l);
    size_t e = 0;
    for (auto sh : {std::array<int64_t, 3>{m, l, n}, {n, l, m}, {l, l, m}, {l, l, n}, {m, l, l}, {n, l, l},
                    {m, n, K}}) {
        const size_t x = gemm_workspace_elems(sh[0], sh[1], sh[2]);
        if (x > e) e = x;
    }
    b->ws_elems = e;
    b->ws = ar.take<double>(e);
    e = 0;
    for (auto sh : {std::array<int64_t, 3>{l, l, l}, {n, l, l}, {l, l, n}, {l, n, l}, {n, l, m}}) {
        const size_t x = gemm_workspace_elems(sh[0], sh[1], sh[2]);
        if (x > e) e = x;
    }
    b->dws_elems = e;
    b->dws = ar.take<double>(e);
    b->RinvV = ar.take<double>((q + 1) * l * l);
    b->RinvW = ar.take<double>((q > 0 ? q : 1) * l * l);
    b->B = ar.take<double>(l * n);
    b->B32 = sizeof(T) == sizeof(float) ? ar.take<float>(l * n) : nullptr;
    b->C1 = ar.take<double>(l * l);
    b->C1b = ar.take<double>(l * l);
    b->RT01 = ar.take<double>(l * l);
    b->Rinv01 = ar.take<double>(l * l);
    b->R0t = ar.take<double>(n * l);
    b->Mm = ar.take<double>(n * l);
    b->Mm2 = ar.take<double>(n * l);
    b->RTL = ar.take<double>(l * l);
    b->RinvL = ar.take<double>(l * l);
    b->dLt = ar.take<double>(l * l);
    b->dM = ar.take<double>(n * l);
    b->dR0t = ar.take<double>(n * l);
    b->dR0o = ar.take<double>(l * n);
    b->dR01 = ar.take<double>(l * l);
    b->dB = ar.take<double>(l * n);
    b->dQ0 = ar.take<double>(l * l);
    b->dX1 = ar.take<double>(l * l);
    b->Md = ar.take<double>(l * l);
    b->Pd = ar.take<double>(l * l);
    b->Ld = ar.take<double>(l * l);
    b->Lid = ar.take<double>(l * l);
    b->Rtmp = ar.take<double>(l * l);
    b->X1 = ar.take<double>(l * l);
    b->X2 = ar.take<double>(l * l);
    b->X3 = ar.take<double>(l * l);
    b->Gt = ar.take<T>(l * l);
    b->St = ar.take<T>(l * l);
    b->RinvT_T = ar.take<T>(l * l);
    b->Li32 = ar.take<float>(l * l);
    b->sync = ar.take<unsigned>(CHOL_SYNC_WORDS);
    b->shifted = ar.take<int32_t>(1);
    b->info = ar.take<int32_t>(1);
}

// Products of panels in T with FP64 MFMA arithmetic: FP64 operands as they
// are, FP32 operands converted on load (exact products, FP64 sums).
template <typename T>
int pgemm(BwdBufs<T>& b, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
          int64_t ldb, T* C, int64_t ldc, double alpha, double beta, hipStream_t s, const int32_t* gate = nullptr,
          int gate_mode = 0) {
    if constexpr (sizeof(T) == sizeof(double))
        return gemm<double>(ta, tb, M, N, K, (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, false,
                            alpha, beta, b.ws, b.ws_elems, s, gate, gate_mode);
    else
        return gemm_f32_acc64(ta, tb, M, N, K, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, false,
                              alpha, beta, b.ws, b.ws_elems, s, gate, gate_mode);
}

// ---------------------------------------------------------------------------
// QR of a rows x c panel (buf0, leading dimension ld) by CholeskyQR, recording
// R^T (optional) and R^{-T}; FP64: two passes, FP32: shifted CholeskyQR3 (the
// third pass conditional on a shift).  Returns the buffer holding Q.
template <typename T>
int qr_record(BwdBufs<T>& b, hipStream_t s, int64_t rows, int64_t c, T* buf0, T* buf1, int64_t ld, double* RT,
              double* RinvT, T** out) {
    constexpr bool F32 = sizeof(T) == sizeof(float);
    const int npass = F32 ? 3 : 2;
    const double u = F32 ? 1.1920928955078125e-7 : 2.220446049250313e-16;
    const double shift = F32 ? 11.0 * (sqrt((double)rows) + (double)c + 1.0) * u
                             : 11.0 * ((double)rows * c + (double)c * (c + 1)) * u;
    T* cur = buf0;
    T* nxt = buf1;
    for (int pass = 0; pass < npass; ++pass) {
        const int32_t* gate = (F32 && pass == 2) ? b.shifted : nullptr;
        RQLP_TRY(pgemm<T>(b, true, false, c, c, rows, cur, ld, cur, ld, b.Gt, c, 1.0, 0.0, s,
                         gate, 1));
        RQLP_TRY(chol_inv<T>(c, b.Gt, c, b.Ld, b.Lid, F32 ? b.Li32 : nullptr, c, shift, b.info, s, gate,
                             pass < 2 ? b.shifted : nullptr, b.sync, pass == 0 ? 1 : 2));
        const T* Lup = F32 ? (const T*)b.Li32 : (const T*)b.Lid;
        RQLP_TRY(pgemm<T>(b, false, true, rows, c, c, cur, ld, Lup, c, nxt, ld, 1.0, 0.0, s,
                         gate, 2));
        if (pass == 0) {
            RQLP_TRY(copy_matrix(c, c, b.Lid, c, RinvT, c, s));
            if (RT) RQLP_TRY(copy_matrix(c, c, b.Ld, c, RT, c, s));
        } else {
            RQLP_TRY(gemm<double>(false, false, c, c, c, b.Lid, c, RinvT, c, b.Rtmp, c, false, 1.0, 0.0, b.dws,
                                  b.dws_elems, s));
            RQLP_TRY(copy_matrix(c, c, b.Rtmp, c, RinvT, c, s));
            if (RT) {
                RQLP_TRY(gemm<double>(false, false, c, c, c, RT, c, b.Ld, c, b.Rtmp, c, false, 1.0, 0.0, b.dws,
                                      b.dws_elems, s));
                RQLP_TRY(copy_matrix(c, c, b.Rtmp, c, RT, c, s));
            }
        }
        T* t = cur;
        cur = nxt;
        nxt = t;
    }
    *out = cur;
    return 0;
}

// dX = (dQ + Q sym(M)) R^{-T}, M = R dR^T - dQ^T Q, for the rows x c thin QR
// X = Q R.  dQ, RT (= R^T) and dR are optional (absent = zero).  dX may not
// alias dQ.  FP64 c x c algebra; the panel products in T.
template <typename T>
int qr_adjoint(BwdBufs<T>& b, hipStream_t s, int64_t rows, int64_t c, const T* Q, int64_t ldq, const T* dQ,
               int64_t lddq, const double* RT, const double* dR, const double* RinvT, T* dX, int64_t lddx) {
    const double* Pd = nullptr;
    const double* Dd = nullptr;
    if (RT && dR) {
        // R dR^T = (dR R^T)^T: keep P = dR RT, used transposed in sym_lower
        RQLP_TRY(gemm<double>(false, false, c, c, c, dR, c, RT, c, b.Pd, c, false, 1.0, 0.0, b.dws, b.dws_elems, s));
        Pd = b.Pd;
    }
    if (dQ) {
        RQLP_TRY(pgemm<T>(b, true, false, c, c, rows, dQ, lddq, Q, ldq, b.Gt, c, 1.0, 0.0, s));
        if constexpr (sizeof(T) == sizeof(double)) RQLP_TRY(copy_matrix(c, c, (const double*)b.Gt, c, b.Md, c, s));
        else RQLP_TRY((cast_matrix<float, double>(c, c, (const float*)b.Gt, c, b.Md, c, s)));
        Dd = b.Md;
    }
    hipLaunchKernelGGL((sym_lower_kernel<T>), grid_for(c * c), dim3(256), 0, s, c, Pd, c, Dd, c, b.St, c);
    RQLP_HIP_TRY(hipGetLastError());
    // tmp = dQ + Q S
    if (dQ) {
        RQLP_TRY(copy_panel<T>(rows, c, dQ, lddq, b.tmp, rows, s));
        RQLP_TRY(pgemm<T>(b, false, false, rows, c, c, Q, ldq, b.St, c, b.tmp, rows, 1.0, 1.0, s));
    } else {
        RQLP_TRY(pgemm<T>(b, false, false, rows, c, c, Q, ldq, b.St, c, b.tmp, rows, 1.0, 0.0, s));
    }
    RQLP_TRY(from_double<T>(c, c, RinvT, c, b.RinvT_T, c, s));
    return pgemm<T>(b, false, false, rows, c, c, b.tmp, rows, b.RinvT_T, c, dX, lddx, 1.0, 0.0, s);
}

template <typename T>
int backward_impl(const T* A, int64_t lda, int64_t m, int64_t n, int64_t l, int q, uint64_t seed, int precision,
                  const T* Omega, int64_t ldo, const int64_t* piv0, const int64_t* piv1, const double* dT,
                  int64_t lddt, T* dA, int64_t ldda, int32_t* info_user, BwdBufs<T>& b, hipStream_t s) {
    const int64_t K = (2 * q + 2) * l;
    int32_t* info = info_user ? info_user : b.info;
    if (info_user) b.info = info_user;
    RQLP_TRY(fill_zero_bytes(info, sizeof(int32_t), s));
    {
        // the check keeps a bit per index in LDS (up to 2^19 columns)
        const size_t words = (size_t)((n + 31) / 32 + (l + 31) / 32);
        if (words * sizeof(unsigned) <= 65536) {
            hipLaunchKernelGGL(check_pivots_kernel, dim3(1), dim3(256), words * sizeof(unsigned), s, l, n, piv0,
                               piv1, info);
            RQLP_HIP_TRY(hipGetLastError());
        }
    }
    auto Lblk = [&](int blk) { return b.Left + (int64_t)blk * l * m; };
    auto Rblk = [&](int blk) { return b.Right + (int64_t)blk * l * n; };
    // ---- Omega into the last block of Right ----
    T* OmB = Rblk(2 * q + 1);
    if (Omega) RQLP_TRY(copy_panel<T>(n, l, Omega, ldo, OmB, n, s));
    else RQLP_TRY(generate_omega(n, l, seed, precision, OmB, n, s));
    // ---- forward recompute of the range finder ----
    T* Q = nullptr;
    RQLP_TRY(pgemm<T>(b, false, false, m, l, n, A, lda, OmB, n, b.Ya, m, 1.0, 0.0, s));
    RQLP_TRY(qr_record<T>(b, s, m, l, b.Ya, b.Yb, m, nullptr, b.RinvV, &Q));
    RQLP_TRY(copy_panel<T>(m, l, Q, m, Lblk(2 * q), m, s));                       // V_0
    for (int it = 1; it <= q; ++it) {
        const T* Vprev = Lblk(2 * (q - it + 1));
        RQLP_TRY(pgemm<T>(b, true, false, n, l, m, A, lda, Vprev, m, b.Ya, n, 1.0, 0.0, s));
        RQLP_TRY(qr_record<T>(b, s, n, l, b.Ya, b.Yb, n, nullptr, b.RinvW + (it - 1) * l * l, &Q));
        T* W = Rblk(2 * (q - it) + 1);
        RQLP_TRY(copy_panel<T>(n, l, Q, n, W, n, s));                             // W_it
        RQLP_TRY(pgemm<T>(b, false, false, m, l, n, A, lda, W, n, b.Ya, m, 1.0, 0.0, s));
        RQLP_TRY(qr_record<T>(b, s, m, l, b.Ya, b.Yb, m, nullptr, b.RinvV + it * l * l, &Q));
        RQLP_TRY(copy_panel<T>(m, l, Q, m, Lblk(2 * (q - it)), m, s));            // V_it
    }
    const T* Vq = Lblk(0);
    // ---- B = V_q^T A, the frozen-pivot small stage ----
    if constexpr (sizeof(T) == sizeof(double)) {
        RQLP_TRY(gemm<double>(true, false, n, l, m, (const double*)A, lda, (const double*)Vq, m, b.B, l, true, 1.0,
                              0.0, b.ws, b.ws_elems, s));
    } else {
        RQLP_TRY(gemm_f32_acc64(true, false, n, l, m, (const float*)A, lda, (const float*)Vq, m, b.B32, l, true, 1.0,
                                0.0, b.ws, b.ws_elems, s));
        RQLP_TRY((cast_matrix<float, double>(l, n, b.B32, l, b.B, l, s)));
    }
    hipLaunchKernelGGL((permute_cols_kernel<double>), grid_for(l * l), dim3(256), 0, s, l, l, b.B, l, piv0, n, b.C1,
                       l, 0);
    RQLP_HIP_TRY(hipGetLastError());
    // the FP64 small QRs use the FP64 view of the same scratch
    BwdBufs<double> sm;
    sm.ws = b.dws;
    sm.ws_elems = b.dws_elems;
    sm.dws = b.dws;
    sm.dws_elems = b.dws_elems;
    sm.Gt = b.Md;
    sm.St = b.Pd;
    sm.RinvT_T = b.Rtmp;
    sm.Li32 = b.Li32;
    sm.Ld = b.Ld;
    sm.Lid = b.Lid;
    sm.Rtmp = b.Rtmp;
    sm.sync = b.sync;
    sm.shifted = b.shifted;
    sm.info = info;
    sm.Md = b.Md;
    sm.Pd = b.Pd;
    double* Q0 = nullptr;
    {
        // Rtmp is RinvT_T of the FP64 view: give qr_record its own product scratch
        BwdBufs<double> sq = sm;
        sq.Rtmp = b.dX1;
        RQLP_TRY(qr_record<double>(sq, s, l, l, b.C1, b.C1b, l, b.RT01, b.Rinv01, &Q0));
    }
    // R0^T (original column order) = B^T Q0, then its columns in piv1 order
    RQLP_TRY(gemm<double>(true, false, n, l, l, b.B, l, Q0, l, b.R0t, n, false, 1.0, 0.0, b.dws, b.dws_elems, s));
    hipLaunchKernelGGL((permute_cols_kernel<double>), grid_for(n * l), dim3(256), 0, s, n, l, b.R0t, n, piv1, l, b.Mm,
                       n, 0);
    RQLP_HIP_TRY(hipGetLastError());
    double* Q1 = nullptr;
    {
        BwdBufs<double> sq = sm;
        sq.Rtmp = b.dX1;
        RQLP_TRY(qr_record<double>(sq, s, n, l, b.Mm, b.Mm2, n, b.RTL, b.RinvL, &Q1));
    }
    // ---- reverse sweep of the small stage ----
    hipLaunchKernelGGL(triu_kernel, grid_for(l * l), dim3(256), 0, s, l, dT, lddt, b.dLt, l, 1);   // dL^T
    RQLP_HIP_TRY(hipGetLastError());
    {
        BwdBufs<double> sa = sm;
        sa.tmp = b.dR0t;                     // n x l scratch of the adjoint (free until the scatter)
        sa.St = b.X1;
        sa.Gt = b.X2;
        sa.Md = b.X3;
        sa.Pd = b.Pd;
        sa.RinvT_T = b.Rtmp;
        RQLP_TRY(qr_adjoint<double>(sa, s, n, l, Q1, n, nullptr, 0, b.RTL, b.dLt, b.RinvL, b.dM, n));
    }
    RQLP_TRY(fill_zero_bytes(b.dR0t, sizeof(double) * n * l, s));
    hipLaunchKernelGGL((permute_cols_kernel<double>), grid_for(n * l), dim3(256), 0, s, n, l, b.dM, n, piv1, l,
                       b.dR0t, n, 1);
    RQLP_HIP_TRY(hipGetLastError());
    RQLP_TRY(transpose_matrix(n, l, b.dR0t, n, b.dR0o, l, 0, s));                    // dR0 (l x n)
    hipLaunchKernelGGL((permute_cols_kernel<double>), grid_for(l * l), dim3(256), 0, s, l, l, b.dR0o, l, piv0, n,
                       b.Md, l, 0);
    RQLP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(triu_kernel, grid_for(l * l), dim3(256), 0, s, l, b.Md, l, b.dR01, l, 0);
    RQLP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(zero_cols_kernel, grid_for(l * l), dim3(256), 0, s, l, l, piv0, n, b.dR0o, l);
    RQLP_HIP_TRY(hipGetLastError());
    RQLP_TRY(gemm<double>(false, false, l, n, l, Q0, l, b.dR0o, l, b.dB, l, false, 1.0, 0.0, b.dws, b.dws_elems, s));
    RQLP_TRY(gemm<double>(false, true, l, l, n, b.B, l, b.dR0o, l, b.dQ0, l, false, 1.0, 0.0, b.dws, b.dws_elems, s));
    {
        BwdBufs<double> sa = sm;
        sa.tmp = b.C1b;                      // l x l scratch (the QR of C1 left Q0 in C1)
        sa.St = b.X1;
        sa.Gt = b.X2;
        sa.Md = b.X3;
        sa.Pd = b.Pd;
        sa.RinvT_T = b.Rtmp;
        RQLP_TRY(qr_adjoint<double>(sa, s, l, l, Q0, l, b.dQ0, l, b.RT01, b.dR01, b.Rinv01, b.dX1, l));
    }
    hipLaunchKernelGGL((permute_cols_kernel<double>), grid_for(l * l), dim3(256), 0, s, l, l, b.dX1, l, piv0, n, b.dB,
                       l, 1);
    RQLP_HIP_TRY(hipGetLastError());
    // ---- reverse sweep of the range finder ----
    T* dBt = Rblk(0);
    hipLaunchKernelGGL((transpose_cast_kernel<T>), dim3((unsigned)ceil_div(l, 32), (unsigned)ceil_div(n, 32)),
                       dim3(256), 0, s, l, n, b.dB, l, dBt, n);
    RQLP_HIP_TRY(hipGetLastError());
    RQLP_TRY(pgemm<T>(b, false, false, m, l, n, A, lda, dBt, n, b.tmp2, m, 1.0, 0.0, s));  // dV_q
    RQLP_TRY(qr_adjoint<T>(b, s, m, l, Vq, m, b.tmp2, m, nullptr, nullptr, b.RinvV + q * l * l, Lblk(1), m));   // dY_q
    for (int it = q; it >= 1; --it) {
        const T* dY = Lblk(2 * (q - it) + 1);
        const T* W = Rblk(2 * (q - it) + 1);
        RQLP_TRY(pgemm<T>(b, true, false, n, l, m, A, lda, dY, m, b.tmp2, n, 1.0, 0.0, s));  // dW
        T* dZ = Rblk(2 * (q - it) + 2);
        RQLP_TRY(qr_adjoint<T>(b, s, n, l, W, n, b.tmp2, n, nullptr, nullptr, b.RinvW + (it - 1) * l * l, dZ, n));
        RQLP_TRY(pgemm<T>(b, false, false, m, l, n, A, lda, dZ, n, b.tmp2, m, 1.0, 0.0, s));  // dV
        const T* Vprev = Lblk(2 * (q - it) + 2);
        RQLP_TRY(qr_adjoint<T>(b, s, m, l, Vprev, m, b.tmp2, m, nullptr, nullptr, b.RinvV + (it - 1) * l * l,
                               Lblk(2 * (q - it) + 3), m));                          // dY_{it-1}
    }
    // ---- dA = Left Right^T ----
    return pgemm<T>(b, false, true, m, n, K, b.Left, m, b.Right, n, dA, ldda, 1.0, 0.0, s);
}

int check_backward_args(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                        int precision) {
    if (m < 1) return -3;
    if (n < 1 || n > m) return -4;
    if (lda < m) return -2;
    if (k < 2) return -5;
    if (p < 2 || k + p > n) return -6;
    if (q < 0) return -7;
    if (d < 0) return -8;
    if (b < 0) return -9;
    if (precision < RQLP_F64 || precision > RQLP_MIXED_BF16X3) return -10;
    if (!A) return -1;
    return 0;
}

template <typename T>
size_t backward_bytes(int64_t m, int64_t n, int64_t l, int q) {
    Arena ar(nullptr, 0);
    BwdBufs<T> b;
    carve_bwd<T>(ar, m, n, l, q, true, &b);
    return ar.used + 256;
}

Arena arena_aligned(void* work, size_t bytes) {
    uintptr_t a = (uintptr_t)work;
    uintptr_t al = (a + 255) & ~uintptr_t(255);
    size_t lost = (size_t)(al - a);
    return Arena(work ? (void*)al : nullptr, bytes > lost ? bytes - lost : 0);
}

}  // namespace
}  // namespace rqlp

using namespace rqlp;

extern "C" {

int rqlp_backward_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b, int precision,
                                 size_t* bytes) {
    RQLP_TRY(check_backward_args((const void*)1, m, m, n, k, p, q, d, b, precision));
    if (!bytes) return -9;
    if (d != 0 || b != 0 || (precision != RQLP_F64 && precision != RQLP_F32)) return RQLP_E_UNSUPPORTED;
    *bytes = precision == RQLP_F64 ? backward_bytes<double>(m, n, k + p, q) : backward_bytes<float>(m, n, k + p, q);
    return 0;
}

int rqlp_backward(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                  int precision, uint64_t seed, const void* Omega, int64_t ldo, const int64_t* piv0,
                  const int64_t* piv1, const double* dT, int64_t lddt, const void* dQ, int64_t lddq, const void* dP,
                  int64_t lddp, const void* saved, void* dA, int64_t ldda, int32_t* info, void* work,
                  size_t work_bytes, void* stream) {
    RQLP_TRY(check_backward_args(A, lda, m, n, k, p, q, d, b, precision));
    const int64_t l = k + p;
    if (Omega && ldo < n) return -13;
    if (!piv0) return -14;
    if (!piv1) return -15;
    if (!dT) return -16;
    if (lddt < l) return -17;
    if (dQ && lddq < m) return -19;
    if (dP && lddp < n) return -21;
    if (!dA) return -23;
    if (ldda < m) return -24;
    if (!work) return -26;
    if (d != 0 || b != 0 || dQ || dP || saved || (precision != RQLP_F64 && precision != RQLP_F32))
        return RQLP_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Arena ar = arena_aligned(work, work_bytes);
    if (precision == RQLP_F64) {
        BwdBufs<double> bb;
        carve_bwd<double>(ar, m, n, l, q, Omega == nullptr, &bb);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        return backward_impl<double>((const double*)A, lda, m, n, l, q, seed, precision, (const double*)Omega, ldo,
                                     piv0, piv1, dT, lddt, (double*)dA, ldda, info, bb, s);
    }
    BwdBufs<float> bb;
    carve_bwd<float>(ar, m, n, l, q, Omega == nullptr, &bb);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    return backward_impl<float>((const float*)A, lda, m, n, l, q, seed, precision, (const float*)Omega, ldo, piv0,
                                piv1, dT, lddt, (float*)dA, ldda, info, bb, s);
}

}  // extern "C"
