// C ABI of the randomized QLP library: argument checks, workspace carve-up
// and the enqueue order of the hot path (Algorithms 2.1, 2.2, 4.1).
#include <string.h>

#include "common.hpp"
#include "kernels.hpp"

using namespace rqlp;

namespace {

constexpr double kEps = 2.220446049250313e-16;

// CholeskyQR shift scale of Fukaya et al. (2020): 11 (m c + c (c + 1)) u.
double shift_scale(int64_t rows, int64_t c) { return 11.0 * ((double)rows * c + (double)c * (c + 1)) * kEps; }

// Scratch for orthonormalising a rows x c panel.
struct OrthoScratch {
    double* G;      // c x c Gram
    double* L1;     // c x c Cholesky factor of pass 1
    double* L2;     // c x c Cholesky factor of pass 2
    double* Li;     // c x c inverse of the current factor
};

void carve_ortho(Arena& ar, int64_t c, OrthoScratch* o) {
    o->G = ar.take<double>(c * c);
    o->L1 = ar.take<double>(c * c);
    o->L2 = ar.take<double>(c * c);
    o->Li = ar.take<double>(c * c);
}

struct Ctx {
    hipStream_t s;
    int32_t* info;
    double* gws;
    size_t gws_elems;
    OrthoScratch o;
};

// CholeskyQR2 of the rows x c panel held in buf0 (leading dimension ld):
// two passes of G = X^T X, G = L L^T, X <- X L^{-T}.  Returns the buffer
// holding the orthonormal result (buf0 or buf1; buf0 is overwritten).  RT
// (c x c, optional) receives R^T = L1 L2 (lower triangular), where
// X_in = V R is the QR factorisation with diag(R) > 0.
int cholqr2(Ctx& cx, int64_t rows, int64_t c, double* buf0, double* buf1, int64_t ld, double* RT,
            double** out) {
    double* cur = buf0;
    double* nxt = buf1;
    for (int pass = 0; pass < 2; ++pass) {
        RQLP_TRY(gemm<double>(true, false, c, c, rows, cur, ld, cur, ld, cx.o.G, c, false, 1.0, 0.0, cx.gws,
                              cx.gws_elems, cx.s));
        double* Lp = pass == 0 ? cx.o.L1 : cx.o.L2;
        RQLP_TRY(chol_inv(c, cx.o.G, c, Lp, cx.o.Li, c, shift_scale(rows, c), cx.info, cx.s));
        RQLP_TRY(gemm<double>(false, true, rows, c, c, cur, ld, cx.o.Li, c, nxt, ld, false, 1.0, 0.0, cx.gws,
                              cx.gws_elems, cx.s));
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (RT)
        RQLP_TRY(gemm<double>(false, false, c, c, c, cx.o.L1, c, cx.o.L2, c, RT, c, false, 1.0, 0.0, cx.gws,
                              cx.gws_elems, cx.s));
    *out = cur;
    return 0;
}

size_t max_gemm_ws(int64_t m, int64_t n, int64_t l) {
    const int64_t shapes[][3] = {{m, l, n}, {n, l, m}, {l, l, m}, {l, l, n}, {m, l, l},
                                 {n, l, l}, {l, l, l}, {l, n, m}};
    size_t mx = 0;
    for (auto& sh : shapes) {
        size_t e = gemm_workspace_elems(sh[0], sh[1], sh[2]);
        if (e > mx) mx = e;
    }
    return mx;
}

// Device buffers of one rqlp_factor call (FP64 path).
struct FactorBufs {
    double* Om;
    double* Y;
    double* Y2;
    double* Z;
    double* Z2;
    double* B;
    double* gws;
    size_t gws_elems;
    OrthoScratch o;
    CpqrScratch cs;
    double* Vh0;
    double* beta0;
    int64_t* piv0;
    double* Vh1;
    double* beta1;
    int64_t* piv1;
    double* Lt;
    double* Rtil;
    double* RtT;
    double* RiT;
    double* Ml;
    double* Mr;
    double* Mt;
    double* Xi;
    double* Xi2;
    int32_t* info;
};

void carve_factor(Arena& ar, int64_t m, int64_t n, int64_t l, bool need_omega, FactorBufs* f) {
    f->Om = need_omega ? ar.take<double>(n * l) : nullptr;
    f->Y = ar.take<double>(m * l);
    f->Y2 = ar.take<double>(m * l);
    f->Z = ar.take<double>(n * l);
    f->Z2 = ar.take<double>(n * l);
    f->B = ar.take<double>(l * n);
    f->gws_elems = max_gemm_ws(m, n, l);
    f->gws = ar.take<double>(f->gws_elems);
    carve_ortho(ar, l, &f->o);
    cpqr_carve(ar, l, n, &f->cs);
    f->Vh0 = ar.take<double>(l * l);
    f->beta0 = ar.take<double>(l);
    f->piv0 = ar.take<int64_t>(l);
    f->Vh1 = ar.take<double>(l * l);
    f->beta1 = ar.take<double>(l);
    f->piv1 = ar.take<int64_t>(l);
    f->Lt = ar.take<double>(l * l);
    f->Rtil = ar.take<double>(l * l);
    f->RtT = ar.take<double>(l * l);
    f->RiT = ar.take<double>(l * l);
    f->Ml = ar.take<double>(l * l);
    f->Mr = ar.take<double>(l * l);
    f->Mt = ar.take<double>(l * l);
    f->Xi = ar.take<double>(l * l);
    f->Xi2 = ar.take<double>(l * l);
    f->info = ar.take<int32_t>(1);
}

bool valid_precision(int p) { return p >= RQLP_F64 && p <= RQLP_MIXED_BF16X3; }

int check_factor_args(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                      int precision) {
    if (m < 1) return -3;
    if (n < 1 || n > m) return -4;
    if (lda < m) return -2;
    if (k < 2) return -5;
    if (p < 2 || k + p > n) return -6;
    if (q < 0) return -7;
    if (d < 0) return -8;
    if (b < 0 || (b > 0 && d != 0)) return -9;
    if (!valid_precision(precision)) return -10;
    if (A == nullptr) return -1;
    return 0;
}

// Aligns the caller's workspace pointer to 256 bytes.
Arena arena_for(void* work, size_t bytes) {
    uintptr_t a = (uintptr_t)work;
    uintptr_t al = (a + 255) & ~uintptr_t(255);
    size_t lost = (size_t)(al - a);
    return Arena(work ? (void*)al : nullptr, bytes > lost ? bytes - lost : 0);
}

}  // namespace

extern "C" {

const char* rqlp_version(void) { return "rqlp-gfx950 0.1"; }

const char* rqlp_status_string(int status) {
    if (status == RQLP_OK) return "success";
    if (status == RQLP_E_WORKSPACE) return "workspace too small";
    if (status == RQLP_E_HIP) return "HIP runtime or launch error";
    if (status == RQLP_E_UNSUPPORTED) return "arguments valid but not supported by this build";
    if (status < 0 && status > -100) return "invalid argument (see the argument index -status)";
    return "unknown status";
}

int rqlp_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b, int precision,
                        size_t* bytes) {
    int st = check_factor_args((const void*)1, m, m, n, k, p, q, d, b, precision);
    if (st) return st;
    if (!bytes) return -9;
    Arena ar(nullptr, 0);
    FactorBufs f;
    carve_factor(ar, m, n, k + p, true, &f);
    *bytes = ar.used + 256;
    return 0;
}

int rqlp_generate_omega(int64_t n, int64_t l, uint64_t seed, int precision, void* Omega, int64_t ldo,
                        void* stream) {
    if (n < 0) return -1;
    if (l < 0) return -2;
    if (!valid_precision(precision)) return -4;
    if (Omega == nullptr && n * l > 0) return -5;
    if (ldo < (n > 1 ? n : 1)) return -6;
    return generate_omega(n, l, seed, precision, Omega, ldo, (hipStream_t)stream);
}

int rqlp_factor(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                int precision, uint64_t seed, const void* Omega, int64_t ldo, void* Q, int64_t ldq, double* T,
                int64_t ldt, void* P, int64_t ldp, int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info,
                char* uplo, void* work, size_t work_bytes, void* stream) {
    RQLP_TRY(check_factor_args(A, lda, m, n, k, p, q, d, b, precision));
    const int64_t l = k + p;
    if (Omega && ldo < n) return -13;
    if (!Q) return -14;
    if (ldq < m) return -15;
    if (!T) return -16;
    if (ldt < l) return -17;
    if (!P) return -18;
    if (ldp < n) return -19;
    if (!work) return -25;
    if (precision != RQLP_F64 || b != 0) return RQLP_E_UNSUPPORTED;

    hipStream_t s = (hipStream_t)stream;
    Arena ar = arena_for(work, work_bytes);
    FactorBufs f;
    carve_factor(ar, m, n, l, Omega == nullptr, &f);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    {
        CpqrPlan pl;
        RQLP_TRY(cpqr_plan(l, n, &pl));
        RQLP_TRY(cpqr_plan(l, l, &pl));
    }
    const double* Ad = (const double*)A;
    int32_t* inf = info ? info : f.info;
    RQLP_TRY(fill_zero_bytes(inf, sizeof(int32_t), s));

    Ctx cx{s, inf, f.gws, f.gws_elems, f.o};

    // ---- range finder: Omega, Y = A Omega, V = qr(Y) (+ q subspace iterations) ----
    const double* Om = (const double*)Omega;
    int64_t ldom = ldo;
    if (!Om) {
        RQLP_TRY(generate_omega(n, l, seed, RQLP_F64, f.Om, n, s));
        Om = f.Om;
        ldom = n;
    }
    RQLP_TRY(gemm<double>(false, false, m, l, n, Ad, lda, Om, ldom, f.Y, m, false, 1.0, 0.0, f.gws, f.gws_elems, s));
    double* V = nullptr;
    RQLP_TRY(cholqr2(cx, m, l, f.Y, f.Y2, m, nullptr, &V));
    for (int it = 0; it < q; ++it) {
        RQLP_TRY(gemm<double>(true, false, n, l, m, Ad, lda, V, m, f.Z, n, false, 1.0, 0.0, f.gws, f.gws_elems, s));
        double* W = nullptr;
        RQLP_TRY(cholqr2(cx, n, l, f.Z, f.Z2, n, nullptr, &W));
        double* ydst = (V == f.Y) ? f.Y2 : f.Y;
        RQLP_TRY(gemm<double>(false, false, m, l, n, Ad, lda, W, n, ydst, m, false, 1.0, 0.0, f.gws, f.gws_elems, s));
        double* other = (ydst == f.Y) ? f.Y2 : f.Y;
        RQLP_TRY(cholqr2(cx, m, l, ydst, other, m, nullptr, &V));
    }
    // ---- projection B = V^T A (as (A^T V)^T, stored l x n) ----
    RQLP_TRY(gemm<double>(true, false, n, l, m, Ad, lda, V, m, f.B, l, true, 1.0, 0.0, f.gws, f.gws_elems, s));
    // ---- first CPQR: B Pi0 = Q0 R0; R0^T kept in original column order (n x l) ----
    RQLP_TRY(cpqr(f.B, l, l, n, f.cs, f.piv0, f.Vh0, l, f.beta0, nullptr, l, f.Z, n, inf, s));
    // ---- second stage: R0^T = Qt Rtil (CholeskyQR2), Rtil^T kept ----
    double* Qt = nullptr;
    RQLP_TRY(cholqr2(cx, n, l, f.Z, f.Z2, n, f.RtT, &Qt));
    char tri = 'L';
    if (d == 0) {
        // Rtil Pi1 = Qhat L^T (pivoted, l x l); Q1 = Qt Qhat
        RQLP_TRY(transpose_matrix(l, l, f.RtT, l, f.Rtil, l, 0, s));
        RQLP_TRY(cpqr(f.Rtil, l, l, l, f.cs, f.piv1, f.Vh1, l, f.beta1, f.Lt, l, nullptr, 1, inf, s));
        RQLP_TRY(apply_householder(l, l, f.Vh1, l, f.beta1, nullptr, 0, nullptr, l, f.Mr, l, s));
        RQLP_TRY(gemm<double>(false, false, n, l, l, Qt, n, f.Mr, l, (double*)P, ldp, false, 1.0, 0.0, f.gws,
                              f.gws_elems, s));
        // Q0 Pi1
        RQLP_TRY(apply_householder(l, l, f.Vh0, l, f.beta0, nullptr, 0, f.piv1, l, f.Ml, l, s));
        RQLP_TRY(transpose_matrix(l, l, f.Lt, l, T, ldt, 'L', s));
    } else {
        // inner unpivoted QR steps R(i-1)^T = Q(i) R(i); R(1)^T = Rtil^T, Q(1) = Qt.
        // Only transposed R factors are formed: the next step's input is R(i)^T.
        double* RprevT = f.RtT;
        bool have_left = false, have_right = false;
        for (int i = 2; i <= d; ++i) {
            RQLP_TRY(copy_matrix(l, l, RprevT, l, f.Xi, l, s));
            double* Qi = nullptr;
            double* RnewT = (RprevT == f.RiT) ? f.RtT : f.RiT;
            RQLP_TRY(cholqr2(cx, l, l, f.Xi, f.Xi2, l, RnewT, &Qi));
            double*& Macc = (i % 2 == 0) ? f.Ml : f.Mr;
            bool& have = (i % 2 == 0) ? have_left : have_right;
            if (!have) {
                RQLP_TRY(copy_matrix(l, l, Qi, l, Macc, l, s));
                have = true;
            } else {
                RQLP_TRY(gemm<double>(false, false, l, l, l, Macc, l, Qi, l, f.Mt, l, false, 1.0, 0.0, f.gws,
                                      f.gws_elems, s));
                double* t = Macc;
                Macc = f.Mt;
                f.Mt = t;
            }
            RprevT = RnewT;
        }
        if (have_right)
            RQLP_TRY(gemm<double>(false, false, n, l, l, Qt, n, f.Mr, l, (double*)P, ldp, false, 1.0, 0.0, f.gws,
                                  f.gws_elems, s));
        else
            RQLP_TRY(copy_matrix(n, l, Qt, n, (double*)P, ldp, s));
        // Q0 * (product of even-index inner factors)
        RQLP_TRY(apply_householder(l, l, f.Vh0, l, f.beta0, have_left ? f.Ml : nullptr, l, nullptr, l, f.Xi, l,
                                   s));
        double* t = f.Ml;
        f.Ml = f.Xi;
        f.Xi = t;
        if (d % 2 == 1) {
            RQLP_TRY(copy_matrix(l, l, RprevT, l, T, ldt, s));                 // L = R(d)^T
        } else {
            RQLP_TRY(transpose_matrix(l, l, RprevT, l, T, ldt, 'U', s));       // R(d) itself
            tri = 'U';
        }
    }
    // ---- assembly: Q = V (Q_B) ----
    RQLP_TRY(gemm<double>(false, false, m, l, l, V, m, f.Ml, l, (double*)Q, ldq, false, 1.0, 0.0, f.gws, f.gws_elems, s));
    RQLP_TRY(finish_lvals(l, T, ldt, lvals, inf, s));
    if (piv0) RQLP_TRY(copy_i64(l, f.piv0, piv0, s));
    if (piv1) RQLP_TRY(copy_i64(l, d == 0 ? f.piv1 : nullptr, piv1, s));
    if (uplo) *uplo = tri;
    return 0;
}

// ---- building blocks ----
int rqlp_gemm_workspace(int64_t m, int64_t n, int64_t c, int precision, size_t* bytes) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (c < 0) return -3;
    if (precision != RQLP_F64 && precision != RQLP_F32) return -4;
    if (!bytes) return -5;
    size_t e1 = gemm_workspace_elems(m, c, n), e2 = gemm_workspace_elems(n, c, m);
    *bytes = (e1 > e2 ? e1 : e2) * (precision == RQLP_F64 ? 8 : 4) + 256;
    return 0;
}

int rqlp_sketch(const void* A, int64_t lda, int64_t m, int64_t n, const void* X, int64_t ldx, int64_t c, void* Y,
                int64_t ldy, int precision, void* work, size_t work_bytes, void* stream) {
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -2;
    if (ldx < (n > 1 ? n : 1)) return -6;
    if (c < 0) return -7;
    if (ldy < (m > 1 ? m : 1)) return -9;
    if (precision != RQLP_F64 && precision != RQLP_F32) return -10;
    if (m * n * c > 0 && (!A || !X || !Y)) return !A ? -1 : (!X ? -5 : -8);
    Arena ar = arena_for(work, work_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (precision == RQLP_F64) {
        size_t e = gemm_workspace_elems(m, c, n);
        double* ws = ar.take<double>(e);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        return gemm<double>(false, false, m, c, n, (const double*)A, lda, (const double*)X, ldx, (double*)Y, ldy, false,
                            1.0, 0.0, ws, e, s);
    }
    size_t e = gemm_workspace_elems(m, c, n);
    float* ws = ar.take<float>(e);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    return gemm<float>(false, false, m, c, n, (const float*)A, lda, (const float*)X, ldx, (float*)Y, ldy, false, 1.0f,
                       0.0f, ws, e, s);
}

int rqlp_project(const void* A, int64_t lda, int64_t m, int64_t n, const void* V, int64_t ldv, int64_t c, void* B,
                 int64_t ldb, int precision, void* work, size_t work_bytes, void* stream) {
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -2;
    if (ldv < (m > 1 ? m : 1)) return -6;
    if (c < 0) return -7;
    if (ldb < (c > 1 ? c : 1)) return -9;
    if (precision != RQLP_F64 && precision != RQLP_F32) return -10;
    if (m * n * c > 0 && (!A || !V || !B)) return !A ? -1 : (!V ? -5 : -8);
    Arena ar = arena_for(work, work_bytes);
    hipStream_t s = (hipStream_t)stream;
    size_t e = gemm_workspace_elems(n, c, m);
    if (precision == RQLP_F64) {
        double* ws = ar.take<double>(e);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        return gemm<double>(true, false, n, c, m, (const double*)A, lda, (const double*)V, ldv, (double*)B, ldb, true,
                            1.0, 0.0, ws, e, s);
    }
    float* ws = ar.take<float>(e);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    return gemm<float>(true, false, n, c, m, (const float*)A, lda, (const float*)V, ldv, (float*)B, ldb, true, 1.0f, 0.0f,
                       ws, e, s);
}

int rqlp_orthonormalize_workspace(int64_t m, int64_t c, size_t* bytes) {
    if (m < 0) return -1;
    if (c < 0 || c > m) return -2;
    if (!bytes) return -3;
    Arena ar(nullptr, 0);
    OrthoScratch o;
    carve_ortho(ar, c, &o);
    size_t e = gemm_workspace_elems(c, c, m);
    if (gemm_workspace_elems(m, c, c) > e) e = gemm_workspace_elems(m, c, c);
    if (gemm_workspace_elems(c, c, c) > e) e = gemm_workspace_elems(c, c, c);
    ar.take<double>(e);
    ar.take<double>(c * c);
    ar.take<double>(m * c);
    ar.take<double>(m * c);
    ar.take<int32_t>(1);
    *bytes = ar.used + 256;
    return 0;
}

int rqlp_orthonormalize(const double* Y, int64_t ldy, int64_t m, int64_t c, double* V, int64_t ldv, double* R,
                        int64_t ldr, int32_t* info, void* work, size_t work_bytes, void* stream) {
    if (m < 0) return -3;
    if (c < 0 || c > m) return -4;
    if (ldy < (m > 1 ? m : 1)) return -2;
    if (ldv < (m > 1 ? m : 1)) return -6;
    if (R && ldr < (c > 1 ? c : 1)) return -8;
    if (m * c > 0 && (!Y || !V)) return !Y ? -1 : -5;
    if (m * c == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    Arena ar = arena_for(work, work_bytes);
    OrthoScratch o;
    carve_ortho(ar, c, &o);
    size_t e = gemm_workspace_elems(c, c, m);
    if (gemm_workspace_elems(m, c, c) > e) e = gemm_workspace_elems(m, c, c);
    if (gemm_workspace_elems(c, c, c) > e) e = gemm_workspace_elems(c, c, c);
    double* gws = ar.take<double>(e);
    double* RT = ar.take<double>(c * c);
    double* b0 = ar.take<double>(m * c);
    double* b1 = ar.take<double>(m * c);
    int32_t* linfo = ar.take<int32_t>(1);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    int32_t* inf = info ? info : linfo;
    RQLP_TRY(fill_zero_bytes(inf, sizeof(int32_t), s));
    RQLP_TRY(copy_matrix(m, c, Y, ldy, b0, m, s));
    Ctx cx{s, inf, gws, e, o};
    double* out = nullptr;
    RQLP_TRY(cholqr2(cx, m, c, b0, b1, m, R ? RT : nullptr, &out));
    if (R) RQLP_TRY(transpose_matrix(c, c, RT, c, R, ldr, 'U', s));
    return copy_matrix(m, c, out, m, V, ldv, s);
}

int rqlp_cpqr_workspace(int64_t rows, int64_t cols, size_t* bytes) {
    if (rows < 0) return -1;
    if (cols < 0) return -2;
    if (!bytes) return -3;
    const int64_t kmax = rows < cols ? rows : cols;
    Arena ar(nullptr, 0);
    CpqrScratch sc;
    cpqr_carve(ar, rows, cols, &sc);
    ar.take<double>(rows * kmax);
    ar.take<double>(kmax);
    ar.take<int64_t>(kmax);
    ar.take<int32_t>(1);
    *bytes = ar.used + 256;
    return 0;
}

int rqlp_cpqr(const double* M, int64_t ldm, int64_t rows, int64_t cols, int64_t* piv, double* R, int64_t ldr,
              double* Rt, int64_t ldrt, double* Qm, int64_t ldq, int32_t* info, void* work, size_t work_bytes,
              void* stream) {
    if (rows < 0) return -3;
    if (cols < 0) return -4;
    if (ldm < (rows > 1 ? rows : 1)) return -2;
    if (R && ldr < (rows > 1 ? rows : 1)) return -7;
    if (Rt && ldrt < (cols > 1 ? cols : 1)) return -9;
    if (Qm && ldq < (rows > 1 ? rows : 1)) return -11;
    if (rows * cols > 0 && !M) return -1;
    if (rows * cols == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    const int64_t kmax = rows < cols ? rows : cols;
    Arena ar = arena_for(work, work_bytes);
    CpqrScratch sc;
    cpqr_carve(ar, rows, cols, &sc);
    double* Vh = ar.take<double>(rows * kmax);
    double* beta = ar.take<double>(kmax);
    int64_t* pv = ar.take<int64_t>(kmax);
    int32_t* linfo = ar.take<int32_t>(1);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    int32_t* inf = info ? info : linfo;
    RQLP_TRY(fill_zero_bytes(inf, sizeof(int32_t), s));
    RQLP_TRY(cpqr(M, ldm, rows, cols, sc, pv, Vh, rows, beta, R, ldr, Rt, ldrt, inf, s));
    if (piv) RQLP_TRY(copy_i64(kmax, pv, piv, s));
    if (Qm) RQLP_TRY(apply_householder(rows, kmax, Vh, rows, beta, nullptr, 0, nullptr, kmax, Qm, ldq, s));
    return 0;
}

}  // extern "C"
