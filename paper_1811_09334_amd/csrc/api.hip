// C ABI of the randomized QLP library: argument checks, workspace carve-up
// and the enqueue order of the hot path (Algorithms 2.1, 2.2, 4.1).
#include <math.h>
#include <string.h>

#include <array>
#include <initializer_list>

#include "common.hpp"
#include "kernels.hpp"

using namespace rqlp;

namespace {

constexpr double kEps = 2.220446049250313e-16;    // FP64 machine epsilon
constexpr double kEps32 = 1.1920928955078125e-7;  // FP32 machine epsilon

// CholeskyQR shift scale of Fukaya et al. (2020): 11 (m c + c (c + 1)) u.
double shift_scale(int64_t rows, int64_t c) { return 11.0 * ((double)rows * c + (double)c * (c + 1)) * kEps; }

// Shift scale for a Gram matrix accumulated in FP32 (Cholesky itself in FP64):
// the worst-case bound above exceeds 1 at the panel sizes of the mixed path,
// so the probabilistic size of the Gram's rounding error, sqrt(m) u tr(G)
// (Higham & Mary 2019), is covered instead, with the same factor 11.
double shift_scale32(int64_t rows, int64_t c) { return 11.0 * (sqrt((double)rows) + (double)c + 1.0) * kEps32; }

// Scratch for orthonormalising a rows x c panel.
struct OrthoScratch {
    double* G;      // c x c Gram
    double* L1;     // c x c Cholesky factor of pass 1
    double* L2;     // c x c Cholesky factor of pass 2
    double* Li;     // c x c inverse of the current factor
    unsigned* sync; // flags of the multi-workgroup Cholesky
    int32_t* shifted;
};

void carve_ortho(Arena& ar, int64_t c, OrthoScratch* o) {
    o->G = ar.take<double>(c * c);
    o->L1 = ar.take<double>(c * c);
    o->L2 = ar.take<double>(c * c);
    o->Li = ar.take<double>(c * c);
    o->sync = ar.take<unsigned>(CHOL_SYNC_WORDS);
    o->shifted = ar.take<int32_t>(1);
}

struct Ctx {
    hipStream_t s;
    int32_t* info;
    double* gws;
    size_t gws_elems;
    OrthoScratch o;
    int32_t* shifted;   // device word: the first pass used the shifted retry
};

// Relative pivot below which the plain attempt of an FP64 CholeskyQR pass
// counts as a breakdown: a column whose component outside the span of the
// earlier columns is below ~1e-6 of its norm (pivot ratio 1e-12) is
// numerically dependent, and the pass takes the shifted retry instead.
constexpr double kPivotRel = 1e-12;
// Squared column norm below which a column is numerically zero after a
// shifted first pass (its healthy columns have norm ~1): it is replaced by a
// random vector (orthonormal completion).
constexpr double kZeroCol2 = 1e-12;

// CholeskyQR of the rows x c panel held in buf0 (leading dimension ld):
// passes of G = X^T X, G = L L^T, X <- X L^{-T}, in place when the update
// kernel takes the panel.  Returns the buffer holding the orthonormal result
// (buf0 or buf1; buf0 is overwritten).  RT (c x c,
// optional) receives R^T = L1 L2 ... (lower triangular), where X_in = V R
// with diag(R) >= 0.
// final == true (a basis that is returned): CholeskyQR2, plus two more passes
// when any pass needed the shifted retry (device word cx.shifted, sticky
// over the call).  A shifted first pass also marks input that is
// numerically rank deficient (kPivotRel): its dependent directions are
// then still tiny, and each shifted pass scales them up by about
// 1 / sqrt(shift), so a shifted CholeskyQR3 does not always reach an
// orthonormal basis, while four passes do; columns that are exactly zero
// (R0^T after a rank stop) never grow and are replaced by random vectors
// after the first pass (complete_columns), which also zeroes their rows of
// R (col0: the panel's first column in a wider basis, which keeps the
// completions of different blocks of one basis apart).  The conditional
// passes 3 and 4 run or are skipped together, so the result buffer does not
// depend on the gate.
// final == false (an intermediate basis of the subspace iteration, which
// only has to span range(X) and be well conditioned): one pass, and the
// second only when the first needed the shifted retry.
int cholqr2(Ctx& cx, int64_t rows, int64_t c, double* buf0, double* buf1, int64_t ld, double* RT,
            double** out, bool final = true, int64_t col0 = 0, bool reortho = false) {
    // in place (the result stays in buf0) when the update kernel takes the
    // panel, which may write its own input; else the passes alternate buffers
    const bool inplace = trmm_fits<double>(rows, c, buf0, ld, buf0, ld);
    double* cur = buf0;
    double* nxt = inplace ? buf0 : buf1;
    const int npass = final ? 4 : 2;
    double* Ls[4] = {cx.o.L1, cx.o.L2, cx.o.L1, cx.o.L2};
    for (int pass = 0; pass < npass; ++pass) {
        // gate: pass 2 of an intermediate basis, passes 3 and 4 of a final one
        const int32_t* gate = (pass >= (final ? 2 : 1)) ? cx.shifted : nullptr;
        if (final && pass == 2 && RT) {
            // R^T of the first two passes, before their factors are reused
            RQLP_TRY(gemm<double>(false, false, c, c, c, cx.o.L1, c, cx.o.L2, c, RT, c, false, 1.0, 0.0, cx.gws,
                                  cx.gws_elems, cx.s));
        }
        RQLP_TRY(gemm<double>(true, false, c, c, rows, cur, ld, cur, ld, cx.o.G, c, false, 1.0, 0.0, cx.gws,
                              cx.gws_elems, cx.s, gate, 1, 1));
        double* Lp = Ls[pass];
        // shifted word: written by the first pass, only ever set by the later ones
        // the second pass (and the first one after a reorthogonalising
        // projection) sees a Gram matrix within rounding of the identity
        const bool near_id = gate == nullptr && (pass == 1 || reortho);
        RQLP_TRY(chol_inv<double>(c, cx.o.G, c, Lp, cx.o.Li, nullptr, c, shift_scale(rows, c), cx.info, cx.s,
                                  gate, cx.shifted, cx.o.sync, pass == 0 ? 1 : 2, pass == 0 ? kPivotRel : 0.0,
                                  near_id));
        // a skipped second pass of an intermediate basis copies X through (static
        // result buffer), unless the passes run in place
        RQLP_TRY(gemm<double>(false, true, rows, c, c, cur, ld, cx.o.Li, c, nxt, ld, false, 1.0, 0.0, cx.gws,
                              cx.gws_elems, cx.s, gate, (final || inplace) ? 1 : 2, 2));
        if (pass == 0) RQLP_TRY(complete_columns(rows, c, nxt, ld, cx.o.L1, c, kZeroCol2, cx.shifted, cx.s, col0));
        if (!inplace) {
            double* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    if (RT) {
        if (!final) {
            RQLP_TRY(gemm<double>(false, false, c, c, c, cx.o.L1, c, cx.o.L2, c, RT, c, false, 1.0, 0.0, cx.gws,
                                  cx.gws_elems, cx.s));
        } else {
            // RT <- RT L3 L4 when the extra passes ran (else copied through)
            RQLP_TRY(gemm<double>(false, false, c, c, c, RT, c, cx.o.L1, c, cx.o.G, c, false, 1.0, 0.0, cx.gws,
                                  cx.gws_elems, cx.s, cx.shifted, 2));
            RQLP_TRY(gemm<double>(false, false, c, c, c, cx.o.G, c, cx.o.L2, c, RT, c, false, 1.0, 0.0, cx.gws,
                                  cx.gws_elems, cx.s, cx.shifted, 2));
        }
    }
    *out = cur;
    return 0;
}

// FP32 panels for the mixed-precision range finder: the Gram and the update
// X <- X L^{-T} run on FP32 MFMA, the c x c Cholesky and inverse in FP64.
struct Ctx32 {
    hipStream_t s;
    int32_t* info;
    float* ws;
    size_t ws_elems;
    float* G;       // c x c
    float* Li;      // c x c
    double* L;      // c x c (FP64 factor, discarded)
    double* Lid;    // c x c (FP64 inverse)
    int32_t* shifted;   // device word: the first pass used the shifted retry
    unsigned* sync;     // flags of the multi-workgroup Cholesky
};

// CholeskyQR of an FP32 panel as shifted CholeskyQR3 (Fukaya et al. 2020):
// three passes, of which the first `always` run unconditionally (2 for the
// final basis: CholeskyQR2; 1 for an intermediate basis of the subspace
// iteration, which only has to span range(X) and be well conditioned) and
// the rest only when a Cholesky of an earlier pass needed the shifted retry
// (device word cx.shifted, set by any such pass and never cleared by a later
// one).  A skipped pass forms no Gram.  The passes run in place when the
// update kernel takes the panel (result in buf0); otherwise they alternate
// buffers and the result is always in buf1: for the final basis the skipped
// third pass copies X through, and for an intermediate basis the two
// conditional passes run or are skipped together (the second runs only when
// the word is set, and then the third does too), so their updates are simply
// left out when skipped.
int cholqr_f32(Ctx32& cx, int64_t rows, int64_t c, float* buf0, float* buf1, int64_t ld, float** out,
               bool final = true, bool reortho = false) {
    // in place (result in buf0) when the update kernel takes the panel
    const bool inplace = trmm_fits<float>(rows, c, buf0, ld, buf0, ld);
    float* cur = buf0;
    float* nxt = inplace ? buf0 : buf1;
    const int always = final ? 2 : 1;
    const int skip_mode = (final && !inplace) ? 2 : 1;   // gemm gate modes: 2 copy op(A), 1 skip
    for (int pass = 0; pass < 3; ++pass) {
        const int32_t* gate = pass >= always ? cx.shifted : nullptr;
        RQLP_TRY(gemm<float>(true, false, c, c, rows, cur, ld, cur, ld, cx.G, c, false, 1.0f, 0.0f, cx.ws,
                             cx.ws_elems, cx.s, gate, 1, 1));
        // the second pass (and the first one after a reorthogonalising
        // projection) sees a Gram matrix within rounding of the identity
        const bool near_id = gate == nullptr && (pass == 1 || reortho);
        RQLP_TRY(chol_inv<float>(c, cx.G, c, cx.L, cx.Lid, cx.Li, c, shift_scale32(rows, c), cx.info, cx.s,
                                 gate, pass < 2 ? cx.shifted : nullptr, cx.sync, pass == 0 ? 1 : 2, 0.0, near_id));
        RQLP_TRY(gemm<float>(false, true, rows, c, c, cur, ld, cx.Li, c, nxt, ld, false, 1.0f, 0.0f, cx.ws,
                             cx.ws_elems, cx.s, gate, skip_mode, 2));
        if (!inplace) {
            float* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    *out = cur;
    return 0;
}

size_t max_ws(size_t (*f)(int64_t, int64_t, int64_t), std::initializer_list<std::array<int64_t, 3>> shapes) {
    size_t mx = 0;
    for (auto& sh : shapes) {
        size_t e = f(sh[0], sh[1], sh[2]);
        if (e > mx) mx = e;
    }
    return mx;
}

// FP64 buffers of the small stage (CPQR of B, second factorisation, Q_B / P_B).
struct SmallBufs {
    double* B;      // l x n
    double* Z;      // n x l   R0^T
    double* Z2;     // n x l
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

// extra FP64 product shapes (M, N, K) of the caller that share gws
void carve_small(Arena& ar, int64_t n, int64_t l, int64_t cp_rows, std::initializer_list<std::array<int64_t, 3>> extra,
                 SmallBufs* f) {
    f->B = ar.take<double>(l * n);
    f->Z = ar.take<double>(n * l);
    f->Z2 = ar.take<double>(n * l);
    size_t e = max_ws(gemm_workspace_elems, {{l, l, n}, {n, l, l}, {l, l, l}});
    size_t e2 = max_ws(gemm_workspace_elems, extra);
    f->gws_elems = e > e2 ? e : e2;
    f->gws = ar.take<double>(f->gws_elems);
    carve_ortho(ar, l, &f->o);
    cpqr_carve(ar, cp_rows, n, &f->cs);
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

// Pivoted QLP of the reduced matrix, Algorithm 2.1 (d = 0) or Algorithm 2.2 (d >= 1), on
// the l x n matrix f.B: first CPQR B Pi0 = Q0 R0, then the second
// factorisation of R0^T.  Writes T (l x l, triangle *tri), P_B (n x l, FP64,
// into Pd) and returns Q_B (l x l, FP64) in *QB; B = Q_B T P_B^T.
int qlp_of_B(Ctx& cx, SmallBufs& f, int64_t l, int64_t n, int d, double* Pd, int64_t ldpd, double* T, int64_t ldt,
             char* tri_out, double** QB) {
    hipStream_t s = cx.s;
    int32_t* inf = cx.info;
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
        RQLP_TRY(gemm<double>(false, false, n, l, l, Qt, n, f.Mr, l, Pd, ldpd, false, 1.0, 0.0, f.gws, f.gws_elems,
                              s));
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
            RQLP_TRY(gemm<double>(false, false, n, l, l, Qt, n, f.Mr, l, Pd, ldpd, false, 1.0, 0.0, f.gws,
                                  f.gws_elems, s));
        else
            RQLP_TRY(copy_matrix(n, l, Qt, n, Pd, ldpd, s));
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
    *QB = f.Ml;
    *tri_out = tri;
    return 0;
}

// FP64 range finder buffers.
struct RangeBufs64 {
    double* Om;
    double* Y;
    double* Y2;
};

void carve_range64(Arena& ar, int64_t m, int64_t n, int64_t l, bool need_omega, RangeBufs64* r) {
    r->Om = need_omega ? ar.take<double>(n * l) : nullptr;
    r->Y = ar.take<double>(m * l);
    r->Y2 = ar.take<double>(m * l);
}

// Mixed-precision range finder buffers.
struct RangeBufsLP {
    unsigned short* Ac;     // m x n, column-major 16-bit copy of A (FP16: A D^{-1})
    unsigned short* Ar;     // n x m, i.e. A row-major
    unsigned short* Aclo;   // bf16x3 remainders (else NULL)
    unsigned short* Arlo;
    int* colexp;            // n (FP16 only)
    int* gexp;              // 1
    float* Om;              // n x l (generated test matrix)
    unsigned short* X16;    // tiled 16-bit panel operand (Omega^T, W^T or V^T: l x max(m, n))
    unsigned short* X16lo;
    float* Y;               // m x l
    float* Y2;
    float* Z;               // n x l
    float* Z2;
    float* lpws;
    size_t lpws_elems;
    float* fws;
    size_t fws_elems;
    float* G;               // l x l
    float* Li;              // l x l
    float* QB;              // l x l
    double* Pd;             // n x l
    int32_t* shifted;       // 1 word
    float* B32;             // l x n (FP32 form: projection before widening)
};

// Buffers of the FP32 and mixed-precision range finders (the FP32 form needs
// no 16-bit copies and runs every product as an FP32 MFMA product).
void carve_range_lp(Arena& ar, int64_t m, int64_t n, int64_t l, int precision, bool need_omega, RangeBufsLP* r) {
    const bool x3 = precision == RQLP_MIXED_BF16X3;
    const bool f32 = precision == RQLP_F32;
    const size_t ec = lp_tiled_elems(n, m), er = lp_tiled_elems(m, n);
    r->Ac = f32 ? nullptr : ar.take<unsigned short>(ec);
    r->Ar = f32 ? nullptr : ar.take<unsigned short>(er);
    r->Aclo = x3 ? ar.take<unsigned short>(ec) : nullptr;
    r->Arlo = x3 ? ar.take<unsigned short>(er) : nullptr;
    r->colexp = ar.take<int>(n);
    r->gexp = ar.take<int>(1);
    r->Om = need_omega ? ar.take<float>(n * l) : nullptr;
    const int64_t mx = m > n ? m : n;
    r->X16 = f32 ? nullptr : ar.take<unsigned short>(lp_tiled_elems(l, mx));
    r->X16lo = x3 ? ar.take<unsigned short>(lp_tiled_elems(l, mx)) : nullptr;
    r->Y = ar.take<float>(m * l);
    r->Y2 = ar.take<float>(m * l);
    r->Z = ar.take<float>(n * l);
    r->Z2 = ar.take<float>(n * l);
    r->lpws_elems = f32 ? 0 : max_ws(gemm_lp_workspace_elems, {{m, l, n}, {n, l, m}});
    r->lpws = f32 ? nullptr : ar.take<float>(r->lpws_elems);
    r->fws_elems = f32 ? max_ws(gemm_workspace_elems, {{l, l, m}, {l, l, n}, {m, l, l}, {n, l, l}, {m, l, n}, {n, l, m}})
                       : max_ws(gemm_workspace_elems, {{l, l, m}, {l, l, n}, {m, l, l}, {n, l, l}});
    r->fws = ar.take<float>(r->fws_elems);
    r->B32 = f32 ? ar.take<float>(l * n) : nullptr;
    r->G = ar.take<float>(l * l);
    r->Li = ar.take<float>(l * l);
    r->QB = ar.take<float>(l * l);
    r->Pd = ar.take<double>(n * l);
    r->shifted = ar.take<int32_t>(1);
}

// Scratch of the block reorthogonalisation.
struct BcgsScratch {
    void* C;        // l x ob coefficients (ob: the column block of ortho_block)
    void* p1;       // rows x ob panel
    void* ws;       // split-K partials (T)
    size_t ws_elems;
};

// Block classical Gram-Schmidt (the reorthogonalisation of Algorithm 4.1) over the rows x l
// panel V whose first bs-column block is already orthonormal: every later
// block V_j is projected against the earlier blocks,
// V_j <- V_j - V_{<j} (V_{<j}^T V_j), and orthonormalised in place by one
// CholeskyQR pass (plus the conditional passes after a shifted retry).  A
// final basis takes the projection and the CholeskyQR twice (BCGS2, the
// reorthogonalisation of Algorithm 4.1; the second CholeskyQR sees an almost
// orthonormal block, so one FP32 pass gives orthogonality to working
// precision; the FP64 path keeps the full form there).
// An intermediate basis of the subspace iteration only has to span the same
// block prefixes and be well conditioned: one projection and one CholeskyQR,
// which leave a loss of orthogonality between blocks of about u / f (f: the
// part of a block outside the span of the earlier ones, well above u here).
template <typename T, typename CtxT>
int bcgs2(CtxT& cx, int64_t rows, int64_t l, int64_t bs, T* V, int64_t ld, BcgsScratch& sc, bool final,
          hipStream_t s) {
    T* C = (T*)sc.C;
    T* p1 = (T*)sc.p1;
    T* ws = (T*)sc.ws;
    for (int64_t s0 = bs; s0 < l; s0 += bs) {
        const int64_t bj = (l - s0) < bs ? (l - s0) : bs;
        T* Vj = V + s0 * ld;
        for (int pass = 0; pass < (final ? 2 : 1); ++pass) {
            RQLP_TRY(gemm<T>(true, false, s0, bj, rows, V, ld, Vj, ld, C, s0, false, T(1), T(0), ws, sc.ws_elems, s));
            RQLP_TRY(gemm<T>(false, false, rows, bj, s0, V, ld, C, s0, Vj, ld, false, T(-1), T(1), ws, sc.ws_elems, s));
            // FP64: the full form for the final basis (four passes after a
            // shifted retry make numerically dependent blocks orthonormal)
            const bool full = pass == 1 && final && sizeof(T) == sizeof(double);
            T* o = nullptr;
            if constexpr (sizeof(T) == sizeof(double)) {
                RQLP_TRY(cholqr2(cx, rows, bj, (double*)Vj, (double*)p1, ld, nullptr, (double**)&o, full, s0, pass == 1));
                if ((void*)o != (void*)Vj) RQLP_TRY(copy_matrix(rows, bj, (const double*)o, ld, (double*)Vj, ld, s));
            } else {
                RQLP_TRY(cholqr_f32(cx, rows, bj, (float*)Vj, (float*)p1, ld, (float**)&o, full, pass == 1));
                if ((void*)o != (void*)Vj)
                    RQLP_TRY((cast_matrix<float, float>(rows, bj, (const float*)o, ld, (float*)Vj, ld, s)));
            }
        }
    }
    return 0;
}

// Column block of the block orthonormalisation for the block size bs of
// Algorithm 4.1: the largest multiple of bs that one CholeskyQR pass on the
// matrix cores takes (512 columns), or the whole panel.  Any
// such blocking gives the same basis up to rounding: every form here is
// triangular (column j of the result lies in the span of columns 0..j of the
// input, with a positive diagonal), so the leading blocks of the range
// finder's basis span the images of the leading blocks of Omega and are
// those of Algorithm 4.1's one-block-at-a-time construction (for a fixed
// Omega the block and unblocked range finders agree).  Wider blocks turn the
// many narrow projections into a few wide products.
int64_t ortho_block(int64_t bs, int64_t l, bool f64) {
    (void)f64;                                      // the same for FP64 and FP32
    const int64_t cap = 512;
    if (bs <= 0 || bs >= l) return l;
    int64_t ob = bs <= cap ? (cap / bs) * bs : bs;
    return ob >= l ? l : ob;
}

// Orthonormalisation of a rows x l panel: as a whole (bs == 0, or one block
// covers it: CholeskyQR), or by the column blocks of ortho_block (the last
// one ragged): a QR of the first block, then block Gram-Schmidt for the
// others.  The result is in *out (buf0 or buf1).
int ortho_f64(Ctx& cx, int64_t rows, int64_t l, int64_t bs, double* buf0, double* buf1, int64_t ld, double** out,
              bool final, BcgsScratch& bc) {
    const int64_t ob = ortho_block(bs, l, true);
    if (ob >= l) return cholqr2(cx, rows, l, buf0, buf1, ld, nullptr, out, final);
    double* o = nullptr;
    RQLP_TRY(cholqr2(cx, rows, ob, buf0, buf1, ld, nullptr, &o, final));
    if (o != buf0) RQLP_TRY(copy_matrix(rows, ob, o, ld, buf0, ld, cx.s));
    RQLP_TRY((bcgs2<double, Ctx>(cx, rows, l, ob, buf0, ld, bc, final, cx.s)));
    *out = buf0;
    return 0;
}

int ortho_f32(Ctx32& cx, int64_t rows, int64_t l, int64_t bs, float* buf0, float* buf1, int64_t ld, float** out,
              bool final, BcgsScratch& bc) {
    const int64_t ob = ortho_block(bs, l, false);
    if (ob >= l) return cholqr_f32(cx, rows, l, buf0, buf1, ld, out, final);
    float* o = nullptr;
    RQLP_TRY(cholqr_f32(cx, rows, ob, buf0, buf1, ld, &o, final));
    if (o != buf0) RQLP_TRY((cast_matrix<float, float>(rows, ob, o, ld, buf0, ld, cx.s)));
    RQLP_TRY((bcgs2<float, Ctx32>(cx, rows, l, ob, buf0, ld, bc, final, cx.s)));
    *out = buf0;
    return 0;
}

// FP32 range finder and projection (RQLP_F32): every pass over A is an FP32
// MFMA product, the panels are orthonormalised by FP32 CholeskyQR, and
// B = V^T A is widened to FP64 for the small stage.  Returns V (m x l).
int range_and_project_f32(Ctx32& c32, RangeBufsLP& r, SmallBufs& f, const float* A, int64_t lda, int64_t m,
                          int64_t n, int64_t l, int q, uint64_t seed, const float* Om, int64_t ldom, float** Vout,
                          int64_t bs, BcgsScratch& bc) {
    hipStream_t s = c32.s;
    if (!Om) {
        RQLP_TRY(generate_omega(n, l, seed, RQLP_F32, r.Om, n, s));
        Om = r.Om;
        ldom = n;
    }
    RQLP_TRY(gemm<float>(false, false, m, l, n, A, lda, Om, ldom, r.Y, m, false, 1.0f, 0.0f, r.fws, r.fws_elems, s));
    float* V = nullptr;
    RQLP_TRY(ortho_f32(c32, m, l, bs, r.Y, r.Y2, m, &V, q == 0, bc));
    for (int it = 0; it < q; ++it) {
        RQLP_TRY(gemm<float>(true, false, n, l, m, A, lda, V, m, r.Z, n, false, 1.0f, 0.0f, r.fws, r.fws_elems, s));
        float* W = nullptr;
        RQLP_TRY(ortho_f32(c32, n, l, bs, r.Z, r.Z2, n, &W, false, bc));
        float* ydst = (V == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(gemm<float>(false, false, m, l, n, A, lda, W, n, ydst, m, false, 1.0f, 0.0f, r.fws, r.fws_elems, s));
        float* other = (ydst == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(ortho_f32(c32, m, l, bs, ydst, other, m, &V, it == q - 1, bc));
    }
    RQLP_TRY(gemm<float>(true, false, n, l, m, A, lda, V, m, r.B32, l, true, 1.0f, 0.0f, r.fws, r.fws_elems, s));
    RQLP_TRY((cast_matrix<float, double>(l, n, r.B32, l, f.B, l, s)));
    *Vout = V;
    return 0;
}

bool valid_precision(int p) { return p >= RQLP_F64 && p <= RQLP_MIXED_BF16X3; }
bool is_mixed(int p) { return p == RQLP_MIXED_BF16 || p == RQLP_MIXED_FP16 || p == RQLP_MIXED_BF16X3; }

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

}  // namespace

namespace rqlp {
int factor_arg_status(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                      int precision, const void* Omega, int64_t ldo, const void* Q, int64_t ldq, const double* T,
                      int64_t ldt, const void* P, int64_t ldp) {
    RQLP_TRY(check_factor_args(A, lda, m, n, k, p, q, d, b, precision));
    const int64_t l = k + p;
    if (Omega && ldo < n) return -13;
    if (!Q) return -14;
    if (ldq < m) return -15;
    if (!T) return -16;
    if (ldt < l) return -17;
    if (!P) return -18;
    if (ldp < n) return -19;
    return 0;
}
}  // namespace rqlp

namespace {

// Workspace layout of one rqlp_factor call (shared by the size query and
// the call itself).
struct FactorLayout {
    RangeBufs64 r64;
    RangeBufsLP rlp;
    SmallBufs sm;
    BcgsScratch bc;     // block RQLP only
    double* Bj;         // block RQLP: one block row of B (bs x n)
    BqlpScratch bq;     // block RQLP with blocks of <= 64 rows: batched per-block QLP
};

// bs: block size of block RQLP (0: unblocked).
void carve_factor(Arena& ar, int64_t m, int64_t n, int64_t l, int precision, bool need_omega, int64_t bs,
                  FactorLayout* L) {
    const int64_t cp_rows = bs > 0 ? bs : l;     // rows of the reduced matrices the CPQR sees
    if (precision == RQLP_F64) {
        carve_range64(ar, m, n, l, need_omega, &L->r64);
        carve_small(ar, n, l, cp_rows, {{m, l, n}, {n, l, m}, {l, l, m}, {m, l, l}, {l, n, m}}, &L->sm);
    } else {
        carve_range_lp(ar, m, n, l, precision, need_omega, &L->rlp);
        carve_small(ar, n, l, cp_rows, {}, &L->sm);
    }
    L->bc = BcgsScratch{nullptr, nullptr, nullptr, 0};
    L->Bj = nullptr;
    if (bs > 0) {
        const size_t es = precision == RQLP_F64 ? sizeof(double) : sizeof(float);
        const int64_t ob = ortho_block(bs, l, precision == RQLP_F64);
        const int64_t mx = m > n ? m : n;            // rows of the Y (m) and Z (n) panels
        L->bc.C = ar.take<char>(l * ob * es);
        L->bc.p1 = ar.take<char>(mx * ob * es);
        L->bc.ws_elems = max_ws(gemm_workspace_elems, {{l, ob, m}, {m, ob, l}, {l, ob, n}, {n, ob, l}});
        L->bc.ws = ar.take<char>(L->bc.ws_elems * es);
        L->Bj = ar.take<double>(bs * n);
        if (bs <= 64) bqlp_carve(ar, n, l, bs, &L->bq);
    }
}

// Aligns the caller's workspace pointer to 256 bytes.
Arena arena_for(void* work, size_t bytes) {
    uintptr_t a = (uintptr_t)work;
    uintptr_t al = (a + 255) & ~uintptr_t(255);
    size_t lost = (size_t)(al - a);
    return Arena(work ? (void*)al : nullptr, bytes > lost ? bytes - lost : 0);
}

// FP64 range finder of Algorithm 2.1 (with q subspace iterations) and the
// projection B = V^T A.  Returns V (m x l) in *Vout.
int range_and_project_f64(Ctx& cx, RangeBufs64& r, SmallBufs& f, const double* A, int64_t lda, int64_t m, int64_t n,
                          int64_t l, int q, uint64_t seed, const double* Om, int64_t ldom, double** Vout, int64_t bs,
                          BcgsScratch& bc) {
    hipStream_t s = cx.s;
    if (!Om) {
        RQLP_TRY(generate_omega(n, l, seed, RQLP_F64, r.Om, n, s));
        Om = r.Om;
        ldom = n;
    }
    RQLP_TRY(gemm<double>(false, false, m, l, n, A, lda, Om, ldom, r.Y, m, false, 1.0, 0.0, f.gws, f.gws_elems, s));
    double* V = nullptr;
    RQLP_TRY(ortho_f64(cx, m, l, bs, r.Y, r.Y2, m, &V, q == 0, bc));
    for (int it = 0; it < q; ++it) {
        // Z = A^T V into the small stage's n x l buffers (free until the CPQR)
        RQLP_TRY(gemm<double>(true, false, n, l, m, A, lda, V, m, f.Z, n, false, 1.0, 0.0, f.gws, f.gws_elems, s));
        double* W = nullptr;
        RQLP_TRY(ortho_f64(cx, n, l, bs, f.Z, f.Z2, n, &W, false, bc));
        double* ydst = (V == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(gemm<double>(false, false, m, l, n, A, lda, W, n, ydst, m, false, 1.0, 0.0, f.gws, f.gws_elems, s));
        double* other = (ydst == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(ortho_f64(cx, m, l, bs, ydst, other, m, &V, it == q - 1, bc));
    }
    // B = V^T A, computed as (A^T V)^T and stored l x n
    RQLP_TRY(gemm<double>(true, false, n, l, m, A, lda, V, m, f.B, l, true, 1.0, 0.0, f.gws, f.gws_elems, s));
    *Vout = V;
    return 0;
}

// Mixed-precision range finder and projection: the 2q + 2 passes over A run
// as 16-bit MFMA products (FP32 accumulation), the panels are orthonormalised
// by FP32 CholeskyQR2, and B = V^T A is widened to FP64 for the small stage.
// Returns V (m x l, FP32) in *Vout.
int range_and_project_lp(Ctx32& c32, RangeBufsLP& r, SmallBufs& f, int kind, const float* A, int64_t lda,
                         int64_t m, int64_t n, int64_t l, int q, uint64_t seed, const float* Om, int64_t ldom,
                         float** Vout, int64_t bs, BcgsScratch& bc) {
    hipStream_t s = c32.s;
    const bool fp16 = kind == RQLP_MIXED_FP16;
    const int* cexp = fp16 ? r.colexp : nullptr;
    const int* gexp = fp16 ? r.gexp : nullptr;
    if (fp16) RQLP_TRY(column_exponents(m, n, A, lda, r.colexp, r.gexp, s));
    RQLP_TRY(encode_tiled(kind, m, n, A, lda, r.Ac, r.Aclo, r.Ar, r.Arlo, cexp, s));
    if (!Om) {
        RQLP_TRY(generate_omega(n, l, seed, kind, r.Om, n, s));
        Om = r.Om;
        ldom = n;
    }
    // Y = A Omega  (FP16: (A D^-1)(2^-g D Omega) 2^g)
    RQLP_TRY(cast_panel(kind, l, n, Om, ldom, r.X16, r.X16lo, cexp, gexp, s));
    RQLP_TRY(gemm_lp<float>(kind, m, l, n, r.Ar, r.Arlo, r.X16, r.X16lo, r.Y, m, false, nullptr, gexp, r.lpws,
                            r.lpws_elems, s));
    float* V = nullptr;
    RQLP_TRY(ortho_f32(c32, m, l, bs, r.Y, r.Y2, m, &V, q == 0, bc));
    for (int it = 0; it < q; ++it) {
        // Z = A^T V  (FP16: D (A D^-1)^T V)
        RQLP_TRY(cast_panel(kind, l, m, V, m, r.X16, r.X16lo, nullptr, nullptr, s));
        RQLP_TRY(gemm_lp<float>(kind, n, l, m, r.Ac, r.Aclo, r.X16, r.X16lo, r.Z, n, false, cexp, nullptr,
                                r.lpws, r.lpws_elems, s));
        float* W = nullptr;
        RQLP_TRY(ortho_f32(c32, n, l, bs, r.Z, r.Z2, n, &W, false, bc));
        // Y = A W
        RQLP_TRY(cast_panel(kind, l, n, W, n, r.X16, r.X16lo, cexp, gexp, s));
        float* ydst = (V == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(gemm_lp<float>(kind, m, l, n, r.Ar, r.Arlo, r.X16, r.X16lo, ydst, m, false, nullptr, gexp,
                                r.lpws, r.lpws_elems, s));
        float* other = (ydst == r.Y) ? r.Y2 : r.Y;
        RQLP_TRY(ortho_f32(c32, m, l, bs, ydst, other, m, &V, it == q - 1, bc));
    }
    // B = V^T A = (A^T V)^T, FP32 accumulation, stored l x n in FP64
    RQLP_TRY(cast_panel(kind, l, m, V, m, r.X16, r.X16lo, nullptr, nullptr, s));
    RQLP_TRY(gemm_lp<double>(kind, n, l, m, r.Ac, r.Aclo, r.X16, r.X16lo, f.B, l, true, cexp, nullptr, r.lpws,
                             r.lpws_elems, s));
    *Vout = V;
    return 0;
}

}  // namespace

extern "C" {

const char* rqlp_version(void) { return "rqlp-gfx950 0.1"; }

const char* rqlp_status_string(int status) {
    if (status == RQLP_OK) return "success";
    if (status == RQLP_E_WORKSPACE) return "workspace too small";
    if (status == RQLP_E_HIP) return "HIP runtime or launch error";
    if (status == RQLP_E_UNSUPPORTED) return "arguments valid but not supported by this library";
    if (status == RQLP_E_SCRATCH_LIMIT)
        return "rqlp_factor_noalloc: the problem needs more workspace than the library's static scratch "
               "(RQLP_NOALLOC_SCRATCH_BYTES); use rqlp_factor with a caller workspace";
    if (status < 0 && status > -100) return "invalid argument (see the argument index -status)";
    return "unknown status";
}

int rqlp_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b, int precision,
                        size_t* bytes) {
    int st = check_factor_args((const void*)1, m, m, n, k, p, q, d, b, precision);
    if (st) return st;
    if (!bytes) return -9;
    Arena ar(nullptr, 0);
    FactorLayout L;
    carve_factor(ar, m, n, k + p, precision, true, (b > 0 && b < k + p) ? b : 0, &L);
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

}  // extern "C"

namespace {

// Auto-rank request of factor_core: after the range finder, the first block
// count J with ||A||_F^2 - ||B_1..J||_F^2 <= eps is read back to the host
// (the one synchronisation of the call) and only those blocks are factorised.
struct AutoRank {
    double eps;
    int64_t* rank;      // host out: columns taken
    double* err2;       // host out: indicator at the rank (may be NULL)
};

// The enqueue order of rqlp_factor (arguments already checked) over l
// columns; with ar != NULL the auto-rank truncation described above.
int factor_core(const void* A, int64_t lda, int64_t m, int64_t n, int64_t l, int q, int d, int64_t bs, int precision,
                uint64_t seed, const void* Omega, int64_t ldo, void* Q, int64_t ldq, double* T, int64_t ldt, void* P,
                int64_t ldp, int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info, char* uplo, void* work,
                size_t work_bytes, hipStream_t s, AutoRank* arq) {
    Arena ar = arena_for(work, work_bytes);
    FactorLayout Lay;
    carve_factor(ar, m, n, l, precision, Omega == nullptr, bs, &Lay);
    double* ar_out = nullptr;
    double* ar_scratch = nullptr;
    if (arq) {
        ar_out = ar.take<double>(4);
        ar_scratch = ar.take<double>(autorank_scratch_doubles(n, l, bs));
    }
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    SmallBufs& f = Lay.sm;
    {
        const int64_t rows = bs > 0 ? bs : l;
        CpqrPlan pl;
        RQLP_TRY(cpqr_plan(rows, n, &pl));
        RQLP_TRY(cpqr_plan(rows, rows, &pl));
    }
    int32_t* inf = info ? info : f.info;
    RQLP_TRY(fill_zero_bytes(inf, sizeof(int32_t), s));
    Ctx cx{s, inf, f.gws, f.gws_elems, f.o, f.o.shifted};
    char tri = 'L';
    double* QB = nullptr;
    const bool f64 = precision == RQLP_F64;
    RangeBufsLP& r = Lay.rlp;
    Ctx32 c32{s, inf, r.fws, r.fws_elems, r.G, r.Li, f.o.L1, f.o.Li, r.shifted, f.o.sync};
    double* V64 = nullptr;
    float* V32 = nullptr;
    if (f64)
        RQLP_TRY(range_and_project_f64(cx, Lay.r64, f, (const double*)A, lda, m, n, l, q, seed, (const double*)Omega,
                                       ldo, &V64, bs, Lay.bc));
    else if (precision == RQLP_F32)
        RQLP_TRY(range_and_project_f32(c32, r, f, (const float*)A, lda, m, n, l, q, seed, (const float*)Omega, ldo,
                                       &V32, bs, Lay.bc));
    else
        RQLP_TRY(range_and_project_lp(c32, r, f, precision, (const float*)A, lda, m, n, l, q, seed,
                                      (const float*)Omega, ldo, &V32, bs, Lay.bc));
    double* Pd = f64 ? (double*)P : r.Pd;
    const int64_t ldpd = f64 ? ldp : n;
    // leading columns factorised (all l, or the auto-rank prefix)
    int64_t le = l;
    if (arq) {
        if (f64)
            RQLP_TRY(autorank_indicator<double>((const double*)A, lda, m, n, f.B, l, l, bs, arq->eps, ar_scratch,
                                                ar_out, s));
        else
            RQLP_TRY(autorank_indicator<float>((const float*)A, lda, m, n, f.B, l, l, bs, arq->eps, ar_scratch,
                                               ar_out, s));
        double h[3] = {0.0, 0.0, 0.0};
        RQLP_HIP_TRY(hipMemcpyAsync(h, ar_out, sizeof(h), hipMemcpyDeviceToHost, s));
        RQLP_HIP_TRY(hipStreamSynchronize(s));
        const int64_t J = (int64_t)h[0];
        le = (bs > 0 && J * bs < l) ? J * bs : l;
        *arq->rank = le;
        if (arq->err2) *arq->err2 = h[1];
        if (!(h[1] <= arq->eps)) RQLP_TRY(set_info_flag(inf, RQLP_INFO_NOT_CONVERGED, s));
        // outputs past the rank: zero columns, pivots -1 (T is cleared below)
        RQLP_TRY(zero_cols<double>(l, 0, l, T, ldt, s));
        if (le < l) {
            if (f64) RQLP_TRY(zero_cols<double>(m, le, l, (double*)Q, ldq, s));
            else RQLP_TRY(zero_cols<float>(m, le, l, (float*)Q, ldq, s));
            RQLP_TRY(zero_cols<double>(n, le, l, Pd, ldpd, s));
            if (piv0) RQLP_TRY(fill_i64(l - le, piv0 + le, -1, s));
            if (piv1) RQLP_TRY(fill_i64(l - le, piv1 + le, -1, s));
        }
    }
    if (bs == 0) {
        RQLP_TRY(qlp_of_B(cx, f, l, n, d, Pd, ldpd, T, ldt, &tri, &QB));
        // assembly: Q = V Q_B
        if (f64) {
            RQLP_TRY(gemm<double>(false, false, m, l, l, V64, m, QB, l, (double*)Q, ldq, false, 1.0, 0.0, f.gws,
                                  f.gws_elems, s));
        } else {
            RQLP_TRY((cast_matrix<double, float>(l, l, QB, l, r.QB, l, s)));
            RQLP_TRY(gemm<float>(false, false, m, l, l, V32, m, r.QB, l, (float*)Q, ldq, false, 1.0f, 0.0f, r.fws,
                                 r.fws_elems, s));
        }
        if (piv0) RQLP_TRY(copy_i64(l, f.piv0, piv0, s));
        if (piv1) RQLP_TRY(copy_i64(l, d == 0 ? f.piv1 : nullptr, piv1, s));
    } else if (bqlp_supported(n, le, bs)) {
        // the block rows B_j and their QLPs (Algorithm 4.1) for all blocks at once (batched kernels)
        if (f64)
            RQLP_TRY(bqlp<double>(f.B, l, n, le, bs, Lay.bq, f.Z, V64, m, m, (double*)Q, ldq, Pd, ldpd, T, ldt,
                                  f.piv0, f.piv1, inf, s));
        else
            RQLP_TRY(bqlp<float>(f.B, l, n, le, bs, Lay.bq, f.Z, V32, m, m, (float*)Q, ldq, Pd, ldpd, T, ldt,
                                 f.piv0, f.piv1, inf, s));
        if (piv0) RQLP_TRY(copy_i64(le, f.piv0, piv0, s));
        if (piv1) RQLP_TRY(copy_i64(le, f.piv1, piv1, s));
    } else {
        // Algorithm 4.1 block by block: B_j = V_j^T A is block row j
        // of B; pivoted QLP of B_j; Q_j = V_j Q_B(j), P_j = P_B(j); T = blkdiag(L_j)
        RQLP_TRY(set_identity(le, T, ldt, s));
        for (int64_t s0 = 0; s0 < le; s0 += bs) {
            const int64_t bj = (le - s0) < bs ? (le - s0) : bs;
            RQLP_TRY(copy_matrix(bj, n, f.B + s0, l, Lay.Bj, bj, s));
            SmallBufs fj = f;
            fj.B = Lay.Bj;
            char tj = 'L';
            RQLP_TRY(qlp_of_B(cx, fj, bj, n, 0, Pd + s0 * ldpd, ldpd, T + s0 + s0 * ldt, ldt, &tj, &QB));
            if (f64) {
                RQLP_TRY(gemm<double>(false, false, m, bj, bj, V64 + s0 * m, m, QB, bj, (double*)Q + s0 * ldq, ldq,
                                      false, 1.0, 0.0, f.gws, f.gws_elems, s));
            } else {
                RQLP_TRY((cast_matrix<double, float>(bj, bj, QB, bj, r.QB, bj, s)));
                RQLP_TRY(gemm<float>(false, false, m, bj, bj, V32 + s0 * m, m, r.QB, bj, (float*)Q + s0 * ldq, ldq,
                                     false, 1.0f, 0.0f, r.fws, r.fws_elems, s));
            }
            if (piv0) RQLP_TRY(copy_i64(bj, f.piv0, piv0 + s0, s));
            if (piv1) RQLP_TRY(copy_i64(bj, f.piv1, piv1 + s0, s));
        }
    }
    if (!f64) RQLP_TRY((cast_matrix<double, float>(n, l, r.Pd, n, (float*)P, ldp, s)));
    RQLP_TRY(finish_lvals(l, T, ldt, lvals, inf, s));
    if (uplo) *uplo = tri;
    return 0;
}

}  // namespace

extern "C" {

int rqlp_factor(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                int precision, uint64_t seed, const void* Omega, int64_t ldo, void* Q, int64_t ldq, double* T,
                int64_t ldt, void* P, int64_t ldp, int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info,
                char* uplo, void* work, size_t work_bytes, void* stream) {
    RQLP_TRY(rqlp::factor_arg_status(A, lda, m, n, k, p, q, d, b, precision, Omega, ldo, Q, ldq, T, ldt, P, ldp));
    const int64_t l = k + p;
    if (!work) return -25;
    // block RQLP with b >= l is a single block: plain RQLP
    const int64_t bs = (b > 0 && b < l) ? b : 0;
    return factor_core(A, lda, m, n, l, q, d, bs, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp, piv0, piv1,
                       lvals, info, uplo, work, work_bytes, (hipStream_t)stream, nullptr);
}

namespace {
int check_autorank_args(const void* A, int64_t lda, int64_t m, int64_t n, int64_t lmax, int64_t b, int q, double eps,
                        int precision) {
    if (m < 1) return -3;
    if (n < 1 || n > m) return -4;
    if (lda < m) return -2;
    if (lmax < 1 || lmax > n) return -5;
    if (b < 1) return -6;
    if (q < 0) return -7;
    if (!(eps >= 0.0)) return -8;
    if (!valid_precision(precision)) return -9;
    if (A == nullptr) return -1;
    return 0;
}
}  // namespace

// ---- deterministic truncated pivoted QLP (eq. (1.2)) ----
namespace {
struct QlpLayout {
    double* M;
    double* Vh;
    double* beta;
    double* mu;
    int* colstep;
    unsigned long long* slots;
    unsigned* counter;
    int* state;
    double* dstate;
    SmallBufs sm;
};
void carve_qlp(Arena& ar, int64_t m, int64_t n, int64_t kt, QlpLayout* L) {
    L->M = ar.take<double>(m * n);
    L->Vh = ar.take<double>(m * kt);
    L->beta = ar.take<double>(kt);
    L->mu = ar.take<double>(kt);
    L->colstep = ar.take<int>(n);
    L->slots = ar.take<unsigned long long>(4 * (size_t)qlp_grid(n));
    L->counter = ar.take<unsigned>(32);
    L->state = ar.take<int>(2);
    L->dstate = ar.take<double>(1);
    carve_small(ar, n, kt, kt, {}, &L->sm);
}
int check_qlp_args(const double* A, int64_t lda, int64_t m, int64_t n, int64_t kt) {
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (lda < m) return -2;
    if (kt < 1 || kt > (m < n ? m : n)) return -5;
    if (m > qlp_max_rows()) return RQLP_E_UNSUPPORTED;
    if (A == nullptr) return -1;
    return 0;
}
}  // namespace

int rqlp_qlp_workspace_size(int64_t m, int64_t n, int64_t kt, size_t* bytes) {
    RQLP_TRY(check_qlp_args((const double*)8, m, m, n, kt));
    if (!bytes) return -4;
    Arena ar(nullptr, 0);
    QlpLayout L;
    carve_qlp(ar, m, n, kt, &L);
    *bytes = ar.used + 256;
    return 0;
}

int rqlp_qlp(const double* A, int64_t lda, int64_t m, int64_t n, int64_t kt, double* Q, int64_t ldq, double* T,
             int64_t ldt, double* P, int64_t ldp, int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info,
             void* work, size_t work_bytes, void* stream) {
    RQLP_TRY(check_qlp_args(A, lda, m, n, kt));
    if (!Q) return -6;
    if (ldq < m) return -7;
    if (!T) return -8;
    if (ldt < kt) return -9;
    if (!P) return -10;
    if (ldp < n) return -11;
    if (!work) return -16;
    hipStream_t s = (hipStream_t)stream;
    Arena ar = arena_for(work, work_bytes);
    QlpLayout L;
    carve_qlp(ar, m, n, kt, &L);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    SmallBufs& f = L.sm;
    {
        CpqrPlan pl;
        RQLP_TRY(cpqr_plan(kt, kt, &pl));
    }
    int32_t* inf = info ? info : f.info;
    RQLP_TRY(fill_zero_bytes(inf, sizeof(int32_t), s));
    // first CPQR: kt steps on a working copy of A
    RQLP_TRY(copy_matrix(m, n, A, lda, L.M, m, s));
    RQLP_TRY(qlp_first_cpqr(L.M, m, m, n, kt, L.Vh, m, L.beta, L.mu, f.piv0, L.colstep, L.slots, L.counter, L.state,
                            L.dstate, inf, s));
    RQLP_TRY(qlp_extract_rt(L.M, m, n, kt, L.colstep, L.mu, L.state, f.Z, n, s));
    // second stage: R^T = Qt Rtil (CholeskyQR2), Rtil Pi1 = Qhat L^T, P = Qt Qhat
    Ctx cx{s, inf, f.gws, f.gws_elems, f.o, f.o.shifted};
    double* Qt = nullptr;
    RQLP_TRY(cholqr2(cx, n, kt, f.Z, f.Z2, n, f.RtT, &Qt));
    RQLP_TRY(transpose_matrix(kt, kt, f.RtT, kt, f.Rtil, kt, 0, s));
    RQLP_TRY(cpqr(f.Rtil, kt, kt, kt, f.cs, f.piv1, f.Vh1, kt, f.beta1, f.Lt, kt, nullptr, 1, inf, s));
    RQLP_TRY(apply_householder(kt, kt, f.Vh1, kt, f.beta1, nullptr, 0, nullptr, kt, f.Mr, kt, s));
    RQLP_TRY(gemm<double>(false, false, n, kt, kt, Qt, n, f.Mr, kt, P, ldp, false, 1.0, 0.0, f.gws, f.gws_elems, s));
    RQLP_TRY(transpose_matrix(kt, kt, f.Lt, kt, T, ldt, 'L', s));
    // Q = Qhat(:, 1:kt) Pi1: the first CPQR's reflectors applied to e_{piv1(c)}
    RQLP_TRY(householder_tall(m, kt, L.Vh, m, L.beta, f.piv1, kt, Q, ldq, s));
    if (piv0) RQLP_TRY(copy_i64(kt, f.piv0, piv0, s));
    if (piv1) RQLP_TRY(copy_i64(kt, f.piv1, piv1, s));
    RQLP_TRY(finish_lvals(kt, T, ldt, lvals, inf, s));
    return 0;
}

int rqlp_autorank_workspace_size(int64_t m, int64_t n, int64_t lmax, int64_t b, int q, int precision,
                                 size_t* bytes) {
    RQLP_TRY(check_autorank_args((const void*)1, m, m, n, lmax, b, q, 0.0, precision));
    if (!bytes) return -7;
    const int64_t bs = b < lmax ? b : 0;
    Arena ar(nullptr, 0);
    FactorLayout L;
    carve_factor(ar, m, n, lmax, precision, true, bs, &L);
    ar.take<double>(4);
    ar.take<double>(autorank_scratch_doubles(n, lmax, bs));
    *bytes = ar.used + 256;
    return 0;
}

int rqlp_factor_autorank(const void* A, int64_t lda, int64_t m, int64_t n, int64_t lmax, int64_t b, int q,
                         double eps, int precision, uint64_t seed, const void* Omega, int64_t ldo, void* Q,
                         int64_t ldq, double* T, int64_t ldt, void* P, int64_t ldp, int64_t* piv0, int64_t* piv1,
                         double* lvals, int32_t* info, int64_t* rank, double* err2, void* work, size_t work_bytes,
                         void* stream) {
    RQLP_TRY(check_autorank_args(A, lda, m, n, lmax, b, q, eps, precision));
    if (Omega && ldo < n) return -12;
    if (!Q) return -13;
    if (ldq < m) return -14;
    if (!T) return -15;
    if (ldt < lmax) return -16;
    if (!P) return -17;
    if (ldp < n) return -18;
    if (!rank) return -23;
    if (!work) return -25;
    AutoRank arq{eps, rank, err2};
    const int64_t bs = b < lmax ? b : 0;
    return factor_core(A, lda, m, n, lmax, q, 0, bs, precision, seed, Omega, ldo, Q, ldq, T, ldt, P, ldp, piv0, piv1,
                       lvals, info, nullptr, work, work_bytes, (hipStream_t)stream, &arq);
}

// ---- building blocks ----
namespace {
// scratch of one 16-bit product over A (m x n) with a c-column panel
struct LpOp {
    unsigned short* Ah;
    unsigned short* Al;
    unsigned short* Xh;
    unsigned short* Xl;
    int* colexp;
    int* gexp;
    float* ws;
    size_t ws_elems;
};
void carve_lp_op(Arena& ar, int64_t m, int64_t n, int64_t c, int precision, LpOp* o) {
    const bool x3 = precision == RQLP_MIXED_BF16X3;
    const int64_t mx = m > n ? m : n;
    const size_t ea = lp_tiled_elems(m, n) > lp_tiled_elems(n, m) ? lp_tiled_elems(m, n) : lp_tiled_elems(n, m);
    o->Ah = ar.take<unsigned short>(ea);
    o->Al = x3 ? ar.take<unsigned short>(ea) : nullptr;
    o->Xh = ar.take<unsigned short>(lp_tiled_elems(c, mx));
    o->Xl = x3 ? ar.take<unsigned short>(lp_tiled_elems(c, mx)) : nullptr;
    o->colexp = ar.take<int>(n > 0 ? n : 1);
    o->gexp = ar.take<int>(1);
    o->ws_elems = max_ws(gemm_lp_workspace_elems, {{m, c, n}, {n, c, m}});
    o->ws = ar.take<float>(o->ws_elems);
}
bool gemm_precision(int p) { return p == RQLP_F64 || p == RQLP_F32 || is_mixed(p); }
}  // namespace

int rqlp_gemm_workspace(int64_t m, int64_t n, int64_t c, int precision, size_t* bytes) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (c < 0) return -3;
    if (!gemm_precision(precision)) return -4;
    if (!bytes) return -5;
    Arena ar(nullptr, 0);
    if (is_mixed(precision)) {
        LpOp o;
        carve_lp_op(ar, m, n, c, precision, &o);
    } else {
        const size_t e = max_ws(gemm_workspace_elems, {{m, c, n}, {n, c, m}});
        if (precision == RQLP_F64) ar.take<double>(e);
        else ar.take<float>(e);
    }
    *bytes = ar.used + 256;
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
    if (!gemm_precision(precision)) return -10;
    if (m * n * c > 0 && (!A || !X || !Y)) return !A ? -1 : (!X ? -5 : -8);
    if (m * c == 0) return 0;
    Arena ar = arena_for(work, work_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (is_mixed(precision)) {
        LpOp o;
        carve_lp_op(ar, m, n, c, precision, &o);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        const bool fp16 = precision == RQLP_MIXED_FP16;
        const float* Af = (const float*)A;
        if (fp16) RQLP_TRY(column_exponents(m, n, Af, lda, o.colexp, o.gexp, s));
        RQLP_TRY(encode_tiled(precision, m, n, Af, lda, nullptr, nullptr, o.Ah, o.Al, fp16 ? o.colexp : nullptr, s));
        RQLP_TRY(cast_panel(precision, c, n, (const float*)X, ldx, o.Xh, o.Xl, fp16 ? o.colexp : nullptr,
                            fp16 ? o.gexp : nullptr, s));
        return gemm_lp<float>(precision, m, c, n, o.Ah, o.Al, o.Xh, o.Xl, (float*)Y, ldy, false, nullptr,
                              fp16 ? o.gexp : nullptr, o.ws, o.ws_elems, s);
    }
    size_t e = gemm_workspace_elems(m, c, n);
    if (precision == RQLP_F64) {
        double* ws = ar.take<double>(e);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        return gemm<double>(false, false, m, c, n, (const double*)A, lda, (const double*)X, ldx, (double*)Y, ldy, false,
                            1.0, 0.0, ws, e, s);
    }
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
    if (!gemm_precision(precision)) return -10;
    if (m * n * c > 0 && (!A || !V || !B)) return !A ? -1 : (!V ? -5 : -8);
    if (n * c == 0) return 0;
    Arena ar = arena_for(work, work_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (is_mixed(precision)) {
        LpOp o;
        carve_lp_op(ar, m, n, c, precision, &o);
        if (!ar.ok()) return RQLP_E_WORKSPACE;
        const bool fp16 = precision == RQLP_MIXED_FP16;
        const float* Af = (const float*)A;
        if (fp16) RQLP_TRY(column_exponents(m, n, Af, lda, o.colexp, o.gexp, s));
        RQLP_TRY(encode_tiled(precision, m, n, Af, lda, o.Ah, o.Al, nullptr, nullptr, fp16 ? o.colexp : nullptr, s));
        RQLP_TRY(cast_panel(precision, c, m, (const float*)V, ldv, o.Xh, o.Xl, nullptr, nullptr, s));
        return gemm_lp<float>(precision, n, c, m, o.Ah, o.Al, o.Xh, o.Xl, (float*)B, ldb, true,
                              fp16 ? o.colexp : nullptr, nullptr, o.ws, o.ws_elems, s);
    }
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

int rqlp_encoded_elems(int64_t m, int64_t n, int form, size_t* elems) {
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (form != RQLP_ENC_COLS && form != RQLP_ENC_ROWS) return -3;
    if (!elems) return -4;
    *elems = form == RQLP_ENC_COLS ? lp_tiled_elems(n, m) : lp_tiled_elems(m, n);
    return 0;
}

int rqlp_encode(const float* A, int64_t lda, int64_t m, int64_t n, int precision, int form, uint16_t* Ahi,
                uint16_t* Alo, int32_t* colexp, int32_t* gexp, void* stream) {
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -2;
    if (!is_mixed(precision)) return -5;
    if (form != RQLP_ENC_COLS && form != RQLP_ENC_ROWS) return -6;
    if (m * n == 0) return 0;
    if (!A) return -1;
    if (!Ahi) return -7;
    if ((Alo != nullptr) != (precision == RQLP_MIXED_BF16X3)) return -8;
    const bool fp16 = precision == RQLP_MIXED_FP16;
    if (fp16 && !colexp) return -9;
    if (fp16 && !gexp) return -10;
    hipStream_t s = (hipStream_t)stream;
    if (fp16) RQLP_TRY(column_exponents(m, n, A, lda, colexp, gexp, s));
    unsigned short* hi = (unsigned short*)Ahi;
    unsigned short* lo = (unsigned short*)Alo;
    if (form == RQLP_ENC_COLS) return encode_tiled(precision, m, n, A, lda, hi, lo, nullptr, nullptr, fp16 ? colexp : nullptr, s);
    return encode_tiled(precision, m, n, A, lda, nullptr, nullptr, hi, lo, fp16 ? colexp : nullptr, s);
}

namespace {
// Shared argument checks of the two products on an encoded A: the panel P
// (prow x c, ldp) and the output O (leading dimension ldo >= orow, oelems
// entries), inner dimension K.
// Returns 1 when there is nothing to compute (empty output), 0 to proceed.
int check_encoded_args(const uint16_t* Ahi, const uint16_t* Alo, const int32_t* colexp, const int32_t* gexp,
                       bool need_gexp, int64_t m, int64_t n, const float* P, int64_t ldp, int64_t prow, int64_t c,
                       const float* O, int64_t ldo, int64_t orow, int64_t oelems, int64_t K, int precision) {
    if (m < 0) return -5;
    if (n < 0) return -6;
    if (ldp < (prow > 1 ? prow : 1)) return -8;
    if (c < 0) return -9;
    if (ldo < (orow > 1 ? orow : 1)) return -11;
    if (!is_mixed(precision)) return -12;
    if (oelems == 0) return 1;
    if (!O) return -10;
    if (K == 0) return 0;
    if (!Ahi) return -1;
    if ((Alo != nullptr) != (precision == RQLP_MIXED_BF16X3)) return -2;
    if (precision == RQLP_MIXED_FP16 && !colexp) return -3;
    if (precision == RQLP_MIXED_FP16 && need_gexp && !gexp) return -4;
    if (!P) return -7;
    return 0;
}
}  // namespace

int rqlp_project_encoded(const uint16_t* Ahi, const uint16_t* Alo, const int32_t* colexp, const int32_t* gexp,
                         int64_t m, int64_t n, const float* V, int64_t ldv, int64_t c, float* B, int64_t ldb,
                         int precision, void* work, size_t work_bytes, void* stream) {
    const int chk = check_encoded_args(Ahi, Alo, colexp, gexp, false, m, n, V, ldv, m, c, B, ldb, c, n * c, m, precision);
    if (chk != 0) return chk < 0 ? chk : 0;
    Arena ar = arena_for(work, work_bytes);
    unsigned short* Vh = ar.take<unsigned short>(lp_tiled_elems(c, m));
    unsigned short* Vl = precision == RQLP_MIXED_BF16X3 ? ar.take<unsigned short>(lp_tiled_elems(c, m)) : nullptr;
    const size_t e = gemm_lp_workspace_elems(n, c, m);
    float* ws = ar.take<float>(e);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    RQLP_TRY(cast_panel(precision, c, m, V, ldv, Vh, Vl, nullptr, nullptr, s));
    return gemm_lp<float>(precision, n, c, m, (const unsigned short*)Ahi, (const unsigned short*)Alo, Vh, Vl, B, ldb,
                          true, precision == RQLP_MIXED_FP16 ? colexp : nullptr, nullptr, ws, e, s);
}

int rqlp_sketch_encoded(const uint16_t* Ahi, const uint16_t* Alo, const int32_t* colexp, const int32_t* gexp,
                        int64_t m, int64_t n, const float* X, int64_t ldx, int64_t c, float* Y, int64_t ldy,
                        int precision, void* work, size_t work_bytes, void* stream) {
    const int chk = check_encoded_args(Ahi, Alo, colexp, gexp, true, m, n, X, ldx, n, c, Y, ldy, m, m * c, n, precision);
    if (chk != 0) return chk < 0 ? chk : 0;
    Arena ar = arena_for(work, work_bytes);
    unsigned short* Xh = ar.take<unsigned short>(lp_tiled_elems(c, n));
    unsigned short* Xl = precision == RQLP_MIXED_BF16X3 ? ar.take<unsigned short>(lp_tiled_elems(c, n)) : nullptr;
    const size_t e = gemm_lp_workspace_elems(m, c, n);
    float* ws = ar.take<float>(e);
    if (!ar.ok()) return RQLP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const bool fp16 = precision == RQLP_MIXED_FP16;
    RQLP_TRY(cast_panel(precision, c, n, X, ldx, Xh, Xl, fp16 ? colexp : nullptr, fp16 ? gexp : nullptr, s));
    return gemm_lp<float>(precision, m, c, n, (const unsigned short*)Ahi, (const unsigned short*)Alo, Xh, Xl, Y, ldy,
                          false, nullptr, fp16 ? gexp : nullptr, ws, e, s);
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
    Ctx cx{s, inf, gws, e, o, o.shifted};
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
