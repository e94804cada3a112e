// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include "common.hpp"

namespace rqlp {

// --- api.hip ----------------------------------------------------------------
// Synchronous argument checks of rqlp_factor up to (not including) the
// workspace: 0, or -i for the first invalid argument i (rqlp_factor's numbering).
int factor_arg_status(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                      int precision, const void* Omega, int64_t ldo, const void* Q, int64_t ldq, const double* T,
                      int64_t ldt, const void* P, int64_t ldp);

// --- gemm.hip ---------------------------------------------------------------
// C = alpha * op(A) * op(B) + beta * C, op(A) = A (ta = false, A is M x K)
// or A^T (ta = true, A is K x M); op(B) = B (tb = false, B is K x N) or B^T
// (tb = true, B is N x K; not combined with ta); C is M x N, or N x M when
// trans_out (C = (op(A) op(B))^T).  ws must hold gemm_workspace_elems(M, N, K)
// elements unless the product goes straight to C.  Conditional products:
// gate (device word, optional) read at run time; when it is 0, gate_mode 1
// computes nothing, gate_mode 2 copies op(A) to C (the product with an
// identity B, direct products with op(A) = A and K == N only).
size_t gemm_workspace_elems(int64_t M, int64_t N, int64_t K);
template <typename T>
int gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B, int64_t ldb,
         T* C, int64_t ldc, bool trans_out, T alpha, T beta, T* ws, size_t ws_elems, hipStream_t s,
         const int32_t* gate = nullptr, int gate_mode = 0, int tri = 0);
// tri = 1: only the lower triangle of C is computed and written (the Gram
// matrix op(A) op(B) = X^T X of CholeskyQR; no transposed output, beta 0);
// tri = 2: op(B) = B^T with B lower triangular (its strict upper part is not
// read), e.g. X L^{-T}.
// --- cholqr_mm.hip: the products of a CholeskyQR pass on a tall panel ------
// G = X^T X (lower triangle; X: R x c, c <= 512) and Y = X Li^T (Li lower
// triangular c x c, strict upper part not read), used by gemm for tri = 1 / 2
// when the operands qualify (*_fits); ws: gram_workspace_elems(R, c).
size_t gram_workspace_elems(int64_t R, int64_t c);
template <typename T>
bool gram_fits(int64_t R, int64_t c, const T* X, int64_t ldx, const T* ws, size_t ws_elems);
template <typename T>
int gram(int64_t R, int64_t c, const T* X, int64_t ldx, T* G, int64_t ldg, T* ws, size_t ws_elems, hipStream_t s,
         const int32_t* gate);
template <typename T>
bool trmm_fits(int64_t R, int64_t c, const T* X, int64_t ldx, const T* Y, int64_t ldy);
template <typename T>
int trmm_lt(int64_t R, int64_t c, const T* X, int64_t ldx, const T* Li, int64_t ldl, T* Y, int64_t ldy,
            hipStream_t s, const int32_t* gate, int gate_mode);
// The same product with FP32 operands and result but FP64 MFMA arithmetic
// (exact products, FP64 sums; split-K partials in ws are FP64).
int gemm_f32_acc64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                   int64_t ldb, float* C, int64_t ldc, bool trans_out, double alpha, double beta, double* ws,
                   size_t ws_elems, hipStream_t s, const int32_t* gate = nullptr, int gate_mode = 0);

// --- gemm_lp.hip ------------------------------------------------------------
// 16-bit operands are "fragment tiled": an R x K operand X is stored as
// ceil(R / 16) x ceil(K / 32) blocks of 512 elements, block (rb, kb) at
// (rb * ceil(K / 32) + kb) * 512, holding X(16 rb + t % 16, 32 kb + 8 (t / 16) + e)
// at 8 t + e (t < 64, e < 8); entries outside X are zero.
size_t lp_tiled_elems(int64_t rows, int64_t K);
// C(i, j) = 2^(gexp + rexp[i]) sum_k X(i, k) Y(j, k) with X (M x K, tiled P /
// lo part Plo) and Y (N x K, tiled Q / Qlo) 16-bit (bfloat16 or IEEE half per
// kind) and FP32 accumulation; M x N output C (or its transpose when
// trans_out) of type TO.  Plo / Qlo: split bfloat16 only, else NULL.
// rexp / gexp may be NULL (no scaling).  ws: gemm_lp_workspace_elems floats.
size_t gemm_lp_workspace_elems(int64_t M, int64_t N, int64_t K);
template <typename TO>
int gemm_lp(int kind, int64_t M, int64_t N, int64_t K, const unsigned short* P, const unsigned short* Plo,
            const unsigned short* Q, const unsigned short* Qlo, TO* C, int64_t ldc, bool trans_out, const int* rexp,
            const int* gexp, float* ws, size_t ws_elems, hipStream_t s);
// Tiled 16-bit copies of the FP32 matrix A (m x n) in one pass: Tc = A^T
// (n x m operand), Tr = A (m x n operand), either may be NULL; lo parts for
// the split form; FP16 columns scaled by 2^-cexp[j].
int encode_tiled(int kind, int64_t m, int64_t n, const float* A, int64_t lda, unsigned short* Tc,
                 unsigned short* Tclo, unsigned short* Tr, unsigned short* Trlo, const int* cexp, hipStream_t s);
// Tiled 16-bit copy of the panel operand X (R x K), X(r, k) = 2^(kexp[k] - gexp) src[k + r ld].
int cast_panel(int kind, int64_t R, int64_t K, const float* src, int64_t ld, unsigned short* dst, unsigned short* dlo,
               const int* kexp, const int* gexp, hipStream_t s);
// per-column power-of-two exponents of an FP32 matrix for IEEE half storage
int column_exponents(int64_t rows, int64_t cols, const float* A, int64_t lda, int* colexp, int* gexp,
                     hipStream_t s);
template <typename S, typename D>
int cast_matrix(int64_t rows, int64_t cols, const S* src, int64_t lds, D* dst, int64_t ldd, hipStream_t s);

// --- chol.hip ---------------------------------------------------------------
// Cholesky G = L L^T of the c x c Gram matrix (lower triangle read) and the
// inverse of L, in one workgroup.  On breakdown the factorisation restarts
// from G + shift_scale * trace(G) * I (RQLP_INFO_CHOLQR_SHIFTED).  Outputs:
// L and Linv (c x c lower triangular, leading dimension ld, zero above the
// diagonal); both are also the kernel's working storage.  G may be FP32 (it
// is widened); Linv32 (optional, leading dimension ld) gets Linv in FP32.
// run_flag (optional device word): when it reads 0 the kernel only writes
// identities (a conditional extra pass); shifted_out (optional): with
// shifted_mode 1 it receives 1 when the shifted retry was used, else 0; with
// shifted_mode 2 it is only ever set to 1 (accumulates over passes).
// pivot_rel: in the plain attempt a pivot <= pivot_rel * G(j, j) counts as a
// breakdown (column j numerically dependent on the earlier ones).
// sync: CHOL_SYNC_WORDS words of device scratch (flags of the multi-workgroup
// kernel used for c <= CHOL_MW_MAXC, and the partial sums and flag of the
// near-identity form); NULL selects the one-workgroup kernel.
// near_identity (with sync, c <= CHOL_MW_MAXC and no run_flag): G is
// expected within rounding of I (a second CholeskyQR pass); when
// ||G - I||_F is small enough L and L^{-1} come from the first-order form,
// else the factorisation runs as usual.
constexpr int CHOL_MW_MAXC = 512;
constexpr int CHOL_SYNC_WORDS = 1024;
constexpr int NEARID_PART_WORD = 128;   // 256 doubles of partial sums
constexpr int NEARID_FLAG_WORD = 640;   // int32: 1 when the full factorisation must run
size_t chol_inv_lds_bytes(int64_t c);
template <typename TG>
int chol_inv(int64_t c, const TG* G, int64_t ldg, double* L, double* Linv, float* Linv32, int64_t ld,
             double shift_scale, int32_t* info, hipStream_t s, const int32_t* run_flag = nullptr,
             int32_t* shifted_out = nullptr, unsigned* sync = nullptr, int shifted_mode = 1,
             double pivot_rel = 0.0, bool near_identity = false);
// gate_mode: 1 (default with run_flag) writes identities when *run_flag is 0,
// 2 returns without writing.
template <typename TG>
int chol_mw(int64_t c, const TG* G, int64_t ldg, double* L, double* Linv, float* Linv32, int64_t ld,
            double shift_scale, int32_t* info, unsigned* sync, hipStream_t s, const int32_t* run_flag,
            int32_t* shifted_out, int shifted_mode, double pivot_rel, int gate_mode = -1);

// --- cpqr.hip ---------------------------------------------------------------
struct CpqrScratch {
    unsigned long long* keys;   // kmax
    double* candcol;            // 2 * G * rows
    double* partial;            // G
    unsigned* bar;              // 2
};
struct CpqrPlan {
    int G;          // workgroups
    int cpw;        // columns per workgroup
    size_t lds;     // dynamic LDS bytes
    bool single;    // one workgroup: no grid-wide exchange
    int rpt;        // > 0: columns held in registers, rpt rows per lane (16 lanes per column)
    int wg_rpt;     // > 0: one workgroup of 512 threads holds the whole matrix in registers
    int wg_ct;      //      (wg_rpt rows per lane, wg_ct column groups of 32)
};
int cpqr_plan(int64_t rows, int64_t cols, CpqrPlan* plan);
size_t cpqr_scratch_bytes(int64_t rows, int64_t cols);
void cpqr_carve(Arena& ar, int64_t rows, int64_t cols, CpqrScratch* sc);
// M: rows x cols.  Outputs (any may be NULL except as noted): piv (kmax,
// int64), Vh (rows x kmax Householder vectors, v_j(j) = 1), beta (kmax),
// Rpiv (rows x kmax, pivoted columns of R), Rt (cols x rows: R^T in
// original column order).
int cpqr(const double* M, int64_t ldm, int64_t rows, int64_t cols, const CpqrScratch& sc, int64_t* piv,
         double* Vh, int64_t ldv, double* beta, double* Rpiv, int64_t ldr, double* Rt, int64_t ldrt,
         int32_t* info, hipStream_t s);

// Y = H_0 H_1 ... H_{k-1} X  (rows x ncols, in place on Y), where X is either
// given (X != NULL, copied into Y) or the unit columns e_{unit[c]} (unit !=
// NULL) or the leading identity columns (both NULL).
int apply_householder(int64_t rows, int64_t k, const double* Vh, int64_t ldv, const double* beta,
                      const double* X, int64_t ldx, const int64_t* unit, int64_t ncols, double* Y,
                      int64_t ldy, hipStream_t s);

// --- bqlp.hip: batched pivoted QLP of the block rows of B (block RQLP) ----
struct BqlpScratch {
    unsigned long long* keys;   // per block: bs steps x G workgroups x 2 key words
    unsigned long long* gw;     // per block: result word (one 128-byte line)
    double* frop;               // per block: G partial ||B_j||_F^2
    double* candcol;            // per block: 2 x G x 64 candidate columns
    double* Vh0;                // per block: bs x bs reflectors of the first CPQR
    double* beta0;              // l
    int* rank;                  // per block
    int32_t* shifted;           // per block: a Cholesky of R0_j^T needed the shift
    double* part;               // per block: ceil(n / 256) Gram partials of 64 x 64
    double* Ls;                 // 4 passes x per block 64 x 64 Cholesky factors
    double* Linv;               // per block 64 x 64
    double* RT;                 // per block 64 x 64: Rt_j^T
    double* Qhat;               // per block 64 x 64
    double* QB;                 // per block 64 x 64
};
void bqlp_carve(Arena& ar, int64_t n, int64_t l, int64_t bs, BqlpScratch* sc);
// blocks of bs <= 64 rows, n <= 65536 and a first-CPQR grid that fits on the device
bool bqlp_supported(int64_t n, int64_t l, int64_t bs);
// B (l x n, FP64): per block row j (rows [j bs, min(l, (j + 1) bs))): the
// pivoted QLP B_j = Q_B^(j) L_j P_B^(j)^T; outputs T = blkdiag(L_j) (l x l),
// Pd (n x l, FP64, column block j = P_B^(j)), Q (m x l, column block j =
// V_j Q_B^(j)), piv0 (original column indices), piv1 (0-based within the
// block).  Z: n x l FP64 scratch (R0^T, then Qt).
template <typename TV>
int bqlp(const double* B, int64_t ldb, int64_t n, int64_t l, int64_t bs, const BqlpScratch& sc, double* Z,
         const TV* V, int64_t ldv, int64_t m, TV* Q, int64_t ldq, double* Pd, int64_t ldpd, double* T, int64_t ldt,
         int64_t* piv0, int64_t* piv1, int32_t* info, hipStream_t s);

// --- autorank.hip: the error indicator of auto-rank RQLP (Section 6) --------
constexpr int AR_FROB_PARTS = 1024;
// doubles of scratch autorank_indicator needs
size_t autorank_scratch_doubles(int64_t n, int64_t l, int64_t bs);
// From A (m x n) and the block rows of B (l x n, blocks of bs rows; bs = 0:
// one block): out3[0] = J, the first block count (1-based) at which
// ||A||_F^2 - ||B_{1..J}||_F^2 <= eps (the number of blocks when none),
// out3[1] = that indicator, out3[2] = ||A||_F^2 (device doubles).
template <typename T>
int autorank_indicator(const T* A, int64_t lda, int64_t m, int64_t n, const double* B, int64_t ldb, int64_t l,
                       int64_t bs, double eps, double* scratch, double* out3, hipStream_t s);
// X(:, c0:c1) = 0 (rows x ..., leading dimension ldx)
template <typename T>
int zero_cols(int64_t rows, int64_t c0, int64_t c1, T* X, int64_t ldx, hipStream_t s);
int fill_i64(int64_t n, int64_t* p, int64_t v, hipStream_t s);
// *info |= bit (device word, one thread)
int set_info_flag(int32_t* info, int32_t bit, hipStream_t s);

// --- qlp.hip: deterministic truncated pivoted QLP (eq. (1.2)) -------------
int qlp_max_rows();
int qlp_grid(int64_t n);
// kt steps of the column-pivoted QR of M (m x n, in place, a working copy):
// pivots, reflectors Vh (m x kt, v(j) = 1, zero above), beta, mu (the diagonal
// of R); colstep (n ints): the step a column was taken at, -1 if never;
// slots: 4 * qlp_grid(n) words; counter: 1 word; state: 2 ints (stopped,
// rank); dstate: 1 double.
int qlp_first_cpqr(double* M, int64_t ldm, int64_t m, int64_t n, int64_t kt, double* Vh, int64_t ldv, double* beta,
                   double* mu, int64_t* piv, int* colstep, unsigned long long* slots, unsigned* counter, int* state,
                   double* dstate, int32_t* info, hipStream_t s);
// Z (n x kt) = R^T of that CPQR in original column order (rows of R past the rank zero)
int qlp_extract_rt(const double* M, int64_t ldm, int64_t n, int64_t kt, const int* colstep, const double* mu,
                   const int* state, double* Z, int64_t ldz, hipStream_t s);
// Y(:, c) = H_0 ... H_{k-1} e_{unit[c]} for tall reflectors (rows up to the LDS size / 8)
int householder_tall(int64_t rows, int64_t k, const double* Vh, int64_t ldv, const double* beta, const int64_t* unit,
                     int64_t ncols, double* Y, int64_t ldy, hipStream_t s);

// --- misc.hip ---------------------------------------------------------------
// Columns of X (rows x c) whose squared norm is <= tau2 are replaced by
// N(0, 1/rows) vectors (Philox4x32-10 counter (i, col0 + j, 1, 0), fixed
// key; col0 = the panel's first column in a wider basis, so that blocks of
// one basis get different vectors), and the diagonal entry L(j, j) of the
// optional c x c factor is zeroed.  Runs only when the device word *gate is
// non-zero.
int complete_columns(int64_t rows, int64_t c, double* X, int64_t ldx, double* L, int64_t ldl, double tau2,
                     const int32_t* gate, hipStream_t s, int64_t col0 = 0);
int fill_zero_bytes(void* p, size_t bytes, hipStream_t s);
int copy_matrix(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y, int64_t ldy,
                hipStream_t s);
// Y (cols x rows) = X^T, optionally keeping only the lower/upper triangle of Y.
// tri: 0 = full, 'L' = keep lower of Y, 'U' = keep upper of Y (rest zero).
int transpose_matrix(int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     int tri, hipStream_t s);
int set_identity(int64_t n, double* Y, int64_t ldy, hipStream_t s);
// lvals = diag(T), flags NaN/Inf in T into *info
int finish_lvals(int64_t l, const double* T, int64_t ldt, double* lvals, int32_t* info, hipStream_t s);
// dst[i] = src[i], or dst[i] = i when src is NULL
int copy_i64(int64_t n, const int64_t* src, int64_t* dst, hipStream_t s);
int generate_omega(int64_t n, int64_t l, uint64_t seed, int precision, void* Omega, int64_t ldo,
                   hipStream_t s);

}  // namespace rqlp
