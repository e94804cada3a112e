/*
 * rqlp.h - C ABI of the MI355X (gfx950) randomized QLP library.
 *
 * The library computes the rank-l randomized QLP factorisation
 *     A  ~=  Q T P^T
 * of Wu & Xiang, "Randomized QLP algorithm and error analysis":
 * Algorithm 2.1 (RQLP), Algorithm 2.2 (ERQLP, d inner QR steps) and
 * Algorithm 4.1 (block RQLP).  A is m x n (k <= n <= m), l = k + p,
 * Q is m x l and P is n x l with orthonormal columns, T is l x l triangular
 * and diag(T) are the "L-values" (Section 1).  q >= 0 subspace iterations
 * (Y <- A orth(A^T orth(Y))) may be added to the range finder of Section 2.
 *
 * Conventions for every entry point
 *   - matrices are column-major with an explicit leading dimension
 *     (element (i, j) of X is X[i + j * ldx]); ld >= rows;
 *   - all matrix / vector pointers are DEVICE pointers unless marked "host";
 *   - sizes are int64_t;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     every call only enqueues work on it and returns without waiting,
 *     except where stated;
 *   - the caller owns every buffer, including the workspace `work`; the
 *     library allocates and frees no device memory and keeps no per-call
 *     state (it caches immutable device properties only);
 *   - return value (synchronous, host): 0 on success, -i when argument i
 *     (1-based, LAPACK style) is invalid, or one of the RQLP_E_* codes.
 *     Numerical events found on the device are reported through the device
 *     word *info (bit flags RQLP_INFO_*), valid once the stream has reached
 *     the end of the call.
 */
#ifndef RQLP_H
#define RQLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the hot path.
 *   RQLP_F64       : everything in FP64 (A, Q, P are double).
 *   RQLP_F32       : A, Q, P float; GEMMs and orthonormalisation in FP32;
 *                    CPQR and the second stage in FP64.
 *   RQLP_MIXED_BF16: A, Q, P float; A, Omega and the orthonormal bases are
 *                    rounded to bfloat16 for the MFMA GEMMs (FP32 accumulate),
 *                    orthonormalisation by CholeskyQR2 with FP32 panels,
 *                    CPQR / second stage / L in FP64.
 *   RQLP_MIXED_FP16: as BF16 with IEEE half and per-column power-of-two
 *                    scaling of A.
 *   RQLP_MIXED_BF16X3: as BF16 with A and the bases split into hi + lo
 *                    bfloat16 parts (three MFMA products per pass).       */
enum rqlp_precision {
    RQLP_F64 = 0,
    RQLP_F32 = 1,
    RQLP_MIXED_BF16 = 2,
    RQLP_MIXED_FP16 = 3,
    RQLP_MIXED_BF16X3 = 4
};

enum rqlp_status {
    RQLP_OK = 0,
    RQLP_E_WORKSPACE = -1000,   /* work_bytes smaller than rqlp_workspace_size() */
    RQLP_E_HIP = -1001,         /* a HIP launch / runtime call failed            */
    RQLP_E_UNSUPPORTED = -1002, /* valid arguments the library does not handle  */
    RQLP_E_SCRATCH_LIMIT = -1003 /* rqlp_factor_noalloc: problem needs more than
                                    RQLP_NOALLOC_SCRATCH_BYTES of workspace      */
};

/* bit flags written to *info (device int32) */
#define RQLP_INFO_CHOLQR_SHIFTED   0x1  /* a Cholesky broke down; shifted retry used */
#define RQLP_INFO_RANK_DEFICIENT   0x2  /* a CPQR stopped early: trailing L-values 0 */
#define RQLP_INFO_NONFINITE        0x4  /* NaN / Inf met in A or an intermediate     */
#define RQLP_INFO_BARRIER_TIMEOUT  0x8  /* a grid-wide wait exceeded its spin bound  */
#define RQLP_INFO_CHOL_FAILED      0x10 /* Cholesky failed even after the shift      */
#define RQLP_INFO_BAD_PIVOTS       0x20 /* rqlp_backward: frozen pivots not valid    */
#define RQLP_INFO_NOT_CONVERGED    0x40 /* rqlp_factor_autorank: eps not reached     */

/* Library version string (host, static storage). */
const char* rqlp_version(void);

/* Human-readable text for a return code (host, static storage). */
const char* rqlp_status_string(int status);

/* Bytes of device workspace rqlp_factor needs for these arguments
 * (written to *bytes, a host pointer).  Arguments as for rqlp_factor. */
int rqlp_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                        int precision, size_t* bytes);

/* Gaussian test matrix (Section 2, the range finder's random matrix;
 * Algorithm 2.1): Omega (n x l, leading dimension ldo) with N(0,1) entries.
 * Element (i, j) is Box-Muller applied to the first two 32-bit words of
 * Philox4x32-10 (Salmon et al., SC'11) with counter (i, j, 0, 0) and key
 * (low 32 bits of seed, high 32 bits of seed):
 *     U1 = (w0 + 1) 2^-32,  U2 = w1 2^-32,
 *     Omega(i, j) = sqrt(-2 ln U1) cos(2 pi U2),
 * computed in FP64 and stored as double (RQLP_F64) or float (other
 * precisions; mixed precisions round further to the 16-bit GEMM type, and
 * store that exactly representable value as float). */
int rqlp_generate_omega(int64_t n, int64_t l, uint64_t seed, int precision,
                        void* Omega, int64_t ldo, void* stream);

/* Randomized QLP of A (Algorithms 2.1, 2.2, 4.1).
 *
 *   A      m x n, lda >= m; double for RQLP_F64, float otherwise.  Read only.
 *   k, p   target rank k >= 2 and oversampling p >= 2 (Algorithm 2.1 input),
 *          l = k + p <= n <= m (Section 1 problem statement).
 *   q      number of subspace iterations of the range finder, q >= 0.
 *   d      0: RQLP, second factorisation pivoted (Algorithm 2.1);
 *          d >= 1: ERQLP with d unpivoted inner QR steps (Algorithm 2.2).
 *   b      0: unblocked; b >= 1: block RQLP with blocks of b columns of
 *          Omega (Algorithm 4.1; the last block is ragged when b does not
 *          divide l); requires d == 0.
 *   precision  one of rqlp_precision.
 *   seed   used when Omega == NULL (see rqlp_generate_omega).
 *   Omega  optional n x l test matrix (ldo >= n), same element type as A;
 *          NULL => generated from seed into the workspace.
 *   Q      m x l output (ldq >= m), element type of A.
 *   T      l x l output (ldt >= l), double: lower triangular ("L") for d = 0
 *          and odd d, upper triangular for even d >= 2 (the inner-QR
 *          assembly of Algorithm 2.2 puts R^(d) itself, not its transpose,
 *          between the orthogonal factors when d is even); *uplo says which.
 *          Block RQLP: T = blkdiag(L_1, ..., L_h).
 *   P      n x l output (ldp >= n), element type of A.  Block RQLP: each
 *          b-column block is orthonormal (the blocks are not mutually
 *          orthogonal).
 *   piv0   l int64 (may be NULL): the first l pivots of the CPQR of B
 *          (original column indices of A, 0-based); block RQLP: per block.
 *   piv1   l int64 (may be NULL): pivots of the second CPQR (d = 0), the
 *          identity otherwise; block RQLP: per block, 0-based within it.
 *   lvals  l doubles (may be NULL): diag(T) (>= 0).
 *   info   device int32 (may be NULL): RQLP_INFO_* flags, overwritten.
 *   uplo   host char (may be NULL): 'L' or 'U', the triangle of T.
 *   work   device workspace of work_bytes >= rqlp_workspace_size(); its
 *          contents on entry are ignored.  Alignment 256 bytes.
 *
 * Arguments are checked before any work is enqueued.  Outputs are written
 * with plain stores; on RQLP_E_* nothing useful is in them. */
int rqlp_factor(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p,
                int q, int d, int b, int precision, uint64_t seed,
                const void* Omega, int64_t ldo,
                void* Q, int64_t ldq, double* T, int64_t ldt, void* P, int64_t ldp,
                int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info, char* uplo,
                void* work, size_t work_bytes, void* stream);

/* rqlp_factor for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid
 * allocation).  No workspace argument: the workspace is a fixed device array
 * of RQLP_NOALLOC_SCRATCH_BYTES bytes inside the library, one copy per device
 * the library runs on, held until the process ends.  A problem whose
 * rqlp_workspace_size() exceeds that size returns RQLP_E_SCRATCH_LIMIT
 * before any work is enqueued.  Arguments 1-24, outputs, argument errors and
 * the asynchronous *info flags are those of rqlp_factor; argument 25 is the
 * stream.  Everything that must start at zero is cleared by kernels inside
 * the call.  All calls on one device share its array: calls that may overlap
 * in time on one device (different streams, or host threads without ordering
 * between them) race and give wrong results; calls on one stream are
 * ordered and safe.  Capturing a call into a HIP graph for replay is not
 * supported (the flag epochs of the multi-workgroup Cholesky are fixed when
 * the call is enqueued). */
#define RQLP_NOALLOC_SCRATCH_BYTES (64u << 20)
int rqlp_factor_noalloc(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p,
                        int q, int d, int b, int precision, uint64_t seed,
                        const void* Omega, int64_t ldo,
                        void* Q, int64_t ldq, double* T, int64_t ldt, void* P, int64_t ldp,
                        int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info, char* uplo,
                        void* stream);

/* Auto-rank (fixed-accuracy) randomized QLP (Section 6): the rank is set by
 * an accuracy tolerance instead of k.  The basis grows one block of b
 * columns of Omega at a time as in Algorithm 4.1 (q subspace iterations,
 * block orthonormalisation against the earlier blocks), and stops at the
 * first block where the error indicator
 *     ||E||_F^2 = ||A||_F^2 - ||B||_F^2,   B = V^T A of the blocks so far,
 * (equal to ||A - Q T P^T||_F^2 by the identity (fixedrank) of Section 2) is
 * <= eps, or when lmax columns are used.  The factorisation of the columns
 * taken is block RQLP's (T = blkdiag(L_j), each b-column block of P
 * orthonormal).
 *
 *   A, lda, m, n, q, precision, seed, Omega (n x lmax), ldo: as for
 *          rqlp_factor.
 *   lmax   largest rank, 1 <= lmax <= n (the columns of Omega).
 *   b      block size >= 1 (b >= lmax: one block, plain RQLP of lmax columns).
 *   eps    tolerance on ||E||_F^2 (absolute, >= 0).  It must lie above the
 *          rounding level of ||A||_F^2 - ||B||_F^2 in the chosen precision:
 *          about 1e-15 ||A||_F^2 in FP64, 1e-6 in FP32, 1e-3 for the 16-bit
 *          products.
 *   Q (m x lmax), T (lmax x lmax, lower triangular), P (n x lmax),
 *   piv0, piv1, lvals (lmax each): as for rqlp_factor on the columns taken;
 *          past the rank the columns of Q and P and all of T there are zero,
 *          the pivots -1 and the L-values 0.
 *   info   device word: RQLP_INFO_* flags; RQLP_INFO_NOT_CONVERGED when eps
 *          was not reached with lmax columns.
 *   rank   host out: the number of columns taken (a multiple of b, or lmax).
 *   err2   host out (may be NULL): ||E||_F^2 at that rank.
 *   work   device workspace of rqlp_autorank_workspace_size() bytes.
 * The stopping block is read back to the host: unlike the other entry points
 * this call synchronises `stream` once (after the range finder) and returns
 * after enqueueing the rest.  This implementation evaluates the basis over
 * all lmax columns in one blocked pass (every prefix of its blocks is the
 * basis the block-by-block loop builds) and factorises only the blocks taken,
 * so its cost grows with lmax, not with the rank found. */
int rqlp_autorank_workspace_size(int64_t m, int64_t n, int64_t lmax, int64_t b, int q, int precision,
                                 size_t* bytes);
int rqlp_factor_autorank(const void* A, int64_t lda, int64_t m, int64_t n, int64_t lmax, int64_t b,
                         int q, double eps, int precision, uint64_t seed,
                         const void* Omega, int64_t ldo,
                         void* Q, int64_t ldq, double* T, int64_t ldt, void* P, int64_t ldp,
                         int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info,
                         int64_t* rank, double* err2, void* work, size_t work_bytes, void* stream);

/* Deterministic truncated pivoted QLP (Stewart's QLP, eq. (1.2) of
 * Section 1; the "QLP" comparison method of Section 5), FP64: kt steps of the
 * column-pivoted Householder QR of A itself, A Pi0 ~= Qhat R with R its first
 * kt rows, then the pivoted QR of R^T (the second factorisation of
 * Algorithm 2.1): A ~= Q T P^T with Q (m x kt) and P (n x kt)
 * orthonormal, T (kt x kt) lower triangular, diag(T) the L-values.  With
 * kt = min(m, n) this is Stewart's full pivoted QLP (exact reconstruction).
 *
 *   A      m x n double (lda >= m), read only; m <= 6144 in this library
 *          (RQLP_E_UNSUPPORTED beyond).
 *   kt     number of pivot steps, 1 <= kt <= min(m, n).
 *   Q, T, P  outputs (ldq >= m, ldt >= kt, ldp >= n).
 *   piv0   kt int64 (may be NULL): pivots of the QR of A (original columns).
 *   piv1   kt int64 (may be NULL): pivots of the QR of R^T.
 *   lvals  kt doubles (may be NULL): diag(T).
 *   info   device int32 (may be NULL): RQLP_INFO_* flags (rank stop of
 *          either pivoted QR: RQLP_INFO_RANK_DEFICIENT, trailing L-values 0).
 *   work   device workspace of rqlp_qlp_workspace_size() bytes (holds an
 *          m x n working copy of A).
 * Pivot rule, ties and rank stop as for rqlp_cpqr.  The QR of A streams the
 * working copy through the device once per pivot step (one launch each). */
int rqlp_qlp_workspace_size(int64_t m, int64_t n, int64_t kt, size_t* bytes);
int rqlp_qlp(const double* A, int64_t lda, int64_t m, int64_t n, int64_t kt,
             double* Q, int64_t ldq, double* T, int64_t ldt, double* P, int64_t ldp,
             int64_t* piv0, int64_t* piv1, double* lvals, int32_t* info,
             void* work, size_t work_bytes, void* stream);

/* ---- building blocks (the steps of Algorithm 2.1, usable on their own) ---- */

/* Adjoint of rqlp_factor with frozen pivots: dA = d<dT, T>/dA, the gradient
 * of any loss of the triangular factor T (the L-values of Section 1 are
 * diag(T)) with respect to A.  The pivot sequences piv0 / piv1 returned by
 * the forward call are held fixed, which makes T a smooth function of A
 * (any fixed pivot order gives a valid QLP).  The forward pipeline
 * (Algorithm 2.1 with q subspace iterations) is recomputed from A and Omega
 * inside the call; nothing has to be kept from the forward call.
 *
 *   A, lda, m, n, k, p, q, d, b, precision, seed, Omega, ldo: as for the
 *          forward call that produced the pivots (same Omega, or same seed
 *          with Omega == NULL).  Supported here: d == 0, b == 0,
 *          precision RQLP_F64 or RQLP_F32 (others: RQLP_E_UNSUPPORTED).
 *   piv0   l int64: the forward's first pivots (distinct, in [0, n)).
 *   piv1   l int64: the forward's second pivots (a permutation of [0, l)).
 *          Invalid pivots set RQLP_INFO_BAD_PIVOTS in *info; dA is then
 *          meaningless but no memory outside the arguments is touched.
 *   dT     l x l double (lddt >= l): cotangent of T; entries above the
 *          diagonal are ignored (T is lower triangular for d == 0).
 *   dQ, dP cotangents of Q and P: must be NULL (not supported here).
 *   saved  must be NULL (no forward state is kept; always recomputed).
 *   dA     m x n output (ldda >= m), element type of A; overwritten.
 *   info   device int32 (may be NULL): RQLP_INFO_* flags, overwritten.
 *   work   device workspace, >= rqlp_backward_workspace_size() bytes.
 * Arithmetic: the passes over A and the panel orthonormalisations in the
 * precision of A; the l x l and n x l algebra in FP64. */
int rqlp_backward(const void* A, int64_t lda, int64_t m, int64_t n, int64_t k, int64_t p,
                  int q, int d, int b, int precision, uint64_t seed,
                  const void* Omega, int64_t ldo, const int64_t* piv0, const int64_t* piv1,
                  const double* dT, int64_t lddt, const void* dQ, int64_t lddq,
                  const void* dP, int64_t lddp, const void* saved,
                  void* dA, int64_t ldda, int32_t* info, void* work, size_t work_bytes,
                  void* stream);

/* Bytes of device workspace rqlp_backward needs (host out).  Arguments as
 * for rqlp_backward; RQLP_E_UNSUPPORTED for the combinations it rejects. */
int rqlp_backward_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int d, int b,
                                 int precision, size_t* bytes);

/* Y = A X  (the sketch of Algorithm 2.1, and every pass of the subspace iteration):
 * A m x n, X n x c, Y m x c, all double (RQLP_F64) or all float (any other
 * precision).  The mixed precisions round A and X to their 16-bit type as
 * rqlp_encode does and accumulate in FP32 (RQLP_MIXED_FP16 scales column j
 * of A by 2^-e_j and row j of X by 2^(e_j - g), and Y by 2^g).
 * Uses `work` for split-K partial sums and the 16-bit copies; query the size
 * with rqlp_gemm_workspace. */
int rqlp_sketch(const void* A, int64_t lda, int64_t m, int64_t n, const void* X, int64_t ldx,
                int64_t c, void* Y, int64_t ldy, int precision, void* work, size_t work_bytes,
                void* stream);

/* B = V^T A  (the projection of Algorithm 2.1): V m x c, A m x n, B c x n; element
 * types and 16-bit rounding as for rqlp_sketch (FP16: B(:, j) carries the
 * column scale 2^e_j back). */
int rqlp_project(const void* A, int64_t lda, int64_t m, int64_t n, const void* V, int64_t ldv,
                 int64_t c, void* B, int64_t ldb, int precision, void* work, size_t work_bytes,
                 void* stream);

/* Bytes of work rqlp_sketch / rqlp_project / rqlp_project_encoded /
 * rqlp_sketch_encoded need for
 * these shapes (host out). */
int rqlp_gemm_workspace(int64_t m, int64_t n, int64_t c, int precision, size_t* bytes);

/* 16-bit encoding of the FP32 matrix A (m x n) used by the MFMA products of
 * the mixed precisions (the sketch / projection operands of Algorithm 2.1
 * in reduced precision).  precision is RQLP_MIXED_BF16,
 * RQLP_MIXED_FP16 or RQLP_MIXED_BF16X3; each element x of A becomes
 *   BF16   : hi = bf16(x) (round to nearest even);
 *   BF16X3 : hi = bf16(x), lo = bf16(x - hi);
 *   FP16   : hi = half(x 2^-e_j) for x in column j, with e_j chosen per
 *            column so that max_i |A(i, j)| 2^-e_j lies in [2^14, 2^15) (0 for
 *            a zero column); colexp (n int32) receives e_j and gexp (1 int32)
 *            max_j e_j.  colexp / gexp are not used by the other types and
 *            may be NULL there.
 * Layout ("fragment tiles", the order in which the 16x16x32 matrix-core
 * instruction consumes its operands): the encoded operand X (R x K) is
 *   form RQLP_ENC_COLS: X = A^T (R = n, K = m), the operand of B = V^T A;
 *   form RQLP_ENC_ROWS: X = A   (R = m, K = n), the operand of Y = A X;
 * it is stored as ceil(R/16) * ceil(K/32) blocks of 512 elements, block
 * (rb, kb) starting at element (rb * ceil(K/32) + kb) * 512 and holding
 * X(16 rb + t % 16, 32 kb + 8 (t / 16) + e) at offset 8 t + e (t < 64, e < 8);
 * entries beyond X are zero.  rqlp_encoded_elems gives the element count of
 * Ahi (and of Alo, which must be NULL unless BF16X3).  Elements are raw
 * 16-bit patterns.  The caller owns all buffers. */
#define RQLP_ENC_COLS 0
#define RQLP_ENC_ROWS 1
int rqlp_encoded_elems(int64_t m, int64_t n, int form, size_t* elems);
int rqlp_encode(const float* A, int64_t lda, int64_t m, int64_t n, int precision, int form,
                uint16_t* Ahi, uint16_t* Alo, int32_t* colexp, int32_t* gexp, void* stream);

/* B = V^T A (the projection of Algorithm 2.1) with A given by rqlp_encode in form
 * RQLP_ENC_COLS (Ahi, Alo; colexp for RQLP_MIXED_FP16, else NULL; gexp is
 * not used and may be NULL); V is m x c float, rounded to the same 16-bit
 * type inside; B is c x n float, FP32 accumulation.  Lets a caller encode A
 * once and reuse it.  Work: rqlp_gemm_workspace(m, n, c). */
int rqlp_project_encoded(const uint16_t* Ahi, const uint16_t* Alo, const int32_t* colexp,
                         const int32_t* gexp, int64_t m, int64_t n, const float* V, int64_t ldv,
                         int64_t c, float* B, int64_t ldb, int precision, void* work,
                         size_t work_bytes, void* stream);

/* Y = A X (the sketch of Algorithm 2.1 and the subspace iterations) with A given by
 * rqlp_encode in form RQLP_ENC_ROWS (colexp and gexp required for
 * RQLP_MIXED_FP16); X is n x c float, rounded inside (FP16: row j scaled by
 * 2^(e_j - g), Y by 2^g); Y is m x c float.  Same error conventions as
 * rqlp_project_encoded (argument numbers in this order). */
int rqlp_sketch_encoded(const uint16_t* Ahi, const uint16_t* Alo, const int32_t* colexp,
                        const int32_t* gexp, int64_t m, int64_t n, const float* X, int64_t ldx,
                        int64_t c, float* Y, int64_t ldy, int precision, void* work,
                        size_t work_bytes, void* stream);

/* Orthonormalisation of the range finder (Algorithm 2.1): V (m x c) gets an orthonormal basis
 * of range(Y) by CholeskyQR2 (shifted retry on breakdown); Y is m x c,
 * double.  R (c x c upper, ldr >= c, may be NULL) receives the triangular
 * factor with Y = V R, diag(R) > 0.  V may alias Y. */
int rqlp_orthonormalize(const double* Y, int64_t ldy, int64_t m, int64_t c, double* V,
                        int64_t ldv, double* R, int64_t ldr, int32_t* info, void* work,
                        size_t work_bytes, void* stream);
int rqlp_orthonormalize_workspace(int64_t m, int64_t c, size_t* bytes);

/* Column-pivoted Householder QR of the rows x cols double matrix M
 * (the first CPQR of Algorithm 2.1; the CPQR of Section 1): M Pi = Qm R with the
 * Businger-Golub pivot rule (largest residual column norm, residual norms
 * recomputed each step), diag(R) >= 0.  Outputs (any may be NULL):
 *   piv   min(rows, cols) int64 pivots (original column indices);
 *   R     rows x min(rows, cols) (ldr >= rows): the pivoted columns of R
 *         (upper triangular block R11);
 *   Rt    cols x rows (ldrt >= cols): row c holds column c of R in the
 *         ORIGINAL column order (R Pi^T transposed);
 *   Qm    rows x min(rows, cols) (ldq >= rows), explicit orthonormal factor.
 * Pivots whose residual norms are within a relative 2^-36 may be taken in
 * either order; the numerical-rank stop (residual <= max(rows, cols) eps
 * ||M||_F) zeroes the trailing rows of R and sets RQLP_INFO_RANK_DEFICIENT. */
int rqlp_cpqr(const double* M, int64_t ldm, int64_t rows, int64_t cols, int64_t* piv,
              double* R, int64_t ldr, double* Rt, int64_t ldrt, double* Qm, int64_t ldq,
              int32_t* info, void* work, size_t work_bytes, void* stream);
int rqlp_cpqr_workspace(int64_t rows, int64_t cols, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* RQLP_H */
