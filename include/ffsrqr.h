/*
 * ffsrqr.h - C ABI of the MI355X (gfx950) Flip-Flop SRQR hot path.
 *
 * Method: Feng, Xiao & Gu, "Low-Rank Matrix Approximations with Flip-Flop
 * Spectrum-Revealing QR Factorization".  Given A (m x n), a target rank k and
 * an oversampling size p, the library computes, with l = min(k+p, m, n):
 *
 *   Omega  l x m i.i.d. N(0,1)                    (Algorithm 2, first step)
 *   B      = Omega A                              (Algorithm 2, sample matrix)
 *   S      l pivots of partial QRCP on B          (Algorithm 1 applied to B)
 *   Q1,R11 Householder QR of A(:, S)              (Algorithm 2, QR of the block;
 *                                                  compact WY, Section 2.1)
 *   R      = Q1^T A Pi = [R11 R12]                (partial QRCP block form,
 *                                                  Sections 2.1 and 3.1)
 *   g2     SRQR test and round-robin swaps        (Section 2.2, definitions of
 *                                                  R-tilde, g1, g2; Algorithm 4)
 *   L, V   QR without pivoting of R^T: R^T = Qhat1 Rhat11, L = Rhat11^T,
 *          V = Pi Qhat1                           (Section 3.1, flip-flop step)
 *   sigma  singular values of L                   (Section 3.1; Algorithm 9)
 *
 * so that A ~ Q1 L V^T, and the diagonal of L tracks the singular values.
 *
 * Conventions for every entry point:
 *  - Matrices are column-major with an explicit leading dimension.
 *  - Pointers named A, B, Q, R, L, V, W, omega, perm, cols, piv, margins,
 *    anorm2, gamma2, sigma and work are DEVICE pointers (hipMalloc'd memory
 *    of the current device); info and bytes are HOST pointers.
 *  - The caller owns every buffer.  A is read-only.  No entry point allocates
 *    device memory (scratch lives in the caller's workspace), except
 *    ffsrqr_server_create, which allocates the server's pool once.
 *  - precision: FFSRQR_FP64 means double storage and arithmetic everywhere;
 *    FFSRQR_FP32 means float storage of A and of the float outputs and
 *    intermediates (Q, L, V, B, R, W, the panel between its 16-column
 *    blocks), FP32 MFMA GEMMs (sketch and projection), and FP64 arithmetic
 *    everywhere else: QRCP on B, the Householder panel steps and their
 *    trailing updates, column and residual norms, the SRQR test and the
 *    singular values.  FFSRQR_MIXED has the storage of FFSRQR_FP32 and
 *    replaces its two GEMMs: the sketch multiplies BF16 operands
 *    (Omega rounded to bfloat16 from its FP64 value, A rounded from FP32,
 *    both to nearest even) on MFMA with FP32 accumulation, with the column
 *    norms summed in FP64 from the FP32 entries; the projection is the
 *    split-BF16 product Q^T A ~ Qhi^T Ahi + Qhi^T Alo + Qlo^T Ahi
 *    (x = hi + lo, hi = bf16(x), lo = bf16(x - hi)) with FP32 accumulation.
 *    Everything after the GEMMs is as in FFSRQR_FP32.
 *  - stream is a hipStream_t (NULL = the default stream).  Stage entry points
 *    only enqueue work; ffsrqr_factor synchronises the stream once per SRQR
 *    test (the swap decision is read back on the host) and on return.
 *  - Errors: argument checks return FFSRQR_EINVAL, a too-small workspace
 *    FFSRQR_EWORKSPACE, a HIP failure FFSRQR_EHIP, no usable gfx950 device
 *    FFSRQR_ENODEV; nothing is enqueued when a check fails.
 *    ffsrqr_last_error() returns a thread-local message for the last failure.
 *    Conditions found on the device are reported through ffsrqr_info.flags.
 *  - Calls on one workspace must not overlap; distinct workspaces may be used
 *    concurrently on distinct streams.
 */
#ifndef FFSRQR_H
#define FFSRQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ffsrqr_stream_t; /* the same type as hipStream_t */

typedef enum {
  FFSRQR_OK = 0,
  FFSRQR_EINVAL = 1,
  FFSRQR_EWORKSPACE = 2,
  FFSRQR_EHIP = 3,
  FFSRQR_ENODEV = 4,
  FFSRQR_EBUSY = 5 /* a server request ended unrun: the server was destroyed first */
} ffsrqr_status;

typedef enum { FFSRQR_FP64 = 0, FFSRQR_FP32 = 1, FFSRQR_MIXED = 2 } ffsrqr_precision;

/* ffsrqr_info.flags bits */
enum {
  FFSRQR_FLAG_RANK_DEFICIENT = 1u, /* alpha or a diagonal of R11 <= tau_r (below)                */
  FFSRQR_FLAG_SWAPCAP = 2u,        /* the swap loop stopped at max_swaps with g2 > g            */
  FFSRQR_FLAG_NONFINITE = 4u,      /* A holds a NaN or Inf; outputs are NaN                     */
  FFSRQR_FLAG_L_CLAMPED = 8u,      /* k + p > min(m, n); l was clamped to min(m, n)             */
  FFSRQR_FLAG_TIMEOUT = 16u        /* a device-wide wait exceeded its spin limit (never expected) */
};

typedef struct {
  int32_t precision; /* ffsrqr_precision                                          */
  int32_t max_swaps; /* cap of the SRQR swap loop; < 0 selects the default 4*l     */
  double g;          /* SRQR tolerance for g2 (Section 2.2: g > 1, e.g. 2.0);
                        0 selects 2.0                                             */
  int32_t block;     /* 0: the l pivots from one partial QRCP on an l-row sketch;
                        1..64: Algorithm 2's blocked selection (TRQRCP): blocks
                        of min(block, k) pivots, each from partial QRCP on a
                        min(block + p, m)-row sample of the columns in play,
                        the sample updated after each block (needs
                        n - l + 1 >= min(block + p, m))                          */
  int32_t g2_probe;  /* 0: the SRQR test's g2 is exact (|alpha| times the largest
                        row norm of R-tilde^{-1}); d in 1..64: Algorithm 4's
                        randomized estimate, |alpha| / sqrt(d) times the largest
                        column norm of P_q R-tilde^{-T}, with a fresh d x (l+1)
                        Gaussian probe P_q for the q-th test of the call
                        (ffsrqr_srqr_probe).  When the argmax is the (l+1)-st
                        position the rotation is the identity and the next test
                        draws P_{q+1}; max_swaps counts these too.               */
  int32_t est_norms; /* 0: j* is chosen by exact residual norms; 1: by
                        Algorithm 4's estimates r_i = ||B(:, i)||^2 / rows
                        from the sample after the last block's update (block
                        0: the l-row sketch updated with all l pivots as one
                        block, B(:, rest) -= B(:, S) R11^{-1} R12, which needs
                        an l x n product more workspace), kept through the
                        swaps by the exact changes of the
                        squared residual norms (the rows of R that leave and
                        enter); alpha stays the exact residual norm of j*, and
                        after an identity rotation r_{j*} = alpha^2.  Not for
                        the tensor and robust PCA drivers.                        */
  int32_t reserved;  /* 0                                                         */
} ffsrqr_opts;

typedef struct {
  int64_t l;              /* number of QR steps, min(k+p, m, n)                    */
  int32_t swaps;          /* SRQR swaps performed                                  */
  uint32_t flags;         /* FFSRQR_FLAG_* bits                                    */
  double g2;              /* g2 of the final leading set (1 when rank deficient)   */
  double alpha;           /* largest residual column norm of the trailing columns  */
  int64_t jstar;          /* original index of that column (-1 when l == n)        */
  int64_t numerical_rank; /* l unless RANK_DEFICIENT                               */
  double min_margin;      /* min over QRCP-on-B steps of (r_max - r_2nd) / r_max   */
  int32_t jacobi_sweeps;  /* sweeps of the one-sided Jacobi on L                   */
  int32_t probes;         /* SRQR tests that drew a random probe (0 when g2 is exact) */
  double jstar_margin;    /* (gamma_j*^2 - g_2nd) / gamma_j*^2: how clearly j* won;
                             g_2nd bounds every other trailing gamma_j^2 (1 when
                             l == n or one column trails)                         */
  int64_t jstar_candidates; /* trailing columns whose residual norm was recomputed
                               exactly to choose j*                                */
} ffsrqr_info;

/* Rank tolerance tau_r of the SRQR test: max(m, n) 2^-52 max_j ||a_j|| for
 * FFSRQR_FP64; 8 sqrt(max(m, n)) 2^-24 max_j ||a_j|| for FFSRQR_FP32 (Q1, the
 * panel between blocks and W are rounded to float, so exactly dependent
 * columns leave residuals of order sqrt(l) 2^-24 ||a_j||).  When alpha or a
 * diagonal entry of R11 is <= tau_r, RANK_DEFICIENT is set, numerical_rank is
 * the number of |R11_ii| > tau_r, g2 = 1 and no swap is made. */

/* Default options: FP64, g = 2, max_swaps = 4 l. */
void ffsrqr_default_opts(ffsrqr_opts* opts);

/* Destroy the second stream and the events that this host thread's calls
 * created (they are created again by the next call).  For an orderly
 * shutdown: call it before the HIP runtime is unloaded, e.g. at exit. */
void ffsrqr_release(void);

/* Text of a status code (static storage). */
const char* ffsrqr_status_string(ffsrqr_status s);

/* Thread-local description of the last failure in this thread ("" if none). */
const char* ffsrqr_last_error(void);

/*
 * Workspace size in bytes (written to *bytes, a host pointer) that is enough
 * for ffsrqr_factor and for every stage entry point on a problem of the
 * given dimensions.  Pure host computation; needs no device.
 * Errors: FFSRQR_EINVAL for m, n < 1, k < 1, k > min(m, n), p < 0, a NULL
 * bytes pointer, an unknown precision, or sizes beyond the supported range:
 * l = min(k + p, m, n) <= 1024, and the Householder QR of the m x l and
 * n x l panels must fit a 256-CU gfx950 with 160 KiB of LDS per workgroup
 * (one row block per workgroup, at most 1024 rows, stored in LDS beside the
 * panel's exchange tile): m and n at most about 256 min(1024, 1259 - l) rows,
 * e.g. 252672 at l = 272, 183040 at l = 544, 30080 at l = 1024.
 * ffsrqr_factor re-checks against the device in use.
 */
ffsrqr_status ffsrqr_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p,
                                    const ffsrqr_opts* opts, size_t* bytes);

/*
 * The whole hot path (Algorithm 9 up to the LQ, with Algorithm 4 inside).
 *   A      m x n, lda >= m, element type per opts->precision.
 *   k, p   target rank 1 <= k <= min(m, n) and oversampling p >= 0;
 *          l = min(k + p, m, n) columns are factored.
 *   seed   key of the Omega stream: Omega[i, t] = sqrt(-2 ln u1) cos(2 pi u2)
 *          with (x0, x1, x2, x3) = Philox4x64-10(counter (t, i, 0, 0),
 *          key (seed, 0)) and u = ((x >> 12) + 0.5) 2^-52 for x0 and x1.
 *   perm   [n] int64: perm[0:l] the leading columns in order, then the other
 *          columns in ascending order (Pi).
 *   Q      m x l (ldq >= m): orthonormal columns, diag(R11) > 0.
 *   L      l x l (ldl >= l): lower triangular, diag(L) >= 0.
 *   V      n x l (ldv >= n): V = Pi Qhat1, orthonormal columns; A ~ Q L V^T.
 *   sigma  [l] double: singular values of L, descending.
 *   info   host pointer, filled on success (may be NULL); also filled
 *          (flags with FFSRQR_FLAG_TIMEOUT) when a device-wide wait ran out
 *          and FFSRQR_EHIP is returned: the outputs are then incomplete.
 * Errors as ffsrqr_workspace_size, plus lda < m, ldq < m, ldl < l, ldv < n,
 * g <= 1 or a NULL output (FFSRQR_EINVAL), all checked before anything is
 * enqueued.
 *   work   device workspace of work_bytes >= ffsrqr_workspace_size(...).
 * A swap of Algorithm 4 (leading position i* out, trailing column j* in as
 * the last leading column) updates the factorization in place: plane
 * rotations restore the triangle of R11 after its column i* is removed and
 * act on the columns of Q1 and the rows of W = Q1^T A; the new column of Q1
 * comes from two Gram-Schmidt passes against the others, and the new row of
 * W from one pass over A.  The LQ and the singular values are computed for
 * the first leading set (concurrently with the first SRQR test) and, when
 * swaps follow, once more for the final one.
 * The call returns after the stream has completed the solve.
 */
ffsrqr_status ffsrqr_factor(const void* A, int64_t m, int64_t n, int64_t lda,
                            int64_t k, int64_t p, uint64_t seed,
                            int64_t* perm, void* Q, int64_t ldq, void* L, int64_t ldl,
                            void* V, int64_t ldv, double* sigma, ffsrqr_info* info,
                            void* work, size_t work_bytes, const ffsrqr_opts* opts,
                            ffsrqr_stream_t stream);

/* ---------------------------------------------------------------------------
 * Stage entry points: one per step of the path, on the same conventions.
 * Each enqueues its kernels on the stream and returns; the outputs are valid
 * after the stream synchronises.  They let a caller (or a test) run and check
 * one step at a time.  Their workspace must be at least
 * ffsrqr_workspace_size(m, n, k, p, opts) for the dimensions involved.
 * ------------------------------------------------------------------------- */

/*
 * Omega^T (Algorithm 2, first step): omega_t is m x l, ldo >= m, with
 * omega_t[t + i*ldo] = Omega[i, t] from the stream documented above.
 */
ffsrqr_status ffsrqr_omega(uint64_t seed, int64_t l, int64_t m, void* omega_t, int64_t ldo,
                           int32_t precision, ffsrqr_stream_t stream);

/*
 * Sketch (Algorithm 2, "form the initial sample matrix"): B = Omega A with
 * Omega l x m from seed, B l x n (ldb >= l), and the column norms
 * anorm2[j] = ||A(:, j)||^2 (FP64 accumulation, n doubles) in the same pass.
 * FFSRQR_MIXED: A and B float, B = bf16(Omega) bf16(A) with FP32 sums.
 */
ffsrqr_status ffsrqr_sketch(const void* A, int64_t m, int64_t n, int64_t lda, uint64_t seed,
                            int64_t l, void* B, int64_t ldb, double* anorm2,
                            void* work, size_t work_bytes, int32_t precision,
                            ffsrqr_stream_t stream);

/*
 * Partial QRCP on the sketch (Algorithm 1 on B, l steps; l <= rows of B):
 * at each step the trailing column with the largest residual norm (ties to
 * the smallest original index) is chosen and a Householder reflector is
 * applied to the remaining columns.  B (l x n, ldb) is read-only.
 *   piv      [l] int64: the chosen original column indices, in order.
 *   margins  [l] double: (r_max - r_second) / r_max at each step (1 when one
 *            column is left).
 */
ffsrqr_status ffsrqr_qrcp(const void* B, int64_t l, int64_t n, int64_t ldb, int64_t* piv,
                          double* margins, void* work, size_t work_bytes, int32_t precision,
                          ffsrqr_stream_t stream);

/*
 * Householder QR without pivoting of the gathered columns A(:, cols[0:c])
 * (Algorithm 2, QR of the pivoted block, compact WY of Section 2.1), c <= m:
 *   Q  m x c (ldq >= m), explicit, orthonormal columns;
 *   R  c x c (ldr >= c), upper triangular with diag(R) >= 0; A(:, cols) = Q R.
 */
ffsrqr_status ffsrqr_panel_qr(const void* A, int64_t m, int64_t n, int64_t lda,
                              const int64_t* cols, int64_t c, void* Q, int64_t ldq,
                              void* R, int64_t ldr, void* work, size_t work_bytes,
                              int32_t precision, ffsrqr_stream_t stream);

/*
 * Projection (partial QR block form, Sections 2.1 and 3.1): W = Q^T A
 * (c x n, ldw >= c) for every column of A in the original order, and the
 * residual norms gamma2[j] = anorm2[j] - ||W(:, j)||^2 (FP64).
 * Q is m x c (ldq >= m).  anorm2 as returned by ffsrqr_sketch.
 * FFSRQR_MIXED: Q, A and W float, W by the split-BF16 product.
 */
ffsrqr_status ffsrqr_project(const void* Q, int64_t m, int64_t c, int64_t ldq,
                             const void* A, int64_t n, int64_t lda, void* W, int64_t ldw,
                             const double* anorm2, double* gamma2, void* work,
                             size_t work_bytes, int32_t precision, ffsrqr_stream_t stream);

/*
 * SRQR test (Section 2.2, definitions of R-tilde and g2; Algorithm 4):
 *   R11    l x l upper triangular (ldr >= l), FP64 or FP32 per precision;
 *   a      [l] the column R(:, j*) (same element type);
 *   alpha  the residual norm of column j* (> 0).
 * Writes rho[0:l] (FP64): rho_i = |alpha| ||row i of R-tilde^{-1}||, so that
 * g2 = max(1, max_i rho_i) and the swap candidate is argmax_i rho_i.
 */
ffsrqr_status ffsrqr_srqr_rho(const void* R11, int64_t l, int64_t ldr, const void* a,
                              double alpha, double* rho, void* work, size_t work_bytes,
                              int32_t precision, ffsrqr_stream_t stream);

/*
 * Randomized g2 estimate of the SRQR test (Algorithm 4, the g2 step;
 * Section 2.2, definition of g2).  R11, a, alpha as for ffsrqr_srqr_rho;
 * d in 1..64 rows of the probe, q >= 1 its stream.  The probe P (d x (l+1))
 * has entry (t, i) = sqrt(-2 ln u1) cos(2 pi u2), u_j = ((x_j >> 12) + 0.5)
 * 2^-52 from words x0, x1 of Philox4x64-10 with counter (i, t, q, 0) and
 * key (seed, 0) (stream 0 is Omega's, ffsrqr_omega).  Writes est[0:l+1]
 * (FP64, device): est_i = |alpha| / sqrt(d) * ||column i of P R-tilde^{-T}||,
 * an estimate of rho_i whose square is unbiased; est_l = ||P(:, l)|| /
 * sqrt(d).  work: device scratch of at least 8 ((d + 1) l + d (l + 1)) + 512
 * bytes (the probe and the d + 1 triangular solves).  FFSRQR_EINVAL for
 * d outside 1..64, q = 0 or alpha <= 0.
 */
ffsrqr_status ffsrqr_srqr_probe(const void* R11, int64_t l, int64_t ldr, const void* a,
                                double alpha, int32_t d, uint64_t seed, uint64_t q,
                                double* est, void* work, size_t work_bytes,
                                int32_t precision, ffsrqr_stream_t stream);

/*
 * Flip-flop LQ (Section 3.1): QR without pivoting of R^T, R = [R11 R12]
 * l x n (ldr >= l) in Pi order: R^T = Qhat1 Rhat11.
 *   L  l x l (ldl >= l) = Rhat11^T, lower triangular, diag(L) >= 0;
 *   V  n x l (ldv >= n) = Pi Qhat1: V(perm[i], :) = Qhat1(i, :).
 */
ffsrqr_status ffsrqr_lq(const void* R, int64_t l, int64_t n, int64_t ldr, const int64_t* perm,
                        void* L, int64_t ldl, void* V, int64_t ldv, void* work,
                        size_t work_bytes, int32_t precision, ffsrqr_stream_t stream);

/*
 * Singular values of L (l x l, ldl >= l, FP64 or FP32 per precision) by
 * one-sided Jacobi in FP64 (Algorithm 9 asks for the SVD of the small
 * factor); sigma[0:l] descending.
 */
ffsrqr_status ffsrqr_svd_small(const void* L, int64_t l, int64_t ldl, double* sigma,
                               void* work, size_t work_bytes, int32_t precision,
                               ffsrqr_stream_t stream);

/*
 * Algorithm 9, last steps: the rank-k approximate SVD from the flip-flop
 * factors (Section 3.1).  With V = Pi Qhat1 (n x l) from ffsrqr_factor:
 *   tmp = A V (m x l, a third pass over A),
 *   tmp = U_tmp Sigma V_tmp^T, its thin SVD (Householder QR of tmp, then
 *         one-sided Jacobi with the rotations accumulated on its l x l
 *         triangular factor),
 *   U = U_tmp(:, 1:k) (m x k, ldu >= m), V_k = V V_tmp(:, 1:k) (n x k,
 *   ldvk >= n), sigma[0:l] = Sigma (descending; sigma[0:k] is Sigma_k),
 * so that A ~ U diag(sigma[0:k]) V_k^T.  Each pair (U(:, j), V_k(:, j)) is
 * signed so that the entry of U(:, j) of largest magnitude (the first on
 * ties) is positive.  A, V, U and V_k have the element type of precision
 * (FFSRQR_MIXED: float, FP32 GEMMs); everything else as ffsrqr_factor.
 * 1 <= k <= l <= min(m, n), the size limits of ffsrqr_workspace_size; the
 * workspace comes from ffsrqr_alg9_workspace_size.  The call returns after
 * the stream has completed.
 */
ffsrqr_status ffsrqr_alg9_workspace_size(int64_t m, int64_t n, int64_t l, int64_t k, int32_t precision,
                                         size_t* bytes);
ffsrqr_status ffsrqr_alg9_svd(const void* A, int64_t m, int64_t n, int64_t lda, const void* V, int64_t ldv,
                              int64_t l, int64_t k, void* U, int64_t ldu, double* sigma, void* Vk,
                              int64_t ldvk, void* work, size_t work_bytes, int32_t precision,
                              ffsrqr_stream_t stream);

/*
 * ST-HOSVD with Flip-Flop SRQR as the rank-k SVD (Section 2, tensor
 * notation and the ST-HOSVD algorithm; Section 4, the tensor experiment).
 *   X      tensor of order d (1 <= d <= 8) with dimensions dims[0:d] (host
 *          array), Fortran order (the first index runs fastest), element
 *          type of opts->precision (FFSRQR_MIXED: float).  Read-only.
 *   ranks  host array, 1 <= ranks[j] <= dims[j]: the Tucker rank.
 *   order  host array, the processing order (a permutation of 0..d-1), or
 *          NULL for 0, 1, .., d-1.
 *   p, seed  oversampling and Omega key of every mode's factorization.
 * For each mode r in the processing order: the mode-r unfolding G_(r) of the
 * current tensor (n_r rows; column c = the Fortran-order linear index of
 * the other indices in order) is factored by ffsrqr_factor's path (target
 * rank ranks[r], oversampling p, the options in opts; opts->block must be 0:
 * the one-block selection) and completed by
 * Algorithm 9 to G_(r) ~ U_r Sigma V^T; U_r is written to U[r]
 * (dims[r] x ranks[r], ldu[r] >= dims[r]; U and ldu are host arrays of
 * device pointers and leading dimensions), and the tensor is reduced to
 * G_(r) <- U_r^T G_(r) (the mode-r product with U_r^T).  core receives the
 * final tensor (ranks[0] x .. x ranks[d-1], Fortran order), so that
 * X ~ core x_1 U_0 x_2 U_1 .. x_d U_{d-1}.
 * Errors: FFSRQR_EINVAL for an order outside 1..8, a rank outside
 * 1..dims[j], an order that is not a permutation, a NULL pointer, or a step
 * whose unfolding breaks the limits of ffsrqr_workspace_size (its message
 * names the mode); the workspace comes from ffsrqr_st_hosvd_workspace_size.
 * The call returns after the stream has completed.
 */
ffsrqr_status ffsrqr_st_hosvd_workspace_size(int32_t d, const int64_t* dims, const int64_t* ranks,
                                             const int32_t* order, int64_t p, const ffsrqr_opts* opts,
                                             size_t* bytes);
ffsrqr_status ffsrqr_st_hosvd(const void* X, int32_t d, const int64_t* dims, const int64_t* ranks,
                              const int32_t* order, int64_t p, uint64_t seed, void* core, void* const* U,
                              const int64_t* ldu, void* work, size_t work_bytes, const ffsrqr_opts* opts,
                              ffsrqr_stream_t stream);

/*
 * Many independent problems in one call (for the batched shapes: tensor
 * unfoldings, the rank-k SVDs of singular value thresholding).  Each
 * ffsrqr_problem carries the arguments of one ffsrqr_factor call (device
 * pointers for A and the outputs, host pointer for info, which may be NULL);
 * opts applies to all (its precision fixes the element type).  The problems
 * run one after another on `stream` through one workspace of
 * ffsrqr_batched_workspace_size bytes (enough for the largest problem);
 * their cooperative stages could not run side by side on one device anyway,
 * since cooperative launches are serialised.  Errors: FFSRQR_EINVAL for
 * count < 1, a NULL probs, or any problem that ffsrqr_factor would reject
 * (checked for all problems before any work is enqueued; the message names
 * the problem); a failure while running stops the batch and is returned.
 * The call returns after the stream has completed every problem.
 */
typedef struct ffsrqr_problem {
  const void* A;
  int64_t m, n, lda, k, p;
  uint64_t seed;
  int64_t* perm;
  void* Q;
  int64_t ldq;
  void* L;
  int64_t ldl;
  void* V;
  int64_t ldv;
  double* sigma;
  ffsrqr_info* info;
} ffsrqr_problem;

ffsrqr_status ffsrqr_batched_workspace_size(int32_t count, const ffsrqr_problem* probs, const ffsrqr_opts* opts,
                                            size_t* bytes);
ffsrqr_status ffsrqr_factor_batched(int32_t count, const ffsrqr_problem* probs, void* work, size_t work_bytes,
                                    const ffsrqr_opts* opts, ffsrqr_stream_t stream);

/*
 * Serving: a request loop over the path (continuous batching).  A server
 * owns one device allocation of cfg->hbm_budget bytes (made by
 * ffsrqr_server_create on the current device) and cfg->slots worker threads
 * (1..16), each with its own stream.  ffsrqr_submit queues a request (an
 * ffsrqr_problem: A and the outputs are device pointers the caller owns and
 * keeps alive until the request is done; its info field is ignored) and
 * returns a ticket; requests are admitted in arrival order as soon as a
 * slot is free and the request's workspace (ffsrqr_workspace_size with the
 * server's precision) fits the free part of the budget, so requests that
 * arrive while others run join them as slots and memory free up.  Each runs
 * ffsrqr_factor with cfg->precision and default options.  ffsrqr_poll sets
 * *done; once done, it returns the request's status and its info (host
 * pointer, may be NULL) and forgets the ticket.  ffsrqr_server_destroy
 * waits for the running requests, ends the queued ones unrun (their status
 * FFSRQR_EBUSY) and frees the pool.
 * Errors: create returns NULL for a NULL cfg, a budget below 1 MiB, slots
 * outside 1..16, an unknown precision or a failed allocation; submit returns
 * what ffsrqr_workspace_size returns for the problem, FFSRQR_EWORKSPACE when
 * its workspace exceeds the budget, FFSRQR_EBUSY once the server is being
 * destroyed; poll returns FFSRQR_EINVAL for an unknown ticket.
 */
typedef struct ffsrqr_server_cfg {
  size_t hbm_budget;  /* bytes of the device pool                               */
  int32_t slots;      /* worker threads (requests running at once), 1..16        */
  int32_t precision;  /* ffsrqr_precision of every request                       */
} ffsrqr_server_cfg;
typedef struct ffsrqr_server ffsrqr_server;

ffsrqr_server* ffsrqr_server_create(const ffsrqr_server_cfg* cfg);
ffsrqr_status ffsrqr_submit(ffsrqr_server* server, const ffsrqr_problem* prob, uint64_t* ticket);
ffsrqr_status ffsrqr_poll(ffsrqr_server* server, uint64_t ticket, ffsrqr_info* out, int32_t* done);
void ffsrqr_server_destroy(ffsrqr_server* server);

/*
 * Robust PCA by the inexact augmented Lagrange multiplier method with
 * Flip-Flop SRQR as its SVD (Section 2, nuclear norm minimization and the
 * robust PCA algorithm; Section 4, the robust PCA experiment): splits
 * M (m x n, ldm) into a low-rank X and a sparse E (min ||X||_* +
 * lambda ||E||_1 with M = X + E).  Iteration: D = M - E + Y / mu; the
 * rank-sv SVD of D by ffsrqr_factor's path (target rank sv, oversampling p,
 * Omega key seed, the options in opts; opts->block must be 0) completed by
 * Algorithm 9;
 * X = U S_{1/mu}(Sigma) V^T over the singular values above 1 / mu;
 * E = S_{lambda/mu}(M - X + Y / mu); Y += mu (M - X - E); mu <- min(1.5 mu,
 * 1e7 mu_0); until ||M - X - E||_F / ||M||_F < tol or max_iter iterations
 * (S_w(x) = sgn(x) max(|x| - w, 0)).  Start: E = 0, Y = M / J(M),
 * J(M) = max(||M||_2, max |M_ij|), mu_0 = 1.25 / ||M||_2, with ||M||_2
 * estimated by sigma_1 of the flip-flop factor L of M (k = 1); sv starts at
 * 10 and follows the number svp of singular values kept: svp + 1 when
 * svp < sv, else svp + round(0.05 n), capped at min(m, n), 1024 - p and
 * max_rank (when > 0).  lambda <= 0 selects 1 / sqrt(max(m, n)).
 *   X (ldx >= m), E (lde >= m): outputs, element type of the precision.
 *   info  host pointer (may be NULL).
 * The FP32 forms cannot reach residuals much below 1e-6: use tol >= 1e-5
 * there.  Errors: FFSRQR_EINVAL for m or n < 1, p outside 0..1023,
 * tol <= 0, max_iter < 1, a leading dimension too small, a NULL pointer or
 * sizes beyond the path's limits at l = min(cap + p, m, n); the workspace
 * comes from ffsrqr_rpca_workspace_size.  The call returns after the
 * stream has completed.
 */
typedef struct ffsrqr_rpca_info {
  int32_t iterations;   /* iterations run                                    */
  int32_t rank;         /* singular values kept in the final X               */
  double residual;      /* ||M - X - E||_F / ||M||_F at exit                  */
  double mu;            /* mu after the last iteration                        */
  double norm2;         /* the estimate of ||M||_2                            */
  int32_t converged;    /* residual < tol                                     */
  int32_t rank_capped;  /* the predicted rank reached its cap                 */
} ffsrqr_rpca_info;

ffsrqr_status ffsrqr_rpca_workspace_size(int64_t m, int64_t n, int64_t p, int64_t max_rank,
                                         const ffsrqr_opts* opts, size_t* bytes);
ffsrqr_status ffsrqr_rpca_ialm(const void* M, int64_t m, int64_t n, int64_t ldm, double lambda, double tol,
                               int32_t max_iter, int64_t p, uint64_t seed, int64_t max_rank, void* X,
                               int64_t ldx, void* E, int64_t lde, ffsrqr_rpca_info* info, void* work,
                               size_t work_bytes, const ffsrqr_opts* opts, ffsrqr_stream_t stream);

/*
 * ffsrqr_svd_small without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid allocation): the same kernels and results as
 * ffsrqr_svd_small, with their scratch in a static device array of the
 * library (about 12.6 MB per GPU, held until the process ends; the call
 * itself allocates nothing).  l <= 1024, else FFSRQR_EINVAL.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Each call clears what must start at zero with kernels on its stream.
 */
ffsrqr_status ffsrqr_svd_small_noalloc(const void* L, int64_t l, int64_t ldl, double* sigma,
                                       int32_t precision, ffsrqr_stream_t stream);

/* ---------------------------------------------------------------------------
 * Device-time accounting of ffsrqr_factor, for benchmarks.  When enabled,
 * ffsrqr_factor records HIP events around each step on the caller's stream
 * and adds the elapsed times (milliseconds) and launch counts to per-step
 * accumulators after its final synchronisation.  Steps:
 * ------------------------------------------------------------------------- */
enum {
  FFSRQR_STEP_OMEGA = 0,     /* Omega generation                              */
  FFSRQR_STEP_SKETCH = 1,    /* sketch GEMM B = Omega A (+ column norms)      */
  FFSRQR_STEP_CHECK = 2,     /* non-finite scan of the column norms           */
  FFSRQR_STEP_QRCP = 3,      /* partial QRCP on the sketch                    */
  FFSRQR_STEP_PANEL = 4,     /* gather + Householder QR of A(:, S)            */
  FFSRQR_STEP_PROJECT = 5,   /* projection GEMM W = Q1^T A                    */
  FFSRQR_STEP_RESID = 6,     /* residual norms gamma^2                        */
  FFSRQR_STEP_SRQR = 7,      /* selection, exact alpha, rho and g2            */
  FFSRQR_STEP_LQ = 8,        /* R^T assembly + Householder QR of R^T          */
  FFSRQR_STEP_SVD = 9,       /* one-sided Jacobi singular values of L         */
  FFSRQR_STEP_SWAP = 10,     /* one SRQR swap: update of Q, R11, W            */
  FFSRQR_NUM_STEPS = 11
};

/* Enable (on != 0) or disable the accounting; either call resets it.
 * Process-wide; meant for single-threaded benchmark drivers. */
void ffsrqr_profile_enable(int on);

/* Copy min(nsteps, FFSRQR_NUM_STEPS) accumulators (host arrays) and return
 * FFSRQR_NUM_STEPS. */
int ffsrqr_profile_read(double* ms, int64_t* launches, int nsteps);

#ifdef __cplusplus
}
#endif

#endif /* FFSRQR_H */
