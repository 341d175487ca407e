// Internal launchers of the gfx950 Flip-Flop SRQR library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ffsrqr {

struct DeviceInfo {
  int id = -1;
  int num_cu = 0;
  size_t lds_max = 0;
  bool coop = false;
  bool gfx950 = false;
};
// Cached properties of the current device.
const DeviceInfo& device_info(hipError_t* err);

// Workspace carving: bump allocator over the caller's buffer (256-byte aligned).
struct Arena {
  char* base;
  size_t cap;
  size_t used;
  template <typename U>
  U* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(U);
    return (base && used <= cap) ? reinterpret_cast<U*>(base + off) : nullptr;
  }
};

hipError_t zero_words(unsigned* p, int n, hipStream_t s);
// Fills n 64-bit words with the empty-slot pattern kVoid.
hipError_t fill_void(uint64_t* p, size_t n, hipStream_t s);

// Omega^T (m x l, ldo): Ot[t + i*ldo] = Omega[i, t] (Philox4x64-10 + Box-Muller).
template <typename T>
hipError_t launch_omega(uint64_t seed, int64_t l, int64_t m, T* Ot, int64_t ldo, hipStream_t s);
// The q-th random probe (q >= 1) of the SRQR test, d x c, FP64:
// P[t * c + i] from counter (i, t, q, 0), key (seed, 0).
hipError_t launch_probe(uint64_t seed, uint64_t q, int64_t d, int64_t c, double* P, hipStream_t s);
// Largest probe height d of the randomized g2 estimate.
constexpr int32_t kMaxProbe = 64;

// C (M x N, ldc) = X^T Y with X K x M (ldx), Y K x N (ldy).  If colnorm is
// non-null it receives ||Y(:, j)||^2 (FP64).  Scratch comes from the arena.
template <typename T>
size_t gemm_tn_scratch(int64_t M, int64_t N, int64_t K, int num_cu);
// y_ncontig: Y is stored with its columns contiguous instead (element
// (k, j) at Y[k ldy + j]), i.e. C = X^T Z^T for a column-major Z (N x K,
// ldy); M <= 1152 in that case.
template <typename T>
hipError_t gemm_tn(int64_t M, int64_t N, int64_t K, const T* X, int64_t ldx, const T* Y,
                   int64_t ldy, T* C, int64_t ldc, double* colnorm, Arena& ar, int num_cu,
                   hipStream_t s, bool y_ncontig = false);

// Mixed form (BF16 MFMA, FP32 accumulation), C (M x N, FP32) = X^T Y with
// X M x K stored K-major (ldx, a multiple of 8) as BF16 parts and Y FP32
// K x N (ldy, a multiple of 4).  nprod 1: C = Xhi^T bf16(Y) (the sketch;
// colnorm, if non-null, gets ||Y(:, j)||^2 in FP64 from the FP32 entries).
// nprod 3: the split-BF16 product Xhi^T Yhi + Xhi^T Ylo + Xlo^T Yhi.
size_t gemm_bf16_scratch(int64_t M, int64_t N, int64_t K, int num_cu);
hipError_t gemm_bf16(int nprod, int64_t M, int64_t N, int64_t K, const __bf16* Xhi, const __bf16* Xlo, int64_t ldx,
                     const float* Y, int64_t ldy, float* C, int64_t ldc, double* colnorm, Arena& ar, int num_cu,
                     hipStream_t s);
// hi = bf16(X), lo = bf16(X - hi) for a rows x cols FP32 block (ld), into
// K-major arrays with leading dimension ldo.
hipError_t split_bf16(const float* X, int64_t rows, int64_t cols, int64_t ld, __bf16* hi, __bf16* lo, int64_t ldo,
                      hipStream_t s);

// Partial QRCP on B (l x n): piv[0:l], margins[0:l].
template <typename T>
size_t qrcp_scratch(int64_t l, int64_t n, const DeviceInfo& d);
template <typename T>
hipError_t qrcp(const T* B, int64_t l, int64_t n, int64_t ldb, int64_t* piv, double* margins,
                Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s);

// P (mrows x c) <- A(:, cols[0:c]).
// Indices outside [0, n) yield NaN columns instead of a read.
template <typename T>
hipError_t gather_cols(const T* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols, int64_t c, T* P,
                       int64_t ldp, hipStream_t s);

// Householder QR of P (mrows x c, in place): explicit Q (mrows x c, ldq) and
// R (c x c, or its transpose when transpose_r), with diag(R) >= 0.
// Whether tall_qr supports mrows x c on device d (c <= 1024, the row blocks
// fit the LDS and the co-resident grid).
bool tallqr_fits(int64_t mrows, int64_t c, const DeviceInfo& d);
template <typename T>
size_t tallqr_scratch(int64_t mrows, int64_t c, const DeviceInfo& d);
template <typename T>
hipError_t tall_qr(T* P, int64_t mrows, int64_t c, int64_t ldp, T* Qout, int64_t ldq, T* R, int64_t ldr,
                   bool transpose_r, Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s,
                   hipEvent_t r_ready = nullptr);  // recorded on s once R is written (before Q is formed)
// V(rowmap[i], :) = Q(i, :) for i < mrows (entries outside [0, mrows) skipped).
template <typename T>
hipError_t scatter_rows(const T* Q, int64_t mrows, int64_t c, int64_t ldq, const int64_t* rowmap, T* V,
                        int64_t ldv, hipStream_t s);

// Rt (n x l): row i = R11(:, i)^T for i < l, W(:, perm[i])^T for i >= l.
template <typename T>
hipError_t assemble_rt(const T* R11, int64_t ldr11, const T* W, int64_t ldw, const int64_t* perm,
                       int64_t l, int64_t n, T* Rt, int64_t ldrt, hipStream_t s);
// R (l x n, ldr) in perm order from R11 and W.
template <typename T>
hipError_t assemble_r(const T* R11, int64_t ldr11, const T* W, int64_t ldw, const int64_t* perm,
                      int64_t l, int64_t n, T* R, int64_t ldr, hipStream_t s);

// perm[n] = [S (l entries), the rest ascending]; inS[n] = 1 for members of S.
// cnt: scratch of ceil(n / 1024) int64.
hipError_t build_perm(const int64_t* S, int64_t l, int64_t n, int64_t* perm, unsigned char* inS, int64_t* cnt,
                      hipStream_t s);

// SRQR small stage.  State shared between kernels and read back by the host.
struct SrqrState {
  double gamma2_max;   // largest approximate residual^2 over the trailing set
  int64_t jstar;       // its original index (-1 if none)
  double anorm_max;    // max_j ||a_j||
  double alpha;        // exact residual norm of column jstar
  double min_diag;     // min |R11_ii|
  double g2;           // max(1, max rho)
  int64_t istar;       // argmax rho (leading position)
  unsigned nonfinite;  // A held a NaN/Inf
  unsigned pad;
  double jmargin;      // (gamma_j*^2 - next largest) / gamma_j*^2 after the recomputation
  int64_t ncand;       // trailing columns whose residual was recomputed exactly
  double ub_noncand;   // largest upper bound of gamma^2 over the other trailing columns
};
template <typename T>
hipError_t residual_norms(const T* W, int64_t l, int64_t n, int64_t ldw, const double* anorm2,
                          double* gamma2, hipStream_t s);
template <typename T>
size_t srqr_scratch(int64_t m, int64_t n, int64_t l);
template <typename T>
hipError_t srqr_select(const double* gamma2, const double* anorm2, const unsigned char* inS, int64_t n,
                       const T* A, int64_t m, int64_t lda, const T* Q, int64_t ldq, const T* W,
                       int64_t ldw, const T* R11, int64_t ldr, int64_t l, SrqrState* st,
                       Arena& ar, hipStream_t s, double win = 0.0);
// rho of R-tilde = [[R11, a], [0, alpha]].  With sel non-null, a is column
// sel->jstar of the matrix at `a` (column stride a_stride) and alpha is
// sel->alpha; otherwise a and alpha_host are used as given.  g2 and istar go
// to st_out when non-null.
template <typename T>
hipError_t srqr_rho(const T* R11, int64_t ldr, const T* a, int64_t a_stride, const SrqrState* sel,
                    double alpha_host, int64_t l, double* rho, SrqrState* st_out, Arena& ar, hipStream_t s);
// Algorithm 4's randomized g2 estimate with the q-th d-row probe:
// est[0:l+1], est_i = |alpha| / sqrt(d) * ||column i of P R-tilde^{-T}||;
// st_out->g2 = max_i est_i, st_out->istar = its argmax in 0..l (l: the
// (l+1)-st position, whose round-robin rotation is the identity).
template <typename T>
hipError_t srqr_probe(const T* R11, int64_t ldr, const T* a, int64_t a_stride, const SrqrState* sel,
                      double alpha_host, int64_t l, int32_t d, uint64_t seed, uint64_t q, double* est,
                      SrqrState* st_out, Arena& ar, hipStream_t s);

// Algorithm 2's blocked pivot selection: l pivots S (and their QRCP
// margins) in blocks of b <= 64 from the sample B (rows x n, ldb = rows,
// rows = trqrcp_rows(m, b, p) = min(b + p, m), formed by the caller and
// updated in place); needs n - l + 1 >= rows.  Synchronises the stream.
int64_t trqrcp_rows(int64_t m, int64_t b, int64_t p);
size_t trqrcp_lds(int64_t b, int64_t rows);
template <typename T>
size_t trqrcp_scratch(int64_t m, int64_t n, int64_t l, int64_t b, int64_t p, const DeviceInfo& d);
template <typename T>
hipError_t trqrcp_select(const T* A, int64_t m, int64_t n, int64_t lda, int64_t l, int64_t b, int64_t p, T* B,
                         int64_t* S, double* margins, Arena& ar, unsigned* err, const DeviceInfo& d,
                         hipStream_t s, bool final_update = false);
// Algorithm 4's residual norm estimates from the updated sample:
// r[c] = ||B(:, c)||^2 / rows (B rows x n, ldb = rows).
template <typename T>
hipError_t sample_norms(const T* B, int64_t rows, int64_t n, double* r, hipStream_t s);
// The estimates for the one-block selection: r[c] = ||B(:, c) - G W(:, c)||^2
// / l with G = B(:, S) R11^{-1}, i.e. the sample update of Algorithm 2 with
// all l pivots as one block (B l x n, ldb = l; W = Q1^T A, l x n).
// one_block_stage copies B (Bc) and gathers B(:, S) (Bs) from the arena, so
// that the rest can run while B's buffer is reused; one_block_estimates then
// forms r from them.
template <typename T>
size_t one_block_estimates_scratch(int64_t l, int64_t n, const DeviceInfo& d);
template <typename T>
hipError_t one_block_stage(const T* B, int64_t l, int64_t n, const int64_t* S, T** Bc, T** Bs, Arena& ar,
                           hipStream_t s);
template <typename T>
hipError_t one_block_estimates(const T* Bc, const T* Bs, int64_t l, int64_t n, const T* R11, int64_t ldr, const T* W,
                               int64_t ldw, double* r, Arena& ar, const DeviceInfo& d, hipStream_t s);
// est[st->jstar] = st->alpha^2 (the estimate of j* after an identity rotation)
hipError_t est_reset_jstar(double* est, const SrqrState* st, hipStream_t s);

// One swap of Algorithm 4 as an update in place of A(:, S) = Q R11 and
// W = Q^T A: leading position istar leaves, trailing column jstar becomes
// the last leading column (rotations on R11, W and Q, one new column of Q by
// two Gram-Schmidt passes, one new row of W by a pass over A).
template <typename T>
size_t swap_scratch(int64_t m, int64_t l);
template <typename T>
// With est non-null the residual norm estimates follow the swap:
// est[c] += W_rot(l-1, c)^2 - W_new(l-1, c)^2, the exact change of c's
// squared residual norm (W_rot: W after the rotations, whose last row belongs
// to the removed column's direction; W_new: with the new last row), and
// est[icol] (the removed column, original index) starts from 0, so that it
// ends exact.
hipError_t srqr_swap_update(const T* A, int64_t m, int64_t n, int64_t lda, T* Q, int64_t ldq, T* W, int64_t ldw,
                            T* R11, int64_t ldr, int64_t l, int64_t istar, int64_t jstar, Arena& ar, hipStream_t s,
                            double* est = nullptr, int64_t icol = -1);

// Tensors (the ST-HOSVD driver), order at most kMaxTensorOrder.  The mode-a
// unfolding holds entry (i_0..i_{d-1}) at i_a + n_a c_a, c_a the
// Fortran-order linear index of the other indices in order (the mode-0
// unfolding is the tensor in Fortran order).  reunfold copies a tensor from
// its mode-a unfolding to its mode-b unfolding (a == b: a plain copy).
constexpr int kMaxTensorOrder = 8;
template <typename T>
hipError_t reunfold(const T* src, int a, T* dst, int b, int d, const int64_t* dims, hipStream_t s);

// Elementwise steps of robust PCA by IALM (D, E, Y with leading dimension
// m; M, X with their own).  Reductions write kIalmBlocks partials (part) and
// their total to out[0] (sum of squares) and out[1] (largest magnitude).
constexpr int kIalmBlocks = 1024;
template <typename T>  // D = M - E + Y / mu
hipError_t ialm_shift(const T* M, int64_t ldm, const T* E, const T* Y, int64_t m, int64_t n, double inv_mu, T* D,
                      hipStream_t s);
template <typename T>  // Y = M / J, E = 0
hipError_t ialm_init(const T* M, int64_t ldm, int64_t m, int64_t n, double inv_j, T* Y, T* E, hipStream_t s);
template <typename T>  // E = S_w(M - X + Y / mu); Z = M - X - E; Y += mu Z; out[0] = ||Z||_F^2
hipError_t ialm_update(const T* M, int64_t ldm, const T* X, int64_t ldx, int64_t m, int64_t n, double mu, double w,
                       T* E, T* Y, double* part, double* out, hipStream_t s);
template <typename T>  // out[0] = ||M||_F^2, out[1] = max |M_ij|; part: 2 kIalmBlocks doubles
hipError_t matrix_norms(const T* M, int64_t ldm, int64_t m, int64_t n, double* part, double* out, hipStream_t s);
template <typename T>  // B (k x rows, ldb): B(j, i) = A(i, j) (sigma[j] - inv_mu)
hipError_t scaled_transpose(const T* A, int64_t rows, int64_t k, int64_t lda, const double* sigma, double inv_mu,
                            T* B, int64_t ldb, hipStream_t s);
template <typename T>
hipError_t zero_matrix(T* X, int64_t ldx, int64_t m, int64_t n, hipStream_t s);

// Singular values of L (l x l) by block one-sided Jacobi (FP64).
template <typename T>
size_t jacobi_scratch(int64_t l, const DeviceInfo& d);
template <typename T>
hipError_t jacobi_sigma(const T* L, int64_t l, int64_t ldl, double* sigma, Arena& ar, unsigned* err,
                        const DeviceInfo& d, hipStream_t s, int* sweeps = nullptr);
// Singular values and vectors of L (l x l): L V = U diag(sigma), sigma
// descending (ties by index), U and V l x l (ldu, ldv >= l) in T; the same
// Jacobi iteration with the rotations accumulated in stacked rows.
template <typename T>
hipError_t jacobi_svd_vectors(const T* L, int64_t l, int64_t ldl, double* sigma, T* U, int64_t ldu, T* V,
                              int64_t ldv, Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s,
                              int* sweeps = nullptr);

// B (cols x rows, ldb) = A^T for A rows x cols (lda).
template <typename T>
hipError_t transpose(const T* A, int64_t rows, int64_t cols, int64_t lda, T* B, int64_t ldb, hipStream_t s);
// For j < k: flip U(:, j) (m rows) and V(:, j) (n rows) together when the
// entry of U(:, j) of largest magnitude (the first on ties) is negative; sg
// is k doubles of scratch.
template <typename T>
hipError_t normalize_pair_signs(T* U, int64_t m, int64_t ldu, T* V, int64_t n, int64_t ldv, int64_t k, double* sg,
                                hipStream_t s);

}  // namespace ffsrqr
