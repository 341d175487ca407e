// SRQR small stage (Section 2.2, definitions of R-tilde, g1, g2; Algorithm 4)
// and the bookkeeping around the projection.
//
//   residual norms  gamma_j^2 = ||a_j||^2 - ||W(:, j)||^2 in FP64, W = Q1^T A
//                   (the part of a_j outside span(Q1)); one wave per column.
//   select          the difference of squares loses the relative accuracy of
//                   gamma_j^2 when gamma_j << ||a_j|| (an absolute error of
//                   about c u ||a_j||^2, u the unit roundoff of W's arithmetic),
//                   so it only preselects: every trailing column whose
//                   approximate gamma_j^2 lies within the window
//                   (4 sqrt(m) + l) u (||a_j||^2 + ||a_max||^2) of the largest
//                   one is a candidate, and each candidate's residual is
//                   recomputed as ||a_j - Q1 W(:, j)||^2 in FP64 (the error of
//                   W then enters only to second order, since Q1 dW lies in
//                   span(Q1), orthogonal to the residual).  j* is the argmax
//                   of the recomputed values (ties to the smallest index),
//                   alpha = gamma_j*, and the margin of the choice is
//                   (gamma_j*^2 - g_2nd) / gamma_j*^2 with g_2nd the largest of
//                   the other candidates' recomputed values and the upper
//                   bounds gamma_j^2 + window of the non-candidates.
//   rho             X = R11^{-1} and z = R11^{-1} a by column-oriented back
//                   substitution (one workgroup per column, R staged in LDS in
//                   chunks of 16 columns), then
//                   rho_i^2 = alpha^2 ||X(i, :)||^2 + z_i^2, the squared norm of
//                   row i of |alpha| R-tilde^{-1}; g2 = max(1, max_i rho_i).
//   probe           Algorithm 4's randomized estimate: the q-th probe P
//                   (d x (l+1), Philox stream q) split as [P1 p2], then
//                   Y = R11^{-1} P1^T and z = R11^{-1} a by the same back
//                   substitution (d + 1 columns instead of l + 1), and
//                   est_i = ||alpha Y(i, :) - z_i p2^T|| / sqrt(d) (i < l),
//                   est_l = ||p2|| / sqrt(d): row i of R-tilde^{-1} P^T
//                   scaled by |alpha| / sqrt(d), i.e. column i of
//                   P R-tilde^{-T}.  g2 = max_i est_i over all l + 1
//                   positions, i* its argmax (ties to the smaller index).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256;

template <typename T>
__global__ void resid_kernel(const T* __restrict__ W, int64_t l, int64_t n, int64_t ldw,
                             const double* __restrict__ anorm2, double* __restrict__ gamma2) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (j >= n) return;
  double s = 0.0;
  for (int64_t i = lane; i < l; i += 64) {
    const double w = (double)W[j * ldw + i];
    s += w * w;
  }
  s = wave_sum(s);
  if (lane == 0) gamma2[j] = anorm2[j] - s;
}

// Block partials of (masked argmax gamma2, max anorm2, non-finite).
__global__ void select_partial(const double* __restrict__ gamma2, const double* __restrict__ anorm2,
                               const unsigned char* __restrict__ inS, int64_t n, double* pv, int64_t* pi,
                               double* pa, unsigned* pnf) {
  __shared__ double rv[NT / 64];
  __shared__ int64_t ri[NT / 64];
  ArgMax b{0.0, -1};
  double amax = 0.0;
  unsigned nf = 0;
  for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < n; j += (int64_t)gridDim.x * NT) {
    const double a = anorm2[j];
    if (!(a <= 1.7976931348623157e308)) nf = 1;  // NaN or Inf
    else if (a > amax) amax = a;
    if (!inS[j] && better(gamma2[j], j, b.v, b.i)) b = ArgMax{gamma2[j], j};
  }
  b = block_argmax(b, rv, ri);
  ArgMax am = block_argmax(ArgMax{amax, 0}, rv, ri);
  ArgMax nfm = block_argmax(ArgMax{(double)nf, 0}, rv, ri);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = b.v;
    pi[blockIdx.x] = b.i;
    pa[blockIdx.x] = am.v;
    pnf[blockIdx.x] = nfm.v > 0.0 ? 1u : 0u;
  }
}

template <typename T>
__global__ void select_final(int nb, const double* pv, const int64_t* pi, const double* pa, const unsigned* pnf,
                             const T* __restrict__ R11, int64_t ldr, int64_t l, SrqrState* st) {
  __shared__ double rv[NT / 64];
  __shared__ int64_t ri[NT / 64];
  ArgMax b{0.0, -1};
  double amax = 0.0;
  unsigned nf = 0;
  for (int q = threadIdx.x; q < nb; q += NT) {
    if (better(pv[q], pi[q], b.v, b.i)) b = ArgMax{pv[q], pi[q]};
    amax = pa[q] > amax ? pa[q] : amax;
    nf |= pnf[q];
  }
  b = block_argmax(b, rv, ri);
  ArgMax am = block_argmax(ArgMax{amax, 0}, rv, ri);
  ArgMax nfm = block_argmax(ArgMax{(double)nf, 0}, rv, ri);
  double dmin = 1.7976931348623157e308;
  for (int64_t i = threadIdx.x; i < l; i += NT) {
    const double d = fabs((double)R11[i * ldr + i]);
    dmin = d < dmin ? d : dmin;
  }
  ArgMax dm = block_argmax(ArgMax{-dmin, 0}, rv, ri);
  if (threadIdx.x == 0) {
    st->gamma2_max = b.v;
    st->jstar = b.i;
    st->anorm_max = sqrt(am.v);
    st->nonfinite = nfm.v > 0.0 ? 1u : 0u;
    st->min_diag = -dm.v;
    st->alpha = 0.0;
  }
}

// ------------------------------------------------------- j* candidates
// Window of the preselection (see the header): the approximate gamma_j^2 of
// a trailing column may exceed the true value by at most win (a_j + a_max)
// where a = ||a||^2, so column j can beat the approximate maximum only when
// gamma_j^2 >= gmax - win (a_j + a_max).
__device__ inline bool is_cand(double g, double a, double gmax, double amax2, double win, bool lead) {
  return !lead && g >= gmax - win * (a + amax2);
}

constexpr int CB_N = 1024;  // columns per block of the candidate compaction

// Per block of CB_N columns: the number of candidates and the largest upper
// bound gamma_j^2 + win a_j over the non-candidates (-1 when there is none).
__global__ void cand_count(const double* __restrict__ gamma2, const double* __restrict__ anorm2,
                           const unsigned char* __restrict__ inS, int64_t n, const SrqrState* st, double win,
                           int64_t* cnt, double* ub) {
  __shared__ double red[CB_N / 64];
  __shared__ int64_t ri[CB_N / 64];
  const int64_t j = (int64_t)blockIdx.x * CB_N + threadIdx.x;
  const double gmax = st->gamma2_max, amax2 = anorm2[st->jstar >= 0 ? st->jstar : 0];
  double c = 0.0, u = -1.0;
  if (j < n && !inS[j]) {
    if (is_cand(gamma2[j], anorm2[j], gmax, amax2, win, false)) c = 1.0;
    else u = gamma2[j] + win * anorm2[j];
  }
  c = block_sum(c, red);
  const ArgMax m = block_argmax(ArgMax{u, 0}, red, ri);
  if (threadIdx.x == 0) {
    cnt[blockIdx.x] = (int64_t)c;
    ub[blockIdx.x] = m.v;
  }
}

// Exclusive prefix of the block counts (in place); the total and the
// largest non-candidate bound go to the state.
__global__ void cand_scan(int64_t* cnt, const double* ub, int nb, SrqrState* st) {
  if (threadIdx.x == 0) {
    int64_t run = 0;
    double u = -1.0;
    for (int q = 0; q < nb; ++q) {
      const int64_t c = cnt[q];
      cnt[q] = run;
      run += c;
      u = ub[q] > u ? ub[q] : u;
    }
    st->ncand = run;
    st->ub_noncand = u;
  }
}

// list[0:ncand] = the candidates in ascending column order.
__global__ void cand_scatter(const double* __restrict__ gamma2, const double* __restrict__ anorm2,
                             const unsigned char* __restrict__ inS, int64_t n, const SrqrState* st, double win,
                             const int64_t* cnt, int64_t* list) {
  __shared__ int sc[CB_N];
  const int64_t j = (int64_t)blockIdx.x * CB_N + threadIdx.x;
  const double gmax = st->gamma2_max, amax2 = anorm2[st->jstar >= 0 ? st->jstar : 0];
  const int f = (j < n && is_cand(gamma2[j], anorm2[j], gmax, amax2, win, inS[j] != 0)) ? 1 : 0;
  sc[threadIdx.x] = f;
  __syncthreads();
  for (int o = 1; o < CB_N; o <<= 1) {  // inclusive Hillis-Steele scan
    const int v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  if (f) list[cnt[blockIdx.x] + sc[threadIdx.x] - 1] = j;
}

// Row-block partial sums of e_i^2, e = a_c - Q W(:, c), for the candidates
// c of chunks of CC: blockIdx.x strides over the rows, blockIdx.y over the
// chunks.  part[t * gridDim.x + blockIdx.x] for candidate t of the list.
constexpr int CC = 8;
template <typename T>
__global__ void cand_exact(const T* __restrict__ A, int64_t m, int64_t lda, const T* __restrict__ Q, int64_t ldq,
                           const T* __restrict__ W, int64_t ldw, int64_t l, const int64_t* __restrict__ list,
                           const SrqrState* st, double* __restrict__ part) {
  extern __shared__ double wl[];  // wl[s * CC + c] = W(s, list[chunk * CC + c])
  __shared__ double red[NT / 64];
  const int64_t nc = st->ncand;
  const int64_t nchunk = (nc + CC - 1) / CC;
  for (int64_t ch = blockIdx.y; ch < nchunk; ch += gridDim.y) {
    int64_t col[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int64_t t = ch * CC + c;
      col[c] = t < nc ? list[t] : -1;
    }
    __syncthreads();
    for (int64_t e = threadIdx.x; e < l * CC; e += NT) {
      const int c = (int)(e % CC);
      const int64_t sidx = e / CC;
      wl[e] = col[c] >= 0 ? (double)W[col[c] * ldw + sidx] : 0.0;
    }
    __syncthreads();
    double acc[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) acc[c] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < m; i += (int64_t)gridDim.x * NT) {
      double ev[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c) ev[c] = col[c] >= 0 ? (double)A[col[c] * lda + i] : 0.0;
      for (int64_t sidx = 0; sidx < l; ++sidx) {
        const double q = (double)Q[sidx * ldq + i];
#pragma unroll
        for (int c = 0; c < CC; ++c) ev[c] = fma(-q, wl[sidx * CC + c], ev[c]);
      }
#pragma unroll
      for (int c = 0; c < CC; ++c) acc[c] = fma(ev[c], ev[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const double t = block_sum(acc[c], red);
      if (threadIdx.x == 0 && col[c] >= 0) part[(ch * CC + c) * gridDim.x + blockIdx.x] = t;
    }
  }
}

// j* = argmax of the recomputed gamma^2 (ties to the smallest index),
// alpha = gamma_j*, and the margin of the choice.
__global__ void cand_final(const int64_t* __restrict__ list, const double* __restrict__ part, int na,
                           SrqrState* st) {
  __shared__ double rv[NT / 64];
  __shared__ int64_t ri[NT / 64];
  const int64_t nc = st->ncand;
  ArgMax b{0.0, -1};
  for (int64_t t = threadIdx.x; t < nc; t += NT) {
    double g = 0.0;
    for (int x = 0; x < na; ++x) g += part[t * na + x];
    if (better(g, list[t], b.v, b.i)) b = ArgMax{g, list[t]};
  }
  const ArgMax top = block_argmax(b, rv, ri);
  ArgMax s2{-1.0, -1};
  for (int64_t t = threadIdx.x; t < nc; t += NT) {
    if (list[t] == top.i) continue;
    double g = 0.0;
    for (int x = 0; x < na; ++x) g += part[t * na + x];
    if (g > s2.v) s2 = ArgMax{g, 0};
  }
  const ArgMax second = block_argmax(s2, rv, ri);
  if (threadIdx.x == 0) {
    if (top.i < 0) {
      st->alpha = 0.0;
      st->jmargin = 1.0;
      return;
    }
    const double g1 = top.v > 0.0 ? top.v : 0.0;
    const double g2nd = second.v > st->ub_noncand ? second.v : st->ub_noncand;
    st->jstar = top.i;
    st->gamma2_max = g1;
    st->alpha = sqrt(g1);
    st->jmargin = g1 > 0.0 ? (g2nd < 0.0 ? 1.0 : (g1 - g2nd) / g1) : 0.0;
  }
}

// Back substitution with R11, one right-hand side per workgroup j:
// j < ncol: e_j (rhs null; column j of R11^{-1}, length j + 1) or row j of
// rhs (stride rstride, length l); j == ncol: z = R11^{-1} a.
template <typename T>
__global__ void trinv_kernel(const T* __restrict__ R, int64_t ldr, int64_t l, const T* __restrict__ a_base,
                             int64_t a_stride, const SrqrState* st, const double* __restrict__ rhs,
                             int64_t rstride, int64_t ncol, double* __restrict__ X) {
  extern __shared__ double sm[];
  constexpr int CH = 16;
  double* b = sm;              // l
  double* xo = b + l;          // l
  double* Rc = xo + l;         // l x CH staging
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t len = (j < ncol && !rhs) ? j + 1 : l;
  const T* a = nullptr;
  if (j == ncol) {
    // st selects the column of W; no trailing column leaves a = 0
    if (!st) a = a_base;
    else if (st->jstar >= 0) a = a_base + st->jstar * a_stride;
  }
  for (int64_t r = tid; r < l; r += NT) {
    double v;
    if (j < ncol) v = rhs ? rhs[j * rstride + r] : (r == j ? 1.0 : 0.0);
    else v = a ? (double)a[r] : 0.0;
    b[r] = v;
    xo[r] = 0.0;
  }
  for (int64_t hi = len - 1; hi >= 0; hi -= CH) {
    const int64_t lo = hi - CH + 1 > 0 ? hi - CH + 1 : 0;
    const int nc = (int)(hi - lo + 1);
    __syncthreads();
    // stage R(0:hi, lo:hi)
    for (int64_t e = tid; e < (hi + 1) * nc; e += NT) {
      const int64_t r = e % (hi + 1), c = e / (hi + 1);
      Rc[c * l + r] = (double)R[(lo + c) * ldr + r];
    }
    for (int64_t i = hi; i >= lo; --i) {
      __syncthreads();
      const double* col = Rc + (i - lo) * l;
      const double xi = b[i] / col[i];
      if (tid == 0) xo[i] = xi;
      for (int64_t r = tid; r < i; r += NT) b[r] -= xi * col[r];
    }
  }
  __syncthreads();
  for (int64_t r = tid; r < l; r += NT) X[j * l + r] = xo[r];
}

// rho_i = sqrt(alpha^2 ||X(i, 0:l)||^2 + X(i, l)^2); g2, istar.
__global__ void rho_kernel(const double* __restrict__ X, int64_t l, const SrqrState* st_in, double alpha_host,
                           double* __restrict__ rho, SrqrState* st) {
  __shared__ double rv[NT / 64];
  __shared__ int64_t ri[NT / 64];
  const double alpha = st_in ? st_in->alpha : alpha_host;
  ArgMax b{0.0, -1};
  for (int64_t i = threadIdx.x; i < l; i += NT) {
    double s = 0.0;
    for (int64_t j = i; j < l; ++j) {
      const double x = X[j * l + i];
      s += x * x;
    }
    const double z = X[l * l + i];
    const double r = sqrt(alpha * alpha * s + z * z);
    rho[i] = r;
    if (better(r, i, b.v, b.i)) b = ArgMax{r, i};
  }
  b = block_argmax(b, rv, ri);
  if (threadIdx.x == 0 && st) {
    st->g2 = b.v > 1.0 ? b.v : 1.0;
    st->istar = b.i;
  }
}

// est_i from Y = R11^{-1} P1^T (column t at X + t l), z = R11^{-1} a (at
// X + d l) and p2 = P(:, l); g2 and istar over positions 0..l.
__global__ void probe_rho_kernel(const double* __restrict__ X, int64_t l, int d, const double* __restrict__ P,
                                 const SrqrState* st_in, double alpha_host, double* __restrict__ est,
                                 SrqrState* st) {
  __shared__ double rv[NT / 64];
  __shared__ int64_t ri[NT / 64];
  const double alpha = st_in ? st_in->alpha : alpha_host;
  const double inv_d = 1.0 / (double)d;
  ArgMax b{0.0, -1};
  for (int64_t i = threadIdx.x; i <= l; i += NT) {
    double s = 0.0;
    if (i < l) {
      const double z = X[(int64_t)d * l + i];
      for (int t = 0; t < d; ++t) {
        const double v = alpha * X[(int64_t)t * l + i] - z * P[(int64_t)t * (l + 1) + l];
        s += v * v;
      }
    } else {
      for (int t = 0; t < d; ++t) {
        const double v = P[(int64_t)t * (l + 1) + l];
        s += v * v;
      }
    }
    const double r = sqrt(s * inv_d);
    est[i] = r;
    if (better(r, i, b.v, b.i)) b = ArgMax{r, i};
  }
  b = block_argmax(b, rv, ri);
  if (threadIdx.x == 0 && st) {
    st->g2 = b.v;
    st->istar = b.i;
  }
}

__global__ void est_reset_kernel(double* est, const SrqrState* st) {
  if (threadIdx.x == 0 && st->jstar >= 0) est[st->jstar] = st->alpha * st->alpha;
}

// ------------------------------------------------------------------ perm
__global__ void perm_clear(int64_t n, unsigned char* inS) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    inS[j] = 0;
}
__global__ void perm_set(const int64_t* __restrict__ S, int64_t l, int64_t n, unsigned char* inS, int64_t* perm) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < l; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = S[k];
    if (c >= 0 && c < n) inS[c] = 1;
    perm[k] = c;
  }
}
constexpr int PB = 1024;
__global__ void perm_count(const unsigned char* __restrict__ inS, int64_t n, int64_t* cnt) {
  __shared__ double red[PB / 64];
  const int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x;
  double c = (j < n && !inS[j]) ? 1.0 : 0.0;
  c = block_sum(c, red);
  if (threadIdx.x == 0) cnt[blockIdx.x] = (int64_t)c;
}
__global__ void perm_scan(int64_t* cnt, int nb) {
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int q = 0; q < nb; ++q) {
      const int64_t c = cnt[q];
      cnt[q] = run;
      run += c;
    }
  }
}
__global__ void perm_scatter(const unsigned char* __restrict__ inS, int64_t n, int64_t l, const int64_t* cnt,
                             int64_t* perm) {
  __shared__ int sc[PB];
  const int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int f = (j < n && !inS[j]) ? 1 : 0;
  sc[threadIdx.x] = f;
  __syncthreads();
  // inclusive Hillis-Steele scan
  for (int o = 1; o < PB; o <<= 1) {
    const int v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  const int64_t dst = l + cnt[blockIdx.x] + sc[threadIdx.x] - 1;
  if (f && dst < n) perm[dst] = j;
}

// ------------------------------------------------------------- assembly
template <typename T>
__global__ void assemble_rt_kernel(const T* __restrict__ R11, int64_t ldr11, const T* __restrict__ W, int64_t ldw,
                                   const int64_t* __restrict__ perm, int64_t l, int64_t n, T* __restrict__ Rt,
                                   int64_t ldrt) {
  __shared__ T tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, s0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t i = i0 + k, s = s0 + tx;
    T v = 0;
    if (i < n && s < l) {
      if (i < l) v = R11[i * ldr11 + s];
      else {
        const int64_t c = perm ? perm[i] : i;
        v = (c >= 0 && c < n) ? W[c * ldw + s] : T(0);
      }
    }
    tile[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t s = s0 + k, i = i0 + tx;
    if (i < n && s < l) Rt[s * ldrt + i] = tile[tx][k];
  }
}

template <typename T>
__global__ void assemble_r_kernel(const T* __restrict__ R11, int64_t ldr11, const T* __restrict__ W, int64_t ldw,
                                  const int64_t* __restrict__ perm, int64_t l, int64_t n, T* __restrict__ R,
                                  int64_t ldr) {
  const int64_t i = blockIdx.y;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < l; s += (int64_t)gridDim.x * blockDim.x)
    R[i * ldr + s] = (i < l) ? R11[i * ldr11 + s] : W[perm[i] * ldw + s];
}

}  // namespace

template <typename T>
hipError_t residual_norms(const T* W, int64_t l, int64_t n, int64_t ldw, const double* anorm2, double* gamma2,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  resid_kernel<T><<<(unsigned)((n + 3) / 4), 256, 0, s>>>(W, l, n, ldw, anorm2, gamma2);
  return hipGetLastError();
}

constexpr int kCandRowBlocks = 32;  // row blocks of the candidate recomputation

template <typename T>
size_t srqr_scratch(int64_t m, int64_t n, int64_t l) {
  const size_t nb = (size_t)(n + CB_N - 1) / CB_N;
  // the exact rho's R11^{-1} and z, or the largest probe with its solves
  const size_t xs = std::max((size_t)(l + 1) * l, (size_t)(kMaxProbe + 1) * l + (size_t)kMaxProbe * (l + 1) + 32);
  return sizeof(double) * (xs + 4 * 1024) + sizeof(int64_t) * 1024 + 4 * 1024 + 8 * 256 +
         nb * (sizeof(int64_t) + sizeof(double)) + (size_t)n * sizeof(int64_t) +
         (size_t)n * kCandRowBlocks * sizeof(double) + 8 * 256;
}

template <typename T>
hipError_t srqr_select(const double* gamma2, const double* anorm2, const unsigned char* inS, int64_t n, const T* A,
                       int64_t m, int64_t lda, const T* Q, int64_t ldq, const T* W, int64_t ldw, const T* R11,
                       int64_t ldr, int64_t l, SrqrState* st, Arena& ar, hipStream_t s, double win) {
  int nb = (int)((n + NT - 1) / NT);
  if (nb > 1024) nb = 1024;
  double* pv = ar.take<double>(1024);
  int64_t* pi = ar.take<int64_t>(1024);
  double* pa = ar.take<double>(1024);
  unsigned* pnf = ar.take<unsigned>(1024);
  if (!pv || !pi || !pa || !pnf) return hipErrorOutOfMemory;
  select_partial<<<nb, NT, 0, s>>>(gamma2, anorm2, inS, n, pv, pi, pa, pnf);
  select_final<T><<<1, NT, 0, s>>>(nb, pv, pi, pa, pnf, R11, ldr, l, st);
  if (l <= 0) return hipGetLastError();  // only the non-finite / norm scan was wanted
  const int cb = (int)((n + CB_N - 1) / CB_N);
  int64_t* cnt = ar.take<int64_t>(cb);
  double* ub = ar.take<double>(cb);
  int64_t* list = ar.take<int64_t>(n);
  double* part = ar.take<double>((size_t)n * kCandRowBlocks);
  if (!cnt || !ub || !list || !part) return hipErrorOutOfMemory;
  cand_count<<<cb, CB_N, 0, s>>>(gamma2, anorm2, inS, n, st, win, cnt, ub);
  cand_scan<<<1, 64, 0, s>>>(cnt, ub, cb, st);
  cand_scatter<<<cb, CB_N, 0, s>>>(gamma2, anorm2, inS, n, st, win, cnt, list);
  int na = (int)((m + NT - 1) / NT);
  if (na > kCandRowBlocks) na = kCandRowBlocks;
  const size_t lds = (size_t)l * CC * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)cand_exact<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  cand_exact<T><<<dim3((unsigned)na, 32u), NT, lds, s>>>(A, m, lda, Q, ldq, W, ldw, l, list, st, part);
  cand_final<<<1, NT, 0, s>>>(list, part, na, st);
  return hipGetLastError();
}

template <typename T>
hipError_t srqr_rho(const T* R11, int64_t ldr, const T* a, int64_t a_stride, const SrqrState* sel,
                    double alpha_host, int64_t l, double* rho, SrqrState* st_out, Arena& ar, hipStream_t s) {
  double* X = ar.take<double>((size_t)(l + 1) * l);
  if (!X) return hipErrorOutOfMemory;
  const size_t lds = (size_t)(2 * l + 16 * l) * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)trinv_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  trinv_kernel<T><<<(unsigned)(l + 1), NT, lds, s>>>(R11, ldr, l, a, a_stride, sel, nullptr, 0, l, X);
  rho_kernel<<<1, NT, 0, s>>>(X, l, sel, alpha_host, rho, st_out);
  return hipGetLastError();
}

template <typename T>
hipError_t srqr_probe(const T* R11, int64_t ldr, const T* a, int64_t a_stride, const SrqrState* sel,
                      double alpha_host, int64_t l, int32_t d, uint64_t seed, uint64_t q, double* est,
                      SrqrState* st_out, Arena& ar, hipStream_t s) {
  if (d < 1 || d > kMaxProbe || q < 1) return hipErrorInvalidValue;
  double* P = ar.take<double>((size_t)d * (l + 1));
  double* X = ar.take<double>((size_t)(d + 1) * l);
  if (!P || !X) return hipErrorOutOfMemory;
  const size_t lds = (size_t)(2 * l + 16 * l) * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)trinv_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_probe(seed, q, d, l + 1, P, s);
  if (e != hipSuccess) return e;
  trinv_kernel<T><<<(unsigned)(d + 1), NT, lds, s>>>(R11, ldr, l, a, a_stride, sel, P, l + 1, d, X);
  probe_rho_kernel<<<1, NT, 0, s>>>(X, l, d, P, sel, alpha_host, est, st_out);
  return hipGetLastError();
}

hipError_t est_reset_jstar(double* est, const SrqrState* st, hipStream_t s) {
  est_reset_kernel<<<1, 64, 0, s>>>(est, st);
  return hipGetLastError();
}

hipError_t build_perm(const int64_t* S, int64_t l, int64_t n, int64_t* perm, unsigned char* inS, int64_t* cnt,
                      hipStream_t s) {
  const int nb = (int)((n + PB - 1) / PB);
  const unsigned gc = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  perm_clear<<<gc, 256, 0, s>>>(n, inS);
  perm_set<<<(unsigned)((l + 255) / 256), 256, 0, s>>>(S, l, n, inS, perm);
  perm_count<<<nb, PB, 0, s>>>(inS, n, cnt);
  perm_scan<<<1, 64, 0, s>>>(cnt, nb);
  perm_scatter<<<nb, PB, 0, s>>>(inS, n, l, cnt, perm);
  return hipGetLastError();
}

template <typename T>
hipError_t assemble_rt(const T* R11, int64_t ldr11, const T* W, int64_t ldw, const int64_t* perm, int64_t l, int64_t n,
                       T* Rt, int64_t ldrt, hipStream_t s) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((l + 31) / 32));
  assemble_rt_kernel<T><<<grid, 256, 0, s>>>(R11, ldr11, W, ldw, perm, l, n, Rt, ldrt);
  return hipGetLastError();
}

template <typename T>
hipError_t assemble_r(const T* R11, int64_t ldr11, const T* W, int64_t ldw, const int64_t* perm, int64_t l, int64_t n,
                      T* R, int64_t ldr, hipStream_t s) {
  dim3 grid((unsigned)((l + 255) / 256), (unsigned)n);
  assemble_r_kernel<T><<<grid, 256, 0, s>>>(R11, ldr11, W, ldw, perm, l, n, R, ldr);
  return hipGetLastError();
}

#define INST(T)                                                                                                   \
  template hipError_t residual_norms<T>(const T*, int64_t, int64_t, int64_t, const double*, double*, hipStream_t); \
  template size_t srqr_scratch<T>(int64_t, int64_t, int64_t);                                                       \
  template hipError_t srqr_select<T>(const double*, const double*, const unsigned char*, int64_t, const T*, int64_t, \
                                     int64_t, const T*, int64_t, const T*, int64_t, const T*, int64_t, int64_t,      \
                                     SrqrState*, Arena&, hipStream_t, double);                                      \
  template hipError_t srqr_rho<T>(const T*, int64_t, const T*, int64_t, const SrqrState*, double, int64_t, double*, \
                                  SrqrState*, Arena&, hipStream_t);                                                 \
  template hipError_t srqr_probe<T>(const T*, int64_t, const T*, int64_t, const SrqrState*, double, int64_t,        \
                                    int32_t, uint64_t, uint64_t, double*, SrqrState*, Arena&, hipStream_t);        \
  template hipError_t assemble_rt<T>(const T*, int64_t, const T*, int64_t, const int64_t*, int64_t, int64_t, T*,   \
                                     int64_t, hipStream_t);                                                         \
  template hipError_t assemble_r<T>(const T*, int64_t, const T*, int64_t, const int64_t*, int64_t, int64_t, T*,    \
                                    int64_t, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
