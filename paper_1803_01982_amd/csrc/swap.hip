// One swap of Algorithm 4 (SRQR) as an update of the factorization in place.
//
// State before the swap: the ordered leading set S (l columns of A), the
// thin QR A(:, S) = Q R11 (Q m x l with orthonormal columns, R11 l x l upper
// triangular with a positive diagonal) and the projection W = Q^T A (l x n,
// columns in the original order).  The swap moves S[istar] out of the
// leading set and appends the trailing column jstar (the round-robin order
// of Algorithm 4).  Instead of a new Householder QR of A(:, S'), a new
// projection and new residual norms from scratch:
//
//   1. Deleting column istar of R11 leaves columns istar..l-2 upper
//      Hessenberg.  Plane rotations G_k in rows (k, k+1), k = istar..l-2,
//      restore the triangle; each maps (x, y) to (hypot(x, y), 0), so the
//      new diagonal stays positive (the sign convention of the Householder
//      QR, under which the thin QR is unique).  The same rotations act on
//      the rows of W and on the columns of Q, so that afterwards
//      Q(:, 0:l-2) R11(0:l-2, 0:l-2) = A(:, S without S[istar]) and W = Q^T A
//      still hold; Q(:, l-1) is the unit vector left over in span(Q).
//   2. The new last column: with w = W(:, jstar) after step 1, the residual
//      v = a_jstar - Q(:, 0:l-2) w(0:l-2) is orthogonalised a second time
//      against Q(:, 0:l-2) (classical Gram-Schmidt, second pass:
//      c = Q(:, 0:l-2)^T v, v <- v - Q(:, 0:l-2) c), then
//      R11(:, l-1) = (w(0:l-2) + c, ||v||) and Q(:, l-1) = v / ||v||.
//      ||v||^2 = alpha^2 + w(l-1)^2 >= alpha^2 > 0 (alpha = gamma_jstar, the
//      largest residual norm, which the caller has checked against the rank
//      tolerance).
//   3. Row l-1 of W becomes Q(:, l-1)^T A: the one pass over A a swap needs.
//
// Arithmetic is FP64 throughout, on T (FP32 or FP64) storage.  Work per
// swap: about 2(l - istar)(m + n) flops for the rotations, 6 m l for the
// new column and 2 m n for the new row (the pass over A).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256;
constexpr int GNT = 1024;  // threads of the rotation-choosing workgroup
constexpr int GCH = 8;     // rows of R11 each thread prefetches per chunk
constexpr int RCOLS = 4;   // columns of A per workgroup in the row pass

// (x, y) -> (r, 0) with r = hypot(x, y) >= 0: c = x / r, s = y / r, scaled
// by the larger magnitude first so that the squares neither overflow nor
// underflow.  r = 0 gives the identity.
__device__ inline void plane_rotation(double x, double y, double& c, double& s, double& r) {
  const double ax = fabs(x), ay = fabs(y);
  const double big = ax > ay ? ax : ay;
  if (big == 0.0) {
    c = 1.0;
    s = 0.0;
    r = 0.0;
    return;
  }
  const double xs = x / big, ys = y / big;
  const double h = sqrt(fma(xs, xs, ys * ys));
  r = big * h;
  c = xs / h;
  s = ys / h;
}

// Step 1 on R11: Rn (ldn) receives the retriangularised columns 0..l-2
// (column c < istar copied, column c >= istar the rotated column c + 1 of
// R11); rotation k is stored as (cs[2k], cs[2k+1]) = (c_k, s_k).  One
// workgroup; thread t owns the columns istar + t + GNT u.  In step k the
// owner of column k chooses G_k from its running entry (row k of the column
// after G_istar..G_{k-1}) and R11(k+1, k+1); after one workgroup barrier the
// owners of the later columns apply it.  The rotation of step k is
// published in one of two LDS slots (by parity of k), so one barrier per
// step suffices.  Entries R11(k+1, c+1) are prefetched GCH rows ahead into
// registers by the owner of column c (one column per thread when
// l - 1 - istar <= GNT; otherwise direct loads).
template <typename T>
__global__ __launch_bounds__(GNT) void swap_givens_kernel(const T* __restrict__ R, int64_t ldr, int l, int istar,
                                                          T* __restrict__ Rn, int64_t ldn, double* __restrict__ cs) {
  extern __shared__ double carry[];  // running entry of each column c >= istar (index c - istar)
  __shared__ double slot[2][2];
  const int tid = threadIdx.x;
  const int nc = l - 1 - istar;  // columns istar..l-2 of the new triangle
  // parts that no rotation touches
  for (int64_t e = tid; e < (int64_t)l * (l - 1); e += GNT) {
    const int i = (int)(e % l), c = (int)(e / l);
    double v;
    if (c < istar) v = i <= c ? (double)R[(int64_t)c * ldr + i] : 0.0;
    else if (i < istar) v = (double)R[(int64_t)(c + 1) * ldr + i];
    else if (i > c) v = 0.0;
    else continue;  // rows istar..c of column c >= istar: written by the steps
    Rn[(int64_t)c * ldn + i] = (T)v;
  }
  for (int c = tid; c < nc; c += GNT) carry[c] = (double)R[(int64_t)(istar + c + 1) * ldr + istar];
  __syncthreads();
  if (nc <= GNT) {
    // one column per thread: c = istar + tid
    const int c = istar + tid;
    const bool own = tid < nc;
    const T* col = R + (int64_t)(c + 1) * ldr;  // column c of the Hessenberg block
    double cur[GCH], nxt[GCH];
#pragma unroll
    for (int i = 0; i < GCH; ++i) {
      const int row = istar + 1 + i;
      cur[i] = (own && row <= c + 1) ? (double)col[row] : 0.0;
    }
    double x = own ? carry[tid] : 0.0;
    for (int k0 = istar; k0 < l - 1; k0 += GCH) {
#pragma unroll
      for (int i = 0; i < GCH; ++i) {
        const int row = k0 + GCH + 1 + i;
        nxt[i] = (own && row <= c + 1) ? (double)col[row] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < GCH; ++i) {
        const int k = k0 + i;
        if (k >= l - 1) break;
        const int b = k & 1;
        if (own && c == k) {
          // y = R11(k+1, k+1), the subdiagonal entry of column k
          double cr, sr, r;
          plane_rotation(x, cur[i], cr, sr, r);
          Rn[(int64_t)c * ldn + k] = (T)r;
          slot[b][0] = cr;
          slot[b][1] = sr;
          cs[2 * k] = cr;
          cs[2 * k + 1] = sr;
        }
        __syncthreads();
        if (own && c > k) {
          const double cr = slot[b][0], sr = slot[b][1], y = cur[i];
          Rn[(int64_t)c * ldn + k] = (T)fma(cr, x, sr * y);
          x = fma(-sr, x, cr * y);
        }
      }
#pragma unroll
      for (int i = 0; i < GCH; ++i) cur[i] = nxt[i];
    }
  } else {
    for (int k = istar; k < l - 1; ++k) {
      const int b = k & 1;
      if (k - istar < nc && (k - istar) % GNT == tid) {
        double cr, sr, r;
        plane_rotation(carry[k - istar], (double)R[(int64_t)(k + 1) * ldr + k + 1], cr, sr, r);
        Rn[(int64_t)k * ldn + k] = (T)r;
        slot[b][0] = cr;
        slot[b][1] = sr;
        cs[2 * k] = cr;
        cs[2 * k + 1] = sr;
      }
      __syncthreads();
      const double cr = slot[b][0], sr = slot[b][1];
      for (int c = k + 1 + ((tid - (k + 1 - istar)) % GNT + GNT) % GNT; c < l - 1; c += GNT) {
        const double x = carry[c - istar], y = (double)R[(int64_t)(c + 1) * ldr + k + 1];
        Rn[(int64_t)c * ldn + k] = (T)fma(cr, x, sr * y);
        carry[c - istar] = fma(-sr, x, cr * y);
      }
    }
  }
}

// Applies G_istar..G_{l-2} to nvec vectors of l entries: entry k of vector
// v at X[v * vs + k * es] (the columns of W: vs = ldw, es = 1; the rows of
// Q: vs = 1, es = ldq).  One thread per vector; the running entry is carried
// in a register, each element is loaded and stored once.
template <typename T>
__global__ void swap_rotate_kernel(T* __restrict__ X, int64_t nvec, int64_t vs, int64_t es, int l, int istar,
                                   const double* __restrict__ cs) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  T* x = X + v * vs;
  double run = (double)x[(int64_t)istar * es];
#pragma unroll 8
  for (int k = istar; k < l - 1; ++k) {
    const double c = cs[2 * k], s = cs[2 * k + 1];
    const double y = (double)x[(int64_t)(k + 1) * es];
    x[(int64_t)k * es] = (T)fma(c, run, s * y);
    run = fma(-s, run, c * y);
  }
  x[(int64_t)(l - 1) * es] = (T)run;
}

// est[c] += sign W(l-1, c)^2 over all columns; with sign > 0, est[icol]
// starts from 0.
template <typename T>
__global__ void est_row_kernel(const T* __restrict__ W, int64_t ldw, int l, int64_t n, double* __restrict__ est,
                               int64_t icol, double sign) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const double w = (double)W[c * ldw + l - 1];
    const double base = (c == icol) ? 0.0 : est[c];
    est[c] = fma(sign * w, w, base);
  }
}

// v = a_jstar - Q(:, 0:l-2) w(0:l-2), w = W(:, jstar); one thread per row.
template <typename T>
__global__ void swap_resid_kernel(const T* __restrict__ A, int64_t lda, int64_t jstar, const T* __restrict__ Q,
                                  int64_t ldq, const T* __restrict__ W, int64_t ldw, int64_t m, int l,
                                  double* __restrict__ v) {
  extern __shared__ double w[];
  for (int k = threadIdx.x; k < l - 1; k += blockDim.x) w[k] = (double)W[jstar * ldw + k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc = (double)A[jstar * lda + i];
  for (int k = 0; k < l - 1; ++k) acc = fma(-(double)Q[(int64_t)k * ldq + i], w[k], acc);
  v[i] = acc;
}

// c_k = Q(:, k)^T v for k < l - 1: one workgroup per k, fixed summation order.
template <typename T>
__global__ void swap_proj_kernel(const T* __restrict__ Q, int64_t ldq, int64_t m, const double* __restrict__ v,
                                 double* __restrict__ c) {
  __shared__ double red[NT / kWave];
  const int64_t k = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += NT) acc = fma((double)Q[k * ldq + i], v[i], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) c[k] = acc;
}

// v <- v - Q(:, 0:l-2) c; part[block] = the block's sum of v_i^2.
template <typename T>
__global__ void swap_correct_kernel(const T* __restrict__ Q, int64_t ldq, int64_t m, int l,
                                    const double* __restrict__ c, double* __restrict__ v,
                                    double* __restrict__ part) {
  extern __shared__ double cc[];
  __shared__ double red[NT / kWave];
  for (int k = threadIdx.x; k < l - 1; k += blockDim.x) cc[k] = c[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < m) {
    double acc = v[i];
    for (int k = 0; k < l - 1; ++k) acc = fma(-(double)Q[(int64_t)k * ldq + i], cc[k], acc);
    v[i] = acc;
    sq = acc * acc;
  }
  sq = block_sum(sq, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sq;
}

// R11(:, l-1) = (W(0:l-2, jstar) + c, ||v||); rho_out = ||v||.
template <typename T>
__global__ void swap_finish_kernel(const double* __restrict__ part, int nb, const T* __restrict__ W, int64_t ldw,
                                   int64_t jstar, const double* __restrict__ c, int l, T* __restrict__ R11,
                                   int64_t ldr, double* __restrict__ rho_out) {
  __shared__ double red[NT / kWave];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) acc += part[b];
  const double rho = sqrt(block_sum(acc, red));
  for (int k = threadIdx.x; k < l - 1; k += NT) R11[(int64_t)(l - 1) * ldr + k] = (T)((double)W[jstar * ldw + k] + c[k]);
  if (threadIdx.x == 0) {
    R11[(int64_t)(l - 1) * ldr + l - 1] = (T)rho;
    *rho_out = rho;
  }
}

// Q(:, l-1) = v / rho.
template <typename T>
__global__ void swap_qcol_kernel(const double* __restrict__ v, const double* __restrict__ rho, int64_t m, int l,
                                 T* __restrict__ Q, int64_t ldq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) Q[(int64_t)(l - 1) * ldq + i] = (T)(v[i] / *rho);
}

// W(l-1, j) = Q(:, l-1)^T a_j for RCOLS columns per workgroup (Q(:, l-1)
// read once for all of them), fixed summation order.
template <typename T>
__global__ void swap_row_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n, const T* __restrict__ Q,
                                int64_t ldq, int l, T* __restrict__ W, int64_t ldw) {
  __shared__ double red[NT / kWave];
  const int64_t j0 = (int64_t)blockIdx.x * RCOLS;
  const T* q = Q + (int64_t)(l - 1) * ldq;
  double acc[RCOLS];
#pragma unroll
  for (int u = 0; u < RCOLS; ++u) acc[u] = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += NT) {
    const double qi = (double)q[i];
#pragma unroll
    for (int u = 0; u < RCOLS; ++u)
      if (j0 + u < n) acc[u] = fma(qi, (double)A[(j0 + u) * lda + i], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < RCOLS; ++u) {
    const double t = block_sum(acc[u], red);
    if (threadIdx.x == 0 && j0 + u < n) W[(j0 + u) * ldw + l - 1] = (T)t;
  }
}

}  // namespace

template <typename T>
size_t swap_scratch(int64_t m, int64_t l) {
  const size_t nb = (size_t)((m + NT - 1) / NT);
  return 8 * 256 + (size_t)l * l * sizeof(T) + sizeof(double) * (2 * (size_t)l + (size_t)m + (size_t)l + nb + 1);
}

template <typename T>
hipError_t srqr_swap_update(const T* A, int64_t m, int64_t n, int64_t lda, T* Q, int64_t ldq, T* W, int64_t ldw,
                            T* R11, int64_t ldr, int64_t l, int64_t istar, int64_t jstar, Arena& ar, hipStream_t s,
                            double* est, int64_t icol) {
  if (l < 1 || istar < 0 || istar >= l || jstar < 0 || jstar >= n || m < 1 || l > INT32_MAX / 2)
    return hipErrorInvalidValue;
  if (est && (icol < 0 || icol >= n)) return hipErrorInvalidValue;
  const unsigned eb = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 4096);
  const int li = (int)l, is = (int)istar;
  T* Rn = ar.take<T>((size_t)l * l);
  double* cs = ar.take<double>(2 * (size_t)l);
  double* v = ar.take<double>((size_t)m);
  double* c = ar.take<double>((size_t)l);
  const int nb = (int)((m + NT - 1) / NT);
  double* part = ar.take<double>((size_t)nb);
  double* rho = ar.take<double>(1);
  if (!Rn || !cs || !v || !c || !part || !rho) return hipErrorOutOfMemory;
  const size_t lds_c = (size_t)l * sizeof(double);
  if (lds_c > 65536) {
    for (const void* f : {(const void*)swap_givens_kernel<T>, (const void*)swap_resid_kernel<T>,
                          (const void*)swap_correct_kernel<T>}) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_c);
      if (e != hipSuccess) return e;
    }
  }
  if (l > 1) {
    // 1. rotations, the retriangularised columns, W's rows and Q's columns
    swap_givens_kernel<T><<<1, GNT, lds_c, s>>>(R11, ldr, li, is, Rn, l, cs);
    if (is < li - 1) {
      swap_rotate_kernel<T><<<(unsigned)((n + NT - 1) / NT), NT, 0, s>>>(W, n, ldw, 1, li, is, cs);
      swap_rotate_kernel<T><<<(unsigned)((m + NT - 1) / NT), NT, 0, s>>>(Q, m, 1, ldq, li, is, cs);
    }
  }
  // the rotated last row belongs to the removed column's direction
  if (est) est_row_kernel<T><<<eb, NT, 0, s>>>(W, ldw, li, n, est, icol, 1.0);
  // 2. the new last column of Q and R11
  swap_resid_kernel<T><<<(unsigned)nb, NT, lds_c, s>>>(A, lda, jstar, Q, ldq, W, ldw, m, li, v);
  if (l > 1) swap_proj_kernel<T><<<(unsigned)(l - 1), NT, 0, s>>>(Q, ldq, m, v, c);
  swap_correct_kernel<T><<<(unsigned)nb, NT, lds_c, s>>>(Q, ldq, m, li, c, v, part);
  if (l > 1) {
    hipError_t e = hipMemcpy2DAsync(R11, (size_t)ldr * sizeof(T), Rn, (size_t)l * sizeof(T), (size_t)l * sizeof(T),
                                    (size_t)(l - 1), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  swap_finish_kernel<T><<<1, NT, 0, s>>>(part, nb, W, ldw, jstar, c, li, R11, ldr, rho);
  swap_qcol_kernel<T><<<(unsigned)nb, NT, 0, s>>>(v, rho, m, li, Q, ldq);
  // 3. row l-1 of W: the pass over A
  swap_row_kernel<T><<<(unsigned)((n + RCOLS - 1) / RCOLS), NT, 0, s>>>(A, lda, m, n, Q, ldq, li, W, ldw);
  if (est) est_row_kernel<T><<<eb, NT, 0, s>>>(W, ldw, li, n, est, -1, -1.0);
  return hipGetLastError();
}

#define INST(T)                                                                                                     \
  template size_t swap_scratch<T>(int64_t, int64_t);                                                                \
  template hipError_t srqr_swap_update<T>(const T*, int64_t, int64_t, int64_t, T*, int64_t, T*, int64_t, T*, int64_t, \
                                          int64_t, int64_t, int64_t, Arena&, hipStream_t, double*, int64_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
