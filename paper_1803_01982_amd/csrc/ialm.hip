// Elementwise steps of robust PCA by the inexact augmented Lagrange
// multiplier method (Section 2, the robust PCA algorithm): the shifted
// matrix whose SVD is taken, the shrinkage of the sparse part and the
// multiplier update with the residual norm, the initial multiplier, the
// norms of M, and the scaled transpose that forms U S_{1/mu}(Sigma) for the
// low-rank product.  All HBM-bound, one pass each, FP64 arithmetic on T
// storage; every reduction sums fixed per-block partials in a fixed order.
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256;

inline unsigned ew_blocks(int64_t total) {
  const int64_t b = (total + NT - 1) / NT;
  return (unsigned)(b < kIalmBlocks ? (b > 0 ? b : 1) : kIalmBlocks);
}

// D = M - E + Y / mu (D, E, Y with leading dimension m)
template <typename T>
__global__ void ialm_shift_kernel(const T* __restrict__ M, int64_t ldm, const T* __restrict__ E,
                                  const T* __restrict__ Y, int64_t m, int64_t total, double inv_mu,
                                  T* __restrict__ D) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e % m, j = e / m;
    D[e] = (T)((double)M[j * ldm + i] - (double)E[e] + (double)Y[e] * inv_mu);
  }
}

// Y = M / J, E = 0
template <typename T>
__global__ void ialm_init_kernel(const T* __restrict__ M, int64_t ldm, int64_t m, int64_t total, double inv_j,
                                 T* __restrict__ Y, T* __restrict__ E) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e % m, j = e / m;
    Y[e] = (T)((double)M[j * ldm + i] * inv_j);
    E[e] = (T)0;
  }
}

__device__ inline double shrink(double x, double w) {
  const double a = fabs(x) - w;
  return a > 0.0 ? copysign(a, x) : 0.0;
}

// E = S_w(M - X + Y / mu); Z = M - X - E; Y += mu Z; part[block] = sum Z^2
template <typename T>
__global__ void ialm_update_kernel(const T* __restrict__ M, int64_t ldm, const T* __restrict__ X, int64_t ldx,
                                   int64_t m, int64_t total, double inv_mu, double mu, double w,
                                   T* __restrict__ E, T* __restrict__ Y, double* __restrict__ part) {
  __shared__ double red[NT / kWave];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e % m, j = e / m;
    const double mm = (double)M[j * ldm + i], x = (double)X[j * ldx + i], y = (double)Y[e];
    const T en = (T)shrink(mm - x + y * inv_mu, w);
    E[e] = en;
    const double z = mm - x - (double)en;
    Y[e] = (T)(y + mu * z);
    acc = fma(z, z, acc);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// per-block sum of squares and largest magnitude of M
template <typename T>
__global__ void norms_kernel(const T* __restrict__ M, int64_t ldm, int64_t m, int64_t total,
                             double* __restrict__ psq, double* __restrict__ pmax) {
  __shared__ double red[NT / kWave];
  double sq = 0.0, mx = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e % m, j = e / m;
    const double v = (double)M[j * ldm + i];
    sq = fma(v, v, sq);
    mx = fmax(mx, fabs(v));
  }
  sq = block_sum(sq, red);
  if (threadIdx.x == 0) psq[blockIdx.x] = sq;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < NT / kWave; ++q) t = fmax(t, red[q]);
    pmax[blockIdx.x] = t;
  }
}

// out[0] = sum of psq[0:nb], out[1] = max of pmax[0:nb] (pmax may be null)
__global__ void partials_final_kernel(const double* __restrict__ psq, const double* __restrict__ pmax, int nb,
                                      double* __restrict__ out) {
  __shared__ double red[NT / kWave];
  double s = 0.0, mx = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) {
    s += psq[b];
    if (pmax) mx = fmax(mx, pmax[b]);
  }
  s = block_sum(s, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < NT / kWave; ++q) t = fmax(t, red[q]);
    out[0] = s;
    out[1] = t;
  }
}

// B (k x rows, ldb) with B(j, i) = A(i, j) (sigma[j] - inv_mu)
template <typename T>
__global__ void scaled_transpose_kernel(const T* __restrict__ A, int64_t rows, int64_t k, int64_t lda,
                                        const double* __restrict__ sigma, double inv_mu, T* __restrict__ B,
                                        int64_t ldb) {
  const int64_t total = rows * k;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t j = e % k, i = e / k;
    B[i * ldb + j] = (T)((double)A[j * lda + i] * (sigma[j] - inv_mu));
  }
}

template <typename T>
__global__ void zero_kernel(T* __restrict__ X, int64_t ldx, int64_t m, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    X[(e / m) * ldx + e % m] = (T)0;
}

}  // namespace

template <typename T>
hipError_t ialm_shift(const T* M, int64_t ldm, const T* E, const T* Y, int64_t m, int64_t n, double inv_mu, T* D,
                      hipStream_t s) {
  const int64_t total = m * n;
  ialm_shift_kernel<T><<<ew_blocks(total), NT, 0, s>>>(M, ldm, E, Y, m, total, inv_mu, D);
  return hipGetLastError();
}

template <typename T>
hipError_t ialm_init(const T* M, int64_t ldm, int64_t m, int64_t n, double inv_j, T* Y, T* E, hipStream_t s) {
  const int64_t total = m * n;
  ialm_init_kernel<T><<<ew_blocks(total), NT, 0, s>>>(M, ldm, m, total, inv_j, Y, E);
  return hipGetLastError();
}

template <typename T>
hipError_t ialm_update(const T* M, int64_t ldm, const T* X, int64_t ldx, int64_t m, int64_t n, double mu, double w,
                       T* E, T* Y, double* part, double* out, hipStream_t s) {
  const int64_t total = m * n;
  const unsigned nb = ew_blocks(total);
  ialm_update_kernel<T><<<nb, NT, 0, s>>>(M, ldm, X, ldx, m, total, 1.0 / mu, mu, w, E, Y, part);
  partials_final_kernel<<<1, NT, 0, s>>>(part, nullptr, (int)nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t matrix_norms(const T* M, int64_t ldm, int64_t m, int64_t n, double* part, double* out, hipStream_t s) {
  const int64_t total = m * n;
  const unsigned nb = ew_blocks(total);
  norms_kernel<T><<<nb, NT, 0, s>>>(M, ldm, m, total, part, part + kIalmBlocks);
  partials_final_kernel<<<1, NT, 0, s>>>(part, part + kIalmBlocks, (int)nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t scaled_transpose(const T* A, int64_t rows, int64_t k, int64_t lda, const double* sigma, double inv_mu,
                            T* B, int64_t ldb, hipStream_t s) {
  scaled_transpose_kernel<T><<<ew_blocks(rows * k), NT, 0, s>>>(A, rows, k, lda, sigma, inv_mu, B, ldb);
  return hipGetLastError();
}

template <typename T>
hipError_t zero_matrix(T* X, int64_t ldx, int64_t m, int64_t n, hipStream_t s) {
  zero_kernel<T><<<ew_blocks(m * n), NT, 0, s>>>(X, ldx, m, m * n);
  return hipGetLastError();
}

#define INST(T)                                                                                                    \
  template hipError_t ialm_shift<T>(const T*, int64_t, const T*, const T*, int64_t, int64_t, double, T*,           \
                                    hipStream_t);                                                                  \
  template hipError_t ialm_init<T>(const T*, int64_t, int64_t, int64_t, double, T*, T*, hipStream_t);              \
  template hipError_t ialm_update<T>(const T*, int64_t, const T*, int64_t, int64_t, int64_t, double, double, T*,  \
                                     T*, double*, double*, hipStream_t);                                           \
  template hipError_t matrix_norms<T>(const T*, int64_t, int64_t, int64_t, double*, double*, hipStream_t);         \
  template hipError_t scaled_transpose<T>(const T*, int64_t, int64_t, int64_t, const double*, double, T*, int64_t, \
                                          hipStream_t);                                                            \
  template hipError_t zero_matrix<T>(T*, int64_t, int64_t, int64_t, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
