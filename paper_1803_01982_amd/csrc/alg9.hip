// Kernels of the last steps of Algorithm 9 (the rank-k approximate SVD from
// the flip-flop factors): a tiled transpose (the GEMMs of those steps produce
// the transposes of tmp = A Pi Qhat1, of U and of V_k) and the sign
// normalisation of the singular pairs.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

// B (cols x rows, ldb) = A^T for A rows x cols (lda), through a 32 x 33 tile.
template <typename T>
__global__ void transpose_kernel(const T* __restrict__ A, int64_t rows, int64_t cols, int64_t lda, T* __restrict__ B,
                                 int64_t ldb) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + tx, c = c0 + k;
    tile[k][tx] = (r < rows && c < cols) ? A[c * lda + r] : T(0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + tx, r = r0 + k;
    if (r < rows && c < cols) B[r * ldb + c] = tile[tx][k];
  }
}

// Per column j < k: the sign of the entry of U(:, j) of largest magnitude
// (the first one on ties), as +1 or -1 in sg[j].  One workgroup per column.
template <typename T>
__global__ void pair_sign_kernel(const T* __restrict__ U, int64_t m, int64_t ldu, double* __restrict__ sg) {
  __shared__ double rv[256 / 64];
  __shared__ int64_t ri[256 / 64];
  const int64_t j = blockIdx.x;
  ArgMax b{0.0, -1};
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double a = fabs((double)U[j * ldu + i]);
    if (better(a, i, b.v, b.i)) b = ArgMax{a, i};
  }
  b = block_argmax(b, rv, ri);
  if (threadIdx.x == 0) sg[j] = (b.i >= 0 && (double)U[j * ldu + b.i] < 0.0) ? -1.0 : 1.0;
}

// X(:, j) *= sg[j] for the k columns of X (rows x k, ldx).
template <typename T>
__global__ void scale_cols_kernel(T* __restrict__ X, int64_t rows, int64_t k, int64_t ldx,
                                  const double* __restrict__ sg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < rows && j < k && sg[j] < 0.0) X[j * ldx + i] = -X[j * ldx + i];
}

}  // namespace

template <typename T>
hipError_t transpose(const T* A, int64_t rows, int64_t cols, int64_t lda, T* B, int64_t ldb, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32));
  transpose_kernel<T><<<grid, 256, 0, s>>>(A, rows, cols, lda, B, ldb);
  return hipGetLastError();
}

template <typename T>
hipError_t normalize_pair_signs(T* U, int64_t m, int64_t ldu, T* V, int64_t n, int64_t ldv, int64_t k, double* sg,
                                hipStream_t s) {
  if (k <= 0) return hipSuccess;
  pair_sign_kernel<T><<<(unsigned)k, 256, 0, s>>>(U, m, ldu, sg);
  scale_cols_kernel<T><<<dim3((unsigned)((m + 255) / 256), (unsigned)k), 256, 0, s>>>(U, m, k, ldu, sg);
  scale_cols_kernel<T><<<dim3((unsigned)((n + 255) / 256), (unsigned)k), 256, 0, s>>>(V, n, k, ldv, sg);
  return hipGetLastError();
}

#define INST(T)                                                                                                   \
  template hipError_t transpose<T>(const T*, int64_t, int64_t, int64_t, T*, int64_t, hipStream_t);                \
  template hipError_t normalize_pair_signs<T>(T*, int64_t, int64_t, T*, int64_t, int64_t, int64_t, double*,       \
                                              hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
