// Tensor unfoldings for the ST-HOSVD driver (Section 2, tensor notation).
//
// A tensor of order d <= 8 with dimensions n_0..n_{d-1} is held as one of
// its unfoldings: the mode-a unfolding stores entry (i_0..i_{d-1}) at
//   i_a + n_a * c_a,  c_a = the Fortran-order linear index of the other
//                           indices (i_0..i_{a-1}, i_{a+1}..i_{d-1}),
// so the mode-0 unfolding is the tensor in Fortran order.  reunfold copies a
// tensor from its mode-a unfolding to its mode-b unfolding: one thread per
// destination entry (coalesced stores), the source read by gather.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

struct TensorShape {
  int d;
  int64_t n[kMaxTensorOrder];
};

template <typename T>
__global__ void reunfold_kernel(const T* __restrict__ src, int a, T* __restrict__ dst, int b, TensorShape t,
                                int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    int64_t idx[kMaxTensorOrder];
    int64_t r = e / t.n[b];
#pragma unroll
    for (int k = 0; k < kMaxTensorOrder; ++k) {
      if (k >= t.d) break;
      if (k == b) {
        idx[k] = e % t.n[b];
      } else {
        idx[k] = r % t.n[k];
        r /= t.n[k];
      }
    }
    int64_t c = 0, s = 1, ia = 0;
#pragma unroll
    for (int k = 0; k < kMaxTensorOrder; ++k) {
      if (k >= t.d) break;
      if (k == a) {
        ia = idx[k];
      } else {
        c += idx[k] * s;
        s *= t.n[k];
      }
    }
    dst[e] = src[ia + t.n[a] * c];
  }
}

}  // namespace

template <typename T>
hipError_t reunfold(const T* src, int a, T* dst, int b, int d, const int64_t* dims, hipStream_t s) {
  if (d < 1 || d > kMaxTensorOrder || a < 0 || a >= d || b < 0 || b >= d) return hipErrorInvalidValue;
  TensorShape t;
  t.d = d;
  int64_t total = 1;
  for (int k = 0; k < kMaxTensorOrder; ++k) {
    t.n[k] = k < d ? dims[k] : 1;
    if (k < d) total *= dims[k];
  }
  if (total <= 0) return hipSuccess;
  if (a == b) return hipMemcpyAsync(dst, src, (size_t)total * sizeof(T), hipMemcpyDeviceToDevice, s);
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  reunfold_kernel<T><<<(unsigned)blocks, 256, 0, s>>>(src, a, dst, b, t, total);
  return hipGetLastError();
}

template hipError_t reunfold<double>(const double*, int, double*, int, int, const int64_t*, hipStream_t);
template hipError_t reunfold<float>(const float*, int, float*, int, int, const int64_t*, hipStream_t);

}  // namespace ffsrqr
