// Gaussian test matrix Omega (Algorithm 2, first step), the random probes of
// the SRQR test's g2 estimate (Algorithm 4) and small fill kernels.
//
// Omega[i, t] comes from one Philox4x64-10 block (Salmon, Moraes, Dror, Shaw,
// SC'11) with counter (t, i, 0, 0) and key (seed, 0), mapped to N(0,1) by the
// Box-Muller transform of its first two words:
//   u = ((x >> 12) + 0.5) * 2^-52   (exact, inside (0, 1))
//   Omega[i, t] = sqrt(-2 ln u1) * cos(2 pi u2)
// Stored transposed (m x l) so that the sketch GEMM reads both operands along
// the contraction index.  The q-th probe (q >= 1) of a solve, d x c, takes
// entry (t, i) from counter (i, t, q, 0) with the same key and map: the third
// counter word keeps the probe streams apart from Omega's.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

__global__ void fill_u32(unsigned* p, int n, unsigned v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t zero_words(unsigned* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u32<<<(n + 255) / 256, 256, 0, s>>>(p, n, 0u);
  return hipGetLastError();
}

__global__ void fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t fill_void(uint64_t* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  fill_u64<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(p, (int64_t)n, kVoid);
  return hipGetLastError();
}

__device__ inline void philox4x64_10(uint64_t& x0, uint64_t& x1, uint64_t& x2, uint64_t& x3,
                                     uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
}

// Nearest bfloat16 value of x, ties to even, taken from the FP64 value
// directly (no intermediate FP32 rounding): with x = f 2^e, 1/2 <= |f| < 1,
// bfloat16 keeps 8 significant bits, i.e. a spacing of 2^(e - 8) (2^-133
// below 2^-126).  Finite x below the bfloat16 overflow threshold.
__device__ inline __bf16 bf16_from_double(double x) {
  if (x == 0.0) return (__bf16)0.0f;
  int e;
  (void)frexp(x, &e);
  e = e < -125 ? -125 : e;
  const double q = ldexp(rint(ldexp(x, 8 - e)), e - 8);  // exact in FP32 and in BF16
  return (__bf16)(float)q;
}

// N(0,1) from the first two words of a Philox block (Box-Muller)
__device__ inline double gauss_of(uint64_t x0, uint64_t x1) {
  const double u1 = ((double)(x0 >> 12) + 0.5) * 0x1p-52;
  const double u2 = ((double)(x1 >> 12) + 0.5) * 0x1p-52;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

template <typename T>
__device__ inline T omega_value(double z) {
  return (T)z;
}
template <>
__device__ inline __bf16 omega_value<__bf16>(double z) {
  return bf16_from_double(z);
}

template <typename T>
__global__ void omega_kernel(uint64_t seed, int64_t l, int64_t m, T* __restrict__ Ot, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (t >= m || i >= l) return;
  uint64_t x0 = (uint64_t)t, x1 = (uint64_t)i, x2 = 0, x3 = 0;
  philox4x64_10(x0, x1, x2, x3, seed, 0ull);
  Ot[t + i * ldo] = omega_value<T>(gauss_of(x0, x1));
}

// P[t * c + i], t < d, i < c: the q-th probe, FP64
__global__ void probe_kernel(uint64_t seed, uint64_t q, int64_t d, int64_t c, double* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = blockIdx.y;
  if (i >= c || t >= d) return;
  uint64_t x0 = (uint64_t)i, x1 = (uint64_t)t, x2 = q, x3 = 0;
  philox4x64_10(x0, x1, x2, x3, seed, 0ull);
  P[t * c + i] = gauss_of(x0, x1);
}

hipError_t launch_probe(uint64_t seed, uint64_t q, int64_t d, int64_t c, double* P, hipStream_t s) {
  if (d <= 0 || c <= 0) return hipSuccess;
  dim3 grid((unsigned)((c + 255) / 256), (unsigned)d);
  probe_kernel<<<grid, 256, 0, s>>>(seed, q, d, c, P);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_omega(uint64_t seed, int64_t l, int64_t m, T* Ot, int64_t ldo, hipStream_t s) {
  if (l <= 0 || m <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)l);
  omega_kernel<T><<<grid, 256, 0, s>>>(seed, l, m, Ot, ldo);
  return hipGetLastError();
}

template hipError_t launch_omega<double>(uint64_t, int64_t, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_omega<float>(uint64_t, int64_t, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_omega<__bf16>(uint64_t, int64_t, int64_t, __bf16*, int64_t, hipStream_t);

}  // namespace ffsrqr
