// Shared device helpers of the gfx950 Flip-Flop SRQR library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ffsrqr.h"

namespace ffsrqr {

constexpr int kWave = 64;

// Lane layouts of the 16x16x4 MFMA tiles used by the GEMMs (checked by an
// in-bounds probe on gfx950).  Operands: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Results (4 registers r per lane):
//   f32: D[4 * (l / 16) + r][l % 16]
//   f64: D[(l / 16) + 4 * r][l % 16]
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double acc4 __attribute__((ext_vector_type(4)));
  static __device__ inline acc4 fma(double a, double b, acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float acc4 __attribute__((ext_vector_type(4)));
  static __device__ inline acc4 fma(float a, float b, acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over aligned groups of `g` lanes (g a power of two <= 64).
__device__ inline double group_sum(double v, int g) {
  for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide sum; `red` is LDS scratch of at least blockDim.x / 64 doubles.
// Every thread gets the total; the summation order is fixed.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// (value, index) argmax with ties to the smallest index; idx < 0 means empty.
struct ArgMax {
  double v;
  int64_t i;
};
__device__ inline bool better(double v1, int64_t i1, double v2, int64_t i2) {
  if (i2 < 0) return i1 >= 0;
  if (i1 < 0) return false;
  return v1 > v2 || (v1 == v2 && i1 < i2);
}
__device__ inline ArgMax wave_argmax(ArgMax a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double v = __shfl_xor(a.v, o, kWave);
    int64_t i = __shfl_xor(a.i, o, kWave);
    if (better(v, i, a.v, a.i)) { a.v = v; a.i = i; }
  }
  return a;
}
// Block-wide argmax; `rv`, `ri` LDS scratch of blockDim.x / 64 entries.
__device__ inline ArgMax block_argmax(ArgMax a, double* rv, int64_t* ri) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  a = wave_argmax(a);
  __syncthreads();
  if (lane == 0) { rv[w] = a.v; ri[w] = a.i; }
  __syncthreads();
  ArgMax b{0.0, -1};
  for (int i = 0; i < nw; ++i)
    if (better(rv[i], ri[i], b.v, b.i)) { b.v = rv[i]; b.i = ri[i]; }
  return b;
}

// ------------------------------------------------------------ grid barrier
// Device-wide barrier for cooperative (co-resident) launches.
//
// On gfx950 an agent-scope release is an L2 writeback and an agent-scope
// acquire an L2 invalidate, and their cost grows with the number of
// workgroups per XCD, so only one thread per workgroup fences: the
// workgroup barrier before it completes every wave's stores to L2, and the
// invalidate after it covers the CU's vector cache for all waves.  Arrival
// is counted in groups of 16 workgroups, then across groups; the last
// arrival publishes the new generation, which the others poll with relaxed
// loads (no cache maintenance per poll).
//
// `sync` (kSyncWords words, zeroed before each launch) holds the counters;
// every wait is bounded: past the spin limit the block raises `error` and
// returns false, and every other block then leaves within one more bounded
// wait, so the grid always drains.
constexpr int kSyncWords = 1024;
constexpr unsigned kSpinLimit = 1u << 22;
constexpr unsigned kGroup = 16;

struct GridSync {
  unsigned* sync;   // [0]: arrivals of groups, [32]: generation, [64 + 32 g]: group arrivals
  unsigned* error;
  unsigned nblocks;
};

__device__ inline bool grid_barrier(const GridSync& gs, unsigned& epoch) {
  __shared__ int s_ok;
  __syncthreads();
  ++epoch;
  if (gs.nblocks == 1) return true;  // one workgroup: the workgroup barrier suffices
  if (threadIdx.x == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned grp = blockIdx.x / kGroup, ngrp = (gs.nblocks + kGroup - 1) / kGroup;
    const unsigned gsize = (grp == ngrp - 1) ? gs.nblocks - grp * kGroup : kGroup;
    const unsigned old = __hip_atomic_fetch_add(gs.sync + 64 + 32 * grp, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1) {
      const unsigned o2 = __hip_atomic_fetch_add(gs.sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == epoch * ngrp - 1)
        __hip_atomic_store(gs.sync + 32, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned spins = 0;
    while (__hip_atomic_load(gs.sync + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0) {
        if (__hip_atomic_load(gs.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            spins > kSpinLimit) {
          __hip_atomic_fetch_or(gs.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// ------------------------------------------------------------ misc kernels
__global__ void fill_u32(unsigned* p, int n, unsigned v);

}  // namespace ffsrqr
