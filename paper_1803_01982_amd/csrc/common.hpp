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

// Lane exchanges inside a row of 16 lanes through DPP (no LDS round trip).
// Partners: xor 1 and xor 2 (quad permutations), i <-> 7 - i inside each
// half row and i <-> 15 - i inside the row; each pairs lanes that differ in
// bit 0, 1, 2 or 3 respectively.
enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ inline int64_t dpp_mov(int64_t v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xF, 0xF, true);
  return (int64_t)(((uint64_t)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over each row of 16 lanes; every lane of the row gets the same value
// (each level adds two equal-content partial sums, in either order).
__device__ inline double row16_sum(double v) {
  v += dpp_mov<kDppXor1>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppHalfMirror>(v);
  v += dpp_mov<kDppMirror>(v);
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
// Every workgroup announces its arrival by storing the barrier's epoch into
// a flag of its own (one 128-byte line per workgroup), and wave 0 of every
// workgroup polls all the flags with relaxed loads, one flag per lane, until
// each holds at least the epoch.  No atomic read-modify-write is on the
// critical path: a barrier costs the flag store plus one round of loads.
//
// On gfx950 an agent-scope release is an L2 write-back and an acquire an L2
// invalidate, so only thread 0 of each workgroup fences: the workgroup
// barrier before its release orders every wave's earlier accesses, and its
// acquire (an invalidate of the CU's caches) precedes every wave's later
// ones through the closing workgroup barrier.  Flags only grow, so a
// workgroup that is already one barrier ahead still satisfies the test.
//
// `sync` (kSyncWords words, zeroed before each launch) holds the flags;
// every wait is bounded: past the spin limit the workgroup raises `error`
// and returns false, and every other workgroup then leaves within one more
// bounded wait, so the grid always drains.
constexpr int kFlagStride = 32;  // words between the flags of two workgroups
constexpr int kMaxGridBlocks = 256;
constexpr int kSyncWords = kFlagStride * kMaxGridBlocks;
constexpr unsigned kSpinLimit = 1u << 22;

struct GridSync {
  unsigned* sync;   // flag of workgroup q at sync[kFlagStride * q]
  unsigned* error;
  unsigned nblocks;
};

__device__ inline bool grid_barrier(const GridSync& gs, unsigned& epoch) {
  __shared__ int s_ok;
  __syncthreads();
  ++epoch;
  if (gs.nblocks == 1) return true;  // one workgroup: the workgroup barrier suffices
  if (threadIdx.x < kWave) {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(gs.sync + kFlagStride * blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      bool here = true;
      for (unsigned q = threadIdx.x; q < gs.nblocks; q += kWave)
        here = here && __hip_atomic_load(gs.sync + kFlagStride * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      if (__all(here)) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0) {
        const bool bad = __hip_atomic_load(gs.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (__any(bad) || spins > kSpinLimit) {
          if (threadIdx.x == 0) __hip_atomic_fetch_or(gs.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_ok = ok;
    }
  }
  __syncthreads();
  return s_ok != 0;
}

// ------------------------------------------------------- write-once slots
// A slot exists once per exchange (step, column, workgroup), is filled with
// kVoid before the launch and is written exactly once with a relaxed
// agent-scope atomic store: a slot that no longer holds kVoid holds its final
// value, so a reader needs neither a grid barrier nor a fence, only a bounded
// poll with relaxed agent-scope atomic loads.  Doubles travel as their bits;
// the bit pattern kVoid (a signalling NaN with a payload, which no arithmetic
// produces) is replaced by the default NaN before it is posted.
constexpr uint64_t kVoid = 0xFFF4DEADBEEF0001ull;

__device__ inline void post_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t peek_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t slot_bits(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return b == kVoid ? 0x7FF8000000000000ull : b;
}
__device__ inline double slot_double(uint64_t b) { return __longlong_as_double((long long)b); }

// ------------------------------------------------------------ misc kernels
__global__ void fill_u32(unsigned* p, int n, unsigned v);

}  // namespace ffsrqr
