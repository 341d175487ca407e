// Partial QRCP on the sketch B (Algorithm 1 applied to B for l steps; the
// pivot search of Algorithm 2).
//
// One cooperative launch on as few 1024-thread workgroups as LDS allows.
// Workgroup g owns a
// contiguous slice of nc columns of B, kept in LDS (or in a global copy when
// the slice does not fit) for all l steps.  Step j:
//   1. each workgroup publishes its best active column (largest residual
//      norm, ties to the smallest original index), its runner-up norm, and
//      that column's rows j..l-1;
//   2. one grid barrier;
//   3. every workgroup reads the candidates and takes the same winner
//      (fixed comparison order, so no broadcast is needed), builds the
//      Householder reflector of the winner's rows j..l-1 (LAPACK xLARFG
//      convention, FP64), retires the winner and applies the reflector to
//      its own active columns, recomputing their residual norms from
//      scratch over rows j+1..l-1 (the same definition as the oracle; no
//      downdating drift to guard against).
// Candidate slots are double-buffered by step parity, so one barrier per
// step suffices.  The register-resident variant below (l <= 544) replaces
// the barrier by write-once slots per step.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 1024;

struct QrcpSlots {
  double* r;      // [2][G]
  double* r2;     // [2][G]
  int64_t* idx;   // [2][G]
  double* col;    // [2][G][l]
};

// Column stride of the B slices: l rounded up so that it is an odd number of
// 8-byte words.
__host__ __device__ inline int ldbl_for(int64_t l, size_t tsize) {
  if (tsize == 8) return (int)(l | 1);
  int64_t w = (l + 1) / 2;  // 8-byte words per float column
  if (!(w & 1)) ++w;
  return (int)(2 * w);
}

// Top-2 of (value, index) pairs: the best pair (largest value, ties to the
// smallest index) and the largest other value (v2 < 0 when there is none).
struct Top2 {
  double v1;
  int64_t i1;
  double v2;
};
__device__ inline Top2 top2_merge(Top2 a, Top2 b) {
  if (better(b.v1, b.i1, a.v1, a.i1)) {
    const Top2 t = a;
    a = b;
    b = t;
  }
  // a holds the overall best; the runner-up is b's best or either second
  double v2 = a.v2;
  if (b.i1 >= 0 && b.v1 > v2) v2 = b.v1;
  if (b.v2 > v2) v2 = b.v2;
  return Top2{a.v1, a.i1, v2};
}
__device__ inline Top2 wave_top2(Top2 x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Top2 y{__shfl_xor(x.v1, o, kWave), __shfl_xor(x.i1, o, kWave), __shfl_xor(x.v2, o, kWave)};
    x = top2_merge(x, y);
  }
  return x;
}

// Top-2 over each row of 16 lanes through DPP exchanges (the merge is
// commutative and associative, so every lane of the row ends with the same
// result).
template <int CTRL>
__device__ inline Top2 top2_dpp(Top2 x) {
  const Top2 y{dpp_mov<CTRL>(x.v1), dpp_mov<CTRL>(x.i1), dpp_mov<CTRL>(x.v2)};
  return top2_merge(x, y);
}
__device__ inline Top2 row16_top2(Top2 x) {
  x = top2_dpp<kDppXor1>(x);
  x = top2_dpp<kDppXor2>(x);
  x = top2_dpp<kDppHalfMirror>(x);
  return top2_dpp<kDppMirror>(x);
}

__device__ inline int group_size_for(int nc) {
  int g = 1;
  while (g * 2 * nc <= NT && g < 64) g *= 2;
  return g;
}

template <typename T, bool IN_LDS>
__global__ __launch_bounds__(NT) void qrcp_kernel(const T* __restrict__ B, int64_t ldb, int l, int64_t n,
                                                  int nc, T* __restrict__ Bw, QrcpSlots sl,
                                                  int64_t* __restrict__ piv, double* __restrict__ margins,
                                                  GridSync gs) {
  extern __shared__ double smem[];
  __shared__ double redv[NT / 64];
  __shared__ int64_t redi[NT / 64];
  __shared__ double s_bcast[4];
  __shared__ int64_t s_ibcast[2];

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int64_t c0 = (int64_t)g * nc;
  const int ncl = (int)((n - c0) < nc ? ((n - c0) > 0 ? (n - c0) : 0) : nc);
  double* v = smem;            // l
  double* rloc = v + l;        // nc
  int* act = (int*)(rloc + nc);  // nc (padded to an even count)
  // column slices with an odd stride (in 8-byte words) so that lanes working
  // on different columns fall in different LDS banks
  const int ldb_l = ldbl_for(l, sizeof(T));
  T* Bl = IN_LDS ? (T*)(smem + l + nc + (nc + 1) / 2) : Bw + (int64_t)g * nc * ldb_l;

  for (int64_t e = tid; e < (int64_t)ncl * l; e += NT) {
    const int c = (int)(e / l), i = (int)(e % l);
    Bl[(int64_t)c * ldb_l + i] = B[(c0 + c) * ldb + i];
  }
  for (int c = tid; c < nc; c += NT) act[c] = c < ncl ? 1 : 0;
  const int gsz = group_size_for(nc), ngrp = NT / gsz, q = tid % gsz;
  __syncthreads();
  for (int c = tid / gsz; c < ncl; c += ngrp) {
    double s = 0.0;
    for (int i = q; i < l; i += gsz) {
      const double b = (double)Bl[(int64_t)c * ldb_l + i];
      s += b * b;
    }
    s = group_sum(s, gsz);
    if (q == 0) rloc[c] = s;
  }
  __syncthreads();

  unsigned epoch = 0;
  for (int j = 0; j < l; ++j) {
    const int par = j & 1;
    // ---- 1. local best and runner-up among the active columns (wave 0)
    if (tid < kWave) {
      Top2 t{0.0, -1, -1.0};
      for (int c = tid; c < ncl; c += kWave)
        if (act[c]) t = top2_merge(t, Top2{rloc[c], c0 + c, -1.0});
      t = wave_top2(t);
      if (tid == 0) {
        sl.r[par * G + g] = t.v1;
        sl.idx[par * G + g] = t.i1;
        sl.r2[par * G + g] = t.v2;
        s_ibcast[0] = t.i1;
      }
    }
    __syncthreads();
    {
      const int64_t bi = s_ibcast[0];
      if (bi >= 0) {
        const int cb = (int)(bi - c0);
        double* dst = sl.col + ((int64_t)par * G + g) * l;
        for (int i = j + tid; i < l; i += NT) dst[i] = (double)Bl[(int64_t)cb * ldb_l + i];
      }
    }
    // ---- 2. exchange
    if (!grid_barrier(gs, epoch)) return;
    // ---- 3. global winner and runner-up (identical in every workgroup; wave 0)
    if (tid < kWave) {
      Top2 t{0.0, -1, -1.0};
      for (int q = tid; q < G; q += kWave)
        t = top2_merge(t, Top2{sl.r[par * G + q], sl.idx[par * G + q], sl.r2[par * G + q]});
      t = wave_top2(t);
      if (tid == 0) {
        s_ibcast[1] = t.i1;
        s_bcast[0] = t.v1;
        if (g == 0) {
          piv[j] = t.i1;
          double mg;
          if (n - j <= 1) mg = 1.0;
          else if (t.v1 > 0.0) mg = (t.v1 - (t.v2 > 0.0 ? t.v2 : 0.0)) / t.v1;
          else mg = 0.0;
          margins[j] = mg;
        }
      }
    }
    __syncthreads();
    const ArgMax w{s_bcast[0], s_ibcast[1]};
    const int wg = (int)(w.i / nc);
    const double* src = sl.col + ((int64_t)par * G + wg) * l;
    for (int i = j + tid; i < l; i += NT) v[i] = src[i];
    __syncthreads();
    double xs = 0.0;
    for (int i = j + 1 + tid; i < l; i += NT) xs += v[i] * v[i];
    const double xnorm2 = block_sum(xs, redv);
    const double x0 = v[j];
    double tau = 0.0;
    if (xnorm2 > 0.0) {
      const double beta = -copysign(sqrt(x0 * x0 + xnorm2), x0);
      tau = (beta - x0) / beta;
      const double scale = 1.0 / (x0 - beta);
      __syncthreads();
      for (int i = j + 1 + tid; i < l; i += NT) v[i] *= scale;
      if (tid == 0) v[j] = 1.0;
    }
    if (wg == g && tid == 0) act[w.i - c0] = 0;
    __syncthreads();
    // ---- update the active local columns, recompute residual norms
    for (int c = tid / gsz; c < ncl; c += ngrp) {
      if (!act[c]) continue;
      T* col = Bl + (int64_t)c * ldb_l;
      if (tau != 0.0) {
        double s = 0.0;
        for (int i = j + q; i < l; i += gsz) s += v[i] * (double)col[i];
        s = group_sum(s, gsz) * tau;
        for (int i = j + q; i < l; i += gsz) col[i] = (T)((double)col[i] - s * v[i]);
      }
      double r = 0.0;
      for (int i = j + 1 + q; i < l; i += gsz) {
        const double b = (double)col[i];
        r += b * b;
      }
      r = group_sum(r, gsz);
      if (q == 0) rloc[c] = r;
    }
    __syncthreads();
  }
}

// Register-resident variant for l <= 16 NR: sixteen threads per column, each
// holding rows q, q + 16, ... of its column (and of CB columns in all) in
// registers, so that the update and the norm recomputation of a step touch
// no LDS except the broadcast reflector.
//
// The workgroups exchange their candidates through slots that exist once per
// step and workgroup, are filled with kVoid before the launch and are written
// exactly once (relaxed agent-scope atomics): a slot that no longer holds
// kVoid holds its final value, so a reader needs neither a grid barrier nor a
// fence, only a bounded poll.  Per step:
//   1. every wave merges the top-2 of its four column groups and posts it to
//      LDS; after one workgroup barrier every wave merges the sixteen posts;
//      the owner of the local winner writes the column's rows j..l-1 to its
//      column slot and wave 0 the candidate (best norm, runner-up, index);
//   2. wave 0 polls the candidate slots of the step until every workgroup's
//      is there, merges them (fixed order, so every workgroup takes the same
//      winner), polls the winner's column slot, builds the reflector (LAPACK
//      xLARFG convention) and broadcasts it through LDS;
//   3. every active column is updated and its residual norm over rows
//      j+1..l-1 recomputed from scratch (sums over the 16 lanes of its group).
// A poll past the spin limit raises `error` and ends the workgroup; the
// others see the error word within their own bounded polls.
struct QrcpPost {
  uint64_t* cand;  // [3][l][G]: best norm, runner-up norm, best index
  uint64_t* col;   // rows j..l-1 of the best column of (j, g) at tri(j) G + g (l - j)
};

// Rows of the column slots of the steps before j: sum over j' < j of (l - j').
__device__ inline int64_t tri_rows(int j, int l) { return (int64_t)j * l - (int64_t)j * (j - 1) / 2; }

// NL > 0 (with CB = 1): the rows q + 16 s with s < NL, the ones that retire
// first, live in LDS (xs[s][tid], 8 NL KiB per workgroup) and only the other
// NR - NL rows in registers, which keeps the l <= 544 variant within 128
// VGPRs; at step j the LDS rows below 16 (j / 16) are dead and skipped.
template <typename T, int NR, int CB, int NL>
__global__ __launch_bounds__(NT) void qrcp_reg_kernel(const T* __restrict__ B, int64_t ldb, int l, int64_t n,
                                                      QrcpPost post, int64_t* __restrict__ piv,
                                                      double* __restrict__ margins, unsigned* __restrict__ error) {
  constexpr int TPC = 16, CPB = NT / TPC;  // threads per column, columns per batch
  constexpr int GQ = kMaxGridBlocks / kWave;  // candidate slots per lane
  constexpr int NRR = NR - NL;                // rows per thread held in registers
  static_assert(NL == 0 || CB == 1, "LDS rows with one column per thread group");
  __shared__ double v[TPC * NR];
  __shared__ double s_tv1[NT / 64], s_tv2[NT / 64];
  __shared__ int64_t s_ti1[NT / 64];
  __shared__ double s_tau;
  __shared__ int64_t s_win;
  __shared__ int s_abort;
  extern __shared__ double xs[];  // [NL][NT]
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, q = tid & (TPC - 1), cl = tid / TPC;
  const int64_t c0 = (int64_t)g * CPB * CB;
  double x[CB][NRR], rn[CB];
  int64_t col[CB];
  bool act[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    col[b] = c0 + (int64_t)b * CPB + cl;
    act[b] = col[b] < n;
    double s2 = 0.0;
    for (int s = 0; s < NL; ++s) {
      const int i = q + TPC * s;
      const double y = (act[b] && i < l) ? (double)B[col[b] * ldb + i] : 0.0;
      xs[s * NT + tid] = y;
      s2 += y * y;
    }
#pragma unroll
    for (int s = 0; s < NRR; ++s) {
      const int i = q + TPC * (s + NL);
      x[b][s] = (act[b] && i < l) ? (double)B[col[b] * ldb + i] : 0.0;
      s2 += x[b][s] * x[b][s];
    }
    rn[b] = row16_sum(s2);
  }
  if (tid == 0) s_abort = 0;
  for (int j = 0; j < l; ++j) {
    // ---- 1. local best and runner-up
    Top2 t{0.0, -1, -1.0};
#pragma unroll
    for (int b = 0; b < CB; ++b)
      if (act[b]) t = top2_merge(t, Top2{rn[b], col[b], -1.0});
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      const Top2 y{__shfl_xor(t.v1, o, kWave), __shfl_xor(t.i1, o, kWave), __shfl_xor(t.v2, o, kWave)};
      t = top2_merge(t, y);
    }
    if (lane == 0) {
      s_tv1[wave] = t.v1;
      s_ti1[wave] = t.i1;
      s_tv2[wave] = t.v2;
    }
    __syncthreads();
    const int64_t tb = tri_rows(j, l) * G;
    {
      static_assert(NT / 64 == 16, "one post per lane of the first row");
      Top2 u{0.0, -1, -1.0};
      if (lane < NT / 64) u = Top2{s_tv1[lane], s_ti1[lane], s_tv2[lane]};
      u = row16_top2(u);
      const int64_t bi = __shfl(u.i1, 0, kWave);
      // the owner group of the local winner posts rows j..l-1 of its column
      uint64_t* dst = post.col + tb + (int64_t)g * (l - j) - j;
#pragma unroll
      for (int b = 0; b < CB; ++b)
        if (bi >= 0 && col[b] == bi) {
          for (int s = j / TPC; s < NL; ++s) {
            const int i = q + TPC * s;
            if (i >= j && i < l) post_u64(dst + i, slot_bits(xs[s * NT + tid]));
          }
#pragma unroll
          for (int s = 0; s < NRR; ++s) {
            const int i = q + TPC * (s + NL);
            if (i >= j && i < l) post_u64(dst + i, slot_bits(x[b][s]));
          }
        }
      if (wave == 0 && lane == 0) {
        post_u64(post.cand + (int64_t)j * G + g, slot_bits(u.v1));
        post_u64(post.cand + ((int64_t)l + j) * G + g, slot_bits(u.v2));
        post_u64(post.cand + (2 * (int64_t)l + j) * G + g, (uint64_t)u.i1);
      }
    }
    // ---- 2. global winner, its reflector (wave 0)
    if (wave == 0) {
      Top2 u{0.0, -1, -1.0};
      bool ok = true;
      unsigned spins = 0;
      for (;;) {
        bool here = true;
        u = Top2{0.0, -1, -1.0};
#pragma unroll
        for (int k = 0; k < GQ; ++k) {
          const int qq = lane + kWave * k;
          if (qq < G) {
            const uint64_t b1 = peek_u64(post.cand + (int64_t)j * G + qq);
            const uint64_t b2 = peek_u64(post.cand + ((int64_t)l + j) * G + qq);
            const uint64_t bi = peek_u64(post.cand + (2 * (int64_t)l + j) * G + qq);
            here = here && b1 != kVoid && b2 != kVoid && bi != kVoid;
            u = top2_merge(u, Top2{slot_double(b1), (int64_t)bi, slot_double(b2)});
          }
        }
        if (__all(here)) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0) {
          const bool bad = __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
          if (__any(bad) || spins > kSpinLimit) {
            ok = false;
            break;
          }
        }
      }
      u = row16_top2(u);
#pragma unroll
      for (int o = 16; o < 64; o <<= 1) {
        const Top2 y{__shfl_xor(u.v1, o, kWave), __shfl_xor(u.i1, o, kWave), __shfl_xor(u.v2, o, kWave)};
        u = top2_merge(u, y);
      }
      const int64_t wi = __shfl(u.i1, 0, kWave);
      if (ok && lane == 0 && g == 0) {
        piv[j] = wi;
        double mg;
        if (n - j <= 1) mg = 1.0;
        else if (u.v1 > 0.0) mg = (u.v1 - (u.v2 > 0.0 ? u.v2 : 0.0)) / u.v1;
        else mg = 0.0;
        margins[j] = mg;
      }
      // the winner's rows j..l-1 (posted by the workgroup that owns it)
      const int wg = ok && wi >= 0 ? (int)(wi / (CPB * CB)) : 0;
      const uint64_t* src = post.col + tb + (int64_t)wg * (l - j) - j;
      // the winner's rows go straight into the reflector buffer v (this
      // wave's own entries i = lane + 64 s), so no register copy is held
      constexpr int WS = (TPC * NR + 63) / 64;
      for (spins = 0; ok;) {
        bool here = true;
#pragma unroll
        for (int s = 0; s < WS; ++s) {
          const int i = lane + 64 * s;
          uint64_t bits = 0;
          if (i >= j && i < l) {
            bits = peek_u64(src + i);
            here = here && bits != kVoid;
          }
          if (i < TPC * NR) v[i] = slot_double(bits);
        }
        if (__all(here)) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0) {
          const bool bad = __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
          if (__any(bad) || spins > kSpinLimit) ok = false;
        }
      }
      if (!ok) {
        if (lane == 0) {
          __hip_atomic_fetch_or(error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_abort = 1;
        }
      } else {
        double xs = 0.0;
#pragma unroll
        for (int s = 0; s < WS; ++s) {
          const int i = lane + 64 * s;
          if (i > j && i < l) xs += v[i] * v[i];
        }
        const double xnorm2 = wave_sum(xs);
        const double x0v = v[j];  // written by lane j % 64 above (same wave, in order)
        double tau = 0.0, scale = 0.0;
        if (xnorm2 > 0.0) {
          const double beta = -copysign(sqrt(x0v * x0v + xnorm2), x0v);
          tau = (beta - x0v) / beta;
          scale = 1.0 / (x0v - beta);
        }
#pragma unroll
        for (int s = 0; s < WS; ++s) {
          const int i = lane + 64 * s;
          if (i < TPC * NR) v[i] = (i < j || i >= l) ? 0.0 : (i == j ? 1.0 : (tau != 0.0 ? v[i] * scale : v[i]));
        }
        if (lane == 0) {
          s_tau = tau;
          s_win = wi;
        }
      }
    }
    __syncthreads();
    if (s_abort) return;
    // ---- 3. update the active columns, recompute their residual norms
    const double tau = s_tau;
    const int64_t wi = s_win;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if (col[b] == wi) act[b] = false;
      if (!act[b]) continue;
      const int s0 = j / TPC;  // LDS rows below 16 s0 are dead (v is zero there)
      if (tau != 0.0) {
        double dt = 0.0;
        for (int s = s0; s < NL; ++s) dt += v[q + TPC * s] * xs[s * NT + tid];
#pragma unroll
        for (int s = 0; s < NRR; ++s) dt += v[q + TPC * (s + NL)] * x[b][s];
        const double f = row16_sum(dt) * tau;
        // compiler barrier: the update reads the reflector from LDS again
        // rather than keeping all of it live in registers beside the column
        asm volatile("" ::: "memory");
        for (int s = s0; s < NL; ++s) xs[s * NT + tid] -= f * v[q + TPC * s];
#pragma unroll
        for (int s = 0; s < NRR; ++s) x[b][s] -= f * v[q + TPC * (s + NL)];
      }
      double r = 0.0;
      for (int s = s0; s < NL; ++s) {
        const int i = q + TPC * s;
        const double y = xs[s * NT + tid];
        if (i > j) r += y * y;
      }
#pragma unroll
      for (int s = 0; s < NRR; ++s) {
        const int i = q + TPC * (s + NL);
        if (i > j) r += x[b][s] * x[b][s];
      }
      rn[b] = row16_sum(r);
    }
  }
}

// Words of the candidate and column slots of the register variant.
inline size_t post_words(int64_t l, int G) { return (size_t)G * (3 * l + l * (l + 1) / 2); }

// Fewest workgroups whose column slices of B still fit in LDS: the per-step
// grid barrier costs more with more workgroups, while the work per step is
// small.  When B does not fit in the LDS of the whole chip, the slices live
// in a global copy instead and one workgroup per CU is used.
void choose(int64_t l, int64_t n, int num_cu, size_t lds_max, size_t tsize, int* nc, int* G, bool* in_lds,
            size_t* lds) {
  const size_t fixed = (size_t)l * sizeof(double) + 2048;
  const size_t per_col = (size_t)ldbl_for(l, tsize) * tsize + sizeof(double) + sizeof(int);
  int64_t c = lds_max > fixed ? (int64_t)((lds_max - fixed) / per_col) : 0;
  if (c > n) c = n;
  if (c >= 1 && (n + c - 1) / c <= num_cu) {
    *in_lds = true;
  } else {
    c = (n + num_cu - 1) / num_cu;
    *in_lds = false;
  }
  if (c < 1) c = 1;
  *nc = (int)c;
  *G = (int)((n + c - 1) / c);
  const size_t base = (size_t)(l + c + (c + 1) / 2) * sizeof(double);
  *lds = *in_lds ? base + (size_t)c * ldbl_for(l, tsize) * tsize : base;
}


// Register variant: rows per thread NR (l <= 16 NR) and columns per thread
// CB, fewest workgroups first (cheaper grid barriers); G <= num_cu.
bool reg_choice(int64_t l, int64_t n, int num_cu, int* NR, int* CB, int* G) {
  static const int nrs[] = {2, 4, 8, 18, 34};
  static const int cbs[] = {4, 4, 2, 1, 1};
  for (int k = 0; k < 5; ++k) {
    if (l > 16 * nrs[k]) continue;
    const int64_t per = (int64_t)(NT / 16) * cbs[k];
    const int64_t g = (n + per - 1) / per;
    if (g > num_cu) return false;
    *NR = nrs[k];
    *CB = cbs[k];
    *G = (int)g;
    return true;
  }
  return false;
}

// rows per thread kept in LDS by the variant for NR rows per thread
inline int reg_lds_rows(int NR) { return NR == 34 ? 16 : 0; }

template <typename T>
const void* reg_kernel(int NR) {
  switch (NR) {
    case 2: return (const void*)qrcp_reg_kernel<T, 2, 4, 0>;
    case 4: return (const void*)qrcp_reg_kernel<T, 4, 4, 0>;
    case 8: return (const void*)qrcp_reg_kernel<T, 8, 2, 0>;
    case 18: return (const void*)qrcp_reg_kernel<T, 18, 1, 0>;
    case 34: return (const void*)qrcp_reg_kernel<T, 34, 1, 16>;
  }
  return nullptr;
}

}  // namespace

template <typename T>
size_t qrcp_scratch(int64_t l, int64_t n, const DeviceInfo& d) {
  int nc, G, NR, CB, Gr;
  bool in_lds;
  size_t lds;
  choose(l, n, d.num_cu, d.lds_max, sizeof(T), &nc, &G, &in_lds, &lds);
  size_t b = (size_t)2 * G * (3 * sizeof(double) + l * sizeof(double)) + 4 * 256;
  if (!in_lds) b += (size_t)G * nc * ldbl_for(l, sizeof(T)) * sizeof(T) + 256;
  if (reg_choice(l, n, d.num_cu, &NR, &CB, &Gr)) b = std::max(b, post_words(l, Gr) * sizeof(uint64_t) + 256);
  return b + kSyncWords * sizeof(unsigned) + 1024;
}

template <typename T>
hipError_t qrcp(const T* B, int64_t l, int64_t n, int64_t ldb, int64_t* piv, double* margins, Arena& ar,
                unsigned* err, const DeviceInfo& d, hipStream_t s) {
  if (l <= 0) return hipSuccess;
  int NR, CB, Gr;
  if (reg_choice(l, n, d.num_cu, &NR, &CB, &Gr)) {
    if (Gr > kMaxGridBlocks) return hipErrorInvalidValue;
    const size_t words = post_words(l, Gr);
    QrcpPost post;
    post.cand = ar.take<uint64_t>(words);
    if (!post.cand) return hipErrorOutOfMemory;
    post.col = post.cand + (size_t)3 * l * Gr;
    hipError_t e = fill_void(post.cand, words, s);
    if (e != hipSuccess) return e;
    int li = (int)l;
    int64_t ln = n, lldb = ldb;
    void* args[] = {(void*)&B, (void*)&lldb, (void*)&li, (void*)&ln, (void*)&post, (void*)&piv, (void*)&margins,
                    (void*)&err};
    const void* fn = reg_kernel<T>(NR);
    const size_t xlds = (size_t)reg_lds_rows(NR) * NT * sizeof(double);
    if (xlds > 65536) {
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)xlds);
      if (e != hipSuccess) return e;
    }
    return hipLaunchCooperativeKernel(fn, dim3(Gr), dim3(NT), args, (unsigned)xlds, s);
  }
  int nc, G;
  bool in_lds;
  size_t lds;
  choose(l, n, d.num_cu, d.lds_max, sizeof(T), &nc, &G, &in_lds, &lds);
  QrcpSlots sl;
  sl.r = ar.take<double>(2 * G);
  sl.r2 = ar.take<double>(2 * G);
  sl.idx = ar.take<int64_t>(2 * G);
  sl.col = ar.take<double>((size_t)2 * G * l);
  unsigned* counter = ar.take<unsigned>(kSyncWords);
  T* Bw = in_lds ? nullptr : ar.take<T>((size_t)G * nc * ldbl_for(l, sizeof(T)));
  if (!sl.r || !sl.r2 || !sl.idx || !sl.col || !counter || (!in_lds && !Bw)) return hipErrorOutOfMemory;
  hipError_t e = zero_words(counter, kSyncWords, s);
  if (e != hipSuccess) return e;
  if (G > kMaxGridBlocks) return hipErrorInvalidValue;
  GridSync gs{counter, err, (unsigned)G};
  int li = (int)l;
  int64_t ln = n, lldb = ldb;
  void* args[] = {(void*)&B, (void*)&lldb, (void*)&li, (void*)&ln, (void*)&nc, (void*)&Bw,
                  (void*)&sl, (void*)&piv, (void*)&margins, (void*)&gs};
  const void* fn = in_lds ? (const void*)qrcp_kernel<T, true> : (const void*)qrcp_kernel<T, false>;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, (unsigned)lds, s);
}

template size_t qrcp_scratch<double>(int64_t, int64_t, const DeviceInfo&);
template size_t qrcp_scratch<float>(int64_t, int64_t, const DeviceInfo&);
template hipError_t qrcp<double>(const double*, int64_t, int64_t, int64_t, int64_t*, double*, Arena&, unsigned*,
                                 const DeviceInfo&, hipStream_t);
template hipError_t qrcp<float>(const float*, int64_t, int64_t, int64_t, int64_t*, double*, Arena&, unsigned*,
                                const DeviceInfo&, hipStream_t);

}  // namespace ffsrqr
