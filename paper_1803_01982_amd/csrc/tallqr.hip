// Householder QR without pivoting of a tall matrix P (mrows x c, mrows >= c).
// Used twice on the path:
//   * the QR of the l pivoted columns A(:, S) (Algorithm 2, QR of the
//     pivoted block; compact WY representation Q = I - Y T Y^T of Section 2.1);
//   * the flip-flop step, QR of R^T (n x l) (Section 3.1).
//
// One cooperative launch factors the matrix.  Workgroup g owns the row block
// [g*rb, (g+1)*rb); the rows of the current 16-column panel stay in
// registers.  Workgroups exchange data only through write-once slots (no
// grid barrier).  Per panel of NB = 16 columns:
//   reflectors: every workgroup posts the Gram matrix of the panel columns
//     over its active rows (rows >= p0), and the owners of rows p0 .. p1-1
//     post those rows (B).  The Grams are summed in a fixed order (two
//     levels), and every workgroup runs the panel's Householder steps (LAPACK
//     xLARFG convention) on (G, B) itself: the Gram matrix over the active
//     rows is invariant under the reflectors, so the dots of column j with
//     the later columns below row jc are G(j, s) minus the products over the
//     top rows 0 .. j of B, which the recurrence keeps transformed.  Each
//     workgroup then applies the reflectors to its own rows.  A column whose
//     remaining squared norm would be recovered with a cancellation worse
//     than 1/16 of G(j, j) stops the recurrence; it and the rest of the
//     panel take one exact reduction per column (partial dots posted to
//     slots, summed in a fixed order);
//   panel end: Z = Y_p^T [Y_p | P_trail] is reduce-scattered and gathered
//     through slots, each workgroup forms the panel's T_p (LAPACK xLARFT,
//     forward, columnwise) from the Gram part and applies
//     P_trail -= Y_p (T_p^T (Y_p^T P_trail)) to its own rows.
//
// Q = H_1 ... H_c [I; 0] = [I; 0] - Y T Y(0:c, :)^T (compact WY form of the
// whole product, Section 2.1) is then formed by three tiled kernels over the
// whole chip instead of panel by panel: S = Y^T Y (split over row chunks,
// then summed in a fixed order); M = T Y(0:c, :)^T by blocked back
// substitution with T^-1 = striu(S) + diag(1/tau) (the identity behind the
// compact WY form; tau = 0 drops the reflector), with the signs that make
// diag(R) >= 0 folded in; Q = [I; 0] diag(sgn) - Y M.  All arithmetic is
// FP64; P and Q are stored as T.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256, NB = 16, NW = NT / 64;
using MF = Mfma<double>;

struct TqSlots {
  uint64_t* gram;   // [npan][G][NB * NB] write-once: Gram of the panel's active rows of workgroup g
  uint64_t* gram2;  // [npan][ceil(G / 8)][NB * NB] write-once: sums of the Grams of eight workgroups
  uint64_t* rowv;   // [c][NB] write-once: row jc of its panel's columns at the panel start (posted by its owner)
  uint64_t* dots;   // [c][G][NB] write-once: partial dots of column jc over the rows of workgroup g
  uint64_t* rowv2;  // [c][NB] write-once: row jc of the remaining panel columns at column step jc
  uint64_t* zpart;  // per panel p: [G][E_p] write-once partials of Z = Y_p^T [Y_p | P_trail], E_p = NB (NB + ntr_p)
  uint64_t* zred;   // per panel p: [E_p] write-once reduced Z
  double* taus;   // [c]      tau of every reflector
};

// Y(gi, s) of panel p0 given the stored value at (gi, p0 + s).
__device__ inline double yval(int64_t gi, int64_t p0, int s, double stored) {
  const int64_t d = p0 + s;
  return gi < d ? 0.0 : (gi == d ? 1.0 : stored);
}

// Posts out[col * NB + s] = sum over the own rows i of Y(i, s) * X(r0 + i, col),
// col < ncol, s < NB; X is column-major in global memory (ldx).  One wave
// per 16-column chunk; MFMA 16x16x4 with A = Y^T from LDS and B = X from
// global memory.  The rows go in groups of four 32-row blocks (32 MFMA K
// steps; the tail in groups of two and one) whose loads are all in flight
// together; every load is issued at a clamped address (row < nrow,
// col < ncol) and rows past nrow get a zero A operand, so no load sits
// behind a branch.
template <typename T>
__device__ __forceinline__ void yt_times_global(const double* Yl, int ldy, int nrow, const T* X, int64_t ldx,
                                                int64_t r0, int ncol, uint64_t* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s = lane & 15, kq = lane >> 4;
  const int nblk = (nrow + 31) / 32;
  for (int col0 = wave * 16; col0 < ncol; col0 += NW * 16) {
    const int col = col0 + s;
    const bool cin = col < ncol;
    const T* xc = X + (int64_t)(cin ? col : ncol - 1) * ldx + r0;
    const double* yc = Yl + s * ldy;
    MF::acc4 a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = MF::acc4{0, 0, 0, 0};
    // groups of four (then two, then one) 32-row blocks: all loads of a
    // group in flight together, no branch inside a group
    auto group = [&](auto gq, int bg) {
      constexpr int GQ = decltype(gq)::value;
      double x[GQ][8];
#pragma unroll
      for (int q = 0; q < GQ; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) x[q][u] = (double)xc[min(32 * (bg + q) + 4 * u + kq, nrow - 1)];
#pragma unroll
      for (int q = 0; q < GQ; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = 32 * (bg + q) + 4 * u + kq;
          const double ya = i < nrow ? yc[i] : 0.0;
          a[u & 3] = MF::fma(ya, cin ? x[q][u] : 0.0, a[u & 3]);
        }
    };
    int bg = 0;
    for (; bg + 4 <= nblk; bg += 4) group(std::integral_constant<int, 4>{}, bg);
    if (bg + 2 <= nblk) {
      group(std::integral_constant<int, 2>{}, bg);
      bg += 2;
    }
    if (bg < nblk) group(std::integral_constant<int, 1>{}, bg);
    if (cin)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        post_u64(out + (int64_t)col * NB + MF::row(lane, r), slot_bits((a[0][r] + a[1][r]) + (a[2][r] + a[3][r])));
  }
}

// X(r0 + i, col) -= sum_s Y(i, s) W(s, col) for the own rows i < nrow and
// col < ncol, W(s, col) = Wl[col * NB + s] in LDS.  A wave takes batches of
// TB row tiles of one 16-column tile.  The MFMA computes the transposed
// tile, D(col, i) = X(i, col) - sum_s W(s, col) Y(i, s) (A = W^T, B = -Y^T),
// so that sixteen lanes hold sixteen consecutive rows of one column: every
// load and store instruction covers four whole 128-byte runs of X.  The next
// batch is loaded while the current one is computed and stored; loads use
// clamped addresses (no branches), stores are masked.
template <typename T>
__device__ __forceinline__ void sub_y_times(const double* Yl, int ldy, int nrow, const double* Wl, T* X, int64_t ldx,
                                            int64_t r0, int ncol) {
  constexpr int TB = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lo = lane & 15, kq = lane >> 4;
  const int ntr = (nrow + 15) / 16, ntc = (ncol + 15) / 16;
  const int nbt = (ntr + TB - 1) / TB, total = ntc * nbt;
  if (wave >= total) return;
  auto load = [&](int k, MF::acc4* acc) {
    const int tc = k / nbt, tr0 = (k % nbt) * TB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = min(tc * 16 + MF::row(lane, r), ncol - 1);
      const T* xc = X + (int64_t)col * ldx + r0;
#pragma unroll
      for (int b = 0; b < TB; ++b) acc[b][r] = (double)xc[min((tr0 + b) * 16 + lo, nrow - 1)];
    }
  };
  auto work = [&](int k, MF::acc4* acc) {
    const int tc = k / nbt, tr0 = (k % nbt) * TB;
    const int wcol = tc * 16 + lo;  // A(m = lo, k = kq) = W(4 k4 + kq, wcol)
    const bool win = wcol < ncol;
    double aw[NB / 4];
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) aw[k4] = win ? Wl[(int64_t)wcol * NB + 4 * k4 + kq] : 0.0;
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int ib = (tr0 + b) * 16 + lo;
#pragma unroll
      for (int k4 = 0; k4 < NB / 4; ++k4) {
        const double bv = ib < nrow ? -Yl[(4 * k4 + kq) * ldy + ib] : 0.0;  // B(k = kq, n = lo)
        acc[b] = MF::fma(aw[k4], bv, acc[b]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = tc * 16 + MF::row(lane, r);
      T* xc = X + (int64_t)(col < ncol ? col : 0) * ldx + r0;
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        const int i = (tr0 + b) * 16 + lo;
        if (col < ncol && i < nrow) xc[i] = (T)acc[b][r];
      }
    }
  };
  MF::acc4 ta[TB], tb[TB];
  load(wave, ta);
  for (int k = wave; k < total; k += 2 * NW) {
    load(min(k + NW, total - 1), tb);
    work(k, ta);
    if (k + NW >= total) break;
    load(min(k + 2 * NW, total - 1), ta);
    work(k + NW, tb);
  }
}

// Gram Y^T Y (NB x NB) of the rows i < nrow of the panel in LDS (Yl,
// column-major, ldy) on MFMA: wave w takes the K steps of rows
// 4 (w + NW t) .. + 3 and leaves its partial tile, entry (s, t) at
// part[w NB NB + t NB + s]; the caller sums the NW tiles in wave order.
__device__ __forceinline__ void gram_tiles(const double* Yl, int ldy, int nrow, double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lo = lane & 15, kq = lane >> 4;
  MF::acc4 ga = {0.0, 0.0, 0.0, 0.0}, gb = {0.0, 0.0, 0.0, 0.0};
  const double* yc = Yl + lo * ldy;
  int i0 = 4 * wave;
  for (; i0 + 4 * NW < nrow; i0 += 8 * NW) {
    const int ia = i0 + kq, ib = i0 + 4 * NW + kq;
    const double va = yc[ia], vb = ib < nrow ? yc[ib] : 0.0;
    ga = MF::fma(va, va, ga);  // A[s = lo][k] = Y(i, lo) = B[k][s = lo]
    gb = MF::fma(vb, vb, gb);
  }
  if (i0 < nrow) {
    const double va = i0 + kq < nrow ? yc[i0 + kq] : 0.0;
    ga = MF::fma(va, va, ga);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave * NB * NB + lo * NB + MF::row(lane, r)] = ga[r] + gb[r];
}

// Broadcast of lane l's value to the whole wave (l wave-uniform).
__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum, in index order, of the n <= N write-once slots p[0], p[stride], ...,
// p[(n - 1) stride] after a bounded poll (all loads of a poll in flight
// together).  False after a timeout or when the error flag is raised.
template <int N>
__device__ inline bool poll_sum(const uint64_t* p, int64_t stride, int n, const unsigned* error, double& sum) {
  double v[N];
  for (unsigned spins = 0;;) {
    bool here = true;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      uint64_t b = 0;
      if (u < n) {
        b = peek_u64(p + u * stride);
        here = here && b != kVoid;
      }
      v[u] = slot_double(b);
    }
    if (here) break;
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 255u) == 0 &&
        (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kSpinLimit))
      return false;
  }
  double s = v[0];
#pragma unroll
  for (int u = 1; u < N; ++u)
    if (u < n) s += v[u];
  sum = s;
  return true;
}

// The n <= N write-once slots p[0], p[stride], ... into v after a bounded poll.
template <int N>
__device__ inline bool poll_vals(const uint64_t* p, int64_t stride, int n, const unsigned* error, double* v) {
  for (unsigned spins = 0;;) {
    bool here = true;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      uint64_t b = 0;
      if (u < n) {
        b = peek_u64(p + u * stride);
        here = here && b != kVoid;
      }
      v[u] = slot_double(b);
    }
    if (here) return true;
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 255u) == 0 &&
        (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kSpinLimit))
      return false;
  }
}

constexpr int kGramGroup = 16;  // workgroups per first-level Gram sum

// A panel column whose remaining squared norm, recovered from the panel's
// Gram matrix, is below this fraction of its squared norm at the panel start
// has lost more than four bits to cancellation; it and the rest of the panel
// go through the exact per-column reductions instead.
constexpr double kPanelTheta = 1.0 / 16.0;

// Reduce-scatter of the E entries of Z over the G partials (write-once
// slots, partial q at zpart[q E]): workgroup g sums the entries
// [E g / G, E (g + 1) / G) in partial order, in batches of 16 partials whose
// sums are added in batch order, and posts them to zred; every workgroup
// then gathers the whole reduced Z into Zl.  No grid barrier: every wait is
// a bounded poll of the slots it reads.  False after a timeout or an error.
__device__ bool reduce_z(const uint64_t* zpart, uint64_t* zred, int64_t E, int G, int g, double* Zl,
                         const unsigned* error) {
  constexpr int RB = 16;
  const int64_t e0 = E * g / G, e1 = E * (g + 1) / G;
  const int ne = (int)(e1 - e0), nb = (G + RB - 1) / RB;
  bool ok = true;
  for (int it0 = 0; it0 < ne * nb && ok; it0 += NT) {
    const int it = it0 + threadIdx.x;
    if (it < ne * nb) {
      const int el = it % ne, q0 = (it / ne) * RB;
      double t = 0.0;
      ok = poll_sum<RB>(zpart + (int64_t)q0 * E + e0 + el, E, min(RB, G - q0), error, t);
      Zl[it] = t;
    }
  }
  if (__syncthreads_or(!ok)) return false;
  for (int el = threadIdx.x; el < ne; el += NT) {
    double t = Zl[el];
    for (int b = 1; b < nb; ++b) t += Zl[b * ne + el];
    post_u64(zred + e0 + el, slot_bits(t));
  }
  __syncthreads();  // Zl is overwritten below
  constexpr int GB = 24;  // gather batch: E <= 24 NT entries (l <= 368) in one round trip
  for (int64_t b = 0; b < E && ok; b += (int64_t)NT * GB) {
    const int64_t e = b + threadIdx.x;
    const int n = e < E ? (int)min((int64_t)GB, (E - e + NT - 1) / NT) : 0;
    double v[GB];
    if (n > 0) ok = poll_vals<GB>(zred + e, NT, n, error, v);
#pragma unroll
    for (int u = 0; u < GB; ++u)
      if (u < n) Zl[e + (int64_t)u * NT] = v[u];
  }
  return !__syncthreads_or(!ok);
}

template <typename T, int RPT>
__global__ __launch_bounds__(NT) void tallqr_kernel(T* __restrict__ P, int64_t mrows, int c, int64_t ldp, int rb,
                                                    T* __restrict__ Qout, int64_t ldq, T* __restrict__ R, int64_t ldr,
                                                    int transpose_r, TqSlots sl, GridSync gs) {
  extern __shared__ double smem[];
  __shared__ double red[NB * NB];
  __shared__ double Tl[NB * NB];
  __shared__ double taul[NB];
  __shared__ int s_jf;  // first panel column left to the per-column reductions
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int64_t r0 = (int64_t)g * rb;
  const int nrow = (int)max((int64_t)0, min((int64_t)rb, mrows - r0));
  // LDS: Y panel of the own rows, column-major with an odd leading dimension
  // so that lanes along rows and lanes along columns both avoid bank conflicts
  const int ldy = rb | 1;
  double* Yl = smem;                    // ldy x NB
  double* Zl = Yl + (int64_t)ldy * NB;  // NB x (c + NB), at least 4 NB NB
  const int npan = (c + NB - 1) / NB;
  int64_t zacc = 0;  // entries of Z in the panels before the current one

  // ------------------------------------------------------------ factorization
  // Within a panel each thread keeps its rows (i = tid + NT u, u < RPT) of the
  // remaining panel columns in registers, the current column always in
  // position 0: after a column step the finished column goes to P and to
  // LDS and the others shift down one position.  The column steps touch no
  // LDS except for the cross-wave part of the reductions, and one copy of
  // the step's code serves all sixteen columns (it stays in the
  // instruction cache).
  for (int pi = 0; pi < npan; ++pi) {
    const int p0 = pi * NB, p1 = min(c, p0 + NB), pw = p1 - p0;
    double y[RPT][NB];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = tid + NT * u;
#pragma unroll
      for (int t = 0; t < NB; ++t)
        y[u][t] = (i < nrow && t < pw) ? (double)P[(int64_t)(p0 + t) * ldp + r0 + i] : 0.0;
    }
    // ---- the panel's reflectors from one exchange.  The Gram matrix G of
    // the panel columns over the active rows (>= p0) is invariant under the
    // reflectors, and the rows p0 .. p1-1 (block B, the only rows the first
    // pw reflectors leave above the diagonal) are posted once.  Before
    // reflector j the dots of column j with the columns s >= j over the rows
    // below jc are then G(j, s) - sum_{i <= j} B(i, j) B(i, s), with B
    // already transformed by reflectors 0 .. j-1; every workgroup runs this
    // recurrence on the same data in the same order (identical reflectors)
    // and applies the reflectors to its own rows without further exchanges.
    {
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = tid + NT * u;
        if (i < nrow) {
          const int64_t gi = r0 + i;
#pragma unroll
          for (int t = 0; t < NB; ++t) Yl[t * ldy + i] = gi >= p0 ? y[u][t] : 0.0;
          if (gi >= p0 && gi < p1)
#pragma unroll
            for (int t = 0; t < NB; ++t) post_u64(sl.rowv + gi * NB + t, slot_bits(y[u][t]));
        }
      }
      __syncthreads();
      gram_tiles(Yl, ldy, nrow, Zl);
      __syncthreads();
      {
        // entry (s, t) posted as the (min, max) sum: G is exactly symmetric
        const int e = tid, lo = min(e & 15, e >> 4), hi = max(e & 15, e >> 4), o = hi * NB + lo;
        const double v = ((Zl[o] + Zl[NB * NB + o]) + Zl[2 * NB * NB + o]) + Zl[3 * NB * NB + o];
        post_u64(sl.gram + ((int64_t)pi * G + g) * NB * NB + e, slot_bits(v));
      }
      // G in two levels (entry e = tid): the first workgroup of each group
      // of kGramGroup sums the group's Grams in workgroup order and posts the
      // sum; every workgroup sums the group sums in group order.  B: row
      // e / NB, column e % NB, from its owner.
      {
        const int ngrp = (G + kGramGroup - 1) / kGramGroup;
        bool ok = true;
        if (g % kGramGroup == 0) {
          double s1 = 0.0;
          ok = poll_sum<kGramGroup>(sl.gram + ((int64_t)pi * G + g) * NB * NB + tid, NB * NB, min(kGramGroup, G - g),
                                    gs.error, s1);
          if (ok) post_u64(sl.gram2 + ((int64_t)pi * ngrp + g / kGramGroup) * NB * NB + tid, slot_bits(s1));
        }
        double acc = 0.0, bv = 0.0;
        for (int k0 = 0; k0 < ngrp && ok; k0 += 16) {
          double s2 = 0.0;
          ok = poll_sum<16>(sl.gram2 + ((int64_t)pi * ngrp + k0) * NB * NB + tid, NB * NB, min(16, ngrp - k0), gs.error,
                            s2);
          acc = k0 == 0 ? s2 : acc + s2;
        }
        const int bi = tid >> 4, bt = tid & 15;
        if (ok && bi < pw) {
          for (unsigned spins = 0;;) {
            const uint64_t b = peek_u64(sl.rowv + (int64_t)(p0 + bi) * NB + bt);
            if (b != kVoid) {
              bv = slot_double(b);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255u) == 0 &&
                (__hip_atomic_load(gs.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kSpinLimit)) {
              ok = false;
              break;
            }
          }
        }
        if (!ok) __hip_atomic_fetch_or(gs.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();  // the partial tiles in Zl are no longer read
        Zl[tid] = acc;
        Zl[NB * NB + tid] = bv;
        if (__syncthreads_or(!ok)) return;
      }
      // the recurrence, by wave 0: lane s keeps column s of B in registers;
      // column j and the diagonal quantities come from lane j
      if (tid < kWave) {
        const int s = tid & (NB - 1);
        double* twl = Zl + 2 * NB * NB;  // tau_j w_j(s), s > j
        double* scl = twl + NB * NB;     // 1 / (x0 - beta) of reflector j
        double* bet = scl + NB;          // beta of reflector j
        double b[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) b[i] = Zl[NB * NB + i * NB + s];
        int jf = pw;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if (j < jf) {
            double bj[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) bj[i] = readlane_d(b[i], j);
            double dsum = 0.0;
#pragma unroll
            for (int i = 0; i <= j; ++i) dsum = fma(bj[i], b[i], dsum);
            const double gjs = Zl[j * NB + s];
            const double d = gjs - dsum;  // dot of columns j and s below row jc
            const double gjj = readlane_d(gjs, j), xnorm2 = readlane_d(d, j), x0 = bj[j];
            if (!(fma(x0, x0, xnorm2) >= kPanelTheta * gjj)) {
              jf = j;
            } else {
              double tau = 0.0, beta = x0, scale = 0.0;
              if (xnorm2 > 0.0) {
                beta = -copysign(sqrt(fma(x0, x0, xnorm2)), x0);
                tau = (beta - x0) / beta;
                scale = 1.0 / (x0 - beta);
              }
              const double tw = tau * fma(scale, d, b[j]);
              if (s > j) {
#pragma unroll
                for (int i = j + 1; i < NB; ++i) b[i] = fma(-tw, bj[i] * scale, b[i]);
                b[j] = b[j] - tw;
              }
              if (tid < NB) twl[j * NB + s] = s > j ? tw : 0.0;
              if (tid == 0) {
                taul[j] = tau;
                scl[j] = scale;
                bet[j] = beta;
              }
            }
          }
        }
        if (tid == 0) s_jf = jf;
      }
      __syncthreads();
    }
    const int jf = s_jf;
    // own rows: reflectors 0 .. jf-1 (the same arithmetic as on B above)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < jf) {
        const int64_t jc = p0 + j;
        const double* twl = Zl + 2 * NB * NB + j * NB;
        const double tau = taul[j], scale = Zl[3 * NB * NB + j], beta = Zl[3 * NB * NB + NB + j];
        double tw[NB];
#pragma unroll
        for (int t = j + 1; t < NB; ++t) tw[t] = twl[t];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = tid + NT * u;
          const int64_t gi = r0 + i;
          if (i < nrow) {
            if (gi >= jc) {
              const double vv = (gi == jc) ? 1.0 : y[u][j] * scale;
#pragma unroll
              for (int t = j + 1; t < NB; ++t) y[u][t] = fma(-tw[t], vv, y[u][t]);
              if (gi == jc) y[u][j] = beta;
              else if (tau != 0.0) y[u][j] = vv;
            }
            P[jc * ldp + gi] = (T)y[u][j];
            Yl[j * ldy + i] = yval(gi, p0, j, y[u][j]);
          }
        }
        if (tid == 0 && g == 0) sl.taus[jc] = tau;
      }
    }
    // the remaining columns (after a cancellation) one reduction each, the
    // current column in register position 0
    for (int k = 0; k < jf && jf < pw; ++k)
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
#pragma unroll
        for (int t = 0; t + 1 < NB; ++t) y[u][t] = y[u][t + 1];
        y[u][NB - 1] = 0.0;
      }
    for (int jt = jf; jt < pw; ++jt) {
      const int jc = p0 + jt;
      // partial dots over the own rows below jc: d_s = sum x_i p_s(i), where
      // position s holds column jc + s
      {
        double d[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) d[t] = 0.0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = tid + NT * u;
          if (i < nrow && r0 + i > jc) {
            const double x = y[u][0];
#pragma unroll
            for (int t = 0; t < NB; ++t) d[t] += x * y[u][t];
          }
        }
        // wave sums of the 16 values by halving exchanges: after the steps
        // over lane bits 5, 4, 3, 2 a lane holds the sum for
        // t = 8 b5 + 4 b4 + 2 b3 + b2, completed over lane bits 1, 0
        const int lane = tid & 63, wave = tid >> 6;
        double h8[8], h4[4], h2[2], h1;
        {
          const bool up = lane & 32;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const double send = up ? d[k] : d[k + 8];
            const double keep = up ? d[k + 8] : d[k];
            h8[k] = keep + __shfl_xor(send, 32, kWave);
          }
        }
        {
          const bool up = lane & 16;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double send = up ? h8[k] : h8[k + 4];
            const double keep = up ? h8[k + 4] : h8[k];
            h4[k] = keep + __shfl_xor(send, 16, kWave);
          }
        }
        // inside a row of 16 lanes the partner of a lane only has to differ in
        // the bit of the level (DPP mirrors and quad permutations)
        {
          const bool up = lane & 8;
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const double send = up ? h4[k] : h4[k + 2];
            const double keep = up ? h4[k + 2] : h4[k];
            h2[k] = keep + dpp_mov<kDppMirror>(send);
          }
        }
        {
          const bool up = lane & 4;
          const double send = up ? h2[0] : h2[1];
          const double keep = up ? h2[1] : h2[0];
          h1 = keep + dpp_mov<kDppHalfMirror>(send);
        }
        h1 += dpp_mov<kDppXor2>(h1);
        h1 += dpp_mov<kDppXor1>(h1);
        if ((lane & 3) == 0) {
          const int t = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
          red[wave * NB + t] = h1;
        }
        // the owner of row jc publishes that row of the remaining columns
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = tid + NT * u;
          if (i < nrow && r0 + i == jc)
#pragma unroll
            for (int t = 0; t < NB; ++t) post_u64(sl.rowv2 + (int64_t)jc * NB + t, slot_bits(y[u][t]));
        }
        __syncthreads();
        if (tid < NB) {
          double sacc = 0.0;
#pragma unroll
          for (int q = 0; q < NW; ++q) sacc += red[q * NB + tid];
          post_u64(sl.dots + ((int64_t)jc * G + g) * NB + tid, slot_bits(sacc));
        }
      }
      // gather the partials of every workgroup (bounded polls of the column's
      // write-once slots) and sum them in a fixed order, identical in every
      // workgroup
      {
        const int t = tid & (NB - 1), gq = tid / NB;
        constexpr int QB = 8;
        double acc = 0.0, rv = 0.0;
        bool ok = true;
        const uint64_t* dj = sl.dots + (int64_t)jc * G * NB + t;
        for (int q0 = gq; q0 < G && ok; q0 += QB * (NT / NB)) {
          double v[QB];
          for (unsigned spins = 0;;) {
            bool here = true;
#pragma unroll
            for (int u = 0; u < QB; ++u) {
              const int q = q0 + u * (NT / NB);
              uint64_t b = 0;
              if (q < G) {
                b = peek_u64(dj + (int64_t)q * NB);
                here = here && b != kVoid;
              }
              v[u] = slot_double(b);
            }
            if (here) break;
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255u) == 0 &&
                (__hip_atomic_load(gs.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kSpinLimit)) {
              ok = false;
              break;
            }
          }
#pragma unroll
          for (int u = 0; u < QB; ++u) acc += v[u];
        }
        if (tid < NB && ok) {
          for (unsigned spins = 0;;) {
            const uint64_t b = peek_u64(sl.rowv2 + (int64_t)jc * NB + tid);
            if (b != kVoid) {
              rv = slot_double(b);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255u) == 0 &&
                (__hip_atomic_load(gs.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > kSpinLimit)) {
              ok = false;
              break;
            }
          }
        }
        if (!ok) __hip_atomic_fetch_or(gs.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        red[gq * NB + t] = acc;
        if (__syncthreads_or(!ok)) return;
        if (tid < NB) {
          double sacc = 0.0;
          for (int q = 0; q < NT / NB; ++q) sacc += red[q * NB + tid];
          Tl[tid] = sacc;      // d_s
          Tl[NB + tid] = rv;   // p_s(jc)
        }
        __syncthreads();
      }
      const double xnorm2 = Tl[0], x0 = Tl[NB];
      double tau = 0.0, beta = x0, scale = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + xnorm2), x0);
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      if (tid == 0) {
        taul[jt] = tau;
        if (g == 0) sl.taus[jc] = tau;
      }
      // own rows: p_s -= tau w_s v, w_s = p_s(jc) + scale d_s; the column
      // becomes v (beta on the diagonal), is stored, and the rest shift down
      double tw[NB];
#pragma unroll
      for (int t = 1; t < NB; ++t) tw[t] = tau * (Tl[NB + t] + scale * Tl[t]);
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = tid + NT * u;
        const int64_t gi = r0 + i;
        if (i < nrow) {
          if (gi >= jc) {
            const double vv = (gi == jc) ? 1.0 : y[u][0] * scale;
#pragma unroll
            for (int t = 1; t < NB; ++t) y[u][t] -= tw[t] * vv;
            if (gi == jc) y[u][0] = beta;
            else if (tau != 0.0) y[u][0] = vv;
          }
          P[(int64_t)jc * ldp + gi] = (T)y[u][0];
          Yl[jt * ldy + i] = yval(gi, p0, jt, y[u][0]);
        }
#pragma unroll
        for (int t = 0; t + 1 < NB; ++t) y[u][t] = y[u][t + 1];
        y[u][NB - 1] = 0.0;
      }
    }
    for (int t = pw; t < NB; ++t)
      for (int i = tid; i < nrow; i += NT) Yl[t * ldy + i] = 0.0;
    __syncthreads();
    const int ntr = c - p1;
    const int64_t E = (int64_t)NB * (NB + ntr);
    uint64_t* zp = sl.zpart + (int64_t)G * zacc + (int64_t)g * E;
    // Gram part Y^T Y (16 x 16) on MFMA, the four partial tiles summed in wave order
    gram_tiles(Yl, ldy, nrow, Zl);
    __syncthreads();
    {
      const int s = tid & (NB - 1), cc = tid / NB;
      post_u64(zp + cc * NB + s,
               slot_bits(((Zl[cc * NB + s] + Zl[NB * NB + cc * NB + s]) + Zl[2 * NB * NB + cc * NB + s]) +
                         Zl[3 * NB * NB + cc * NB + s]));
    }
    if (ntr > 0) yt_times_global<T>(Yl, ldy, nrow, P + (int64_t)p1 * ldp, ldp, r0, ntr, zp + NB * NB);
    if (!reduce_z(sl.zpart + (int64_t)G * zacc, sl.zred + zacc, E, G, g, Zl, gs.error)) {
      if (tid == 0) __hip_atomic_fetch_or(gs.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    zacc += E;
    // T of the panel: T(s,s) = tau_s, T(0:s, s) = -tau_s T(0:s, 0:s) (Y^T y_s),
    // by wave 0 alone: lane j keeps row j of T in registers (T(j, q) = 0 for
    // q < j, so the sums over q < s add exact zeros below the row's start)
    if (tid < kWave) {
      double trow[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) trow[q] = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NB; ++s2) {
        if (s2 < pw) {
          double val = 0.0;
#pragma unroll
          for (int q = 0; q < s2; ++q) val += trow[q] * Zl[s2 * NB + q];
          const double ts = taul[s2];
          trow[s2] = tid < s2 ? -ts * val : (tid == s2 ? ts : 0.0);
        }
      }
      if (tid < NB)
#pragma unroll
        for (int q = 0; q < NB; ++q) Tl[q * NB + tid] = trow[q];
    }
    __syncthreads();
    // W' = T^T Z_trail (in place, column by column)
    for (int u = tid; u < ntr; u += NT) {
      double z[NB], w[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) z[q] = Zl[(NB + u) * NB + q];
#pragma unroll
      for (int s2 = 0; s2 < NB; ++s2) {
        double a = 0.0;
        for (int q = 0; q <= s2; ++q) a += Tl[s2 * NB + q] * z[q];
        w[s2] = a;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) Zl[(NB + u) * NB + q] = w[q];
    }
    __syncthreads();
    // P_trail(own rows) -= Y W'  (rows above p0 have Y = 0); the next panel
    // reads these rows from other waves
    if (ntr > 0) sub_y_times<T>(Yl, ldy, nrow, Zl + NB * NB, P + (int64_t)p1 * ldp, ldp, r0, ntr);
    __syncthreads();
  }

  // --------------------------------------------------- R output, diag(R) >= 0
  // (the own rows only: every entry read here was written by this workgroup)
  if (r0 >= c) return;
  const int rows = (int)min((int64_t)nrow, (int64_t)c - r0);
  double* sgn = Zl;  // sign of diag(R) for the own rows
  for (int i = tid; i < rows; i += NT) sgn[i] = ((double)P[(r0 + i) * ldp + r0 + i] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)rows * c; e += NT) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    const int64_t gi = r0 + i;
    const double val = (j >= gi) ? sgn[i] * (double)P[(int64_t)j * ldp + gi] : 0.0;
    if (transpose_r) R[gi * ldr + j] = (T)val;
    else R[(int64_t)j * ldr + gi] = (T)val;
  }
}

// Y(i, k) of the unit lower trapezoidal Householder block stored in P.
template <typename T>
__device__ inline double yload(const T* P, int64_t ldp, int64_t i, int64_t k) {
  return i < k ? 0.0 : (i == k ? 1.0 : (double)P[k * ldp + i]);
}

// Partial Gram S = Y^T Y over one chunk of rows for one 64 x 64 tile pair
// (I <= J) of the c x c result: spart[split][b * c + a] = sum_{i in chunk}
// Y(i, a) Y(i, b).  K steps of 16 rows through LDS, loaded along the rows
// (sixteen lanes on one column) and one step ahead into registers.
constexpr int WY_T = 64, WY_K = 16, WY_LD = WY_T + 16;

template <typename T>
__global__ __launch_bounds__(256) void gram_y_kernel(const T* __restrict__ P, int64_t mrows, int c, int64_t ldp,
                                                     int64_t chunk, double* __restrict__ spart) {
  constexpr int GY_LD = WY_T + 1;  // odd stride: the row-wise stores below spread over the banks
  __shared__ double Ya[WY_K * GY_LD];
  __shared__ double Yb[WY_K * GY_LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = (c + WY_T - 1) / WY_T;
  int I = 0, J = 0;
  for (int pr = blockIdx.x; pr >= 0; ++I) {  // tile pair index -> (I, J), I <= J
    if (pr < nt - I) {
      J = I + pr;
      break;
    }
    pr -= nt - I;
  }
  const int a0 = I * WY_T, b0 = J * WY_T;
  const int64_t ilo = (int64_t)blockIdx.y * chunk;
  const int64_t ihi = min(mrows, ilo + chunk);
  const int wa = wave & 1, wb = wave >> 1;
  MF::acc4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = MF::acc4{0, 0, 0, 0};
  // loader: element e = tid + 256 u is row k = e % WY_K of column x = e / WY_K,
  // so sixteen lanes read sixteen consecutive rows of one column
  double ra[4], rb[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, k = e & (WY_K - 1), x = e / WY_K;
      const int64_t gi = k0 + k;
      const bool rin = gi < ihi;
      ra[u] = (rin && a0 + x < c) ? yload(P, ldp, gi, a0 + x) : 0.0;
      rb[u] = (rin && b0 + x < c) ? yload(P, ldp, gi, b0 + x) : 0.0;
    }
  };
  load(ilo);
  for (int64_t k0 = ilo; k0 < ihi; k0 += WY_K) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, k = e & (WY_K - 1), x = e / WY_K;
      Ya[k * GY_LD + x] = ra[u];
      Yb[k * GY_LD + x] = rb[u];
    }
    __syncthreads();
    if (k0 + WY_K < ihi) load(k0 + WY_K);
#pragma unroll
    for (int kk = 0; kk < WY_K; kk += 4) {
      const int k = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = Yb[k * GY_LD + wb * 32 + x * 16 + (lane & 15)];  // A(b, i)
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = Ya[k * GY_LD + wa * 32 + y * 16 + (lane & 15)];  // B(i, a)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = MF::fma(av[x], bv[y], acc[x][y]);
    }
  }
  double* out = spart + (int64_t)blockIdx.y * c * c;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = b0 + wb * 32 + x * 16 + MF::row(lane, r);
        const int a = a0 + wa * 32 + y * 16 + (lane & 15);
        if (a < c && b < c) out[(int64_t)b * c + a] = acc[x][y][r];
      }
}

// S = sum of the row-chunk partials in split order (upper triangle a <= b).
__global__ void gram_sum_kernel(const double* __restrict__ spart, int nsplit, int c, double* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)c * c) return;
  const int a = (int)(e % c), b = (int)(e / c);
  if (a > b) return;
  double t = 0.0;
  for (int s = 0; s < nsplit; ++s) t += spart[(int64_t)s * c * c + e];
  S[e] = t;
}


// Column j of M' = (T Y(0:c, :)^T) diag(sgn), row-major in mt, by back
// substitution with U = T^-1 = striu(S) + diag(1/tau): U m = y_j with
// y_j(k) = Y(j, k) (zero for k > j).  m_k = r_k tau_k, so tau_k = 0 gives
// m_k = 0 (the reflector is the identity).  One wave per column (four per
// workgroup, one per SIMD), lane l holding r_i for the rows i = l + 64 u;
// m_k is broadcast by a lane read, so the steps need no workgroup barrier.
// The columns k of striu(S) come through LDS in blocks of sb (32, or 16 for
// c > 512), loaded by the whole workgroup with all loads in flight together.
constexpr int WM_NT = 256;

template <typename T, int RPL>
__global__ __launch_bounds__(WM_NT) void wy_m_kernel(const T* __restrict__ P, int c, int64_t ldp, int sb,
                                                     const double* __restrict__ S, const double* __restrict__ taus,
                                                     double* __restrict__ mt, double* __restrict__ sgn) {
  extern __shared__ double Sb[];  // [sb][c]: Sb[kk][i] = S(i, K sb + kk), i < K sb + kk
  constexpr int NWV = WM_NT / 64, FB = 40;  // one batch of loads per block for c <= 320
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = blockIdx.x * NWV + wave;
  const bool live = j < c;
  const int jmax = min(c - 1, blockIdx.x * NWV + NWV - 1);
  double r[RPL], tr[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = lane + 64 * u;
    r[u] = (live && i <= j) ? yload(P, ldp, j, i) : 0.0;
    tr[u] = i < c ? taus[i] : 0.0;
  }
  const int nblk = jmax / sb + 1, ne = sb * c;
  for (int K = nblk - 1; K >= 0; --K) {
    __syncthreads();  // the previous block is no longer read
    for (int e0 = 0; e0 < ne; e0 += WM_NT * FB) {
      double pf[FB];
#pragma unroll
      for (int x = 0; x < FB; ++x) {
        const int e = e0 + tid + WM_NT * x, kk = e / c, i = e - kk * c, k = K * sb + kk;
        pf[x] = (e < ne && k <= jmax && i < k) ? S[(int64_t)k * c + i] : 0.0;
      }
#pragma unroll
      for (int x = 0; x < FB; ++x) {
        const int e = e0 + tid + WM_NT * x;
        if (e < ne) Sb[e] = pf[x];
      }
    }
    __syncthreads();
    if (!live) continue;
    for (int kk = sb - 1; kk >= 0; --kk) {
      const int k = K * sb + kk;
      if (k > j) continue;
      const int ku = k >> 6, kl = k & 63;
      double rk = 0.0, tk = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u)
        if (u == ku) {
          rk = r[u];
          tk = tr[u];
        }
      const double mk = readlane_d(rk, kl) * readlane_d(tk, kl);
      double sv[RPL];  // unconditional (clamped) reads, issued together
#pragma unroll
      for (int u = 0; u < RPL; ++u) sv[u] = Sb[kk * c + min(lane + 64 * u, c - 1)];
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int i = lane + 64 * u;
        const double upd = fma(-mk, sv[u], r[u]);
        r[u] = i < k ? upd : (i == k ? mk : r[u]);
      }
    }
  }
  if (!live) return;
  const double sj = ((double)P[(int64_t)j * ldp + j] < 0.0) ? -1.0 : 1.0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int k = lane + 64 * u;
    if (k < c) mt[(int64_t)k * c + j] = (k <= j) ? r[u] * sj : 0.0;
  }
  if (lane == 0) sgn[j] = sj;
}

// The same M' for c <= 592 as a blocked triangular solve: workgroup w
// takes the sixteen right-hand sides j = 16 w .. 16 w + 15 with all their
// rows in LDS, and walks the 16-row blocks from the one holding the largest
// j up to the first.  A block's diagonal part is solved by sixteen lanes of
// wave 0, lane jj holding the block's rows of column jj in registers (the
// solve needs no lane exchange); the rows above are then updated at once,
// r(0:k0, :) -= S(0:k0, block) m(block, :), on FP64 MFMA by all four waves.
// The S columns of the next block are loaded while the current one is
// worked on.
// RS = 256-row slots per column (2 for c <= 512, 3 up to the 592 rows whose
// 34 c16 doubles still fit the LDS).
constexpr int WB_NT = 256, WB_LD = 17;  // LDS row stride of the right-hand sides
constexpr int WB_MAXC = 592;

template <typename T, int RS>
__global__ __launch_bounds__(WB_NT) void wy_m_blocked_kernel(const T* __restrict__ P, int c, int64_t ldp,
                                                             const double* __restrict__ S,
                                                             const double* __restrict__ taus,
                                                             double* __restrict__ mt, double* __restrict__ sgn) {
  extern __shared__ double smem[];
  const int c16 = (c + 15) & ~15;
  double* rl = smem;                         // rl[i * WB_LD + jj]: row i of right-hand side jj
  double* sb = rl + (int64_t)c16 * WB_LD;    // sb[kk * c16 + i] = S(i, k0 + kk), i < k0 + kk
  double* tl = sb + (int64_t)16 * c16;       // tau_k, zero past c
  constexpr int PF = 16 * RS;                // S loads per thread and block (16 c16 <= 256 PF)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j0 = blockIdx.x * 16, jn = min(16, c - j0);
  // thread tid: right-hand side jj = tid % 16, rows tid / 16 + 16 x (all
  // loads in flight together)
  const int jj = tid & 15, ir = tid >> 4;
  for (int k = tid; k < c16; k += WB_NT) tl[k] = k < c ? taus[k] : 0.0;
  {
    constexpr int RX = 256 * RS / 16;
    double v[RX];
#pragma unroll
    for (int x = 0; x < RX; ++x) {
      const int i = ir + 16 * x;
      v[x] = (jj < jn && i < c) ? yload(P, ldp, j0 + jj, i) : 0.0;
    }
#pragma unroll
    for (int x = 0; x < RX; ++x)
      if (ir + 16 * x < c16) rl[(ir + 16 * x) * WB_LD + jj] = v[x];
  }
  // S(0 : k0 + 16, k0 : k0 + 16) of block kb, element x of thread tid:
  // column kk = x / RS, row i = tid + WB_NT (x % RS)
  double pf[PF];
  auto load_s = [&](int kb) {
    const int k0 = kb * 16;
#pragma unroll
    for (int x = 0; x < PF; ++x) {
      const int kk = x / RS, i = tid + WB_NT * (x % RS), k = k0 + kk;
      pf[x] = (i < k && k < c) ? S[(int64_t)k * c + i] : 0.0;
    }
  };
  auto store_s = [&](int kb) {
    const int k0 = kb * 16;
#pragma unroll
    for (int x = 0; x < PF; ++x) {
      const int kk = x / RS, i = tid + WB_NT * (x % RS);
      if (i < k0 + 16) sb[kk * c16 + i] = pf[x];
    }
  };
  const int nb = (j0 + jn - 1) / 16 + 1;
  load_s(nb - 1);
  for (int kb = nb - 1; kb >= 0; --kb) {
    const int k0 = kb * 16;
    __syncthreads();  // the previous block no longer reads sb; rl is up to date
    store_s(kb);
    if (kb > 0) load_s(kb - 1);
    __syncthreads();
    if (wave == 0 && lane < 16) {
      double rr[16], tk[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        rr[t] = rl[(k0 + t) * WB_LD + lane];
        tk[t] = tl[k0 + t];
      }
#pragma unroll
      for (int t = 15; t >= 0; --t) {
        const double m = rr[t] * tk[t];
        rr[t] = m;
#pragma unroll
        for (int i = 0; i < t; ++i) rr[i] = fma(-m, sb[t * c16 + k0 + i], rr[i]);
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) rl[(k0 + t) * WB_LD + lane] = rr[t];
    }
    __syncthreads();
    // rows above: tile rows 16 tt .. 16 tt + 15; A = S(rows, block), B = m(block, :)
    for (int tt = wave; tt < kb; tt += WB_NT / 64) {
      MF::acc4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        const int kk = 4 * k4 + (lane >> 4);
        d = MF::fma(sb[kk * c16 + 16 * tt + (lane & 15)], rl[(k0 + kk) * WB_LD + (lane & 15)], d);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * tt + MF::row(lane, r);
        rl[i * WB_LD + (lane & 15)] -= d[r];
      }
    }
  }
  __syncthreads();
  if (jj < jn) {
    const int j = j0 + jj;
    const double sj = ((double)P[(int64_t)j * ldp + j] < 0.0) ? -1.0 : 1.0;
    for (int k = ir; k < c; k += 16) mt[(int64_t)k * c + j] = k <= j ? rl[k * WB_LD + jj] * sj : 0.0;
    if (ir == 0) sgn[j] = sj;
  }
}

// Q(i, j) = [i == j] sgn_j - sum_{k <= min(i, j)} Y(i, k) M'(k, j), with
// M' = M diag(sgn) row-major (mt) and Y the unit lower trapezoidal
// Householder vectors stored in P.  64 x 64 tiles of Q per workgroup, K in
// steps of 16 through LDS, the next step loaded into registers while the
// current one is computed; the MFMA computes the transposed tile
// (A = M'^T, B = Y^T) so that each result row is a run of 16 consecutive
// entries of a column of Q.  Column tiles stop at K = j0 + 64 (M' is upper
// triangular), row tiles at K = i0 + 64 (Y is lower trapezoidal).

template <typename T>
__global__ __launch_bounds__(256) void wy_apply_kernel(const T* __restrict__ P, int64_t mrows, int c, int64_t ldp,
                                                       const double* __restrict__ mt, const double* __restrict__ sgn,
                                                       T* __restrict__ Q, int64_t ldq) {
  __shared__ double Ys[WY_K * WY_LD];  // Ys[k * WY_LD + i] = Y(i0 + i, k0 + k)
  __shared__ double Ms[WY_K * WY_LD];  // Ms[k * WY_LD + j] = M'(k0 + k, j0 + j)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * WY_T;
  const int j0 = blockIdx.y * WY_T;
  const int wr = wave & 1, wc = wave >> 1;  // 32 x 32 quarter of the tile: rows (i) wr, columns (j) wc
  int64_t kmax = min((int64_t)c, (int64_t)j0 + WY_T);
  kmax = min(kmax, i0 + WY_T);
  MF::acc4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = MF::acc4{0, 0, 0, 0};
  // the next K step is loaded into registers while the current one is computed
  double yr[4], mr[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, k = e / WY_T, x = e % WY_T;
      const int64_t gk = k0 + k, gi = i0 + x;
      double yv = 0.0;
      if (gk < kmax && gi < mrows) yv = gi < gk ? 0.0 : (gi == gk ? 1.0 : (double)P[gk * ldp + gi]);
      yr[u] = yv;
      const int gj = j0 + x;
      mr[u] = (gk < kmax && gj < c) ? mt[gk * c + gj] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < kmax; k0 += WY_K) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u, k = e / WY_T, x = e % WY_T;
      Ys[k * WY_LD + x] = yr[u];
      Ms[k * WY_LD + x] = mr[u];
    }
    __syncthreads();
    if (k0 + WY_K < kmax) load(k0 + WY_K);
#pragma unroll
    for (int kk = 0; kk < WY_K; kk += 4) {
      const int k = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Ms[k * WY_LD + wc * 32 + a * 16 + (lane & 15)];  // A(j, k)
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ys[k * WY_LD + wr * 32 + b * 16 + (lane & 15)];  // B(k, i)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = MF::fma(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + wc * 32 + a * 16 + MF::row(lane, r);
        const int64_t i = i0 + wr * 32 + b * 16 + (lane & 15);
        if (j < c && i < mrows) Q[(int64_t)j * ldq + i] = (T)((i == j ? sgn[j] : 0.0) - acc[a][b][r]);
      }
}

// Row blocks of 64 to 256 rows, aiming at 128 workgroups: more workgroups
// share the streaming trailing updates, fewer keep the panel exchanges
// cheap.  Measured on 16384 x 272 / 8192 x 272: 64 workgroups 1.99 / 1.83
// ms, 128 workgroups 1.66 / 1.39 ms, 256 workgroups 1.74 ms (16384 rows).
// From 32768 rows on the trailing updates dominate and the row blocks stay
// at 128 rows up to one workgroup per CU (32768 x 544: 256 workgroups 4.79
// ms, 128 workgroups 5.71 ms; 16384 x 544: 4.01 and 4.00 ms).
void choose(int64_t mrows, int c, int num_cu, int* G, int* rb, size_t* lds) {
  int64_t rows = (mrows + 127) / 128;
  rows = rows < 64 ? 64 : (rows > 256 ? 256 : rows);
  if (mrows >= 32768) rows = std::max<int64_t>(128, (mrows + num_cu - 1) / num_cu);
  int64_t g = (mrows + rows - 1) / rows;
  if (g > num_cu) g = num_cu;
  if (g < 1) g = 1;
  int64_t r = (mrows + g - 1) / g;
  *G = (int)((mrows + r - 1) / r);
  *rb = (int)r;
  // Zl: Z = Y_p^T [Y_p | P_trail] (NB x (c + NB)), also the four partial
  // Gram tiles (4 NB NB)
  *lds = ((size_t)(r | 1) * NB + std::max((size_t)NB * (c + NB), (size_t)4 * NB * NB) + 64) * sizeof(double);
}

template <typename T>
__global__ void gather_kernel(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                              const int64_t* __restrict__ cols, int64_t c, T* __restrict__ P, int64_t ldp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < m && j < c) {
    const int64_t cj = cols[j];
    P[j * ldp + i] = (cj >= 0 && cj < n) ? A[cj * lda + i] : T(__builtin_nan(""));
  }
}

// V(rowmap[i], :) = Q(i, :)
template <typename T>
__global__ void scatter_rows_kernel(const T* __restrict__ Q, int64_t mrows, int64_t c, int64_t ldq,
                                    const int64_t* __restrict__ rowmap, T* __restrict__ V, int64_t ldv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < mrows && j < c) {
    const int64_t r = rowmap[i];
    if (r >= 0 && r < mrows) V[j * ldv + r] = Q[j * ldq + i];
  }
}

}  // namespace

// Entries of Z = Y_p^T [Y_p | P_trail] over all panels: NB (NB + ntr_p).
static size_t z_entries(int64_t c) {
  size_t t = 0;
  for (int64_t p1 = NB; p1 - NB < c; p1 += NB) t += (size_t)NB * (NB + (p1 < c ? c - p1 : 0));
  return t;
}

// Row chunks of the Gram S = Y^T Y: enough (chunk, tile pair) workgroups to
// fill the chip twice, chunks of at least 256 rows, at most 32 partials.
void gram_split(int64_t mrows, int64_t c, int num_cu, int* nsplit, int64_t* chunk) {
  const int nt = (int)((c + WY_T - 1) / WY_T), npairs = nt * (nt + 1) / 2;
  int64_t s = (2 * (int64_t)num_cu + npairs - 1) / npairs;
  s = std::min<int64_t>(s, std::max<int64_t>(1, mrows / 256));
  s = std::min<int64_t>(s, 32);
  int64_t ch = (mrows + s - 1) / s;
  ch = (ch + WY_K - 1) / WY_K * WY_K;
  *chunk = ch;
  *nsplit = (int)((mrows + ch - 1) / ch);
}

bool tallqr_fits(int64_t mrows, int64_t c, const DeviceInfo& d) {
  if (c < 1 || c > 1024 || mrows < c) return false;
  int G, rb;
  size_t lds;
  choose(mrows, (int)c, d.num_cu, &G, &rb, &lds);
  return lds <= d.lds_max && G <= kMaxGridBlocks && (rb + NT - 1) / NT <= 4;
}

template <typename T>
size_t tallqr_scratch(int64_t mrows, int64_t c, const DeviceInfo& d) {
  int G, rb, nsplit;
  int64_t chunk;
  size_t lds;
  choose(mrows, (int)c, d.num_cu, &G, &rb, &lds);
  gram_split(mrows, c, d.num_cu, &nsplit, &chunk);
  const size_t npan = ((size_t)c + NB - 1) / NB;
  const size_t ngrp = ((size_t)G + kGramGroup - 1) / kGramGroup;
  size_t b = sizeof(double) * (npan * G * NB * NB + npan * ngrp * NB * NB + (size_t)c * NB + (size_t)c * G * NB +
                               (size_t)c * NB + ((size_t)G + 1) * z_entries(c) + c +
                               ((size_t)nsplit + 2) * c * c + c);
  return b + 16 * 256;
}

template <typename T>
hipError_t tall_qr(T* P, int64_t mrows, int64_t c, int64_t ldp, T* Qout, int64_t ldq, T* R, int64_t ldr,
                   bool transpose_r, Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s,
                   hipEvent_t r_ready) {
  if (c <= 0) return hipSuccess;
  if (mrows < c || c > 1024) return hipErrorInvalidValue;
  int G, rb, nsplit;
  int64_t chunk;
  size_t lds;
  choose(mrows, (int)c, d.num_cu, &G, &rb, &lds);
  if (lds > d.lds_max) return hipErrorInvalidValue;
  gram_split(mrows, c, d.num_cu, &nsplit, &chunk);
  const int npan = (int)((c + NB - 1) / NB);
  TqSlots sl;
  const int ngrp = (G + kGramGroup - 1) / kGramGroup;
  sl.gram = ar.take<uint64_t>((size_t)npan * G * NB * NB);
  sl.gram2 = ar.take<uint64_t>((size_t)npan * ngrp * NB * NB);
  sl.rowv = ar.take<uint64_t>((size_t)c * NB);
  sl.dots = ar.take<uint64_t>((size_t)c * G * NB);
  sl.rowv2 = ar.take<uint64_t>((size_t)c * NB);
  const size_t zall = z_entries(c);
  sl.zpart = ar.take<uint64_t>((size_t)G * zall);
  sl.zred = ar.take<uint64_t>(zall);
  sl.taus = ar.take<double>((size_t)c);
  double* spart = ar.take<double>((size_t)nsplit * c * c);
  double* S = ar.take<double>((size_t)c * c);
  double* mt = ar.take<double>((size_t)c * c);
  double* sgn = ar.take<double>((size_t)c);
  if (!sl.gram || !sl.gram2 || !sl.dots || !sl.rowv || !sl.rowv2 || !sl.zpart || !sl.zred || !sl.taus || !spart ||
      !S || !mt || !sgn)
    return hipErrorOutOfMemory;
  // the slot arrays were carved one after the other (gram .. zred): one fill
  // covers them and the alignment gaps between them
  hipError_t e = fill_void(sl.gram, (size_t)(sl.zred + zall - sl.gram), s);
  if (e != hipSuccess) return e;
  if (G > kMaxGridBlocks) return hipErrorInvalidValue;
  GridSync gs{nullptr, err, (unsigned)G};  // the kernel only uses the error word (no grid barrier)
  int ci = (int)c, tr = transpose_r ? 1 : 0;
  void* args[] = {(void*)&P, (void*)&mrows, (void*)&ci, (void*)&ldp, (void*)&rb, (void*)&Qout, (void*)&ldq,
                  (void*)&R, (void*)&ldr, (void*)&tr, (void*)&sl, (void*)&gs};
  const int rpt = (rb + NT - 1) / NT;  // rows per thread in the column steps
  const void* fn = rpt <= 1 ? (const void*)tallqr_kernel<T, 1>
                   : rpt <= 2 ? (const void*)tallqr_kernel<T, 2>
                   : rpt <= 4 ? (const void*)tallqr_kernel<T, 4> : nullptr;
  if (!fn) return hipErrorInvalidValue;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, (unsigned)lds, s);
  if (e != hipSuccess) return e;
  if (r_ready) {
    e = hipEventRecord(r_ready, s);
    if (e != hipSuccess) return e;
  }
  const int nt = (ci + WY_T - 1) / WY_T;
  gram_y_kernel<T><<<dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)nsplit), 256, 0, s>>>(P, mrows, ci, ldp, chunk,
                                                                                        spart);
  gram_sum_kernel<<<(unsigned)((c * c + 255) / 256), 256, 0, s>>>(spart, nsplit, ci, S);
  const size_t blds = ((size_t)((ci + 15) & ~15) * (WB_LD + 16 + 1)) * sizeof(double);
  if (ci <= WB_MAXC && (d.lds_max == 0 || blds <= d.lds_max)) {
    const void* bfn = ci <= 512 ? (const void*)wy_m_blocked_kernel<T, 2> : (const void*)wy_m_blocked_kernel<T, 3>;
    if (blds > 65536) {
      e = hipFuncSetAttribute(bfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)blds);
      if (e != hipSuccess) return e;
    }
    const double* taus_b = sl.taus;
    const double* S_b = S;
    void* bargs[] = {(void*)&P, (void*)&ci, (void*)&ldp, (void*)&S_b, (void*)&taus_b, (void*)&mt, (void*)&sgn};
    e = hipLaunchKernel(bfn, dim3((unsigned)((ci + 15) / 16)), dim3(WB_NT), bargs, blds, s);
    if (e != hipSuccess) return e;
  } else {
  int msb = ci <= 512 ? 32 : 16;
  const size_t mlds = (size_t)msb * ci * sizeof(double);
  const unsigned mgrid = (unsigned)((c + WM_NT / 64 - 1) / (WM_NT / 64));
  const void* mfn = ci <= 64    ? (const void*)wy_m_kernel<T, 1>
                    : ci <= 128 ? (const void*)wy_m_kernel<T, 2>
                    : ci <= 256 ? (const void*)wy_m_kernel<T, 4>
                    : ci <= 512 ? (const void*)wy_m_kernel<T, 8>
                                : (const void*)wy_m_kernel<T, 16>;
  if (mlds > 65536) {
    e = hipFuncSetAttribute(mfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds);
    if (e != hipSuccess) return e;
  }
  const double* taus_c = sl.taus;
  const double* S_c = S;
  void* margs[] = {(void*)&P, (void*)&ci, (void*)&ldp, (void*)&msb, (void*)&S_c, (void*)&taus_c, (void*)&mt, (void*)&sgn};
  e = hipLaunchKernel(mfn, dim3(mgrid), dim3(WM_NT), margs, mlds, s);
  if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)((mrows + WY_T - 1) / WY_T), (unsigned)nt);
  wy_apply_kernel<T><<<grid, 256, 0, s>>>(P, mrows, ci, ldp, mt, sgn, Qout, ldq);
  return hipGetLastError();
}

template <typename T>
hipError_t gather_cols(const T* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols, int64_t c, T* P,
                       int64_t ldp, hipStream_t s) {
  if (c <= 0 || m <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)c);
  gather_kernel<T><<<grid, 256, 0, s>>>(A, m, n, lda, cols, c, P, ldp);
  return hipGetLastError();
}

template <typename T>
hipError_t scatter_rows(const T* Q, int64_t mrows, int64_t c, int64_t ldq, const int64_t* rowmap, T* V, int64_t ldv,
                        hipStream_t s) {
  if (c <= 0 || mrows <= 0) return hipSuccess;
  dim3 grid((unsigned)((mrows + 255) / 256), (unsigned)c);
  scatter_rows_kernel<T><<<grid, 256, 0, s>>>(Q, mrows, c, ldq, rowmap, V, ldv);
  return hipGetLastError();
}

#define INST(T)                                                                                                    \
  template size_t tallqr_scratch<T>(int64_t, int64_t, const DeviceInfo&);                                          \
  template hipError_t tall_qr<T>(T*, int64_t, int64_t, int64_t, T*, int64_t, T*, int64_t, bool, Arena&, unsigned*, \
                                 const DeviceInfo&, hipStream_t, hipEvent_t);                                                  \
  template hipError_t gather_cols<T>(const T*, int64_t, int64_t, int64_t, const int64_t*, int64_t, T*, int64_t,     \
                                     hipStream_t);                                                                 \
  template hipError_t scatter_rows<T>(const T*, int64_t, int64_t, int64_t, const int64_t*, T*, int64_t, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
