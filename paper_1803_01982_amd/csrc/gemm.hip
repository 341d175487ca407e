// C = X^T Y on MFMA: the sketch B = Omega A (Algorithm 2, sample matrix;
// X = Omega^T) and the projection W = Q1^T A (partial QR block form,
// Sections 2.1 and 3.1; X = Q1).  Both operands are column-major and
// contiguous along the contraction index K = m, so one kernel serves both.
//
// Tile 64 x 64 per workgroup (4 waves in 2 x 2, 32 x 32 each as 2 x 2 MFMA
// 16x16x4 blocks), K step 16, double-buffered LDS with a register prefetch
// of the next K step.  Split-K over gridDim.z when the output tiles alone
// cannot fill the chip; partial products are summed in a fixed order.
// The column norms ||Y(:, j)||^2 are accumulated in FP64 from the LDS tiles
// by the workgroups of the first row-tile, so the sketch reads A only once.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2, NT = 256;

template <typename T>
__global__ __launch_bounds__(NT) void gemm_tn_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ C, int64_t ldc, int64_t cstride,
    double* __restrict__ colnorm, int64_t nstride) {
  __shared__ T Xs[2][BK][BM + PAD];
  __shared__ T Ys[2][BK][BN + PAD];
  using MF = Mfma<T>;
  typename MF::acc4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename MF::acc4{0, 0, 0, 0};

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const bool do_norm = colnorm != nullptr && blockIdx.y == 0;

  // loader mapping: 16 consecutive k by 4 columns per wave instruction
  const int lk = tid % BK, lc = tid / BK;  // lc in 0..15
  T xr[4], yr[4];
  auto load = [&](int64_t k0) {
    const int64_t k = k0 + lk;
    const bool kin = k < ke;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t mm = m0 + lc + 16 * q, nn = n0 + lc + 16 * q;
      xr[q] = (kin && mm < M) ? X[mm * ldx + k] : T(0);
      yr[q] = (kin && nn < N) ? Y[nn * ldy + k] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Xs[buf][lk][lc + 16 * q] = xr[q];
      Ys[buf][lk][lc + 16 * q] = yr[q];
    }
  };

  double nrm = 0.0;
  int cur = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) load(k0 + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Xs[cur][kr][wy * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Ys[cur][kr][wx * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MF::fma(a[i], b[j], acc[i][j]);
    }
    if (do_norm && tid < BN) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        const double y = (double)Ys[cur][kk][tid];
        nrm += y * y;
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  T* Cz = C + (int64_t)blockIdx.z * cstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wy * 32 + i * 16 + MF::row(lane, r);
        const int64_t col = n0 + wx * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) Cz[col * ldc + row] = acc[i][j][r];
      }
  if (do_norm && tid < BN && n0 + tid < N) colnorm[(int64_t)blockIdx.z * nstride + n0 + tid] = nrm;
}

// Tall-tile variant for M <= 16 MT (the sketch and projection have M = l
// rows, a few hundred): one workgroup covers all M rows and 64 columns, so
// no row tile is partly empty and X is streamed once per column block.
// Four waves, wave w owning columns 16 w .. 16 w + 15 of the block and all
// MT row tiles (MT accumulators); K step 16, double-buffered LDS with a
// register prefetch of the next step.
constexpr int TBN = 64, TPAD = 2;

template <typename T, int MT>
__global__ __launch_bounds__(NT) void gemm_tall_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ C, int64_t ldc, int64_t cstride,
    double* __restrict__ colnorm, int64_t nstride) {
  constexpr int TBM = 16 * MT;
  constexpr int XL = (TBM * BK + NT - 1) / NT;  // X elements loaded per thread per K step
  constexpr int YL = TBN * BK / NT;             // Y elements per thread (4)
  __shared__ T Xs[2][BK][TBM + TPAD];
  __shared__ T Ys[2][BK][TBN + TPAD];
  using MF = Mfma<T>;
  typename MF::acc4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = typename MF::acc4{0, 0, 0, 0};

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n0 = (int64_t)blockIdx.x * TBN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const bool do_norm = colnorm != nullptr;

  // loader: element e = tid + NT q of a tile is (row e / BK, k e % BK), so
  // sixteen consecutive threads read one 16-element run along K
  T xr[XL], yr[YL];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int e = tid + NT * q, row = e / BK;
      const int64_t k = k0 + (e % BK);
      xr[q] = (row < TBM && row < M && k < ke) ? X[(int64_t)row * ldx + k] : T(0);
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int e = tid + NT * q, col = e / BK;
      const int64_t k = k0 + (e % BK), nn = n0 + col;
      yr[q] = (nn < N && k < ke) ? Y[nn * ldy + k] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int e = tid + NT * q, row = e / BK;
      if (row < TBM) Xs[buf][e % BK][row] = xr[q];
    }
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      const int e = tid + NT * q;
      Ys[buf][e % BK][e / BK] = yr[q];
    }
  };

  double nrm = 0.0;
  int cur = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) load(k0 + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      const T b = Ys[cur][kr][wave * 16 + (lane & 15)];
      T a[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) a[t] = Xs[cur][kr][t * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = MF::fma(a[t], b, acc[t]);
    }
    if (do_norm && tid < TBN) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        const double y = (double)Ys[cur][kk][tid];
        nrm += y * y;
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  T* Cz = C + (int64_t)blockIdx.z * cstride;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = t * 16 + MF::row(lane, r);
      const int64_t col = n0 + wave * 16 + (lane & 15);
      if (row < M && col < N) Cz[col * ldc + row] = acc[t][r];
    }
  if (do_norm && tid < TBN && n0 + tid < N) colnorm[(int64_t)blockIdx.z * nstride + n0 + tid] = nrm;
}

// Eight-wave form of the tall-tile kernel: two waves per SIMD, so that the
// LDS traffic of one wave overlaps the MFMAs of the other.  Wave w owns
// columns 16 (w % 4) .. 16 (w % 4) + 15; waves 0-3 own the row tiles
// 0 .. MA - 1 and waves 4-7 the tiles MA .. MT - 1 (MA = ceil(MT / 2)).  The
// two wave groups run separate instantiations of one body, selected by a
// wave-uniform branch, so neither carries a per-tile predicate; the second
// group also accumulates the column norms from its B fragments, which cover
// every K index of its 16 columns once.
//
// Within a K step the fragments of the next k4 slice are read while the
// MFMAs of the current one run; the register set holding the next step's
// global loads is stored into the other LDS buffer after the first MFMA
// group and then refilled two steps ahead.  The one barrier per step sits
// before the last MFMA group, and the next step's first fragments are read
// behind it.
//
// LDS layout.  FP64: element (k, r) of a tile sits in row k at column
// r ^ k (the swizzle stays inside the 16-row tile) and the row stride is
// 16 mod 32 elements; then both the transposing stores (16 k by 2 rows per
// 32 lanes) and the fragment reads (2 k by 16 rows per 32 lanes) touch 32
// distinct 8-byte bank pairs.  FP32: a row stride of 2 mod 32 elements,
// which measured best for 4-byte elements.
constexpr int NT8 = 512;

template <typename T>
struct Tall8Layout {
  static constexpr bool swz = sizeof(T) == 8;
  static constexpr int pad = swz ? 16 : 2;
};

template <typename T, int MT, int G, bool YN>
__device__ __forceinline__ void tall8_body(int64_t n0, int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* __restrict__ X,
                                           int64_t ldx, const T* __restrict__ Y, int64_t ldy, T* __restrict__ C,
                                           int64_t ldc, int64_t cstride, double* __restrict__ colnorm, int64_t nstride,
                                           T (*Xs)[BK][32 * ((MT + 1) / 2) + Tall8Layout<T>::pad],
                                           T (*Ys)[BK][TBN + Tall8Layout<T>::pad]) {
  constexpr bool SWZ = Tall8Layout<T>::swz;
  constexpr int PAD = Tall8Layout<T>::pad;
  constexpr int MA = (MT + 1) / 2;
  constexpr int TBM = 32 * MA;                  // rows held in LDS (rows >= M are zero)
  constexpr int NTL = G == 0 ? MA : MT - MA;    // row tiles of this wave group
  constexpr int T0 = G == 0 ? 0 : MA;
  constexpr int XL = TBM * BK / NT8;            // X elements per thread per K step (= MA)
  constexpr int YL = TBN * BK / NT8;            // Y elements per thread (2)
  constexpr int XB = BK * (TBM + PAD), YB = BK * (TBN + PAD);  // elements per LDS buffer
  static_assert(BK == 16 && TBM * BK % NT8 == 0 && TBN * BK % NT8 == 0, "loader covers the tiles exactly");
  using MF = Mfma<T>;
  typename MF::acc4 acc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = typename MF::acc4{0, 0, 0, 0};

  const int tid = threadIdx.x, lane = tid & 63, wc = (tid >> 6) & 3;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;

  // loader: thread tid moves k = tid % 16 of rows tid / 16 + 32 q; every
  // load is issued at an address clamped into the operand and the values
  // outside the tile are zeroed when stored, so the loads carry no branches.
  // YN (Y stored with the columns contiguous, element (k, j) at k ldy + j):
  // thread tid moves column tid % 64 of k = tid / 64 + 8 q instead, so that
  // a wave reads 64 consecutive columns.
  const int sk = tid & 15, sr = tid >> 4;
  const int yk = tid >> 6, yc = tid & 63;
  T xr[XL], yr[YL];
  auto load = [&](int64_t k0) {
    const int64_t k = k0 + sk < K ? k0 + sk : K - 1;
#pragma unroll
    for (int q = 0; q < XL; ++q) xr[q] = X[(int64_t)min(sr + 32 * q, (int)M - 1) * ldx + k];
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      if (YN) {
        const int64_t kk = k0 + yk + 8 * q < K ? k0 + yk + 8 * q : K - 1;
        const int64_t nn = n0 + yc < N ? n0 + yc : N - 1;
        yr[q] = Y[kk * ldy + nn];
      } else {
        const int64_t nn = n0 + sr + 32 * q;
        yr[q] = Y[(nn < N ? nn : N - 1) * ldy + k];
      }
    }
  };
  T* const xst = &Xs[0][sk][SWZ ? (sr ^ sk) : sr];
  T* const yst = &Ys[0][sk][SWZ ? (sr ^ sk) : sr];
  auto store = [&](int buf, int64_t k0) {
    const bool kin = k0 + sk < ke;
#pragma unroll
    for (int q = 0; q < XL; ++q) xst[buf * XB + 32 * q] = (sr + 32 * q < M && kin) ? xr[q] : T(0);
#pragma unroll
    for (int q = 0; q < YL; ++q) {
      if (YN) {
        const int kl = yk + 8 * q;
        Ys[buf][kl][SWZ ? (yc ^ kl) : yc] = (n0 + yc < N && k0 + kl < ke) ? yr[q] : T(0);
      } else {
        yst[buf * YB + 32 * q] = (n0 + sr + 32 * q < N && kin) ? yr[q] : T(0);
      }
    }
  };

  // fragment reads: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of
  // the k4 slice, one base address per slice (the swizzle depends on k)
  const int g = lane >> 4, c = lane & 15;
  const T* xrd[BK / 4];
  const T* yrd[BK / 4];
#pragma unroll
  for (int k4 = 0; k4 < BK / 4; ++k4) {
    const int kr = 4 * k4 + g, cc = SWZ ? (c ^ kr) : c;
    xrd[k4] = &Xs[0][kr][T0 * 16 + cc];
    yrd[k4] = &Ys[0][kr][wc * 16 + cc];
  }
  double nrm = 0.0;
  auto frag = [&](T* a, T& b, int buf, int k4) {
    b = yrd[k4][buf * YB];
#pragma unroll
    for (int t = 0; t < NTL; ++t) a[t] = xrd[k4][buf * XB + 16 * t];
  };
  auto mma = [&](const T* a, T b) {
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = MF::fma(a[t], b, acc[t]);
    if (G == 1) nrm = fma((double)b, (double)b, nrm);
  };

  // one K step from LDS buffer `buf`; on entry a0/b0 and a1/b1 hold its
  // first two k4 slices (the scheduling fences keep the phases in order)
  T a0[NTL], a1[NTL], b0, b1;
  auto step = [&](int buf, int64_t k0) {
    mma(a0, b0);
    store(buf ^ 1, k0 + BK);
    load(k0 + 2 * BK);
    __builtin_amdgcn_sched_barrier(0);
    frag(a0, b0, buf, 2);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    frag(a1, b1, buf, 3);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();  // every read of `buf` has returned; the other buffer is complete
    __builtin_amdgcn_sched_barrier(0);
    frag(a0, b0, buf ^ 1, 0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    frag(a1, b1, buf ^ 1, 1);
    __builtin_amdgcn_sched_barrier(0);
  };

  // an even number of steps: a trailing step past ke multiplies zeros
  const int64_t npair = (ke - kb + 2 * BK - 1) / (2 * BK);
  load(kb);
  store(0, kb);
  load(kb + BK);
  __syncthreads();
  frag(a0, b0, 0, 0);
  frag(a1, b1, 0, 1);
  for (int64_t i = 0; i < npair; ++i) {
    const int64_t k0 = kb + 2 * BK * i;
    step(0, k0);
    step(1, k0 + BK);
  }

  T* Cz = C + (int64_t)blockIdx.z * cstride;
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = (T0 + t) * 16 + MF::row(lane, r);
      const int64_t col = n0 + wc * 16 + c;
      if (row < M && col < N) Cz[col * ldc + row] = acc[t][r];
    }
  if (G == 1 && colnorm != nullptr) {
    nrm += __shfl_xor(nrm, 16, kWave);
    nrm += __shfl_xor(nrm, 32, kWave);
    const int64_t col = n0 + wc * 16 + lane;
    if (lane < 16 && col < N) colnorm[(int64_t)blockIdx.z * nstride + col] = nrm;
  }
}

// More than 16 MT rows (M up to 1152): the rows are split into `groups`
// groups of 16 MT rows, each a workgroup of its own over the same column
// block.  Workgroups are dispatched round-robin over the eight XCDs
// (workgroup b to XCD b % 8), so the groups of one column block take ids
// eight apart: they share an XCD and its L2, which then serves the second
// read of their common columns of Y.
template <typename T, int MT, bool YN>
__global__ __launch_bounds__(NT8) void gemm_tall8_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ C, int64_t ldc, int64_t cstride,
    double* __restrict__ colnorm, int64_t nstride, int groups) {
  constexpr int PAD = Tall8Layout<T>::pad;
  __shared__ T Xs[2][BK][32 * ((MT + 1) / 2) + PAD];
  __shared__ T Ys[2][BK][TBN + PAD];
  int64_t tile = blockIdx.x;
  int grp = 0;
  if (groups > 1) {
    const int64_t per = 8 * (int64_t)groups;
    tile = (int64_t)(blockIdx.x / per) * 8 + blockIdx.x % 8;
    grp = (int)((blockIdx.x % per) / 8);
  }
  const int64_t n0 = tile * TBN, r0 = (int64_t)grp * 16 * MT;
  if (n0 >= N || r0 >= M) return;
  const int64_t Mg = M - r0 < 16 * MT ? M - r0 : 16 * MT;
  X += r0 * ldx;
  C += r0;
  if (grp != 0) colnorm = nullptr;
  if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 8) == 0)
    tall8_body<T, MT, 0, YN>(n0, Mg, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm, nstride, Xs, Ys);
  else
    tall8_body<T, MT, 1, YN>(n0, Mg, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm, nstride, Xs, Ys);
}

// C = sum_z Cpart_z (fixed order); colnorm likewise.
template <typename T>
__global__ void splitk_reduce(int64_t M, int64_t N, int splits, const T* __restrict__ P, T* __restrict__ C,
                              int64_t ldc, const double* __restrict__ np, double* __restrict__ colnorm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < M * N) {
    const int64_t row = idx % M, col = idx / M;
    T s = 0;
    for (int z = 0; z < splits; ++z) s += P[(int64_t)z * M * N + idx];
    C[col * ldc + row] = s;
  }
  if (colnorm && idx < N) {
    double s = 0;
    for (int z = 0; z < splits; ++z) s += np[(int64_t)z * N + idx];
    colnorm[idx] = s;
  }
}

constexpr int TALL_MT = 18;  // one tall-tile workgroup covers at most 16 TALL_MT rows
constexpr int TALL_GROUPS = 4;  // row groups of the tall-tile kernel (M <= 1152)

// Row groups and row tiles per group of the tall-tile kernel for M rows
// (groups == 0: M is too large for it).
void tall_shape(int64_t M, int* groups, int* mt) {
  const int64_t g = (M + 16 * TALL_MT - 1) / (16 * TALL_MT);
  if (g > TALL_GROUPS) {
    *groups = 0;
    *mt = 0;
    return;
  }
  const int64_t rows = (M + g - 1) / g;
  *groups = (int)g;
  *mt = (int)((rows + 15) / 16);
}

int pick_splits(int64_t M, int64_t N, int64_t K, int num_cu) {
  int64_t s = 1;
  int groups, mt;
  tall_shape(M, &groups, &mt);
  if (groups > 0) {
    // one workgroup per CU: as many K splits as needed to cover the chip
    const int64_t tiles = (N + TBN - 1) / TBN * groups;
    while (tiles * s < (int64_t)num_cu && K / (s * 2) >= 1024) s *= 2;
    return (int)s;
  }
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  const int64_t want = 2 * (int64_t)num_cu;
  while (tiles * s < want && K / (s * 2) >= 512) s *= 2;
  return (int)s;
}

template <typename T, int MT, bool YN>
void launch_tall(dim3 grid, hipStream_t s, int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* X, int64_t ldx,
                 const T* Y, int64_t ldy, T* C, int64_t ldc, int64_t cstride, double* colnorm, int64_t nstride,
                 int groups) {
  if constexpr (MT >= 8)
    gemm_tall8_kernel<T, MT, YN><<<grid, NT8, 0, s>>>(M, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm,
                                                      nstride, groups);
  else if constexpr (!YN)
    gemm_tall_kernel<T, MT><<<grid, NT, 0, s>>>(M, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm, nstride);
}

template <typename T, bool YN, int MT = 1>
void dispatch_tall(int mt, dim3 grid, hipStream_t s, int64_t M, int64_t N, int64_t K, int64_t kchunk, const T* X,
                   int64_t ldx, const T* Y, int64_t ldy, T* C, int64_t ldc, int64_t cstride, double* colnorm,
                   int64_t nstride, int groups) {
  if constexpr (MT <= TALL_MT) {
    if (mt == MT)
      launch_tall<T, MT, YN>(grid, s, M, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm, nstride, groups);
    else
      dispatch_tall<T, YN, MT + 1>(mt, grid, s, M, N, K, kchunk, X, ldx, Y, ldy, C, ldc, cstride, colnorm, nstride,
                                   groups);
  }
}

}  // namespace

template <typename T>
size_t gemm_tn_scratch(int64_t M, int64_t N, int64_t K, int num_cu) {
  const int s = pick_splits(M, N, K, num_cu);
  if (s == 1) return 0;
  return (size_t)s * M * N * sizeof(T) + (size_t)s * N * sizeof(double) + 1024;
}

template <typename T>
hipError_t gemm_tn(int64_t M, int64_t N, int64_t K, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                   T* C, int64_t ldc, double* colnorm, Arena& ar, int num_cu, hipStream_t s, bool y_ncontig) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K <= 0) return hipErrorInvalidValue;
  const int splits = pick_splits(M, N, K, num_cu);
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  int groups, mt;
  tall_shape(M, &groups, &mt);
  if (y_ncontig) {
    // only the eight-wave kernel reads Y by columns (rows past M are computed
    // and dropped)
    if (groups == 0) return hipErrorInvalidValue;
    mt = mt < 8 ? 8 : mt;
  }
  const bool tall = groups > 0;
  // groups > 1 only with the eight-wave kernel (mt >= 8 there)
  const int64_t ntile = (N + TBN - 1) / TBN;
  const int64_t gx = groups > 1 ? (ntile + 7) / 8 * 8 * groups : ntile;
  dim3 grid = tall ? dim3((unsigned)gx, 1u, (unsigned)splits)
                   : dim3((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
  T* out = C;
  int64_t ldo = ldc, ostride = 0, nstride = 0;
  double* nout = colnorm;
  T* part = nullptr;
  double* npart = nullptr;
  if (splits > 1) {
    part = ar.take<T>((size_t)splits * M * N);
    npart = colnorm ? ar.take<double>((size_t)splits * N) : nullptr;
    if (!part || (colnorm && !npart)) return hipErrorOutOfMemory;
    out = part;
    ldo = M;
    ostride = M * N;
    nout = npart;
    nstride = N;
  }
  if (tall && y_ncontig)
    dispatch_tall<T, true>(mt, grid, s, M, N, K, kchunk, X, ldx, Y, ldy, out, ldo, ostride, nout, nstride, groups);
  else if (tall)
    dispatch_tall<T, false>(mt, grid, s, M, N, K, kchunk, X, ldx, Y, ldy, out, ldo, ostride, nout, nstride, groups);
  else
    gemm_tn_kernel<T><<<grid, NT, 0, s>>>(M, N, K, kchunk, X, ldx, Y, ldy, out, ldo, ostride, nout, nstride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t total = M * N > N ? M * N : N;
  splitk_reduce<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(M, N, splits, part, C, ldc, npart, colnorm);
  return hipGetLastError();
}

template size_t gemm_tn_scratch<double>(int64_t, int64_t, int64_t, int);
template size_t gemm_tn_scratch<float>(int64_t, int64_t, int64_t, int);
template hipError_t gemm_tn<double>(int64_t, int64_t, int64_t, const double*, int64_t, const double*, int64_t,
                                    double*, int64_t, double*, Arena&, int, hipStream_t, bool);
template hipError_t gemm_tn<float>(int64_t, int64_t, int64_t, const float*, int64_t, const float*, int64_t,
                                   float*, int64_t, double*, Arena&, int, hipStream_t, bool);

}  // namespace ffsrqr
