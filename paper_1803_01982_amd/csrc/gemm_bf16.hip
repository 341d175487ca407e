// The mixed-precision form's GEMM passes on BF16 MFMA with FP32 accumulation:
//
//   sketch      B = Omega A  (Algorithm 2, sample matrix): one product of
//               BF16 operands, X = bf16(Omega^T) (rounded from FP64 when
//               Omega is drawn) and bf16(A) rounded from the FP32 entries of
//               A in registers; the column norms ||A(:, j)||^2 are summed in
//               FP64 from the FP32 entries in the same pass.
//   projection  W = Q1^T A  (partial QR block form, Sections 2.1 and 3.1):
//               split-BF16, x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
//               (x - hi is exact in FP32), and
//                 Q^T A ~ Qhi^T Ahi + Qhi^T Alo + Qlo^T Ahi,
//               dropping Qlo^T Alo (about 2^-16 of a product), three MFMAs
//               into one FP32 accumulator.  Q is split once into BF16 arrays
//               by split_bf16_kernel; A is split in registers.
//
// Both operands are K-contiguous (K = m): X is M x K (stored K-major, ldx a
// multiple of 8 on a 16-byte aligned base), Y is FP32 K x N (ldy).  Two
// kernel forms:
//   wide-column (gemm_bf16_xl_kernel, when K is a multiple of 64 and the
//     columns of Y are 16-byte aligned): X through LDS by direct global ->
//     LDS loads, each wave owning 32 columns of Y for every row of its
//     group, straight from global memory into registers;
//   narrow (gemm_bf16_kernel, any K and alignment): one workgroup of eight
//     waves covers a group of up to 640 rows of C (512 for the
//     three-product form) and a block of 64 columns; wave w owns the row
//     tiles w, w + 8, ... and all four 16-column tiles of the block, its X
//     fragments loaded straight from global memory into registers (16 bytes
//     per lane: eight consecutive k of one row) one K step ahead, while the
//     FP32 columns of Y go through LDS once per K step (loaded one step
//     ahead, rounded or split into BF16, stored as [column][k] rows of 40
//     BF16 so that the 16 lanes reading one k-slice of 16 columns hit
//     distinct banks) and are read by every wave as its B fragments.
// Both use MFMA 16x16x32 (BF16 in, FP32 out) and one workgroup barrier per K
// step, and split K when the grid would not cover the chip (partial sums
// added in a fixed order).
//
// Lane layout of v_mfma_f32_16x16x32_bf16 (checked by an in-bounds probe on
// gfx950): lane l holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]
// for e = 0..7; result register r of lane l is D[4 (l / 16) + r][l % 16].
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MB_NT = 512;            // threads per workgroup (eight waves)
constexpr int MB_BN = 64;             // columns per workgroup
constexpr int MB_MAXT = 40;           // row tiles per group (640 rows)
constexpr int MB_KMAX = 64;           // largest K step (two MFMA k-slices)

__device__ inline f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// BF16 round to nearest even of an FP32 value (the hardware conversion).
__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// NP = 1: C = Xhi^T bf16(Y).  NP = 3: C = Xhi^T Yhi + Xhi^T Ylo + Xlo^T Yhi.
// NTW = row tiles per wave (ceil(MT / 8)).  Xlo is unused for NP = 1.
// KS = MFMA k-slices of 32 per K step: 2 (a 64-deep step, half the barriers
// and twice the bytes in flight per prefetch) unless the three-product form
// with three or more row tiles per wave needs the registers (KS = 1).  The products
// are accumulated in the same order for either KS.
template <int NP, int NTW>
struct Bf16Step {
  static constexpr int KS = (NP == 3 && NTW >= 3) ? 1 : 2;
  static constexpr int BK = 32 * KS;
  static constexpr int YS = BK + 8;  // BF16 per LDS row of a Y column (the padding spreads the banks)
};

template <int NP, int NTW>
__global__ __launch_bounds__(MB_NT) void gemm_bf16_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, const __bf16* __restrict__ Xhi, const __bf16* __restrict__ Xlo,
    int64_t ldx, const float* __restrict__ Y, int64_t ldy, float* __restrict__ C, int64_t ldc, int64_t cstride,
    double* __restrict__ colnorm, int64_t nstride, int groups, int rows_per_group) {
  constexpr int NB = NP == 1 ? 1 : 2;  // BF16 parts of Y held in LDS
  constexpr int KS = Bf16Step<NP, NTW>::KS, MB_BK = Bf16Step<NP, NTW>::BK, MB_YS = Bf16Step<NP, NTW>::YS;
  constexpr int YPT = MB_BK / 8;  // Y values per thread and step (four or eight consecutive k)
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][NB][MB_BN * MB_YS];
  __shared__ double nred[MB_NT];

  // workgroup -> (column block, row group); the groups of one column block
  // take ids eight apart (same XCD, shared L2 for their common A columns)
  int64_t tile = blockIdx.x;
  int grp = 0;
  if (groups > 1) {
    const int64_t per = 8 * (int64_t)groups;
    tile = (int64_t)(blockIdx.x / per) * 8 + blockIdx.x % 8;
    grp = (int)((blockIdx.x % per) / 8);
  }
  const int64_t n0 = tile * MB_BN, r0 = (int64_t)grp * rows_per_group;
  if (n0 >= N || r0 >= M) return;
  const int64_t Mg = M - r0 < rows_per_group ? M - r0 : rows_per_group;
  const int MT = (int)((Mg + 15) / 16);
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;  // fragment row/column and k-group

  // X fragments: tile t = wave + 8 i, row r0 + 16 t + fr, k = k0 + 8 fg .. +7.
  // Rows past Mg read row Mg - 1 (their results are discarded); k past ke
  // is zero-filled.
  const __bf16* xrow_hi[NTW];
  const __bf16* xrow_lo[NTW];
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    int64_t row = (int64_t)16 * (wave + 8 * i) + fr;
    row = row < Mg ? row : Mg - 1;
    xrow_hi[i] = Xhi + (r0 + row) * ldx;
    xrow_lo[i] = NP == 3 ? Xlo + (r0 + row) * ldx : nullptr;
  }
  // fragment (tile i, k-slice ks) at index i * KS + ks
  auto load_x = [&](bf16x8* xh, bf16x8* xl, int64_t k0) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t k = k0 + 32 * ks + 8 * fg;
      const bool full = k + 8 <= ke;
#pragma unroll
      for (int i = 0; i < NTW; ++i) {
        if (full) {
          xh[i * KS + ks] = *reinterpret_cast<const bf16x8*>(xrow_hi[i] + k);
          if (NP == 3) xl[i * KS + ks] = *reinterpret_cast<const bf16x8*>(xrow_lo[i] + k);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            xh[i * KS + ks][e] = k + e < ke ? xrow_hi[i][k + e] : (__bf16)0.0f;
            if (NP == 3) xl[i * KS + ks][e] = k + e < ke ? xrow_lo[i][k + e] : (__bf16)0.0f;
          }
        }
      }
    }
  };

  // Y loader: thread tid moves YPT consecutive k (k0 + YPT (tid % 8)) of
  // column n0 + tid / 8 (16 or 32 bytes); columns past N read column N - 1
  // and k past ke is zeroed.
  const int yc = tid >> 3, yk = (tid & 7) * YPT;
  const int64_t ycol = n0 + yc < N ? n0 + yc : N - 1;
  const float* ysrc = Y + ycol * ldy;
  const bool ycol_ok = n0 + yc < N;
  // 16-byte loads need 16-byte aligned columns (ldy % 4 == 0, aligned base)
  const bool yvec = (ldy & 3) == 0 && (reinterpret_cast<uintptr_t>(Y) & 15) == 0;
  float yv[YPT];
  auto load_y = [&](int64_t k0) {
    const int64_t k = k0 + yk;
    if (yvec && k + YPT <= ke) {
#pragma unroll
      for (int h = 0; h < YPT / 4; ++h) {
        const float4 v = *reinterpret_cast<const float4*>(ysrc + k + 4 * h);
        yv[4 * h] = v.x;
        yv[4 * h + 1] = v.y;
        yv[4 * h + 2] = v.z;
        yv[4 * h + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < YPT; ++e) yv[e] = k + e < ke ? ysrc[k + e] : 0.0f;
    }
  };
  double nrm = 0.0;
  auto store_y = [&](int buf) {
    __bf16 hi[YPT], lo[YPT];
#pragma unroll
    for (int e = 0; e < YPT; ++e) {
      const float y = ycol_ok ? yv[e] : 0.0f;
      hi[e] = to_bf16(y);
      if (NP == 3) lo[e] = to_bf16(y - (float)hi[e]);
      nrm = fma((double)y, (double)y, nrm);
    }
    __bf16* dst = &Ys[buf][0][yc * MB_YS + yk];
#pragma unroll
    for (int e = 0; e < YPT; ++e) dst[e] = hi[e];
    if (NP == 3) {
      __bf16* dl = &Ys[buf][NB - 1][yc * MB_YS + yk];
#pragma unroll
      for (int e = 0; e < YPT; ++e) dl[e] = lo[e];
    }
  };

  f32x4 acc[NTW][4];
#pragma unroll
  for (int i = 0; i < NTW; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // PRE: the next step's X fragments are loaded into a second register set
  // before the current MFMAs; without it (the three-product form with five
  // row tiles per wave, where two sets do not fit the 256 VGPRs of a wave)
  // they are loaded into the same registers right after the MFMAs that read
  // them, and the other wave of the SIMD covers the latency.
  constexpr bool PRE = NP == 1 || NTW <= 4;  // always true with the groups chosen below
  constexpr int NX = PRE ? NTW * KS : 1;
  bf16x8 xh[NTW * KS], xl[NTW * KS], nh[NX], nl[NX];
  const int64_t nsteps = (ke - kb + MB_BK - 1) / MB_BK;
  if (nsteps > 0) {
    load_y(kb);
    store_y(0);
    load_x(xh, xl, kb);
    load_y(kb + MB_BK);
  }
  for (int64_t st = 0; st < nsteps; ++st) {
    const int64_t k0 = kb + st * MB_BK;
    const int buf = (int)(st & 1);
    if (PRE && st + 1 < nsteps) load_x(nh, nl, k0 + MB_BK);
    __syncthreads();  // Ys[buf] complete; every read of Ys[buf ^ 1] done
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int yo = (16 * c + fr) * MB_YS + 32 * ks + 8 * fg;
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Ys[buf][0][yo]);
        bf16x8 bl;
        if (NP == 3) bl = *reinterpret_cast<const bf16x8*>(&Ys[buf][NB - 1][yo]);
#pragma unroll
        for (int i = 0; i < NTW; ++i) {
          if (wave + 8 * i < MT) {
            acc[i][c] = mfma_bf16(xh[i * KS + ks], bh, acc[i][c]);
            if (NP == 3) {
              acc[i][c] = mfma_bf16(xh[i * KS + ks], bl, acc[i][c]);
              acc[i][c] = mfma_bf16(xl[i * KS + ks], bh, acc[i][c]);
            }
          }
        }
      }
    }
    if (st + 1 < nsteps) {
      if (PRE) {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          xh[i] = nh[i];
          if (NP == 3) xl[i] = nl[i];
        }
      } else {
        load_x(xh, xl, k0 + MB_BK);
      }
      store_y(buf ^ 1);
      if (st + 2 < nsteps) load_y(k0 + 2 * MB_BK);
    }
  }

  float* Cz = C + (int64_t)blockIdx.z * cstride + r0;
#pragma unroll
  for (int i = 0; i < NTW; ++i) {
    const int t = wave + 8 * i;
    if (t >= MT) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * t + 4 * fg + r, col = n0 + 16 * c + fr;
        if (row < Mg && col < N) Cz[col * ldc + row] = acc[i][c][r];
      }
  }
  if (colnorm != nullptr && grp == 0) {
    // the eight threads of a column hold disjoint k ranges: fixed-order sum
    nred[tid] = nrm;
    __syncthreads();
    if (tid < MB_BN && n0 + tid < N) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += nred[tid * 8 + q];
      colnorm[(int64_t)blockIdx.z * nstride + n0 + tid] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Wide-column form.  The rows of X (all MTG row tiles of a group) go through
// LDS, the columns of Y straight into registers:
//   - X: per 64-deep K step, MTG x NPART x 2 MFMA operand fragments of 1 KB,
//     each moved by one direct global -> LDS load instruction
//     (global_load_lds_dwordx4) in which lane l fetches the 16 bytes it will
//     later read back as its operand: row 16 t + l % 16, k = 8 (l / 16) ..
//     + 7 of the slice.  LDS then holds every fragment in operand order,
//     read back with one conflict-free 16-byte read per lane.  Two stage
//     buffers (two distinct LDS arrays, so the compiler can tell that the
//     loads into one do not alias the reads of the other), loaded one step
//     ahead.
//   - Y: wave w owns NC 16-column tiles (the workgroup 128 NC columns) for
//     every row tile of the group, so a Y value is needed by one wave only:
//     each lane loads the eight consecutive k of its column that form its B
//     operand (two 16-byte loads per k-slice), one step ahead, and rounds
//     (splits) them to BF16 in registers.
// One wait for this wave's loads and one workgroup barrier per K step; the
// loads of step s + 1 are issued right after that barrier, before the
// MFMAs of step s (a scheduling barrier keeps that order).  The products of
// one accumulator run in the same order as in the narrow form above.
constexpr int XL_NT = 512;
constexpr int XL_BK = 64;
constexpr int XL_FRAG = 1024;  // bytes of one operand fragment: 64 lanes x 16 bytes

template <int NP, int MTG, int NC>
struct XlShape {
  static constexpr int NPART = NP == 1 ? 1 : 2;
  static constexpr int NF = MTG * NPART * 2;  // fragments per K step
  static constexpr int FPW = (NF + 7) / 8;    // fragments loaded per wave
  static constexpr int STAGE = NF * XL_FRAG;  // LDS bytes per K step
  static constexpr int BN = 8 * 16 * NC;      // columns per workgroup
};

// One direct global -> LDS load: 16 bytes per lane from src to
// dst + 16 lane (dst the same for the whole wave).
__device__ __forceinline__ void xl_issue(const __bf16* src, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// Scheduling groups for the MFMAs of one k-slice: the reads of the first
// two row tiles, then per tile its MFMAs with the RPT reads of the tile two
// ahead placed between them.
template <int T, int MTG, int RPT, int MPT>
__device__ __forceinline__ void xl_sched() {
  if constexpr (T == 0) __builtin_amdgcn_sched_group_barrier(0x100, MTG > 1 ? 2 * RPT : RPT, 0);
  if constexpr (T < MTG) {
    constexpr int R = T + 2 < MTG ? RPT : 0;
    constexpr int M0 = (MPT + 1) / 2, M1 = MPT - M0;
    constexpr int R0 = (R + 1) / 2, R1 = R - R0;
    __builtin_amdgcn_sched_group_barrier(0x008, M0, 0);
    if constexpr (R0 > 0) __builtin_amdgcn_sched_group_barrier(0x100, R0, 0);
    if constexpr (M1 > 0) __builtin_amdgcn_sched_group_barrier(0x008, M1, 0);
    if constexpr (R1 > 0) __builtin_amdgcn_sched_group_barrier(0x100, R1, 0);
    xl_sched<T + 1, MTG, RPT, MPT>();
  }
}

template <int NP, int MTG, int NC>
__global__ __launch_bounds__(XL_NT) void gemm_bf16_xl_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, const __bf16* __restrict__ Xhi, const __bf16* __restrict__ Xlo,
    int64_t ldx, const float* __restrict__ Y, int64_t ldy, float* __restrict__ C, int64_t ldc, int64_t cstride,
    double* __restrict__ colnorm, int64_t nstride, int groups, int rows_per_group) {
  typedef XlShape<NP, MTG, NC> S;
  constexpr int NPART = S::NPART, NF = S::NF, FPW = S::FPW;
  __shared__ __attribute__((aligned(16))) unsigned char xs0[S::STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char xs1[S::STAGE];

  int64_t tile = blockIdx.x;
  int grp = 0;
  if (groups > 1) {
    const int64_t per = 8 * (int64_t)groups;
    tile = (int64_t)(blockIdx.x / per) * 8 + blockIdx.x % 8;
    grp = (int)((blockIdx.x % per) / 8);
  }
  const int64_t n0 = tile * S::BN, r0 = (int64_t)grp * rows_per_group;
  if (n0 >= N || r0 >= M) return;
  const int64_t Mg = M - r0 < rows_per_group ? M - r0 : rows_per_group;
  const int MT = (int)((Mg + 15) / 16);
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps fragment indices scalar
  const int fr = lane & 15, fg = lane >> 4;

  // fragment f = (t NPART + p) 2 + s (row tile t, part p, k-slice s) is
  // loaded by wave f % 8.  Lane (fr, fg) of it reads row 16 t + fr,
  // k = 32 s + 8 fg ..: a per-lane offset plus a uniform one, except in a
  // tile that crosses Mg, whose rows past Mg read row Mg - 1 (results
  // discarded).
  const int64_t lane_off = (int64_t)fr * ldx + 8 * fg;
  auto issue_x = [&](unsigned char* buf, int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < FPW; ++i) {
      const int f = wave + 8 * i;
      if (f < NF) {
        const int t = f / (2 * NPART), s = f & 1;
        const __bf16* part = ((f / 2) % NPART) ? Xlo : Xhi;
        const __bf16* src;
        if (16 * t + 16 <= Mg) {
          src = part + (r0 + 16 * t) * ldx + 32 * s + k0 + lane_off;
        } else {
          const int64_t row = 16 * t + fr < Mg ? 16 * t + fr : Mg - 1;
          src = part + (r0 + row) * ldx + 32 * s + 8 * fg + k0;
        }
        xl_issue(src, buf + f * XL_FRAG);
      }
    }
  };

  // Y: column n0 + 16 (NC wave + c) + fr (clamped to N - 1), k = k0 + 32 s + 8 fg
  const float* ycol[NC];
  bool yok[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t col = n0 + 16 * (NC * wave + c) + fr;
    yok[c] = col < N;
    ycol[c] = Y + (col < N ? col : N - 1) * ldy + 8 * fg;
  }
  float yr[NC][2][8];
  auto load_y = [&](int s, int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float* p = ycol[c] + k0 + 32 * s;
      const float4 a = *reinterpret_cast<const float4*>(p);
      const float4 b = *reinterpret_cast<const float4*>(p + 4);
      yr[c][s][0] = a.x; yr[c][s][1] = a.y; yr[c][s][2] = a.z; yr[c][s][3] = a.w;
      yr[c][s][4] = b.x; yr[c][s][5] = b.y; yr[c][s][6] = b.z; yr[c][s][7] = b.w;
    }
  };

  f32x4 acc[MTG][NC];
#pragma unroll
  for (int t = 0; t < MTG; ++t)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  double nrm[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) nrm[c] = 0.0;

  const int64_t nsteps = (ke - kb) / XL_BK;  // K and the chunk are whole steps

  // one K step on stage `cur`, loading step st + 1 into `nxt`.  The two
  // k-slices run one after the other: slice s of Y is rounded to BF16 and
  // its registers reloaded with slice s of the next step before the MFMAs
  // of slice s over all row tiles.
  auto step = [&](const unsigned char* cur, unsigned char* nxt, int64_t st) __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads of step st have landed
    __syncthreads();                     // every wave's loads of step st; every read of nxt done
    const bool more = st + 1 < nsteps;
    const int64_t k1 = kb + (st + 1) * XL_BK;
    const unsigned char* xb = cur + 16 * lane;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 yh[NC], yl[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float y = yok[c] ? yr[c][s][e] : 0.0f;
          const __bf16 h = to_bf16(y);
          yh[c][e] = h;
          if (NP == 3) yl[c][e] = to_bf16(y - (float)h);
          if (NP == 1) nrm[c] = fma((double)y, (double)y, nrm[c]);
        }
      if (more) {
        if (s == 0) issue_x(nxt, k1);
        load_y(s, k1);
      }
      __builtin_amdgcn_sched_barrier(0);
      // operand reads run two row tiles ahead of the MFMAs (a ring of three
      // register sets); the interleave is pinned for the scheduler below
      bf16x8 xh[3], xl[3];
      auto rd = [&](int t) __attribute__((always_inline)) {
        xh[t % 3] = *reinterpret_cast<const bf16x8*>(xb + ((t * NPART) * 2 + s) * XL_FRAG);
        if (NP == 3) xl[t % 3] = *reinterpret_cast<const bf16x8*>(xb + ((t * NPART + 1) * 2 + s) * XL_FRAG);
      };
      rd(0);
      if (MTG > 1) rd(1);
#pragma unroll
      for (int t = 0; t < MTG; ++t) {
        if (t + 2 < MTG) rd(t + 2);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          acc[t][c] = mfma_bf16(xh[t % 3], yh[c], acc[t][c]);
          if (NP == 3) {
            acc[t][c] = mfma_bf16(xh[t % 3], yl[c], acc[t][c]);
            acc[t][c] = mfma_bf16(xl[t % 3], yh[c], acc[t][c]);
          }
        }
      }
      xl_sched<0, MTG, NPART, NP * NC>();
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  if (nsteps > 0) {
    issue_x(xs0, kb);
    load_y(0, kb);
    load_y(1, kb);
  }
  for (int64_t st = 0; st < nsteps; st += 2) {
    step(xs0, xs1, st);
    if (st + 1 < nsteps) step(xs1, xs0, st + 1);
  }

  float* Cz = C + (int64_t)blockIdx.z * cstride + r0;
#pragma unroll
  for (int t = 0; t < MTG; ++t) {
    if (t >= MT) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t col = n0 + 16 * (NC * wave + c) + fr;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * t + 4 * fg + r;
        if (row < Mg) Cz[col * ldc + row] = acc[t][c][r];
      }
    }
  }
  if (NP == 1 && colnorm != nullptr && grp == 0) {
    // the four lanes of a column (k groups fg) hold disjoint k: pairwise sums
    // in a fixed pairing, the same value on every lane
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double v = nrm[c];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int64_t col = n0 + 16 * (NC * wave + c) + fr;
      if (fg == 0 && col < N) colnorm[(int64_t)blockIdx.z * nstride + col] = v;
    }
  }
}

// xhi = bf16(x), xlo = bf16(x - xhi) for an M x K column-major FP32 block
// (ld), written K-major with leading dimension ldo.
__global__ void split_bf16_kernel(const float* __restrict__ X, int64_t rows, int64_t cols, int64_t ld,
                                  __bf16* __restrict__ hi, __bf16* __restrict__ lo, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= rows || j >= cols) return;
  const float x = X[j * ld + i];
  const __bf16 h = to_bf16(x);
  hi[j * ldo + i] = h;
  lo[j * ldo + i] = to_bf16(x - (float)h);
}

__global__ void splitk_reduce_f32(int64_t M, int64_t N, int splits, const float* __restrict__ P,
                                  float* __restrict__ C, int64_t ldc, const double* __restrict__ np,
                                  double* __restrict__ colnorm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < M * N) {
    const int64_t row = idx % M, col = idx / M;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += P[(int64_t)z * M * N + idx];
    C[col * ldc + row] = s;
  }
  if (colnorm && idx < N) {
    double s = 0;
    for (int z = 0; z < splits; ++z) s += np[(int64_t)z * N + idx];
    colnorm[idx] = s;
  }
}

// Row groups: at most 40 row tiles (640 rows) per group for the one-product
// form; 32 (512 rows, four tiles per wave) for the three-product form, whose
// five-tile variant does not fit the 256 VGPRs of a wave.
void bf16_shape(int nprod, int64_t M, int* groups, int* rows_per_group, int* ntw) {
  const int maxt = nprod == 1 ? MB_MAXT : 32;
  const int64_t g = (M + 16 * maxt - 1) / (16 * maxt);
  const int64_t rows = ((M + g - 1) / g + 15) / 16 * 16;
  *groups = (int)g;
  *rows_per_group = (int)rows;
  *ntw = (int)((rows / 16 + 7) / 8);
}

int bf16_splits(int nprod, int64_t M, int64_t N, int64_t K, int num_cu) {
  int groups, rpg, ntw;
  bf16_shape(nprod, M, &groups, &rpg, &ntw);
  const int64_t tiles = (N + MB_BN - 1) / MB_BN * groups;
  int64_t s = 1;
  while (tiles * s < (int64_t)num_cu && K / (s * 2) >= 2048) s *= 2;
  return (int)s;
}

template <int NP, int NTW = 1>
hipError_t launch_bf16(int ntw, dim3 grid, hipStream_t s, int64_t M, int64_t N, int64_t K, int64_t kchunk,
                       const __bf16* Xhi, const __bf16* Xlo, int64_t ldx, const float* Y, int64_t ldy, float* C,
                       int64_t ldc, int64_t cstride, double* colnorm, int64_t nstride, int groups, int rpg) {
  if constexpr (NTW <= (NP == 1 ? 5 : 4)) {
    if (ntw == NTW) {
      gemm_bf16_kernel<NP, NTW><<<grid, MB_NT, 0, s>>>(M, N, K, kchunk, Xhi, Xlo, ldx, Y, ldy, C, ldc, cstride,
                                                       colnorm, nstride, groups, rpg);
      return hipGetLastError();
    }
    return launch_bf16<NP, NTW + 1>(ntw, grid, s, M, N, K, kchunk, Xhi, Xlo, ldx, Y, ldy, C, ldc, cstride,
                                    colnorm, nstride, groups, rpg);
  } else {
    return hipErrorInvalidValue;
  }
}

// Wide-column launch: NP products, MTG row tiles per group, NC column tiles
// per wave; K split into `splits` chunks of whole 64-deep steps.
template <int NP, int MTG, int NC>
hipError_t launch_xl(int64_t M, int64_t N, int64_t K, int splits, const __bf16* Xhi, const __bf16* Xlo, int64_t ldx,
                     const float* Y, int64_t ldy, float* out, int64_t ldo, int64_t ostride, double* nout,
                     int64_t nstride, int groups, int rpg, hipStream_t s) {
  typedef XlShape<NP, MTG, NC> S;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + XL_BK - 1) / XL_BK * XL_BK;
  const int64_t ntile = (N + S::BN - 1) / S::BN;
  const int64_t gx = groups > 1 ? (ntile + 7) / 8 * 8 * groups : ntile;
  gemm_bf16_xl_kernel<NP, MTG, NC><<<dim3((unsigned)gx, 1u, (unsigned)splits), XL_NT, 0, s>>>(
      M, N, K, kchunk, Xhi, Xlo, ldx, Y, ldy, out, ldo, ostride, nout, nstride, groups, rpg);
  return hipGetLastError();
}

}  // namespace

namespace {

// Plan of the wide-column form: K a whole number of 64-deep steps and Y in
// 16-byte aligned columns (its loads are unconditional 16-byte loads); row
// groups of at most 17 tiles, or one group of at most eight for small M;
// K split until the grid covers the chip.
struct XlPlan {
  bool ok;
  int mtg, groups, rpg, splits;
};

XlPlan xl_plan(int64_t M, int64_t N, int64_t K, bool y_aligned, int num_cu) {
  XlPlan p{false, 0, 0, 0, 1};
  if (K % XL_BK != 0 || !y_aligned) return p;
  const int64_t T = (M + 15) / 16;
  if (T <= 8) {
    p.mtg = 8;
    p.groups = 1;
  } else {
    p.mtg = 17;
    p.groups = (int)((T + 16) / 17);
  }
  p.rpg = (int)((T + p.groups - 1) / p.groups * 16);
  const int64_t tiles = (N + XlShape<1, 17, 2>::BN - 1) / XlShape<1, 17, 2>::BN * p.groups;
  int64_t sp = 1;
  while (tiles * sp < (int64_t)num_cu && K / (sp * 2) >= 2048) sp *= 2;
  p.splits = (int)sp;
  p.ok = true;
  return p;
}

}  // namespace

size_t gemm_bf16_scratch(int64_t M, int64_t N, int64_t K, int num_cu) {
  int s = std::max(bf16_splits(1, M, N, K, num_cu), bf16_splits(3, M, N, K, num_cu));
  const XlPlan xp = xl_plan(M, N, K, true, num_cu);
  if (xp.ok) s = std::max(s, xp.splits);
  if (s == 1) return 0;
  return (size_t)s * M * N * sizeof(float) + (size_t)s * N * sizeof(double) + 1024;
}

hipError_t gemm_bf16(int nprod, int64_t M, int64_t N, int64_t K, const __bf16* Xhi, const __bf16* Xlo, int64_t ldx,
                     const float* Y, int64_t ldy, float* C, int64_t ldc, double* colnorm, Arena& ar, int num_cu,
                     hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K <= 0 || (nprod != 1 && nprod != 3) || M > 4 * 16 * MB_MAXT) return hipErrorInvalidValue;
  // 16-byte X fragment loads: rows of X start on 16-byte boundaries
  if ((ldx % 8) != 0 || (reinterpret_cast<uintptr_t>(Xhi) & 15) != 0 ||
      (Xlo != nullptr && (reinterpret_cast<uintptr_t>(Xlo) & 15) != 0))
    return hipErrorInvalidValue;
  const bool y_aligned = (ldy & 3) == 0 && (reinterpret_cast<uintptr_t>(Y) & 15) == 0;
  const XlPlan xp = xl_plan(M, N, K, y_aligned, num_cu);
  int groups, rpg, ntw;
  bf16_shape(nprod, M, &groups, &rpg, &ntw);
  const int splits = xp.ok ? xp.splits : bf16_splits(nprod, M, N, K, num_cu);
  float* out = C;
  int64_t ldo = ldc, ostride = 0, nstride = 0;
  double* nout = colnorm;
  float* part = nullptr;
  double* npart = nullptr;
  if (splits > 1) {
    part = ar.take<float>((size_t)splits * M * N);
    npart = colnorm ? ar.take<double>((size_t)splits * N) : nullptr;
    if (!part || (colnorm && !npart)) return hipErrorOutOfMemory;
    out = part;
    ldo = M;
    ostride = M * N;
    nout = npart;
    nstride = N;
  }
  hipError_t e;
  if (xp.ok) {
    if (nprod == 1)
      e = xp.mtg == 8 ? launch_xl<1, 8, 2>(M, N, K, splits, Xhi, nullptr, ldx, Y, ldy, out, ldo, ostride, nout,
                                           nstride, xp.groups, xp.rpg, s)
                      : launch_xl<1, 17, 2>(M, N, K, splits, Xhi, nullptr, ldx, Y, ldy, out, ldo, ostride, nout,
                                            nstride, xp.groups, xp.rpg, s);
    else
      e = xp.mtg == 8 ? launch_xl<3, 8, 2>(M, N, K, splits, Xhi, Xlo, ldx, Y, ldy, out, ldo, ostride, nout,
                                           nstride, xp.groups, xp.rpg, s)
                      : launch_xl<3, 17, 2>(M, N, K, splits, Xhi, Xlo, ldx, Y, ldy, out, ldo, ostride, nout,
                                            nstride, xp.groups, xp.rpg, s);
  } else {
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + MB_KMAX - 1) / MB_KMAX * MB_KMAX;  // a whole number of K steps for either step depth
    const int64_t ntile = (N + MB_BN - 1) / MB_BN;
    const int64_t gx = groups > 1 ? (ntile + 7) / 8 * 8 * groups : ntile;
    dim3 grid((unsigned)gx, 1u, (unsigned)splits);
    e = nprod == 1 ? launch_bf16<1>(ntw, grid, s, M, N, K, kchunk, Xhi, nullptr, ldx, Y, ldy, out, ldo, ostride,
                                    nout, nstride, groups, rpg)
                   : launch_bf16<3>(ntw, grid, s, M, N, K, kchunk, Xhi, Xlo, ldx, Y, ldy, out, ldo, ostride, nout,
                                    nstride, groups, rpg);
  }
  if (e != hipSuccess || splits == 1) return e;
  const int64_t total = M * N > N ? M * N : N;
  splitk_reduce_f32<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(M, N, splits, part, C, ldc, npart, colnorm);
  return hipGetLastError();
}

hipError_t split_bf16(const float* X, int64_t rows, int64_t cols, int64_t ld, __bf16* hi, __bf16* lo, int64_t ldo,
                      hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)cols);
  split_bf16_kernel<<<grid, 256, 0, s>>>(X, rows, cols, ld, hi, lo, ldo);
  return hipGetLastError();
}

}  // namespace ffsrqr
