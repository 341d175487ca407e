// Singular values of the small factor L (l x l) by one-sided (Hestenes)
// Jacobi in FP64 (Algorithm 9 takes an SVD of the small factor; the
// flip-flop factor L is already QR-preconditioned, which is the setting in
// which one-sided Jacobi converges in few sweeps).
//
// Block form for one cooperative launch: the columns are split into
// P = 2G blocks of bs <= 16 columns; a round-robin tournament (circle method)
// pairs the blocks so that in each of the P-1 rounds of a sweep every block
// meets one other block.  Workgroup g takes pair g of the round and copies
// its 2 bs columns C into LDS.  The rotations of the round are chosen on the
// Gram matrix of those columns: H = C^T C (FP64 MFMA), then each inner round
// rotates bs disjoint column pairs (p, q) at once, updating H <- R^T H R and
// the accumulated J <- J R (the annihilated entry set to zero, the two
// diagonal entries to a - t h and b + t h); finally the columns are replaced
// by C J (FP64 MFMA) in global memory.  Inside a workgroup the inner rounds
// are pipelined: wave 0 chooses the rotations of round ir + 1 while the
// other waves apply round ir to H and J.  The inner rounds take the cross
// pairs (one column of each block); in the first round of a sweep they take
// every pair of the union, which covers the pairs inside each block once per
// sweep.  H is recomputed from the columns at every round, so the rounding
// of the Gram updates never accumulates beyond one round, and the columns
// only ever see orthogonal transformations.  A pair is rotated when
// |h_pq| > tol sqrt(h_pp h_qq) (tol = 1e-14), with Rutishauser's formulas.
// The iteration stops after a sweep with no rotation, or after a sweep in
// which every rotated pair had |h_pq| <= s sqrt(h_pp h_qq) (at most 60
// sweeps).  In that quadratically convergent regime the cosines left after
// the sweep are of order s^2 times a modest factor (about 50 at l = 544),
// and sigma_j = ||c_j|| (sorted descending) is off by at most that much,
// relatively.  s = 1e-8 (leftover of order 1e-16) for FP64 data and for the
// vector form; for FP32 data without vectors s = 1e-4, whose leftover (of
// order 1e-7) lies below the rounding already carried by L's FP32 entries:
// the sweep after it could not change sigma beyond that rounding.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 512;
constexpr int NW = NT / kWave;
constexpr int GW = 32;  // order of the Gram and rotation arrays (2 bs <= GW)
constexpr int GS = 40;  // their row stride in LDS (rows land 16 banks apart)
constexpr double kTol = 1e-14;
constexpr double kSettled = 1e-8;    // a sweep with no larger rotation ends the iteration
constexpr double kSettled32 = 1e-4;  // the same for FP32 data, singular values only
constexpr int kMaxSweeps = 60;

__device__ inline int rr_player(int pos, int r, int P) {
  // circle method: position 0 fixed, positions 1..P-1 rotate by r
  return pos == 0 ? 0 : ((pos - 1 + r) % (P - 1)) + 1;
}
// The block pair that holds block x in round r (pair g holds positions g
// and P - 1 - g).
__device__ inline int rr_pair_of(int x, int r, int P) {
  const int pos = x == 0 ? 0 : ((x - 1 - r) % (P - 1) + (P - 1)) % (P - 1) + 1;
  return pos < P / 2 ? pos : P - 1 - pos;
}

// Barrier over part of the grid: this workgroup posts its flag (the count
// of barriers passed, which advances identically in every workgroup, so the
// flags of grid_barrier serve here too) and waits only for the workgroups
// in [a0, a0 + na) and [a1, a1 + nb), the ones whose writes it reads next.
// The same release/acquire fences and bounded wait as grid_barrier.
__device__ inline bool subset_barrier(const GridSync& gs, unsigned& epoch, int a0, int na, int a1, int nb) {
  __shared__ int s_ok;
  __syncthreads();
  ++epoch;
  if (gs.nblocks == 1) return true;
  if (threadIdx.x < kWave) {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(gs.sync + kFlagStride * blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    unsigned spins = 0;
    const int nt = na + nb;
    for (;;) {
      bool here = true;
      for (int t = threadIdx.x; t < nt; t += kWave) {
        const int q = t < na ? a0 + t : a1 + (t - na);
        here = here && __hip_atomic_load(gs.sync + kFlagStride * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
      }
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

// Entry (i, j) of R^T H R when column k of R holds alpha_k at row k and
// beta_k at the row of its partner: ai, bi and aj, bj for columns i and j,
// hij = H(i, j), hipj = H(i, partner j), hpij = H(partner i, j),
// hpipj = H(partner i, partner j).
__device__ inline double rot_entry(double ai, double bi, double aj, double bj, double hij, double hipj, double hpij,
                                   double hpipj) {
  return fma(bi, fma(bj, hpipj, aj * hpij), ai * fma(bj, hipj, aj * hij));
}

// 1 / sqrt(x) for x > 0: the hardware estimate (about 24 correct bits)
// refined by two Newton steps y <- y + y (1 - x y^2) / 2.
__device__ inline double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}

// Rotation that annihilates h in the 2x2 Gram block [[a, h], [h, b]]
// (Rutishauser's choice, the smaller angle): with d = b - a, e = 2 h,
// r = sqrt(d^2 + e^2) and D = |d| + r,
//   t = sign(d) e / D,   cs = 1 / sqrt(1 + t^2),   sn = cs t.
// Since 1 + t^2 = 2 r / D, cs = D u and sn = sign(d) e u with
// u = 1 / sqrt(2 r D), and t = sign(d) e u (2 r u): two reciprocal square
// roots and no division.  d and e are scaled by the same power of two first
// (t, cs, sn are ratios), so nothing overflows or underflows; e != 0.
__device__ inline void jacobi_rotation(double a, double b, double h, double& cs, double& sn, double& t) {
  double d = b - a, e = 2.0 * h;
  const int k = max(__builtin_amdgcn_frexp_exp(d), __builtin_amdgcn_frexp_exp(e));
  d = __builtin_amdgcn_ldexp(d, -k);
  e = __builtin_amdgcn_ldexp(e, -k);
  const double x = fma(d, d, e * e);  // in [1/4, 2)
  const double r = x * rsqrt_refined(x);
  const double D = fabs(d) + r;
  const double r2 = 2.0 * r;
  const double u = rsqrt_refined(r2 * D);
  const double eu = copysign(1.0, d) * e * u;
  cs = D * u;
  sn = eu;
  t = eu * (r2 * u);
}

// Dynamic LDS: C (ncol columns of ldc = ch + 1 rows: the ch rows of the local
// columns that this workgroup owns; rows past l and columns >= 2 bs stay
// zero), then H and J (GW rows of stride GS each), then the partial Gram sums
// of the row quarters 1..3 (3 x 3 x 256).  When the l rows of a block pair do
// not fit the LDS of one workgroup, rg workgroups share the pair, each with
// ch rows: each computes the Gram matrix of its rows, the partial Gram
// matrices are exchanged through xbuf (two buffers by round parity; a
// barrier among the rg workgroups of the pair only) and summed in a fixed
// order, so every workgroup of the pair takes the same rotations and
// applies them to its own rows.
//
// Between rounds a workgroup waits only for the workgroups that wrote the
// two blocks it takes next (the pairs that held them in the round just
// ended), not for the whole grid; every sweep ends at a grid barrier, where
// the decision to go on is taken.
//
// With vectors (lpad > 0), M holds ldm = lpad + l rows: L in rows 0..l-1,
// zeros up to lpad (a multiple of ch) and the identity in rows lpad ..
// lpad + l - 1.  The Gram matrices take the rows below lpad only, the
// rotations every row, so that after the sweeps M = [L V; 0; V] with
// L V = U diag(sigma): the right singular vectors accumulate in the last l
// rows (one-sided Jacobi on the stacked matrix).
template <typename T, bool MULTI>
__global__ __launch_bounds__(NT) void jacobi_kernel(const T* __restrict__ L, int l, int64_t ldl, double* __restrict__ M,
                                                    int ldm, int lpad, int bs, int P, int ldc, int ncol, int ch,
                                                    int rg, double* __restrict__ xbuf, unsigned* __restrict__ rot,
                                                    double* __restrict__ sig, int* __restrict__ sweeps_out,
                                                    double settled, GridSync gs) {
  typedef Mfma<double> MF;
  extern __shared__ double smem[];
  double* C = smem;
  double* H0 = C + (size_t)ncol * ldc;
  double* H1 = H0 + GW * GS;
  double* J0 = H1 + GW * GS;
  double* Pg = J0 + GW * GS;
  __shared__ double2 s_ab[2][GW];  // (alpha, beta) of column k: c_k <- alpha c_k + beta c_partner
  __shared__ double s_dn[2][GW];   // the diagonal entry of H for column k after the rotation
  __shared__ int s_sweep;  // a pair with |h_pq| > settled sqrt(h_pp h_qq) was rotated this sweep
  __shared__ int s_round;
  __shared__ unsigned short sched_full[31 * 16];
  __shared__ unsigned char part_full[31 * GW];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int W2 = 2 * bs, nct = ncol / 16;
  unsigned epoch = 0;

  for (int64_t e = (int64_t)g * NT + tid; e < (int64_t)ldm * l; e += (int64_t)G * NT) {
    const int64_t r = e % ldm, c = e / ldm;
    M[c * ldm + r] = r < l ? (double)L[c * ldl + r] : (lpad > 0 && r - lpad == c ? 1.0 : 0.0);
  }
  const int rows_gram = lpad > 0 ? lpad : l;  // rows that enter the Gram matrices
  for (int e = tid; e < ncol * ldc + 3 * GW * GS; e += NT) smem[e] = 0.0;  // C, H and J
  if (g == 0 && tid < 3) rot[tid] = 0u;
  if (!grid_barrier(gs, epoch)) return;

  // pair schedules of the local columns:
  //   full: all W2(W2-1)/2 pairs of the union in W2-1 rounds of bs disjoint
  //         pairs (circle method), used in the first round of every sweep,
  //         built once as a table;
  //   cross: the bs*bs pairs (block a, block b) in bs rounds (p, bs + (p+r) % bs),
  //         computed where they are used.
  for (int e = tid; e < (W2 - 1) * bs; e += NT) {
    const int ir = e / bs, pr = e % bs;
    const int p = rr_player(pr, ir, W2), q = rr_player(W2 - 1 - pr, ir, W2);
    sched_full[e] = (unsigned short)((min(p, q) << 8) | max(p, q));
    part_full[ir * GW + p] = (unsigned char)q;
    part_full[ir * GW + q] = (unsigned char)p;
  }
  // work of the update waves in the inner rounds: H block (pair hb_p1,
  // pair hb_p2) for threads 0..bs*bs-1 of waves 1..; J entries of pair jb_pi
  // in rows jb_r0 + jb_rs t for the threads from 256 on
  const int ut = tid - kWave;
  const bool hb_ok = ut >= 0 && ut < bs * bs;
  const int hb_p1 = hb_ok ? ut / bs : 0, hb_p2 = hb_ok ? ut % bs : 0;
  const int jt = tid - kWave - 256, jb_rs = (NT - kWave - 256) / bs;
  const bool jb_ok = jt >= 0 && jt < jb_rs * bs;
  const int jb_pi = jb_ok ? jt % bs : 0, jb_r0 = jb_ok ? jt / bs : 0;
  // Gram tiles: t = 0 -> (0,0), 1 -> (0,1), 2 -> (1,1); four quarters of the rows
  const int ntile = nct * (nct + 1) / 2;
  const int kq = ch / 4;                        // rows of a quarter of the owned rows (ch is a multiple of 16)
  const int pair = MULTI ? g / rg : g;          // block pair of this workgroup in every round
  const int r0 = MULTI ? (g % rg) * ch : 0;     // its first row (MULTI: rg > 1 workgroups per pair)
  __syncthreads();

  int sweep = 0;
  for (sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (g == 0 && tid == 0) rot[(sweep + 1) % 3] = 0u;
    if (tid == 0) s_sweep = 0;
    for (int r = 0; r < P - 1; ++r) {
      // blocks of this workgroup's pair
      const int pa = rr_player(pair, r, P);
      const int pb = rr_player(P - 1 - pair, r, P);
      const int ca0 = pa * bs, cb0 = pb * bs;
      const int na = max(0, min(bs, l - ca0)), nbk = max(0, min(bs, l - cb0));
      // local column k < bs -> block a column k, k >= bs -> block b column k - bs
      auto gcol = [&](int k) -> int {
        return k < bs ? (k < na ? ca0 + k : -1) : (k < W2 && k - bs < nbk ? cb0 + k - bs : -1);
      };
      if (tid == 0) s_round = 0;
      // load rows r0 .. r0 + ch - 1 of the local columns into C (zero past
      // l): wave w takes local columns w + kk NW, all loads in flight together
      auto load_chunk = [&](int r0) {
        for (int i0 = 0; i0 < ch; i0 += 64 * 8) {
          double v[GW / NW][8];
#pragma unroll
          for (int kk = 0; kk < GW / NW; ++kk) {
            const int k = wave + kk * NW;
            const int gc = gcol(k);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int i = i0 + u * 64 + lane;
              v[kk][u] = (gc >= 0 && i < ch && r0 + i < ldm) ? M[(int64_t)gc * ldm + r0 + i] : 0.0;
            }
          }
#pragma unroll
          for (int kk = 0; kk < GW / NW; ++kk) {
            const int k = wave + kk * NW;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int i = i0 + u * 64 + lane;
              if (k < W2 && i < ch) C[k * ldc + i] = v[kk][u];
            }
          }
        }
      };
      // Gram H = C^T C of the local columns: task (tile gt, row quarter gh),
      // task = gt + 3 gh taken by wave task % NW (at most two per wave, their
      // sums kept in registers over the chunks); the quarter-0 sums stay in
      // the registers of waves 0..2, the others go through Pg
      typename MF::acc4 acct[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      {
        load_chunk(r0);
        __syncthreads();
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
          const int task = wave + ti * NW;
          const int gt = task % 3, gh = task / 3;
          if (task >= 12 || gt >= ntile) continue;
          if (r0 >= rows_gram) continue;  // rows of the accumulated vectors: no Gram contribution
          const int gtr = (gt == 2) ? 1 : 0, gtc = (gt == 0) ? 0 : 1;
          typename MF::acc4 acc = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
          const int klo = gh * kq, khi = klo + kq;
          const double* ca = C + (gtr * 16 + (lane & 15)) * ldc + (lane >> 4);
          const double* cb = C + (gtc * 16 + (lane & 15)) * ldc + (lane >> 4);
          int k0 = klo;
          for (; k0 + 16 <= khi; k0 += 16) {
            const double a0 = ca[k0], a1 = ca[k0 + 4], a2 = ca[k0 + 8], a3 = ca[k0 + 12];
            const double b0 = cb[k0], b1 = cb[k0 + 4], b2 = cb[k0 + 8], b3 = cb[k0 + 12];
            acc = MF::fma(a0, b0, acc);
            acc1 = MF::fma(a1, b1, acc1);
            acc = MF::fma(a2, b2, acc);
            acc1 = MF::fma(a3, b3, acc1);
          }
          for (; k0 < khi; k0 += 4) acc = MF::fma(ca[k0], cb[k0], acc);
          acct[ti] = acc + acc1;
        }
      }
      typename MF::acc4 acc0 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        const int task = wave + ti * NW;
        const int gt = task % 3, gh = task / 3;
        if (task >= 12 || gt >= ntile) continue;
        if (gh == 0) {
          acc0 = acct[ti];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) Pg[(gh - 1) * 768 + gt * 256 + q * 64 + lane] = acct[ti][q];
        }
      }
      __syncthreads();
      if (wave < ntile) {
        const int gt = wave, gtr = (gt == 2) ? 1 : 0, gtc = (gt == 0) ? 0 : 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int o = gt * 256 + q * 64 + lane;
          const double v = ((acc0[q] + Pg[o]) + Pg[768 + o]) + Pg[1536 + o];
          const int i = gtr * 16 + MF::row(lane, q), j = gtc * 16 + (lane & 15);
          if (gtr != gtc || i <= j) {
            H0[i * GS + j] = v;
            H0[j * GS + i] = v;
          }
        }
      }
      if (MULTI) {
        // partial Gram matrices of the rg workgroups of the pair: post, one
        // grid barrier, and every workgroup sums all of them in the same
        // order (its own read back from memory like the others)
        __syncthreads();
        double* xb = xbuf + (int64_t)(r & 1) * G * GW * GW;
        for (int e = tid; e < GW * GW; e += NT) xb[(int64_t)g * GW * GW + e] = H0[(e / GW) * GS + e % GW];
        if (!subset_barrier(gs, epoch, pair * rg, rg, 0, 0)) return;
        for (int e = tid; e < GW * GW; e += NT) {
          double v = 0.0;
          for (int h = 0; h < rg; ++h) v += xb[((int64_t)pair * rg + h) * GW * GW + e];
          H0[(e / GW) * GS + e % GW] = v;
        }
      }
      for (int e = tid; e < GW * GW; e += NT) {
        const int ei = e / GW, ej = e % GW;
        J0[ei * GS + ej] = (ei == ej && ei < W2) ? 1.0 : 0.0;
      }
      __syncthreads();
      // skip the round when no scheduled pair needs a rotation
      const bool full = (r == 0);
      int need = 0;
      for (int e = tid; e < W2 * W2; e += NT) {
        const int ei = e / W2, ej = e % W2;
        if (full ? ei < ej : (ei < bs && ej >= bs)) {
          const double a = H0[ei * GS + ei], b = H0[ej * GS + ej], hg = H0[ei * GS + ej];
          need |= !(a == 0.0 || b == 0.0 || hg * hg <= (kTol * kTol) * (a * b)) ? 1 : 0;
        }
      }
      const int nir = __syncthreads_or(need) ? (full ? W2 - 1 : bs) : 0;
      // inner rounds on the Gram matrix.  Round ir rotates the scheduled pairs
      // with (alpha, beta) of every column in s_ab[ir & 1] and the new
      // diagonal entries in s_dn[ir & 1].  In the iteration of round ir,
      // waves 1.. apply it to H (from one buffer into the other) and to J,
      // while wave 0 already chooses the rotations of round ir + 1: of H after
      // round ir it needs two new diagonal entries and one entry given by the
      // same expression the update evaluates.  One workgroup barrier per round.
      auto pair_of = [&](int P, int ir) -> unsigned {
        if (full) return sched_full[ir * bs + P];
        int q = P + ir;
        if (q >= bs) q -= bs;
        return (unsigned)((P << 8) | (bs + q));
      };
      int rot_acc = 0, big_acc = 0;
      // rotation of the pair (p, q) of lane `lane` (lanes >= bs compute a
      // copy of pair 0 and store nothing); a, b, hg: H(p,p), H(q,q), H(p,q)
      auto choose_rot = [&](int p, int q, double a, double b, double hg, int buf) {
        const bool skip = (a == 0.0) | (b == 0.0) | (hg * hg <= (kTol * kTol) * (a * b));
        double cs = 1.0, sn = 0.0, tt = 0.0;
        if (!skip) jacobi_rotation(a, b, hg, cs, sn, tt);
        if (lane < bs) {
          s_ab[buf][p] = make_double2(cs, -sn);
          s_ab[buf][q] = make_double2(cs, sn);
          s_dn[buf][p] = a - tt * hg;
          s_dn[buf][q] = b + tt * hg;
          if (!skip) {
            rot_acc = 1;
            if (hg * hg > (settled * settled) * (a * b)) big_acc = 1;
          }
        }
      };
      if (nir > 0 && wave == 0) {
        const unsigned pq = pair_of(lane < bs ? lane : 0, 0);
        const int p = (int)(pq >> 8), q = (int)(pq & 255u);
        choose_rot(p, q, H0[p * GS + p], H0[q * GS + q], H0[p * GS + q], 0);
      }
      __syncthreads();
      for (int ir = 0; ir < nir; ++ir) {
        const double* Hc = (ir & 1) ? H1 : H0;
        double* Hn = (ir & 1) ? H0 : H1;
        const double2* ab = s_ab[ir & 1];
        const double* dn = s_dn[ir & 1];
        const bool last = ir + 1 == nir;
        if (wave == 0) {
          if (!last) {
            // pair (p, q) of round ir + 1 and the partners x of p, y of q in round ir
            const int P = lane < bs ? lane : 0;
            int p, q, x, y;
            if (full) {
              const unsigned u = sched_full[(ir + 1) * bs + P];
              p = (int)(u >> 8);
              q = (int)(u & 255u);
              x = part_full[ir * GW + p];
              y = part_full[ir * GW + q];
            } else {
              // cross rounds: p = P, q = bs + (P + ir + 1) % bs, x = bs + (P + ir) % bs,
              // y = (P + 1) % bs (here ir + 1 < bs)
              int t1 = P + ir + 1, t0 = P + ir;
              t1 -= t1 >= bs ? bs : 0;
              t0 -= t0 >= bs ? bs : 0;
              p = P;
              q = bs + t1;
              x = bs + t0;
              y = P + 1 == bs ? 0 : P + 1;
            }
            const double hpq = Hc[p * GS + q], hpy = Hc[p * GS + y], hxq = Hc[x * GS + q], hxy = Hc[x * GS + y];
            const double2 fp = ab[p], fq = ab[q];
            const double a = dn[p], b = dn[q];
            const double hg = rot_entry(fp.x, fp.y, fq.x, fq.y, hpq, hpy, hxq, hxy);
            choose_rot(p, q, a, b, hg, (ir + 1) & 1);
          }
        } else {
          if (!last && hb_ok) {
            const unsigned u1 = pair_of(hb_p1, ir), u2 = pair_of(hb_p2, ir);
            const int p1 = (int)(u1 >> 8), q1 = (int)(u1 & 255u), p2 = (int)(u2 >> 8), q2 = (int)(u2 & 255u);
            const double h00 = Hc[p1 * GS + p2], h01 = Hc[p1 * GS + q2];
            const double h10 = Hc[q1 * GS + p2], h11 = Hc[q1 * GS + q2];
            const double2 f1 = ab[p1], g1 = ab[q1], f2 = ab[p2], g2 = ab[q2];
            if (hb_p1 == hb_p2) {
              // the rotated pair itself: new diagonal entries, the annihilated entry
              const double off = f1.y != 0.0 ? 0.0 : h01;
              Hn[p1 * GS + p1] = dn[p1];
              Hn[q1 * GS + q1] = dn[q1];
              Hn[p1 * GS + q1] = off;
              Hn[q1 * GS + p1] = off;
            } else {
              Hn[p1 * GS + p2] = rot_entry(f1.x, f1.y, f2.x, f2.y, h00, h01, h10, h11);
              Hn[p1 * GS + q2] = rot_entry(f1.x, f1.y, g2.x, g2.y, h01, h00, h11, h10);
              Hn[q1 * GS + p2] = rot_entry(g1.x, g1.y, f2.x, f2.y, h10, h11, h00, h01);
              Hn[q1 * GS + q2] = rot_entry(g1.x, g1.y, g2.x, g2.y, h11, h10, h01, h00);
            }
          }
          if (jb_ok) {
            // J <- J R on rows jb_r0 + jb_rs t (jb_rs >= 12, so three rows cover GW)
            const unsigned u = pair_of(jb_pi, ir);
            const int p = (int)(u >> 8), q = (int)(u & 255u);
            const double2 fp = ab[p], fq = ab[q];
            double jp[3], jq[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
              const int i = min(jb_r0 + jb_rs * t, W2 - 1);
              jp[t] = J0[i * GS + p];
              jq[t] = J0[i * GS + q];
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) {
              const int i = jb_r0 + jb_rs * t;
              if (i < W2) {
                J0[i * GS + p] = fma(fp.y, jq[t], fp.x * jp[t]);
                J0[i * GS + q] = fma(fq.y, jp[t], fq.x * jq[t]);
              }
            }
          }
        }
        __syncthreads();
      }
      if (nir > 0 && wave == 0) {
        const bool any_rot = __any(rot_acc), any_big = __any(big_acc);
        if (lane == 0) {
          s_round = any_rot ? 1 : 0;
          if (any_big) s_sweep = 1;
        }
      }
      __syncthreads();
      // columns <- C J, written straight to M (transposed product J^T C^T, so
      // each MFMA result row is a run of 16 consecutive entries of a column);
      // a wave takes a 16-row slice of the owned rows for both column tiles
      if (s_round) {
        const int nit = (min(ch, ldm - r0) + 15) / 16;
        for (int it = wave; it < nit; it += NW) {
          typename MF::acc4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
          const double* ja = J0 + (lane >> 4) * GS + (lane & 15);
          const double* cbp = C + (lane >> 4) * ldc + it * 16 + (lane & 15);
          if (nct == 2) {
#pragma unroll
            for (int hs = 0; hs < 8; hs += 4) {
              double bv[4], av0[4], av1[4];
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                bv[s] = cbp[4 * (hs + s) * ldc];
                av0[s] = ja[4 * (hs + s) * GS];
                av1[s] = ja[4 * (hs + s) * GS + 16];
              }
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                d0 = MF::fma(av0[s], bv[s], d0);
                d1 = MF::fma(av1[s], bv[s], d1);
              }
            }
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) d0 = MF::fma(ja[4 * s * GS], cbp[4 * s * ldc], d0);
          }
          const int i = r0 + it * 16 + (lane & 15);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = MF::row(lane, q);
            const int gc0 = gcol(j);
            if (gc0 >= 0 && i < ldm) M[(int64_t)gc0 * ldm + i] = d0[q];
            const int gc1 = gcol(16 + j);
            if (nct == 2 && gc1 >= 0 && i < ldm) M[(int64_t)gc1 * ldm + i] = d1[q];
          }
        }
      }
      if (r + 1 < P - 1) {
        // the next round's blocks: wait only for the workgroups that wrote
        // them in this round (the sweep's last round ends at the grid
        // barrier below instead)
        const int qa = rr_pair_of(rr_player(pair, r + 1, P), r, P);
        const int qb = rr_pair_of(rr_player(P - 1 - pair, r + 1, P), r, P);
        if (!subset_barrier(gs, epoch, qa * rg, rg, qb * rg, rg)) return;
      }
    }
    if (tid == 0 && s_sweep) __hip_atomic_fetch_or(&rot[sweep % 3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(gs, epoch)) return;
    const unsigned big = __hip_atomic_load(&rot[sweep % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!big) break;  // no rotation, or only rotations below the settled level
  }
  if (g == 0 && tid == 0 && sweeps_out) *sweeps_out = sweep < kMaxSweeps ? sweep + 1 : kMaxSweeps;
  // column norms
  for (int c = g * NW + wave; c < l; c += G * NW) {
    double s = 0.0;
    for (int i = lane; i < l; i += 64) {
      const double x = M[(int64_t)c * ldm + i];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sig[c] = sqrt(s);
  }
}

// sigma sorted descending (rank sort, ties by index).
__global__ void sort_desc(const double* __restrict__ in, int l, double* __restrict__ out) {
  for (int j = threadIdx.x; j < l; j += blockDim.x) {
    const double v = in[j];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = in[i];
      rank += (u > v || (u == v && i < j)) ? 1 : 0;
    }
    out[rank] = v;
  }
}

// Block size bs <= 16 (2 bs local columns <= GW); C holds ch rows (a
// multiple of 16) of the local columns padded to ncol = 16 or 32 columns, with
// ldc = ch + 1 (an odd stride spreads the MFMA operand reads over the LDS
// banks).  ch covers all l rows when they fit the LDS (up to 416 rows with
// 160 KiB), else the rows are split over the fewest workgroups per block pair
// (*rg) whose equal shares fit.  Returns false when not even 16 rows fit.
bool choose(int64_t l, const DeviceInfo& d, int* bs, int* P, int* ldc, int* ncol, int* ch, int* rg, size_t* lds) {
  int b = 16;
  if (l < 2 * b) b = (int)((l + 1) / 2 > 0 ? (l + 1) / 2 : 1);
  const int nc = (2 * b + 15) / 16 * 16;
  auto bytes = [&](int rows) { return ((size_t)nc * (rows + 1) + 3 * GW * GS + 3 * 768) * sizeof(double); };
  const int l16 = (int)((l + 15) & ~(int64_t)15);
  int chunks = 1, rows = l16;
  while (d.lds_max != 0 && bytes(rows) + 4096 > d.lds_max && rows > 16) {
    ++chunks;
    rows = ((l16 + chunks - 1) / chunks + 15) & ~15;
  }
  int p = (int)((l + b - 1) / b);
  if (p < 2) p = 2;
  if (p & 1) ++p;
  *bs = b;
  *P = p;
  *rg = chunks;
  *ch = rows;
  *ldc = rows + 1;
  *ncol = nc;
  *lds = bytes(rows);
  return d.lds_max == 0 || *lds + 4096 <= d.lds_max;
}

// Output of the vector form: column c of M has rank(c) among the column
// norms (descending, ties by index); sigma[rank] = its norm,
// U(:, rank) = M(0:l, c) / sigma (zero when sigma is zero),
// V(:, rank) = M(lpad:lpad+l, c).  One workgroup per column.
template <typename T>
__global__ void svd_vectors_out(const double* __restrict__ M, int l, int ldm, int lpad, const double* __restrict__ sg,
                                double* __restrict__ sigma, T* __restrict__ U, int64_t ldu, T* __restrict__ V,
                                int64_t ldv) {
  __shared__ int s_rank;
  const int c = blockIdx.x;
  if (threadIdx.x == 0) {
    const double v = sg[c];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = sg[i];
      rank += (u > v || (u == v && i < c)) ? 1 : 0;
    }
    s_rank = rank;
    sigma[rank] = v;
  }
  __syncthreads();
  const int rk = s_rank;
  const double sv = sg[c];
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    U[(int64_t)rk * ldu + i] = (T)(M[(int64_t)c * ldm + i] * inv);
    V[(int64_t)rk * ldv + i] = (T)M[(int64_t)c * ldm + lpad + i];
  }
}

// Rows of the stacked matrix of the vector form for block rows of ch.
void vec_rows(int64_t l, int ch, int* lpad, int* ldm, int* rg) {
  const int rg0 = (int)((l + ch - 1) / ch);
  *lpad = rg0 * ch;
  *ldm = *lpad + (int)l;
  *rg = 2 * rg0;
}

}  // namespace

template <typename T>
size_t jacobi_scratch(int64_t l, const DeviceInfo& d) {
  // the stacked M of the vector form (at most (2 l + 416) x l), sigma, the
  // partial-Gram exchange (two buffers of at most kMaxGridBlocks workgroups
  // of GW x GW) and
  // the barrier flags
  return sizeof(double) * ((size_t)(2 * l + 432) * l + l + (size_t)2 * kMaxGridBlocks * GW * GW) +
         (kSyncWords + 64) * sizeof(unsigned) + 8 * 256;
}

namespace {
template <typename T>
hipError_t jacobi_launch(const T* L, int64_t l, int64_t ldl, bool vectors, double* sigma, T* U, int64_t ldu, T* V,
                         int64_t ldv, Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s, int* sweeps) {
  if (l <= 0) return hipSuccess;
  int bs, P, ldc, ncol, ch, rg;
  size_t lds;
  if (!choose(l, d, &bs, &P, &ldc, &ncol, &ch, &rg, &lds)) return hipErrorInvalidValue;
  int lpad = 0, ldm = (int)l;
  if (vectors) vec_rows(l, ch, &lpad, &ldm, &rg);
  const int nwg = P / 2 * rg;  // workgroups: rg per block pair
  if (nwg > kMaxGridBlocks) return hipErrorInvalidValue;
  double* M = ar.take<double>((size_t)ldm * l);
  double* sig = ar.take<double>(l);
  double* xbuf = ar.take<double>((size_t)2 * nwg * GW * GW);
  unsigned* ctl = ar.take<unsigned>(kSyncWords + 64);
  if (!M || !sig || !xbuf || !ctl) return hipErrorOutOfMemory;
  hipError_t e = zero_words(ctl, kSyncWords + 64, s);
  if (e != hipSuccess) return e;
  GridSync gs{ctl, err, (unsigned)nwg};
  unsigned* rot = ctl + kSyncWords;
  int li = (int)l;
  double settled = (vectors || sizeof(T) == 8) ? kSettled : kSettled32;
  void* args[] = {(void*)&L,    (void*)&li,  (void*)&ldl,  (void*)&M,   (void*)&ldm,  (void*)&lpad,
                  (void*)&bs,   (void*)&P,   (void*)&ldc,  (void*)&ncol, (void*)&ch,  (void*)&rg,
                  (void*)&xbuf, (void*)&rot, (void*)&sig,  (void*)&sweeps, (void*)&settled, (void*)&gs};
  const void* fn = rg > 1 ? (const void*)jacobi_kernel<T, true> : (const void*)jacobi_kernel<T, false>;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  e = hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(NT), args, (unsigned)lds, s);
  if (e != hipSuccess) return e;
  if (vectors)
    svd_vectors_out<T><<<(unsigned)l, 256, 0, s>>>(M, li, ldm, lpad, sig, sigma, U, ldu, V, ldv);
  else
    sort_desc<<<1, 1024, 0, s>>>(sig, li, sigma);
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t jacobi_sigma(const T* L, int64_t l, int64_t ldl, double* sigma, Arena& ar, unsigned* err,
                        const DeviceInfo& d, hipStream_t s, int* sweeps) {
  return jacobi_launch<T>(L, l, ldl, false, sigma, nullptr, 0, nullptr, 0, ar, err, d, s, sweeps);
}

template <typename T>
hipError_t jacobi_svd_vectors(const T* L, int64_t l, int64_t ldl, double* sigma, T* U, int64_t ldu, T* V, int64_t ldv,
                              Arena& ar, unsigned* err, const DeviceInfo& d, hipStream_t s, int* sweeps) {
  return jacobi_launch<T>(L, l, ldl, true, sigma, U, ldu, V, ldv, ar, err, d, s, sweeps);
}

template size_t jacobi_scratch<double>(int64_t, const DeviceInfo&);
template size_t jacobi_scratch<float>(int64_t, const DeviceInfo&);
template hipError_t jacobi_sigma<double>(const double*, int64_t, int64_t, double*, Arena&, unsigned*,
                                         const DeviceInfo&, hipStream_t, int*);
template hipError_t jacobi_sigma<float>(const float*, int64_t, int64_t, double*, Arena&, unsigned*,
                                        const DeviceInfo&, hipStream_t, int*);
template hipError_t jacobi_svd_vectors<double>(const double*, int64_t, int64_t, double*, double*, int64_t, double*,
                                               int64_t, Arena&, unsigned*, const DeviceInfo&, hipStream_t, int*);
template hipError_t jacobi_svd_vectors<float>(const float*, int64_t, int64_t, double*, float*, int64_t, float*,
                                              int64_t, Arena&, unsigned*, const DeviceInfo&, hipStream_t, int*);

}  // namespace ffsrqr
