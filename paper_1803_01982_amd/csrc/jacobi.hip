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
// by C J (FP64 MFMA) in global memory.  The inner rounds take the cross
// pairs (one column of each block); in the first round of a sweep they take
// every pair of the union, which covers the pairs inside each block once per
// sweep.  H is recomputed from the columns at every round, so the rounding
// of the Gram updates never accumulates beyond one round, and the columns
// only ever see orthogonal transformations.  A pair is rotated when
// |h_pq| > tol sqrt(h_pp h_qq) (tol = 1e-14), with Rutishauser's formulas;
// the iteration stops after a sweep with no rotation (at most 60 sweeps).
// sigma_j = ||c_j||, sorted descending.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 1024;
constexpr int NW = NT / kWave;
constexpr int GW = 32;  // stride of the Gram and rotation arrays (2 bs <= GW)
constexpr double kTol = 1e-14;
constexpr int kMaxSweeps = 60;

__device__ inline int rr_player(int pos, int r, int P) {
  // circle method: position 0 fixed, positions 1..P-1 rotate by r
  return pos == 0 ? 0 : ((pos - 1 + r) % (P - 1)) + 1;
}

// Dynamic LDS: C (ncol columns of ldc rows; rows >= l and columns >= 2 bs stay
// zero), then H[2][GW * GW] and J[2][GW * GW] (double buffers).
template <typename T>
__global__ __launch_bounds__(NT) void jacobi_kernel(const T* __restrict__ L, int l, int64_t ldl, double* __restrict__ M,
                                                    int bs, int P, int ldc, int ncol, unsigned* __restrict__ rot,
                                                    double* __restrict__ sig, int* __restrict__ sweeps_out,
                                                    GridSync gs) {
  typedef Mfma<double> MF;
  extern __shared__ double smem[];
  double* C = smem;
  double* H0 = C + (size_t)ncol * ldc;
  double* H1 = H0 + GW * GW;
  double* J0 = H1 + GW * GW;
  double* J1 = J0 + GW * GW;
  __shared__ double s_al[GW], s_be[GW], s_dn[GW];
  __shared__ int s_pt[GW];
  __shared__ int s_sweep, s_round, s_inner[2];
  __shared__ unsigned short sched_full[31 * 16];
  __shared__ unsigned short sched_cross[16 * 16];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int W2 = 2 * bs, nct = ncol / 16;
  unsigned epoch = 0;

  for (int64_t e = (int64_t)g * NT + tid; e < (int64_t)l * l; e += (int64_t)G * NT) {
    const int64_t r = e % l, c = e / l;
    M[c * l + r] = (double)L[c * ldl + r];
  }
  for (int e = tid; e < ncol * ldc + 4 * GW * GW; e += NT) smem[e] = 0.0;  // C, H and J
  if (g == 0 && tid < 3) rot[tid] = 0u;
  if (!grid_barrier(gs, epoch)) return;

  // pair schedules of the local columns, built once:
  //   full: all W2(W2-1)/2 pairs of the union in W2-1 rounds of bs disjoint
  //         pairs (circle method), used in the first round of every sweep;
  //   cross: the bs*bs pairs (block a, block b) in bs rounds (p, bs + (p+r) % bs).
  for (int e = tid; e < (W2 - 1) * bs; e += NT) {
    const int ir = e / bs, pr = e % bs;
    const int p = rr_player(pr, ir, W2), q = rr_player(W2 - 1 - pr, ir, W2);
    sched_full[e] = (unsigned short)((min(p, q) << 8) | max(p, q));
  }
  for (int e = tid; e < bs * bs; e += NT) {
    const int ir = e / bs, p = e % bs;
    sched_cross[e] = (unsigned short)((p << 8) | (bs + (p + ir) % bs));
  }
  // this thread's entry of the GW x GW arrays
  const int ei = tid / GW, ej = tid % GW;
  const bool own = ei < W2 && ej < W2;
  // Gram tiles: t = 0 -> (0,0), 1 -> (0,1), 2 -> (1,1); two halves of the rows
  const int ntile = nct * (nct + 1) / 2;
  const int kr = (l + 15) & ~15;
  const int kh = ((kr / 4 + 1) / 2) * 4;
  __syncthreads();

  int sweep = 0;
  for (sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (g == 0 && tid == 0) rot[(sweep + 1) % 3] = 0u;
    if (tid == 0) s_sweep = 0;
    for (int r = 0; r < P - 1; ++r) {
      // blocks of this workgroup's pair
      const int pa = rr_player(g, r, P);
      const int pb = rr_player(P - 1 - g, r, P);
      const int ca0 = pa * bs, cb0 = pb * bs;
      const int na = max(0, min(bs, l - ca0)), nbk = max(0, min(bs, l - cb0));
      // local column k < bs -> block a column k, k >= bs -> block b column k - bs
      auto gcol = [&](int k) -> int {
        return k < bs ? (k < na ? ca0 + k : -1) : (k < W2 && k - bs < nbk ? cb0 + k - bs : -1);
      };
      if (tid == 0) {
        s_round = 0;
        s_inner[0] = 0;
        s_inner[1] = 0;
      }
      // load: wave w takes local columns w and w + NW, all loads in flight together
      for (int i0 = 0; i0 < l; i0 += 64 * 8) {
        double v[2][8];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const int k = wave + kk * NW;
          const int gc = gcol(k);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 64 + lane;
            v[kk][u] = (gc >= 0 && i < l) ? M[(int64_t)gc * l + i] : 0.0;
          }
        }
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const int k = wave + kk * NW;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 64 + lane;
            if (k < W2 && i < l) C[k * ldc + i] = v[kk][u];
          }
        }
      }
      __syncthreads();
      // Gram H = C^T C of the local columns
      typename MF::acc4 acc = {0.0, 0.0, 0.0, 0.0};
      const int t = wave % (ntile > 0 ? ntile : 1), h = wave / (ntile > 0 ? ntile : 1);
      const int tr = (t == 2) ? 1 : 0, tc = (t == 0) ? 0 : 1;
      if (wave < 2 * ntile) {
        typename MF::acc4 acc1 = {0.0, 0.0, 0.0, 0.0};
        const int klo = h ? kh : 0, khi = h ? kr : kh;
        const double* ca = C + (tr * 16 + (lane & 15)) * ldc + (lane >> 4);
        const double* cb = C + (tc * 16 + (lane & 15)) * ldc + (lane >> 4);
        int k0 = klo;
        for (; k0 + 8 <= khi; k0 += 8) {
          acc = MF::fma(ca[k0], cb[k0], acc);
          acc1 = MF::fma(ca[k0 + 4], cb[k0 + 4], acc1);
        }
        if (k0 < khi) acc = MF::fma(ca[k0], cb[k0], acc);
        acc = acc + acc1;
        if (h == 1)
#pragma unroll
          for (int q = 0; q < 4; ++q) H1[t * 256 + q * 64 + lane] = acc[q];
      }
      __syncthreads();
      if (wave < ntile) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double v = acc[q] + H1[t * 256 + q * 64 + lane];
          const int i = tr * 16 + MF::row(lane, q), j = tc * 16 + (lane & 15);
          if (tr != tc || i <= j) {
            H0[i * GW + j] = v;
            H0[j * GW + i] = v;
          }
        }
      }
      J0[tid] = (ei == ej && ei < W2) ? 1.0 : 0.0;
      __syncthreads();
      // inner rounds on the Gram matrix
      const bool full = (r == 0);
      const int nir = full ? W2 - 1 : bs;
      const unsigned short* sched = full ? sched_full : sched_cross;
      for (int ir = 0; ir < nir; ++ir) {
        if (tid < bs) {
          const unsigned pq = sched[ir * bs + tid];
          const int p = (int)(pq >> 8), q = (int)(pq & 255u);
          const double a = H0[p * GW + p], b = H0[q * GW + q], hg = H0[p * GW + q];
          if (a == 0.0 || b == 0.0 || hg * hg <= (kTol * kTol) * (a * b)) {
            s_al[p] = 1.0; s_be[p] = 0.0; s_pt[p] = p; s_dn[p] = a;
            s_al[q] = 1.0; s_be[q] = 0.0; s_pt[q] = q; s_dn[q] = b;
          } else {
            const double zeta = (b - a) / (2.0 * hg);
            const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = rsqrt(1.0 + tt * tt), sn = cs * tt;
            s_al[p] = cs; s_be[p] = -sn; s_pt[p] = q; s_dn[p] = a - tt * hg;
            s_al[q] = cs; s_be[q] = sn; s_pt[q] = p; s_dn[q] = b + tt * hg;
            s_inner[ir & 1] = 1;
            s_round = 1;
            s_sweep = 1;
          }
        }
        if (tid == 0) s_inner[(ir + 1) & 1] = 0;
        __syncthreads();
        if (!s_inner[ir & 1]) continue;  // uniform: nothing rotated in this inner round
        if (own) {
          const int pi = s_pt[ei], pj = s_pt[ej];
          const double ai = s_al[ei], bi = s_be[ei], aj = s_al[ej], bj = s_be[ej];
          double v;
          if (ei == ej) v = s_dn[ei];
          else if (pj == ei) v = 0.0;  // the pair annihilated in this inner round
          else
            v = ai * (aj * H0[ei * GW + ej] + bj * H0[ei * GW + pj]) +
                bi * (aj * H0[pi * GW + ej] + bj * H0[pi * GW + pj]);
          H1[ei * GW + ej] = v;
          J1[ei * GW + ej] = aj * J0[ei * GW + ej] + bj * J0[ei * GW + pj];
        }
        __syncthreads();
        double* x = H0; H0 = H1; H1 = x;
        x = J0; J0 = J1; J1 = x;
      }
      // columns <- C J, written straight to M (transposed product J^T C^T, so
      // each MFMA result row is a run of 16 consecutive entries of a column)
      if (s_round) {
        const int nit = (l + 15) / 16;
        for (int tt = wave; tt < nct * nit; tt += NW) {
          const int jt = tt % nct, it = tt / nct;
          typename MF::acc4 d = {0.0, 0.0, 0.0, 0.0};
          const double* ja = J0 + (lane >> 4) * GW + jt * 16 + (lane & 15);
          const double* cbp = C + (lane >> 4) * ldc + it * 16 + (lane & 15);
          for (int k0 = 0; k0 < ncol; k0 += 4) d = MF::fma(ja[k0 * GW], cbp[k0 * ldc], d);
          const int i = it * 16 + (lane & 15);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = jt * 16 + MF::row(lane, q);
            const int gc = gcol(j);
            if (gc >= 0 && i < l) M[(int64_t)gc * l + i] = d[q];
          }
        }
      }
      if (!grid_barrier(gs, epoch)) return;
    }
    if (tid == 0 && s_sweep) __hip_atomic_fetch_or(&rot[sweep % 3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(gs, epoch)) return;
    const unsigned any = __hip_atomic_load(&rot[sweep % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!any) break;
  }
  if (g == 0 && tid == 0 && sweeps_out) *sweeps_out = sweep < kMaxSweeps ? sweep + 1 : kMaxSweeps;
  // column norms
  for (int c = g * NW + wave; c < l; c += G * NW) {
    double s = 0.0;
    for (int i = lane; i < l; i += 64) {
      const double x = M[(int64_t)c * l + i];
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

// Block size bs <= 16 (2 bs local columns <= GW); C holds the local columns
// padded to ncol = 16 or 32 columns of ldc = roundup(l, 16) + 1 rows (an odd
// stride spreads the MFMA operand reads over the LDS banks).  Returns false
// when the columns of one block pair do not fit in LDS.
bool choose(int64_t l, const DeviceInfo& d, int* bs, int* P, int* ldc, int* ncol, size_t* lds) {
  const int ld = (int)(((l + 15) & ~(int64_t)15) + 1);
  auto bytes = [&](int b) { return ((size_t)((2 * b + 15) / 16 * 16) * ld + 4 * GW * GW) * sizeof(double); };
  int b = 16;
  if (d.lds_max != 0 && bytes(b) + 4096 > d.lds_max) b = 8;  // 16 local columns
  if (l < 2 * b) b = (int)((l + 1) / 2 > 0 ? (l + 1) / 2 : 1);
  int p = (int)((l + b - 1) / b);
  if (p < 2) p = 2;
  if (p & 1) ++p;
  *bs = b;
  *P = p;
  *ldc = ld;
  *ncol = (2 * b + 15) / 16 * 16;
  *lds = bytes(b);
  return d.lds_max == 0 || *lds + 4096 <= d.lds_max;
}

}  // namespace

template <typename T>
size_t jacobi_scratch(int64_t l, const DeviceInfo& d) {
  return sizeof(double) * ((size_t)l * l + l) + (kSyncWords + 64) * sizeof(unsigned) + 8 * 256;
}

template <typename T>
hipError_t jacobi_sigma(const T* L, int64_t l, int64_t ldl, double* sigma, Arena& ar, unsigned* err,
                        const DeviceInfo& d, hipStream_t s, int* sweeps) {
  if (l <= 0) return hipSuccess;
  int bs, P, ldc, ncol;
  size_t lds;
  if (!choose(l, d, &bs, &P, &ldc, &ncol, &lds)) return hipErrorInvalidValue;
  double* M = ar.take<double>((size_t)l * l);
  double* sig = ar.take<double>(l);
  unsigned* ctl = ar.take<unsigned>(kSyncWords + 64);
  if (!M || !sig || !ctl) return hipErrorOutOfMemory;
  hipError_t e = zero_words(ctl, kSyncWords + 64, s);
  if (e != hipSuccess) return e;
  GridSync gs{ctl, err, (unsigned)(P / 2)};
  unsigned* rot = ctl + kSyncWords;
  int li = (int)l;
  void* args[] = {(void*)&L,    (void*)&li,  (void*)&ldl, (void*)&M,   (void*)&bs,     (void*)&P, (void*)&ldc,
                  (void*)&ncol, (void*)&rot, (void*)&sig, (void*)&sweeps, (void*)&gs};
  const void* fn = (const void*)jacobi_kernel<T>;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  e = hipLaunchCooperativeKernel(fn, dim3(P / 2), dim3(NT), args, (unsigned)lds, s);
  if (e != hipSuccess) return e;
  sort_desc<<<1, 1024, 0, s>>>(sig, li, sigma);
  return hipGetLastError();
}

template size_t jacobi_scratch<double>(int64_t, const DeviceInfo&);
template size_t jacobi_scratch<float>(int64_t, const DeviceInfo&);
template hipError_t jacobi_sigma<double>(const double*, int64_t, int64_t, double*, Arena&, unsigned*,
                                         const DeviceInfo&, hipStream_t, int*);
template hipError_t jacobi_sigma<float>(const float*, int64_t, int64_t, double*, Arena&, unsigned*,
                                        const DeviceInfo&, hipStream_t, int*);

}  // namespace ffsrqr
