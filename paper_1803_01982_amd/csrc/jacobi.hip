// Singular values of the small factor L (l x l) by one-sided (Hestenes)
// Jacobi in FP64 (Algorithm 9 takes an SVD of the small factor; the
// flip-flop factor L is already QR-preconditioned, which is the setting in
// which one-sided Jacobi converges in few sweeps).
//
// Block form for one cooperative launch: the columns are split into
// P = 2G blocks of bs columns; a round-robin tournament (circle method) pairs
// the blocks so that in each of the P-1 rounds of a sweep every block meets
// one other block.  Workgroup g takes pair g of the round, copies the two
// blocks into LDS and rotates the cross pairs (one column of each block);
// in the first round of a sweep it rotates every pair of the union, which
// covers the pairs inside each block once per sweep.  Pairs run in parallel
// rounds, one wave per pair; one grid barrier per round.  A pair (p, q) is rotated when
// |c_p . c_q| > tol ||c_p|| ||c_q|| (tol = 1e-14), with Rutishauser's
// formulas; the iteration stops after a sweep with no rotation (at most 60
// sweeps).  sigma_j = ||c_j||, sorted descending.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 1024;
constexpr double kTol = 1e-14;
constexpr int kMaxSweeps = 60;

__device__ inline int rr_player(int pos, int r, int P) {
  // circle method: position 0 fixed, positions 1..P-1 rotate by r
  return pos == 0 ? 0 : ((pos - 1 + r) % (P - 1)) + 1;
}

template <typename T>
__global__ __launch_bounds__(NT) void jacobi_kernel(const T* __restrict__ L, int l, int64_t ldl, double* __restrict__ M,
                                                    int bs, int P, unsigned* __restrict__ rot,
                                                    double* __restrict__ sig, int* __restrict__ sweeps_out,
                                                    GridSync gs) {
  extern __shared__ double C[];  // 2*bs columns of length l
  __shared__ int s_rot;
  __shared__ double dn[64];       // squared norms of the 2*bs local columns
  __shared__ unsigned short sched_full[31 * 16];
  __shared__ unsigned short sched_cross[16 * 16];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = NT / 64;
  unsigned epoch = 0;

  for (int64_t e = (int64_t)g * NT + tid; e < (int64_t)l * l; e += (int64_t)G * NT) {
    const int64_t r = e % l, c = e / l;
    M[c * l + r] = (double)L[c * ldl + r];
  }
  if (g == 0 && tid < 3) rot[tid] = 0u;
  if (!grid_barrier(gs, epoch)) return;

  const int W2 = 2 * bs;
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
  __syncthreads();
  int sweep = 0;
  for (sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (g == 0 && tid == 0) rot[(sweep + 1) % 3] = 0u;
    if (tid == 0) s_rot = 0;
    for (int r = 0; r < P - 1; ++r) {
      // blocks of this workgroup's pair
      const int pa = rr_player(g, r, P);
      const int pb = rr_player(P - 1 - g, r, P);
      const int ca0 = pa * bs, cb0 = pb * bs;
      const int na = max(0, min(bs, l - ca0)), nbk = max(0, min(bs, l - cb0));
      // local column k < bs -> block a column k, k >= bs -> block b column k - bs
      for (int e = tid; e < W2 * l; e += NT) {
        // all loads of the two blocks in flight together
        const int k = e / l, i = e - k * l;
        const int gc = k < bs ? (k < na ? ca0 + k : -1) : (k - bs < nbk ? cb0 + k - bs : -1);
        C[e] = gc >= 0 ? M[(int64_t)gc * l + i] : 0.0;
      }
      __syncthreads();
      for (int k = wave; k < W2; k += nwave) {
        double a = 0.0;
        for (int i = lane; i < l; i += 64) {
          const double x = C[k * l + i];
          a += x * x;
        }
        a = wave_sum(a);
        if (lane == 0) dn[k] = a;  // fresh squared norms of the local columns
      }
      __syncthreads();
      // one pass over the scheduled pairs; the norms follow each rotation
      // (a - t g, b + t g), so each pair needs one dot product
      const bool full = (r == 0);
      const int nir = full ? W2 - 1 : bs;
      const unsigned short* sched = full ? sched_full : sched_cross;
      for (int ir = 0; ir < nir; ++ir) {
        for (int pr = wave; pr < bs; pr += nwave) {
          const unsigned pq = sched[ir * bs + pr];
          const int lo = (int)(pq >> 8), hi = (int)(pq & 255u);
          double* cp = C + lo * l;
          double* cq = C + hi * l;
          double gg = 0.0;
          for (int i = lane; i < l; i += 64) gg += cp[i] * cq[i];
          gg = wave_sum(gg);
          const double a = dn[lo], b = dn[hi];
          if (a == 0.0 || b == 0.0 || gg * gg <= (kTol * kTol) * (a * b)) continue;
          const double zeta = (b - a) / (2.0 * gg);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = rsqrt(1.0 + t * t), sn = cs * t;
          for (int i = lane; i < l; i += 64) {
            const double x = cp[i], y = cq[i];
            cp[i] = cs * x - sn * y;
            cq[i] = sn * x + cs * y;
          }
          if (lane == 0) {
            dn[lo] = a - t * gg;
            dn[hi] = b + t * gg;
            s_rot = 1;
          }
        }
        __syncthreads();
      }
      for (int k = wave; k < W2; k += nwave) {
        const int gc = k < bs ? (k < na ? ca0 + k : -1) : (k - bs < nbk ? cb0 + k - bs : -1);
        if (gc >= 0)
          for (int i = lane; i < l; i += 64) M[(int64_t)gc * l + i] = C[k * l + i];
      }
      if (!grid_barrier(gs, epoch)) return;
    }
    if (tid == 0 && s_rot) __hip_atomic_fetch_or(&rot[sweep % 3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(gs, epoch)) return;
    const unsigned any = __hip_atomic_load(&rot[sweep % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!any) break;
  }
  if (g == 0 && tid == 0 && sweeps_out) *sweeps_out = sweep < kMaxSweeps ? sweep + 1 : kMaxSweeps;
  // column norms
  for (int c = g * nwave + wave; c < l; c += G * nwave) {
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

void choose(int64_t l, const DeviceInfo& d, int* bs, int* P, size_t* lds) {
  int b = 16;  // at most 32 local columns (dn has 64 slots)
  while (b > 1 && (size_t)2 * b * l * sizeof(double) > d.lds_max - 2048) --b;
  if (l < 2 * b) b = (int)((l + 1) / 2 > 0 ? (l + 1) / 2 : 1);
  int p = (int)((l + b - 1) / b);
  if (p < 2) p = 2;
  if (p & 1) ++p;
  *bs = b;
  *P = p;
  *lds = (size_t)2 * b * l * sizeof(double);
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
  int bs, P;
  size_t lds;
  choose(l, d, &bs, &P, &lds);
  double* M = ar.take<double>((size_t)l * l);
  double* sig = ar.take<double>(l);
  unsigned* ctl = ar.take<unsigned>(kSyncWords + 64);
  if (!M || !sig || !ctl) return hipErrorOutOfMemory;
  hipError_t e = zero_words(ctl, kSyncWords + 64, s);
  if (e != hipSuccess) return e;
  GridSync gs{ctl, err, (unsigned)(P / 2)};
  unsigned* rot = ctl + kSyncWords;
  int li = (int)l;
  void* args[] = {(void*)&L, (void*)&li, (void*)&ldl, (void*)&M, (void*)&bs, (void*)&P, (void*)&rot, (void*)&sig,
                  (void*)&sweeps, (void*)&gs};
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
