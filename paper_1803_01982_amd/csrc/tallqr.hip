// Householder QR without pivoting of a tall matrix P (mrows x c, mrows >= c).
// Used twice on the path:
//   * the QR of the l pivoted columns A(:, S) (Algorithm 2, QR of the
//     pivoted block; compact WY representation Q = I - Y T Y^T of Section 2.1);
//   * the flip-flop step, QR of R^T (n x l) (Section 3.1).
//
// One cooperative launch.  Workgroup g owns the row block [g*rb, (g+1)*rb).
// Columns are processed in panels of NB = 16:
//   column step (one grid barrier): every workgroup publishes the partial
//     dot products of the current column with the remaining panel columns
//     over its rows (and the owner of the pivot row publishes that row);
//     after the barrier all workgroups sum the partials in the same fixed
//     order, build the same reflector (LAPACK xLARFG convention) and update
//     their own rows of the panel, which stay in LDS for the whole panel;
//   panel end (two grid barriers): Z = Y^T [Y | P_trail] is reduced
//     (reduce-scatter, then every workgroup reads the whole Z), each
//     workgroup forms the panel's T (LAPACK xLARFT, forward, columnwise)
//     from the Gram part and applies P_trail -= Y (T^T (Y^T P_trail)) to its
//     own rows.
// Then Q = H_1 ... H_c [I; 0] is formed backwards panel by panel with the
// same reduce pattern (Q -= Y (T (Y^T Q))), and signs are normalised so that
// diag(R) >= 0.  All arithmetic is FP64; P and Q are stored as T.
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256, NB = 16, SUB = 128;

struct TqSlots {
  double* dots;   // [2][G][NB]
  double* rowv;   // [2][NB]
  double* zpart;  // [G][NB * c]
  double* zred;   // [2][NB * c]
  double* tst;    // [npan][NB * NB]
  double* tau;    // [c]
};

// Y(gi, s) of panel p0 given the stored value at (gi, p0 + s).
__device__ inline double yval(int64_t gi, int64_t p0, int s, double stored) {
  const int64_t d = p0 + s;
  return gi < d ? 0.0 : (gi == d ? 1.0 : stored);
}

// Partial Z[:, col] = sum over own rows (rows >= p0) of Y(:, s) * X(row, col)
// for NB x ncol entries; X column col lives at X[col * ldx + row] (global,
// with an optional row map).  Yl holds Y of the own rows (nrow x NB, in LDS).
// Result written to out[col * NB + s].
template <typename T>
__device__ void partial_yt_x(const double* Yl, int nrow, int pw, const T* X, int64_t ldx,
                             const int64_t* rowmap, int64_t mrows, int64_t r0, int ncol, double* stage,
                             double* out) {
  const int tid = threadIdx.x;
  const int s = tid % NB, cc = tid / NB;  // 16 x 16 outputs per chunk
  for (int col0 = 0; col0 < ncol; col0 += NB) {
    double acc = 0.0;
    for (int i0 = 0; i0 < nrow; i0 += SUB) {
      const int nr = min(SUB, nrow - i0);
      __syncthreads();
      for (int e = tid; e < nr * NB; e += NT) {
        const int i = e % nr, c = e / nr;
        const int64_t gi = r0 + i0 + i;
        const int64_t row = rowmap ? rowmap[gi] : gi;
        stage[i * NB + c] = (col0 + c < ncol && row >= 0 && row < mrows) ? (double)X[(int64_t)(col0 + c) * ldx + row]
                                                                          : 0.0;
      }
      __syncthreads();
      if (s < pw)
        for (int i = 0; i < nr; ++i) acc += Yl[(i0 + i) * NB + s] * stage[i * NB + cc];
    }
    if (s < NB && col0 + cc < ncol) out[(int64_t)(col0 + cc) * NB + s] = (s < pw) ? acc : 0.0;
  }
}

// Partial Z for the Gram part: Y^T Y over own rows, written to out[col*NB+s].
__device__ void partial_gram(const double* Yl, int nrow, int pw, double* out) {
  const int tid = threadIdx.x;
  const int s = tid % NB, cc = tid / NB;
  double acc = 0.0;
  if (s < pw && cc < pw)
    for (int i = 0; i < nrow; ++i) acc += Yl[i * NB + s] * Yl[i * NB + cc];
  out[cc * NB + s] = acc;
}

// Reduce-scatter of E entries over G partials into zred, then every block
// copies the whole reduced Z into Zl.  Returns false on a barrier timeout.
__device__ bool reduce_z(const double* zpart, double* zred, int64_t E, int64_t estride, int G, int g,
                         double* Zl, const GridSync& gs, unsigned& epoch) {
  if (!grid_barrier(gs, epoch)) return false;
  const int64_t e0 = E * g / G, e1 = E * (g + 1) / G;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += NT) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t += zpart[(int64_t)q * estride + e];
    zred[e] = t;
  }
  if (!grid_barrier(gs, epoch)) return false;
  for (int64_t e = threadIdx.x; e < E; e += NT) Zl[e] = zred[e];
  __syncthreads();
  return true;
}

template <typename T>
__global__ __launch_bounds__(NT) void tallqr_kernel(T* __restrict__ P, int64_t mrows, int c, int64_t ldp, int rb,
                                                    T* __restrict__ Qout, int64_t ldq,
                                                    const int64_t* __restrict__ rowmap, T* __restrict__ R,
                                                    int64_t ldr, int transpose_r, TqSlots sl, GridSync gs) {
  extern __shared__ double smem[];
  __shared__ double red[NB * NB];
  __shared__ double Tl[NB * NB];
  __shared__ double taul[NB];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int64_t r0 = (int64_t)g * rb;
  const int nrow = (int)max((int64_t)0, min((int64_t)rb, mrows - r0));
  double* Yl = smem;                        // rb x NB
  double* stage = Yl + (int64_t)rb * NB;    // SUB x NB
  double* Zl = stage + SUB * NB;            // NB x c
  const int npan = (c + NB - 1) / NB;
  const int64_t estride = (int64_t)NB * (c > NB ? c : NB);
  unsigned epoch = 0;
  int step = 0;

  // ------------------------------------------------------------ factorization
  for (int pi = 0; pi < npan; ++pi) {
    const int p0 = pi * NB, p1 = min(c, p0 + NB), pw = p1 - p0;
    __syncthreads();
    for (int e = tid; e < nrow * NB; e += NT) {
      const int i = e % nrow, t = e / nrow;
      Yl[i * NB + t] = t < pw ? (double)P[(int64_t)(p0 + t) * ldp + r0 + i] : 0.0;
    }
    __syncthreads();
    for (int jc = p0; jc < p1; ++jc, ++step) {
      const int jt = jc - p0, par = step & 1;
      // partial dots d_t = sum_{own rows > jc} x_i p_t(i), t = jt..pw-1
      {
        const int t = tid % NB, rs = tid / NB;
        double acc = 0.0;
        if (t >= jt && t < pw)
          for (int i = rs; i < nrow; i += NT / NB)
            if (r0 + i > jc) acc += Yl[i * NB + jt] * Yl[i * NB + t];
        red[rs * NB + t] = acc;
        __syncthreads();
        if (tid < NB) {
          double sacc = 0.0;
          for (int q = 0; q < NT / NB; ++q) sacc += red[q * NB + tid];
          sl.dots[((int64_t)par * G + g) * NB + tid] = sacc;
        }
        if (jc >= r0 && jc < r0 + nrow && tid < NB)
          sl.rowv[par * NB + tid] = Yl[(jc - r0) * NB + tid];
      }
      if (!grid_barrier(gs, epoch)) return;
      // sum the partials in a fixed order (identical in every workgroup)
      {
        const int t = tid % NB, gs16 = tid / NB;
        double acc = 0.0;
        for (int q = gs16; q < G; q += NT / NB) acc += sl.dots[((int64_t)par * G + q) * NB + t];
        red[gs16 * NB + t] = acc;
        __syncthreads();
        if (tid < NB) {
          double sacc = 0.0;
          for (int q = 0; q < NT / NB; ++q) sacc += red[q * NB + tid];
          Tl[tid] = sacc;                       // d_t
          Tl[NB + tid] = sl.rowv[par * NB + tid];  // p_t(jc)
        }
        __syncthreads();
      }
      const double xnorm2 = Tl[jt], x0 = Tl[NB + jt];
      double tau = 0.0, beta = x0, scale = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + xnorm2), x0);
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      if (tid == 0) taul[jt] = tau;
      if (g == 0 && tid == 0) sl.tau[jc] = tau;
      // own rows: p_t -= tau w_t v, w_t = p_t(jc) + scale d_t
      for (int e = tid; e < nrow * NB; e += NT) {
        const int i = e / NB, t = e % NB;
        const int64_t gi = r0 + i;
        if (t <= jt || t >= pw || gi < jc) continue;
        const double wt = Tl[NB + t] + scale * Tl[t];
        if (gi == jc) Yl[i * NB + t] -= tau * wt;
        else Yl[i * NB + t] -= tau * wt * (Yl[i * NB + jt] * scale);
      }
      __syncthreads();
      for (int i = tid; i < nrow; i += NT) {
        const int64_t gi = r0 + i;
        if (gi == jc) Yl[i * NB + jt] = beta;
        else if (gi > jc && tau != 0.0) Yl[i * NB + jt] *= scale;
      }
      __syncthreads();
    }
    // write the panel back (R above the diagonal, beta on it, v below)
    for (int e = tid; e < nrow * NB; e += NT) {
      const int i = e % nrow, t = e / nrow;
      if (t < pw) P[(int64_t)(p0 + t) * ldp + r0 + i] = (T)Yl[i * NB + t];
    }
    __syncthreads();
    // Y of the own rows (rows >= p0 only contribute)
    for (int e = tid; e < nrow * NB; e += NT) {
      const int i = e / NB, s = e % NB;
      Yl[i * NB + s] = s < pw ? yval(r0 + i, p0, s, Yl[i * NB + s]) : 0.0;
    }
    __syncthreads();
    const int ntr = c - p1;
    double* zp = sl.zpart + (int64_t)g * estride;
    partial_gram(Yl, nrow, pw, zp);
    if (ntr > 0) partial_yt_x<T>(Yl, nrow, pw, P + (int64_t)p1 * ldp, ldp, nullptr, mrows, r0, ntr, stage, zp + NB * NB);
    double* zr = sl.zred + (int64_t)(pi & 1) * estride;
    if (!reduce_z(sl.zpart, zr, (int64_t)NB * (NB + ntr), estride, G, g, Zl, gs, epoch)) return;
    // T of the panel: T(s,s) = tau_s, T(0:s, s) = -tau_s T(0:s, 0:s) (Y^T y_s)
    if (tid < NB * NB) Tl[tid] = 0.0;
    __syncthreads();
    for (int s = 0; s < pw; ++s) {
      const double ts = taul[s];
      double val = 0.0;
      if (tid < s) {
        for (int q = tid; q < s; ++q) val += Tl[q * NB + tid] * Zl[s * NB + q];
        val *= -ts;
      }
      __syncthreads();
      if (tid < s) Tl[s * NB + tid] = val;
      if (tid == s) Tl[s * NB + s] = ts;
      __syncthreads();
    }
    if (g == 0 && tid < NB * NB) sl.tst[(int64_t)pi * NB * NB + tid] = Tl[tid];
    // W' = T^T Z_trail (in place, column by column)
    for (int u = tid; u < ntr; u += NT) {
      double z[NB], w[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) z[q] = Zl[(NB + u) * NB + q];
#pragma unroll
      for (int s2 = 0; s2 < NB; ++s2) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q <= s2) a += Tl[s2 * NB + q] * z[q];
        w[s2] = a;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) Zl[(NB + u) * NB + q] = w[q];
    }
    __syncthreads();
    // P_trail(own rows >= p0) -= Y W'
    for (int e = tid; e < nrow * ntr; e += NT) {
      const int i = e % nrow, u = e / nrow;
      const int64_t gi = r0 + i;
      if (gi < p0) continue;
      double a = 0.0;
#pragma unroll
      for (int s = 0; s < NB; ++s) a += Yl[i * NB + s] * Zl[(NB + u) * NB + s];
      T* pp = P + (int64_t)(p1 + u) * ldp + gi;
      *pp = (T)((double)*pp - a);
    }
  }

  // --------------------------------------------------- explicit Q, backwards
  // the T factors written by workgroup 0 at the panel ends must be visible
  if (!grid_barrier(gs, epoch)) return;
  for (int e = tid; e < nrow * c; e += NT) {
    const int i = e % nrow, j = e / nrow;
    const int64_t gi = r0 + i;
    const int64_t row = rowmap ? rowmap[gi] : gi;
    if (row < 0 || row >= mrows) continue;
    Qout[(int64_t)j * ldq + row] = (T)(gi == j ? 1.0 : 0.0);
  }
  for (int pi = npan - 1; pi >= 0; --pi) {
    const int p0 = pi * NB, p1 = min(c, p0 + NB), pw = p1 - p0;
    const int ncol = c - p0;
    __syncthreads();
    for (int e = tid; e < nrow * NB; e += NT) {
      const int i = e % nrow, s = e / nrow;
      Yl[i * NB + s] = s < pw ? yval(r0 + i, p0, s, (double)P[(int64_t)(p0 + s) * ldp + r0 + i]) : 0.0;
    }
    if (tid < NB * NB) Tl[tid] = sl.tst[(int64_t)pi * NB * NB + tid];
    __syncthreads();
    double* zp = sl.zpart + (int64_t)g * estride;
    partial_yt_x<T>(Yl, nrow, pw, Qout + (int64_t)p0 * ldq, ldq, rowmap, mrows, r0, ncol, stage, zp);
    double* zr = sl.zred + (int64_t)(pi & 1) * estride;
    if (!reduce_z(sl.zpart, zr, (int64_t)NB * ncol, estride, G, g, Zl, gs, epoch)) return;
    // W2 = T Z (T upper triangular)
    for (int u = tid; u < ncol; u += NT) {
      double z[NB], w[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) z[q] = Zl[u * NB + q];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q >= r) a += Tl[q * NB + r] * z[q];
        w[r] = a;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) Zl[u * NB + q] = w[q];
    }
    __syncthreads();
    for (int e = tid; e < nrow * ncol; e += NT) {
      const int i = e % nrow, u = e / nrow;
      const int64_t gi = r0 + i;
      if (gi < p0) continue;
      double a = 0.0;
#pragma unroll
      for (int s = 0; s < NB; ++s) a += Yl[i * NB + s] * Zl[u * NB + s];
      const int64_t row = rowmap ? rowmap[gi] : gi;
      if (row < 0 || row >= mrows) continue;
      T* qq = Qout + (int64_t)(p0 + u) * ldq + row;
      *qq = (T)((double)*qq - a);
    }
  }
  __syncthreads();

  // --------------------------------------------------- signs, R output
  double* sgn = Zl;  // c entries
  for (int j = tid; j < c; j += NT) sgn[j] = ((double)P[(int64_t)j * ldp + j] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  for (int e = tid; e < nrow * c; e += NT) {
    const int i = e % nrow, j = e / nrow;
    const int64_t gi = r0 + i;
    const int64_t row = rowmap ? rowmap[gi] : gi;
    if (sgn[j] < 0.0 && row >= 0 && row < mrows) {
      T* qq = Qout + (int64_t)j * ldq + row;
      *qq = -*qq;
    }
    if (gi < c) {
      const double val = (j >= gi) ? sgn[gi] * (double)P[(int64_t)j * ldp + gi] : 0.0;
      if (transpose_r) R[(int64_t)gi * ldr + j] = (T)val;
      else R[(int64_t)j * ldr + gi] = (T)val;
    }
  }
}

void choose(int64_t mrows, int c, int num_cu, int* G, int* rb, size_t* lds) {
  int64_t g = (mrows + 255) / 256;
  if (g > num_cu) g = num_cu;
  if (g < 1) g = 1;
  int64_t r = (mrows + g - 1) / g;
  *G = (int)((mrows + r - 1) / r);
  *rb = (int)r;
  *lds = ((size_t)r * NB + SUB * NB + (size_t)NB * (c > NB ? c : NB) + 64) * sizeof(double);
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

}  // namespace

template <typename T>
size_t tallqr_scratch(int64_t mrows, int64_t c, const DeviceInfo& d) {
  int G, rb;
  size_t lds;
  choose(mrows, (int)c, d.num_cu, &G, &rb, &lds);
  const int npan = (int)((c + NB - 1) / NB);
  const size_t cz = c > NB ? c : NB;
  size_t b = sizeof(double) * ((size_t)2 * G * NB + 2 * NB + (size_t)G * NB * cz + (size_t)2 * NB * cz +
                               (size_t)npan * NB * NB + c);
  return b + 64 * sizeof(unsigned) + 8 * 256;
}

template <typename T>
hipError_t tall_qr(T* P, int64_t mrows, int64_t c, int64_t ldp, T* Qout, int64_t ldq, const int64_t* rowmap,
                   T* R, int64_t ldr, bool transpose_r, Arena& ar, unsigned* err, const DeviceInfo& d,
                   hipStream_t s) {
  if (c <= 0) return hipSuccess;
  if (mrows < c) return hipErrorInvalidValue;
  int G, rb;
  size_t lds;
  choose(mrows, (int)c, d.num_cu, &G, &rb, &lds);
  if (lds > d.lds_max) return hipErrorInvalidValue;
  const int npan = (int)((c + NB - 1) / NB);
  TqSlots sl;
  sl.dots = ar.take<double>((size_t)2 * G * NB);
  sl.rowv = ar.take<double>(2 * NB);
  const size_t cz = c > NB ? c : NB;
  sl.zpart = ar.take<double>((size_t)G * NB * cz);
  sl.zred = ar.take<double>((size_t)2 * NB * cz);
  sl.tst = ar.take<double>((size_t)npan * NB * NB);
  sl.tau = ar.take<double>(c);
  unsigned* counter = ar.take<unsigned>(64);
  if (!sl.dots || !sl.rowv || !sl.zpart || !sl.zred || !sl.tst || !sl.tau || !counter) return hipErrorOutOfMemory;
  hipError_t e = zero_words(counter, 64, s);
  if (e != hipSuccess) return e;
  GridSync gs{counter, err, (unsigned)G};
  int ci = (int)c, tr = transpose_r ? 1 : 0;
  void* args[] = {(void*)&P, (void*)&mrows, (void*)&ci, (void*)&ldp, (void*)&rb, (void*)&Qout, (void*)&ldq,
                  (void*)&rowmap, (void*)&R, (void*)&ldr, (void*)&tr, (void*)&sl, (void*)&gs};
  const void* fn = (const void*)tallqr_kernel<T>;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, (unsigned)lds, s);
}

template <typename T>
hipError_t gather_cols(const T* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols, int64_t c, T* P,
                       int64_t ldp, hipStream_t s) {
  if (c <= 0 || m <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)c);
  gather_kernel<T><<<grid, 256, 0, s>>>(A, m, n, lda, cols, c, P, ldp);
  return hipGetLastError();
}

template size_t tallqr_scratch<double>(int64_t, int64_t, const DeviceInfo&);
template size_t tallqr_scratch<float>(int64_t, int64_t, const DeviceInfo&);
template hipError_t tall_qr<double>(double*, int64_t, int64_t, int64_t, double*, int64_t, const int64_t*, double*,
                                    int64_t, bool, Arena&, unsigned*, const DeviceInfo&, hipStream_t);
template hipError_t tall_qr<float>(float*, int64_t, int64_t, int64_t, float*, int64_t, const int64_t*, float*,
                                   int64_t, bool, Arena&, unsigned*, const DeviceInfo&, hipStream_t);
template hipError_t gather_cols<double>(const double*, int64_t, int64_t, int64_t, const int64_t*, int64_t, double*,
                                        int64_t, hipStream_t);
template hipError_t gather_cols<float>(const float*, int64_t, int64_t, int64_t, const int64_t*, int64_t, float*,
                                       int64_t, hipStream_t);

}  // namespace ffsrqr
