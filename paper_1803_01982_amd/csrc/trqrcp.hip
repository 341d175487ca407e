// Blocked pivot selection of Algorithm 2 (truncated randomized QRCP with
// the sample update), an alternative to one partial QRCP on an l-row
// sketch: from the sample B = Omega A of rows = min(b + p, m) rows (formed
// by the caller with the path's sketch kernels), per block of
// bj = min(b, l - j) pivots:
//   1. partial QRCP on the sample's columns still in play (the cooperative
//      QRCP on those columns, gathered; its first bj pivots are the block's:
//      partial QRCP is greedy, so the later steps do not change them);
//   2. the chosen columns' residual after the previous blocks, by two
//      classical Gram-Schmidt projections against the blocks' basis Q,
//      then its Householder QR: Q_b (appended to Q) and R11;
//   3. R12 = Q_b^T A (a pass over A) and the sample update of the remaining
//      columns, B(:, c) <- B(:, c) - B(:, piv) R11^{-1} R12(:, c), which is
//      Omega applied to their new residual.
// The blocks' basis only steers the pivot choice: the path then factors the
// chosen columns from scratch (the thin QR with a positive diagonal is
// unique, so it is the factorization Algorithm 2 accumulates).  With
// final_update the last block updates the sample too, so that B(:, c) is
// Omega times the residual of column c after all l pivots: Algorithm 4's
// residual norm estimates are ||B(:, c)||^2 / rows (sample_norms).
#include <numeric>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

constexpr int NT = 256;

// r[c] = ||B(:, c)||^2 / rows (FP64), one thread per column
template <typename T>
__global__ void sample_norms_kernel(const T* __restrict__ B, int64_t rows, int64_t n, double* __restrict__ r) {
  const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (c >= n) return;
  const T* b = B + c * rows;
  double acc = 0.0;
  for (int64_t i = 0; i < rows; ++i) {
    const double v = (double)b[i];
    acc = fma(v, v, acc);
  }
  r[c] = acc / (double)rows;
}

// Row i of G = Bs R11^{-1} (l x l, Bs = B(:, S)) by forward substitution on
// the row vector (g R11 = Bs(i, :)), FP64, written as column i of Gt
// (Gt = G^T): g_j = b_j / R11(j, j), then b_k -= g_j R11(j, k) for k > j.
template <typename T>
__global__ void right_trsm_kernel(const T* __restrict__ Bs, int64_t l, const T* __restrict__ R11, int64_t ldr,
                                  T* __restrict__ Gt) {
  extern __shared__ double bsh[];  // l
  const int64_t i = blockIdx.x;
  for (int64_t j = threadIdx.x; j < l; j += NT) bsh[j] = (double)Bs[j * l + i];
  for (int64_t j = 0; j < l; ++j) {
    __syncthreads();
    const double g = bsh[j] / (double)R11[j * ldr + j];
    for (int64_t k = j + 1 + threadIdx.x; k < l; k += NT) bsh[k] = fma(-g, (double)R11[k * ldr + j], bsh[k]);
    if (threadIdx.x == 0) Gt[i * l + j] = (T)g;
  }
}

// r[c] = ||B(:, c) - C(:, c)||^2 / rows (FP64), one wave per column
// (the lanes read the column's contiguous rows, then a fixed-order wave sum)
template <typename T>
__global__ void sample_resid_kernel(const T* __restrict__ B, const T* __restrict__ Cm, int64_t rows, int64_t n,
                                    double* __restrict__ r) {
  const int64_t c = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (c >= n) return;
  double acc = 0.0;
  for (int64_t i = lane; i < rows; i += kWave) {
    const double v = (double)B[c * rows + i] - (double)Cm[c * rows + i];
    acc = fma(v, v, acc);
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane == 0) r[c] = acc / (double)rows;
}

template <typename T>
__global__ void sub_kernel(T* __restrict__ P, const T* __restrict__ D, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT)
    P[e] = (T)((double)P[e] - (double)D[e]);
}

// For each remaining column c = rest[q]: x = R11^{-1} Rb(:, c) by back
// substitution (in place in Rb), then B(:, c) -= B(:, piv) x.  One thread per
// column; R11 (bj x bj) and B(:, piv) (rows x bj) staged in LDS.
template <typename T>
__global__ void sample_update_kernel(T* __restrict__ B, int64_t ldb, int rows, const int64_t* __restrict__ piv,
                                     int bj, const T* __restrict__ R11, int64_t ldr, T* __restrict__ Rb,
                                     int64_t ldrb, const int64_t* __restrict__ rest, int64_t nr) {
  extern __shared__ double sm[];
  double* r11 = sm;              // r11[t * bj + i] = R11(i, t)
  double* bp = r11 + bj * bj;    // bp[t * rows + i] = B(i, piv[t])
  for (int e = threadIdx.x; e < bj * bj; e += NT) r11[e] = (double)R11[(int64_t)(e / bj) * ldr + e % bj];
  for (int e = threadIdx.x; e < rows * bj; e += NT) bp[e] = (double)B[piv[e / rows] * ldb + e % rows];
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (q >= nr) return;
  const int64_t c = rest[q];
  T* x = Rb + c * ldrb;
  for (int i = bj - 1; i >= 0; --i) {
    double v = (double)x[i];
    for (int t = i + 1; t < bj; ++t) v -= r11[t * bj + i] * (double)x[t];
    x[i] = (T)(v / r11[i * bj + i]);
  }
  T* bc = B + c * ldb;
  for (int i = 0; i < rows; ++i) {
    double v = (double)bc[i];
    for (int t = 0; t < bj; ++t) v -= bp[t * rows + i] * (double)x[t];
    bc[i] = (T)v;
  }
}

template <typename T>
struct TrqLayout {
  T *Bact = nullptr, *P = nullptr, *P2 = nullptr, *Qs = nullptr, *QT = nullptr, *C = nullptr,
    *R11 = nullptr, *Rb = nullptr;
  int64_t *act = nullptr, *pivl = nullptr, *pivd = nullptr, *rest = nullptr;
  double* mg = nullptr;
};

template <typename T>
bool trq_carve(Arena& ar, int64_t m, int64_t n, int64_t l, int64_t b, int64_t rows, TrqLayout<T>* o) {
  o->Bact = ar.take<T>((size_t)rows * n);
  o->P = ar.take<T>((size_t)m * b);
  o->P2 = ar.take<T>((size_t)m * b);
  o->Qs = ar.take<T>((size_t)m * l);
  o->QT = ar.take<T>((size_t)l * m);
  o->C = ar.take<T>((size_t)l * b);
  o->R11 = ar.take<T>((size_t)b * b);
  o->Rb = ar.take<T>((size_t)b * n);
  o->act = ar.take<int64_t>((size_t)n);
  o->pivl = ar.take<int64_t>((size_t)rows);
  o->pivd = ar.take<int64_t>((size_t)b);
  o->rest = ar.take<int64_t>((size_t)n);
  o->mg = ar.take<double>((size_t)rows);
  return o->Bact && o->P && o->P2 && o->Qs && o->QT && o->C && o->R11 && o->Rb && o->act &&
         o->pivl && o->pivd && o->rest && o->mg;
}

}  // namespace

int64_t trqrcp_rows(int64_t m, int64_t b, int64_t p) { return std::min(b + p, m); }

size_t trqrcp_lds(int64_t b, int64_t rows) { return (size_t)(b * b + rows * b) * sizeof(double); }

template <typename T>
size_t trqrcp_scratch(int64_t m, int64_t n, int64_t l, int64_t b, int64_t p, const DeviceInfo& d) {
  const int64_t rows = trqrcp_rows(m, b, p);
  Arena ar{nullptr, 0, 0};
  TrqLayout<T> o;
  trq_carve<T>(ar, m, n, l, b, rows, &o);
  size_t w = qrcp_scratch<T>(rows, n, d);
  w = std::max(w, gemm_tn_scratch<T>(b, n, m, d.num_cu));
  w = std::max(w, gemm_tn_scratch<T>(l, b, m, d.num_cu));
  w = std::max(w, gemm_tn_scratch<T>(m, b, l, d.num_cu));
  w = std::max(w, tallqr_scratch<T>(m, b, d));
  return ar.used + 256 + w + 1024;
}

template <typename T>
hipError_t trqrcp_select(const T* A, int64_t m, int64_t n, int64_t lda, int64_t l, int64_t b, int64_t p, T* B,
                         int64_t* S, double* margins, Arena& ar, unsigned* err, const DeviceInfo& d,
                         hipStream_t s, bool final_update) {
  const int64_t rows = trqrcp_rows(m, b, p);
  if (b < 1 || b > 64 || l < 1 || n - l + 1 < rows) return hipErrorInvalidValue;
  TrqLayout<T> o;
  if (!trq_carve<T>(ar, m, n, l, b, rows, &o)) return hipErrorOutOfMemory;
  const size_t base = ar.used;
  auto scratch = [&]() { return Arena{ar.base, ar.cap, base}; };
  const size_t lds = trqrcp_lds(b, rows);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)sample_update_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipError_t e;
  std::vector<int64_t> active((size_t)n), hS, pl((size_t)rows);
  std::iota(active.begin(), active.end(), int64_t(0));
  std::vector<double> hm, mgh((size_t)rows);
  int64_t j = 0;
  while (j < l) {
    const int64_t bj = std::min(b, l - j);
    const int64_t na = (int64_t)active.size();
    // 1. partial QRCP on the sample of the columns in play
    if ((e = hipMemcpyAsync(o.act, active.data(), (size_t)na * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return e;
    if ((e = gather_cols<T>(B, rows, n, rows, o.act, na, o.Bact, rows, s)) != hipSuccess) return e;
    {
      Arena a = scratch();
      if ((e = qrcp<T>(o.Bact, rows, na, rows, o.pivl, o.mg, a, err, d, s)) != hipSuccess) return e;
    }
    if ((e = hipMemcpyAsync(pl.data(), o.pivl, (size_t)bj * sizeof(int64_t), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(mgh.data(), o.mg, (size_t)bj * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    std::vector<int64_t> piv((size_t)bj);
    std::vector<char> taken((size_t)na, 0);
    for (int64_t t = 0; t < bj; ++t) {
      const int64_t loc = pl[(size_t)t];
      if (loc < 0 || loc >= na || taken[(size_t)loc]) return hipErrorInvalidValue;
      taken[(size_t)loc] = 1;
      piv[(size_t)t] = active[(size_t)loc];
      hS.push_back(piv[(size_t)t]);
      hm.push_back(mgh[(size_t)t]);
    }
    std::vector<int64_t> rest;
    rest.reserve((size_t)(na - bj));
    for (int64_t t = 0; t < na; ++t)
      if (!taken[(size_t)t]) rest.push_back(active[(size_t)t]);
    // 2. the chosen columns' residual, its QR
    if ((e = hipMemcpyAsync(o.pivd, piv.data(), (size_t)bj * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return e;
    if ((e = gather_cols<T>(A, m, n, lda, o.pivd, bj, o.P, m, s)) != hipSuccess) return e;
    if (j > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        Arena a = scratch();
        if ((e = gemm_tn<T>(j, bj, m, o.Qs, m, o.P, m, o.C, j, nullptr, a, d.num_cu, s)) != hipSuccess) return e;
        Arena a2 = scratch();
        if ((e = gemm_tn<T>(m, bj, j, o.QT, l, o.C, j, o.P2, m, nullptr, a2, d.num_cu, s)) != hipSuccess) return e;
        const int64_t tot = m * bj;
        sub_kernel<T><<<(unsigned)std::min<int64_t>((tot + NT - 1) / NT, 4096), NT, 0, s>>>(o.P, o.P2, tot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    T* Qb = o.Qs + j * m;
    {
      Arena a = scratch();
      if ((e = tall_qr<T>(o.P, m, bj, m, Qb, m, o.R11, bj, false, a, err, d, s)) != hipSuccess) return e;
    }
    if ((e = transpose<T>(Qb, m, bj, m, o.QT + j, l, s)) != hipSuccess) return e;
    // 3. R12 and the sample update of the remaining columns
    const int64_t nr = (int64_t)rest.size();
    if (nr > 0 && (j + bj < l || final_update)) {
      if ((e = hipMemcpyAsync(o.rest, rest.data(), (size_t)nr * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
          hipSuccess)
        return e;
      {
        Arena a = scratch();
        if ((e = gemm_tn<T>(bj, n, m, Qb, m, A, lda, o.Rb, bj, nullptr, a, d.num_cu, s)) != hipSuccess) return e;
      }
      sample_update_kernel<T><<<(unsigned)((nr + NT - 1) / NT), NT, lds, s>>>(B, rows, (int)rows, o.pivd, (int)bj,
                                                                              o.R11, bj, o.Rb, bj, o.rest, nr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the host vectors copied above must outlive the copies
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    active.swap(rest);
    j += bj;
  }
  if ((e = hipMemcpyAsync(S, hS.data(), (size_t)l * sizeof(int64_t), hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(margins, hm.data(), (size_t)l * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

template <typename T>
hipError_t sample_norms(const T* B, int64_t rows, int64_t n, double* r, hipStream_t s) {
  if (n <= 0 || rows <= 0) return hipSuccess;
  sample_norms_kernel<T><<<(unsigned)((n + NT - 1) / NT), NT, 0, s>>>(B, rows, n, r);
  return hipGetLastError();
}

template <typename T>
size_t one_block_estimates_scratch(int64_t l, int64_t n, const DeviceInfo& d) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  return 2 * up((size_t)l * l * sizeof(T)) + 2 * up((size_t)l * n * sizeof(T)) +
         gemm_tn_scratch<T>(l, n, l, d.num_cu) + 1024;
}

template <typename T>
hipError_t one_block_stage(const T* B, int64_t l, int64_t n, const int64_t* S, T** Bc, T** Bs, Arena& ar,
                           hipStream_t s) {
  *Bc = ar.take<T>((size_t)l * n);
  *Bs = ar.take<T>((size_t)l * l);
  if (!*Bc || !*Bs) return hipErrorOutOfMemory;
  hipError_t e = hipMemcpyAsync(*Bc, B, (size_t)l * n * sizeof(T), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  return gather_cols<T>(B, l, n, l, S, l, *Bs, l, s);
}

template <typename T>
hipError_t one_block_estimates(const T* Bc, const T* Bs, int64_t l, int64_t n, const T* R11, int64_t ldr, const T* W,
                               int64_t ldw, double* r, Arena& ar, const DeviceInfo& d, hipStream_t s) {
  if (l < 1 || n < 1) return hipSuccess;
  T* Gt = ar.take<T>((size_t)l * l);
  T* Cm = ar.take<T>((size_t)l * n);
  if (!Gt || !Cm) return hipErrorOutOfMemory;
  const size_t lds = (size_t)l * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)right_trsm_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  right_trsm_kernel<T><<<(unsigned)l, NT, lds, s>>>(Bs, l, R11, ldr, Gt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // C = G W, the sample of the projection of every column onto span(A(:, S))
  if ((e = gemm_tn<T>(l, n, l, Gt, l, W, ldw, Cm, l, nullptr, ar, d.num_cu, s)) != hipSuccess) return e;
  constexpr int CPB = NT / kWave;  // columns per block
  sample_resid_kernel<T><<<(unsigned)((n + CPB - 1) / CPB), NT, 0, s>>>(Bc, Cm, l, n, r);
  return hipGetLastError();
}

#define INST(T)                                                                                                   \
  template size_t one_block_estimates_scratch<T>(int64_t, int64_t, const DeviceInfo&);                           \
  template hipError_t one_block_stage<T>(const T*, int64_t, int64_t, const int64_t*, T**, T**, Arena&, hipStream_t); \
  template hipError_t one_block_estimates<T>(const T*, const T*, int64_t, int64_t, const T*, int64_t, const T*,     \
                                             int64_t, double*, Arena&, const DeviceInfo&, hipStream_t);             \
  template size_t trqrcp_scratch<T>(int64_t, int64_t, int64_t, int64_t, int64_t, const DeviceInfo&);             \
  template hipError_t trqrcp_select<T>(const T*, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, T*,       \
                                       int64_t*, double*, Arena&, unsigned*, const DeviceInfo&, hipStream_t,    \
                                       bool);                                                                    \
  template hipError_t sample_norms<T>(const T*, int64_t, int64_t, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace ffsrqr
