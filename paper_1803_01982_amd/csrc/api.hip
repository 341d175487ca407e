// C ABI of the gfx950 Flip-Flop SRQR library: argument checks, workspace
// planning, the stage entry points and the whole path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ffsrqr.h"
#include "common.hpp"
#include "kernels.hpp"

namespace ffsrqr {

namespace {

thread_local std::string g_last_error;

ffsrqr_status fail(ffsrqr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define FF_HIP(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(FFSRQR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));             \
  } while (0)

std::mutex g_dev_mu;
DeviceInfo g_dev[64];

// ---------------------------------------------------------------- profiling
struct Profile {
  std::mutex mu;
  bool on = false;
  double ms[FFSRQR_NUM_STEPS] = {};
  int64_t launches[FFSRQR_NUM_STEPS] = {};
} g_prof;

// Events around the steps of one ffsrqr_factor call, on its stream.
class StepTimer {
 public:
  explicit StepTimer(hipStream_t s) : s_(s) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    on_ = g_prof.on;
  }
  ~StepTimer() {
    for (auto& r : recs_) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
  }
  // begin() returns a handle for end(); end() without one closes the latest
  // step.  A step may be issued on another stream (its interval may then
  // overlap other steps).
  int begin(int step) { return begin(step, s_); }
  void end() { end((int)recs_.size() - 1, s_); }
  int begin(int step, hipStream_t st) {
    if (!on_) return -1;
    Rec r{step, nullptr, nullptr, false};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    hipEventRecord(r.a, st);
    recs_.push_back(r);
    return (int)recs_.size() - 1;
  }
  void end(int h, hipStream_t st) {
    if (!on_ || h < 0 || h >= (int)recs_.size()) return;
    if (hipEventRecord(recs_[h].b, st) == hipSuccess) recs_[h].closed = true;
  }
  // after the stream has been synchronised
  void collect() {
    if (!on_) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto& r : recs_) {
      float ms = 0.f;
      if (r.closed && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        g_prof.ms[r.step] += ms;
        g_prof.launches[r.step] += 1;
      }
    }
  }

 private:
  struct Rec {
    int step;
    hipEvent_t a, b;
    bool closed;
  };
  hipStream_t s_;
  bool on_ = false;
  std::vector<Rec> recs_;
};

bool valid_precision(int32_t p) { return p == FFSRQR_FP64 || p == FFSRQR_FP32 || p == FFSRQR_MIXED; }
size_t elem_size(int32_t p) { return p == FFSRQR_FP64 ? sizeof(double) : sizeof(float); }
// Rows of the K-major BF16 operand arrays of the mixed form: m rounded up to
// a multiple of 8 (16-byte fragment loads).
int64_t bf16_ld(int64_t m) { return (m + 7) / 8 * 8; }

// Conservative device shape for sizing without touching a device.
DeviceInfo sizing_device() {
  DeviceInfo d;
  d.num_cu = 512;
  d.lds_max = 0;  // size the global-memory fallbacks too
  d.coop = true;
  d.gfx950 = true;
  return d;
}

struct Layout {
  int64_t l;
  size_t bytes;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Persistent buffers of the whole path followed by one scratch region shared
// by the stages (they run in stream order).
template <typename T>
size_t scratch_bytes(int64_t m, int64_t n, int64_t l, const DeviceInfo& d, int64_t block = 0, int64_t p = 0,
                     bool est = false) {
  size_t s = 0;
  if (block > 0) s = std::max(s, trqrcp_scratch<T>(m, n, l, block, p, d));
  // the one-block estimates run on the side stream, next to a6 on the other
  if (est && block <= 0) s = std::max(s, align256(tallqr_scratch<T>(n, l, d)) + one_block_estimates_scratch<T>(l, n, d));
  s = std::max(s, gemm_tn_scratch<T>(l, n, m, d.num_cu));
  if (sizeof(T) == 4) s = std::max(s, gemm_bf16_scratch(l, n, m, d.num_cu));
  s = std::max(s, qrcp_scratch<T>(l, n, d));
  s = std::max(s, tallqr_scratch<T>(m, l, d));
  // a6 on one stream while a4's residual norms, a5 and a7 run on the other
  s = std::max(s, align256(tallqr_scratch<T>(n, l, d)) + std::max(srqr_scratch<T>(m, n, l), jacobi_scratch<T>(l, d)));
  s = std::max(s, srqr_scratch<T>(m, n, l));
  s = std::max(s, jacobi_scratch<T>(l, d));
  s = std::max(s, swap_scratch<T>(m, l));
  return s + 16 * 256;
}

template <typename T>
size_t persistent_bytes(int64_t m, int64_t n, int64_t l) {
  size_t b = 0;
  // Omega^T, then the gathered panel, then (mixed form) the BF16 parts of Q
  b += align256((size_t)(sizeof(T) == 4 ? bf16_ld(m) : m) * l * sizeof(T));
  b += align256((size_t)l * n * sizeof(T));                                   // B, then R^T
  b += align256((size_t)l * n * sizeof(T));                                   // W
  b += align256((size_t)n * l * sizeof(T));                                   // Qhat1
  b += align256((size_t)l * l * sizeof(T));                                   // R11
  b += 3 * align256((size_t)n * sizeof(double));                              // anorm2, gamma2, estimates
  b += 2 * align256((size_t)l * sizeof(double));                              // margins, rho
  b += align256((size_t)l * sizeof(int64_t));                                 // S
  b += align256((size_t)n);                                                   // inS
  b += align256((size_t)((n + 1023) / 1024 + 1) * sizeof(int64_t));           // perm counts
  b += align256(sizeof(SrqrState)) + align256(64 * sizeof(unsigned));         // state, error word
  return b + 256;
}

template <typename T>
size_t total_bytes(int64_t m, int64_t n, int64_t l, const DeviceInfo& d, int64_t block = 0, int64_t p = 0,
                   bool est = false) {
  return persistent_bytes<T>(m, n, l) + scratch_bytes<T>(m, n, l, d, block, p, est);
}

ffsrqr_status get_device(const DeviceInfo** out) {
  int id = 0;
  hipError_t e = hipGetDevice(&id);
  if (e != hipSuccess) return fail(FFSRQR_ENODEV, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (id < 0 || id >= 64) return fail(FFSRQR_ENODEV, "device id out of range");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceInfo& d = g_dev[id];
  if (d.id != id) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, id);
    if (e != hipSuccess) return fail(FFSRQR_ENODEV, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    d.num_cu = prop.multiProcessorCount;
    d.lds_max = prop.sharedMemPerBlock;
    d.coop = prop.cooperativeLaunch != 0;
    d.gfx950 = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    d.id = id;
  }
  if (!d.gfx950) return fail(FFSRQR_ENODEV, "the current device is not gfx950");
  if (!d.coop) return fail(FFSRQR_ENODEV, "the current device has no cooperative launch");
  *out = &d;
  return FFSRQR_OK;
}

// A second stream (default priority) with a fork and a join event, one set
// per host thread and device, so that concurrent calls from different host
// threads never share them.  Created on first use, kept until exit.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
thread_local SideStream g_side[64];

ffsrqr_status get_side(int id, SideStream** out) {
  SideStream& ss = g_side[id];
  if (!ss.stream) {
    hipError_t e = hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(FFSRQR_EHIP, std::string("side stream: ") + hipGetErrorString(e));
  }
  *out = &ss;
  return FFSRQR_OK;
}

// ------------------------------------------------------------- no-alloc
// Scratch of the entry points that allocate nothing: a file-scope device
// array of fixed size (one copy per GPU, held until the process ends).  Host
// code never passes the array's name to a kernel (on the host it only names
// a stand-in); it looks the array's address up once per device with
// hipGetSymbolAddress and passes that pointer.
constexpr int64_t kNoAllocMaxL = 1024;
constexpr size_t kNoAllocBytes =
    sizeof(double) * ((size_t)kNoAllocMaxL * kNoAllocMaxL + kNoAllocMaxL + (size_t)2 * kMaxGridBlocks * 32 * 32) +
    (kSyncWords + 64) * sizeof(unsigned) + 64 * sizeof(unsigned) + 16 * 256;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

ffsrqr_status scratch_for(int id, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[id]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(FFSRQR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[id] = ptr;
  }
  *out = g_scratch_ptr[id];
  return FFSRQR_OK;
}

ffsrqr_status check_dims(int64_t m, int64_t n, int64_t k, int64_t p) {
  if (m < 1 || n < 1) return fail(FFSRQR_EINVAL, "m and n must be >= 1");
  if (k < 1 || k > std::min(m, n)) return fail(FFSRQR_EINVAL, "k must satisfy 1 <= k <= min(m, n)");
  if (p < 0) return fail(FFSRQR_EINVAL, "p must be >= 0");
  if (m > (int64_t(1) << 31) || n > (int64_t(1) << 31)) return fail(FFSRQR_EINVAL, "m and n must be < 2^31");
  return FFSRQR_OK;
}

// Sizes the path supports on device d: l <= 1024 and the Householder QR of
// the m x l panel and of the n x l transposed factor fit the device.
ffsrqr_status check_limits(int64_t m, int64_t n, int64_t l, const DeviceInfo& d) {
  if (l > 1024) return fail(FFSRQR_EINVAL, "l = min(k + p, m, n) must be <= 1024");
  if (!tallqr_fits(m, l, d) || !tallqr_fits(n, l, d))
    return fail(FFSRQR_EINVAL, "m or n too large for the panel QR at this l (rows per workgroup exceed the LDS)");
  return FFSRQR_OK;
}

// The blocked selection (opts.block > 0): blocks of at most 64 pivots, and
// enough columns that the sample of the columns in play never has fewer
// columns than rows (n - l + 1 >= min(block + p, m)).
ffsrqr_status check_block(int64_t m, int64_t n, int64_t k, int64_t p, int64_t l, int32_t block) {
  if (block < 0 || block > 64) return fail(FFSRQR_EINVAL, "block must be 0 (one block) or 1..64");
  if (block == 0) return FFSRQR_OK;
  const int64_t b = std::min<int64_t>(block, k);
  if (n - l + 1 < trqrcp_rows(m, b, p))
    return fail(FFSRQR_EINVAL, "blocked selection needs n - l + 1 >= min(block + p, m)");
  return FFSRQR_OK;
}

// The tensor and robust PCA drivers run the one-block selection: their
// per-step ranks (and, for robust PCA, the rank of every iteration) change
// the sample's shape, so opts.block is refused there.
ffsrqr_status check_driver_opts(const ffsrqr_opts* o) {
  if (!o) return FFSRQR_OK;
  if (o->block != 0)
    return fail(FFSRQR_EINVAL, "opts.block is for ffsrqr_factor and ffsrqr_factor_batched; the drivers need 0");
  if (o->g2_probe < 0 || o->g2_probe > kMaxProbe) return fail(FFSRQR_EINVAL, "g2_probe must be 0 (exact) or 1..64");
  if (o->est_norms != 0) return fail(FFSRQR_EINVAL, "est_norms is for ffsrqr_factor and ffsrqr_factor_batched");
  return FFSRQR_OK;
}

// The device the limits are checked against when no device is at hand: a
// 256-CU gfx950 with 160 KiB of LDS per workgroup.
DeviceInfo limits_device() {
  DeviceInfo d;
  d.num_cu = 256;
  d.lds_max = 160 * 1024;
  d.coop = true;
  d.gfx950 = true;
  return d;
}

// Rank tolerance of the SRQR test (alpha or a diagonal entry of R11 at or
// below it counts as zero): max(m, n) 2^-52 max_j ||a_j|| for FP64 storage;
// for FP32 storage, 8 sqrt(max(m, n)) 2^-24 max_j ||a_j||, since Q1, the
// panel between blocks and W are rounded to FP32 and exactly dependent
// columns then leave residuals of order sqrt(l) 2^-24 ||a_j||.
double rank_tol(int64_t m, int64_t n, double anorm_max, bool fp32) {
  const double mn = (double)std::max(m, n);
  return fp32 ? 8.0 * std::sqrt(mn) * 0x1p-24 * anorm_max : mn * 0x1p-52 * anorm_max;
}

// Window of the j* preselection, relative to ||a_j||^2 + ||a_max||^2: the
// rounding of ||a_j||^2 - ||W(:, j)||^2 grows like (4 sqrt(m) + l) u with u
// the unit roundoff of W's arithmetic; the split-BF16 projection adds a
// product error of about 2^-16 per term, i.e. about 2^-16 / sqrt(m) of
// ||a_j||^2 for sums of m terms of random sign, taken with a factor 64.
template <typename T>
double select_window(int64_t m, int64_t l, bool mixed) {
  const double u = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;
  double w = (4.0 * std::sqrt((double)m) + (double)l) * u;
  if (mixed) w += 64.0 * 0x1p-16 / std::sqrt((double)m);
  return w;
}

ffsrqr_opts resolve(const ffsrqr_opts* o, int64_t l) {
  ffsrqr_opts r;
  ffsrqr_default_opts(&r);
  if (o) r = *o;
  if (r.g == 0.0) r.g = 2.0;
  if (r.max_swaps < 0) r.max_swaps = (int32_t)std::min<int64_t>(4 * l, INT32_MAX);
  return r;
}

// --------------------------------------------------------------------------
template <typename T>
ffsrqr_status factor_impl(const T* A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p, uint64_t seed,
                          int64_t* perm, T* Q, int64_t ldq, T* L, int64_t ldl, T* V, int64_t ldv, double* sigma,
                          ffsrqr_info* info, void* work, size_t work_bytes, const ffsrqr_opts& op,
                          const DeviceInfo& d, hipStream_t s) {
  const bool mixed = op.precision == FFSRQR_MIXED;
  const int64_t mp = bf16_ld(m);
  const int64_t l = std::min(k + p, std::min(m, n));
  uint32_t flags = (l < k + p) ? FFSRQR_FLAG_L_CLAMPED : 0u;
  const int64_t blk0 = op.block > 0 ? std::min<int64_t>(op.block, k) : 0;
  if (op.g2_probe < 0 || op.g2_probe > kMaxProbe) return fail(FFSRQR_EINVAL, "g2_probe must be 0 (exact) or 1..64");
  if (op.est_norms != 0 && op.est_norms != 1) return fail(FFSRQR_EINVAL, "est_norms must be 0 or 1");
  const bool est_mode = op.est_norms == 1;
  const size_t need = total_bytes<T>(m, n, l, d, blk0, p, est_mode);
  if (work_bytes < need)
    return fail(FFSRQR_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");

  Arena ar{(char*)work, work_bytes, 0};
  T* region1 = ar.take<T>((size_t)(sizeof(T) == 4 ? mp : m) * l);  // Omega^T, the gathered panel, Q's BF16 parts
  T* region2 = ar.take<T>((size_t)l * n);  // B, later R^T
  T* W = ar.take<T>((size_t)l * n);
  T* Qhat = ar.take<T>((size_t)n * l);
  T* R11 = ar.take<T>((size_t)l * l);
  double* anorm2 = ar.take<double>(n);
  double* gamma2 = ar.take<double>(n);
  double* est = ar.take<double>(n);
  double* margins = ar.take<double>(l);
  double* rho = ar.take<double>(l + 1);
  int64_t* S = ar.take<int64_t>(l);
  unsigned char* inS = ar.take<unsigned char>(n);
  int64_t* cnt = ar.take<int64_t>((n + 1023) / 1024 + 1);
  SrqrState* st = ar.take<SrqrState>(1);
  unsigned* err = ar.take<unsigned>(64);
  const size_t scratch_off = ar.used;
  auto scratch = [&]() { return Arena{(char*)work, work_bytes, scratch_off}; };
  if (!err) return fail(FFSRQR_EWORKSPACE, "workspace carving failed");

  SideStream* side = nullptr;
  {
    const ffsrqr_status sst = get_side(d.id, &side);
    if (sst != FFSRQR_OK) return sst;
  }
  StepTimer tm(s);
  FF_HIP(zero_words(err, 64, s));
  // a1: Omega and the sketch (one pass over A, column norms fused); with
  // the blocked selection (Algorithm 2's blocks) the sample has
  // min(block + p, m) rows instead of l
  const int64_t blk = op.block > 0 ? std::min<int64_t>(op.block, k) : 0;
  const int64_t srows = blk > 0 ? trqrcp_rows(m, blk, p) : l;
  tm.begin(FFSRQR_STEP_OMEGA);
  if (mixed) FF_HIP(launch_omega<__bf16>(seed, srows, m, (__bf16*)region1, mp, s));
  else FF_HIP(launch_omega<T>(seed, srows, m, region1, m, s));
  tm.end();
  {
    Arena a = scratch();
    tm.begin(FFSRQR_STEP_SKETCH);
    if (mixed)
      FF_HIP(gemm_bf16(1, srows, n, m, (const __bf16*)region1, nullptr, mp, (const float*)A, lda, (float*)region2,
                       srows, anorm2, a, d.num_cu, s));
    else
      FF_HIP(gemm_tn<T>(srows, n, m, region1, m, A, lda, region2, srows, anorm2, a, d.num_cu, s));
    tm.end();
  }
  // non-finite input: report and stop before any pivoting
  {
    Arena a = scratch();
    FF_HIP(hipMemsetAsync(inS, 0, (size_t)n, s));
    tm.begin(FFSRQR_STEP_CHECK);
    FF_HIP(srqr_select<T>(anorm2, anorm2, inS, n, A, m, lda, Q, ldq, W, l, R11, l, 0, st, a, s));
    tm.end();
    SrqrState hs;
    FF_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    FF_HIP(hipStreamSynchronize(s));
    if (hs.nonfinite) {
      flags |= FFSRQR_FLAG_NONFINITE;
      const double qnan = std::nan("");
      std::vector<double> nanv((size_t)l, qnan);
      FF_HIP(hipMemcpyAsync(sigma, nanv.data(), (size_t)l * sizeof(double), hipMemcpyHostToDevice, s));
      // NaN-fill Q, L, V column by column; perm = identity
      std::vector<T> col((size_t)std::max(m, n), (T)qnan);
      for (int64_t j = 0; j < l; ++j) {
        FF_HIP(hipMemcpyAsync(Q + j * ldq, col.data(), (size_t)m * sizeof(T), hipMemcpyHostToDevice, s));
        FF_HIP(hipMemcpyAsync(L + j * ldl, col.data(), (size_t)l * sizeof(T), hipMemcpyHostToDevice, s));
        FF_HIP(hipMemcpyAsync(V + j * ldv, col.data(), (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
      }
      std::vector<int64_t> id((size_t)n);
      for (int64_t j = 0; j < n; ++j) id[j] = j;
      FF_HIP(hipMemcpyAsync(perm, id.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, s));
      FF_HIP(hipStreamSynchronize(s));
      if (info) {
        std::memset(info, 0, sizeof(*info));
        info->l = l;
        info->flags = flags;
        info->g2 = qnan;
        info->alpha = qnan;
        info->jstar = -1;
        info->jstar_margin = 0.0;
      }
      return FFSRQR_OK;
    }
  }
  // a2: partial QRCP on the sketch -> S (or Algorithm 2's blocks of it)
  {
    Arena a = scratch();
    tm.begin(FFSRQR_STEP_QRCP);
    if (blk > 0) {
      const hipError_t e = trqrcp_select<T>(A, m, n, lda, l, blk, p, region2, S, margins, a, err, d, s, est_mode);
      if (e == hipErrorInvalidValue) return fail(FFSRQR_EHIP, "blocked pivot selection: invalid pivot");
      FF_HIP(e);
      // Algorithm 4's residual norm estimates from the sample after the last block
      if (est_mode) FF_HIP(sample_norms<T>(region2, srows, n, est, s));
    } else {
      FF_HIP(qrcp<T>(region2, l, n, l, S, margins, a, err, d, s));
    }
    tm.end();
  }
  std::vector<double> hmarg((size_t)l);
  FF_HIP(hipMemcpyAsync(hmarg.data(), margins, (size_t)l * sizeof(double), hipMemcpyDeviceToHost, s));

  int32_t swaps = 0;
  int32_t rotations = 0;  // swap-loop iterations: swaps and the probe's identity rotations
  uint64_t probe_q = 0;   // SRQR tests so far; the q-th draws the probe of stream q
  const bool probe = op.g2_probe > 0;
  int32_t jacobi_sweeps = 0;
  SrqrState hs{};
  double g2 = 1.0;
  int64_t numerical_rank = l;
  // a6 and a7 for the current leading set: the LQ on the caller's stream;
  // as soon as its cooperative kernel has written L, the Jacobi step on the
  // side stream while the caller's stream forms Qhat1 (into a buffer of its
  // own) and V.  Their scratch is carved after the LQ's.
  Arena a_main = scratch();
  Arena a_side{(char*)work, work_bytes, scratch_off + align256(tallqr_scratch<T>(n, l, d))};
  auto issue_lq = [&]() -> ffsrqr_status {
    const int lq_step = tm.begin(FFSRQR_STEP_LQ);
    FF_HIP(assemble_rt<T>(R11, l, W, l, perm, l, n, region2, n, s));
    Arena am = a_main;
    FF_HIP(tall_qr<T>(region2, n, l, n, Qhat, n, L, ldl, true, am, err, d, s, side->fork));
    FF_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
    const int svd_step = tm.begin(FFSRQR_STEP_SVD, side->stream);
    Arena a = a_side;
    FF_HIP(jacobi_sigma<T>(L, l, ldl, sigma, a, err, d, side->stream, (int*)(err + 32)));
    tm.end(svd_step, side->stream);
    FF_HIP(hipEventRecord(side->join, side->stream));
    FF_HIP(scatter_rows<T>(Qhat, n, l, n, perm, V, ldv, s));
    tm.end(lq_step, s);
    FF_HIP(hipStreamWaitEvent(s, side->join, 0));
    return FFSRQR_OK;
  };
  // device-wide waits that ran out of their spin limit end the call
  auto timed_out = [&]() -> ffsrqr_status {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->l = l;
      info->flags = flags | FFSRQR_FLAG_TIMEOUT;
      info->g2 = std::nan("");
      info->alpha = std::nan("");
      info->jstar = -1;
    }
    return fail(FFSRQR_EHIP, "a device-wide wait exceeded its spin limit; the outputs are incomplete");
  };
  bool lq_current = false;  // L, V, sigma belong to the current leading set
  bool redo = false;        // the next test runs on the same leading set (estimates: identity rotation)
  T* ob_Bc = nullptr;       // one-block estimates: the copied sketch and B(:, S), pending on the side stream
  T* ob_Bs = nullptr;
  Arena ob_arena = a_side;
  int64_t removed_col = -1; // original index of the column the next swap removes
  unsigned herr[64];
  std::vector<int64_t> hS;
  for (int iter = 0;; ++iter) {
    if (iter == 0) {
      // a3: Householder QR of A(:, S); a4: projection
      tm.begin(FFSRQR_STEP_PANEL);
      FF_HIP(build_perm(S, l, n, perm, inS, cnt, s));
      FF_HIP(gather_cols<T>(A, m, n, lda, perm, l, region1, m, s));
      {
        Arena a = scratch();
        FF_HIP(tall_qr<T>(region1, m, l, m, Q, ldq, R11, l, false, a, err, d, s));
      }
      tm.end();
      {
        Arena a = scratch();
        tm.begin(FFSRQR_STEP_PROJECT);
        if (mixed) {
          // the panel in region1 is no longer read once Q is formed (stream order)
          __bf16* qh = (__bf16*)region1;
          __bf16* ql = qh + (size_t)mp * l;
          FF_HIP(split_bf16((const float*)Q, m, l, ldq, qh, ql, mp, s));
          FF_HIP(gemm_bf16(3, l, n, m, qh, ql, mp, (const float*)A, lda, (float*)W, l, nullptr, a, d.num_cu, s));
        } else {
          FF_HIP(gemm_tn<T>(l, n, m, Q, ldq, A, lda, W, l, nullptr, a, d.num_cu, s));
        }
        tm.end();
      }
      if (est_mode && blk == 0 && l < n) {
        // Algorithm 4's estimates for the one-block selection: the l-row
        // sketch (still in region2, which a6 reuses) is copied to the side
        // stream's scratch here, and updated there with all l pivots as one
        // block before the SRQR test
        Arena a = a_side;
        FF_HIP(one_block_stage<T>(region2, l, n, S, &ob_Bc, &ob_Bs, a, s));
        ob_arena = a;
      }
    } else if (!redo) {
      // Algorithm 4's swap as an update of Q, R11 and W (rotations, one new
      // column, one pass over A for the new row); S was updated on the host
      tm.begin(FFSRQR_STEP_SWAP);
      {
        Arena a = scratch();
        FF_HIP(srqr_swap_update<T>(A, m, n, lda, Q, ldq, W, l, R11, l, l, hs.istar, hs.jstar, a, s,
                                   est_mode ? est : nullptr, removed_col));
      }
      FF_HIP(build_perm(S, l, n, perm, inS, cnt, s));
      tm.end();
    }
    // The side stream runs a4's residual norms and the SRQR test (a5); in
    // the first test the caller's stream runs a6 meanwhile (issued before the
    // swap decision is known: it is the result unless a swap follows).  They
    // read W and R11 concurrently and write disjoint buffers.
    FF_HIP(hipEventRecord(side->fork, s));
    FF_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
    {
      const int h = tm.begin(FFSRQR_STEP_RESID, side->stream);
      if (!est_mode) FF_HIP(residual_norms<T>(W, l, n, l, anorm2, gamma2, side->stream));
      if (ob_Bc) {
        Arena a = ob_arena;
        FF_HIP(one_block_estimates<T>(ob_Bc, ob_Bs, l, n, R11, l, W, l, est, a, d, side->stream));
        ob_Bc = nullptr;
      }
      tm.end(h, side->stream);
    }
    {
      const int h = tm.begin(FFSRQR_STEP_SRQR, side->stream);
      Arena a = a_side;
      // with the estimates j* is their argmax (a zero window: only exact
      // ties are candidates) and alpha its exact residual norm
      FF_HIP(srqr_select<T>(est_mode ? est : gamma2, anorm2, inS, n, A, m, lda, Q, ldq, W, l, R11, l, l, st, a,
                            side->stream, est_mode ? 0.0 : select_window<T>(m, l, mixed)));
      if (l < n) {
        Arena a2 = a_side;
        ++probe_q;
        if (probe) {
          const hipError_t e = srqr_probe<T>(R11, l, W, l, st, 0.0, l, op.g2_probe, seed, probe_q, rho, st, a2,
                                             side->stream);
          if (e == hipErrorInvalidValue) return fail(FFSRQR_EINVAL, "bad g2 probe");
          FF_HIP(e);
        } else {
          FF_HIP(srqr_rho<T>(R11, l, W, l, st, 0.0, l, rho, st, a2, side->stream));
        }
      }
      tm.end(h, side->stream);
    }
    if (iter == 0) {
      const ffsrqr_status lst = issue_lq();  // joins the side stream
      if (lst != FFSRQR_OK) return lst;
      lq_current = true;
    } else {
      FF_HIP(hipEventRecord(side->join, side->stream));
      FF_HIP(hipStreamWaitEvent(s, side->join, 0));
      if (!redo) lq_current = false;
    }
    redo = false;
    FF_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    FF_HIP(hipMemcpyAsync(herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    FF_HIP(hipStreamSynchronize(s));
    if (herr[0]) return timed_out();
    if (lq_current) jacobi_sweeps = (int32_t)herr[32];
    if (l >= n) {
      g2 = 1.0;
      hs.jstar = -1;
      hs.alpha = 0.0;
      break;
    }
    const double tau_r = rank_tol(m, n, hs.anorm_max, sizeof(T) == 4);
    if (hs.alpha <= tau_r || hs.min_diag <= tau_r) {
      flags |= FFSRQR_FLAG_RANK_DEFICIENT;
      std::vector<T> hr((size_t)l * l);
      FF_HIP(hipMemcpy(hr.data(), R11, hr.size() * sizeof(T), hipMemcpyDeviceToHost));
      numerical_rank = 0;
      for (int64_t i = 0; i < l; ++i)
        if (std::fabs((double)hr[(size_t)i * l + i]) > tau_r) ++numerical_rank;
      g2 = 1.0;
      break;
    }
    // Algorithm 4's loop test.  With the random probe the argmax may be the
    // (l+1)-st position itself: that rotation is the identity, the leading
    // set and its factors stay, and the next test only draws a fresh probe.
    bool done = false;
    for (;;) {
      g2 = hs.g2;
      if (g2 <= op.g) {
        done = true;
        break;
      }
      if (rotations >= op.max_swaps) {
        flags |= FFSRQR_FLAG_SWAPCAP;
        done = true;
        break;
      }
      ++rotations;
      if (!(probe && hs.istar == l)) break;
      if (est_mode) {
        // j* returns to the (l+1)-st position with its exact residual norm:
        // the selection runs again on the same leading set
        FF_HIP(est_reset_jstar(est, st, s));
        redo = true;
        break;
      }
      ++probe_q;
      tm.begin(FFSRQR_STEP_SRQR);
      {
        Arena a2 = a_side;
        FF_HIP(srqr_probe<T>(R11, l, W, l, st, 0.0, l, op.g2_probe, seed, probe_q, rho, st, a2, s));
      }
      tm.end();
      FF_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
      FF_HIP(hipStreamSynchronize(s));
    }
    if (done) break;
    if (redo) continue;
    // round-robin swap: S <- (S without S[istar]) followed by jstar
    if (hs.istar < 0 || hs.istar >= l || hs.jstar < 0 || hs.jstar >= n)
      return fail(FFSRQR_EHIP, "invalid swap candidates");
    if (hS.empty()) {
      hS.resize((size_t)l);
      FF_HIP(hipMemcpy(hS.data(), S, (size_t)l * sizeof(int64_t), hipMemcpyDeviceToHost));
    }
    removed_col = hS[(size_t)hs.istar];
    hS.erase(hS.begin() + hs.istar);
    hS.push_back(hs.jstar);
    FF_HIP(hipMemcpyAsync(S, hS.data(), (size_t)l * sizeof(int64_t), hipMemcpyHostToDevice, s));
    ++swaps;
  }
  if (!lq_current) {
    // the leading set changed after the first LQ: a6 and a7 once more
    const ffsrqr_status lst = issue_lq();
    if (lst != FFSRQR_OK) return lst;
    FF_HIP(hipMemcpyAsync(herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    FF_HIP(hipStreamSynchronize(s));
    if (herr[0]) return timed_out();
    jacobi_sweeps = (int32_t)herr[32];
  }
  tm.collect();
  if (info) {
    double mm = 1.0;
    for (double x : hmarg) mm = std::min(mm, x);
    info->l = l;
    info->swaps = swaps;
    info->flags = flags;
    info->g2 = g2;
    info->alpha = hs.alpha;
    info->jstar = hs.jstar;
    info->numerical_rank = numerical_rank;
    info->min_margin = mm;
    info->jacobi_sweeps = jacobi_sweeps;
    info->probes = probe ? (int32_t)probe_q : 0;
    info->jstar_margin = l < n ? hs.jmargin : 1.0;
    info->jstar_candidates = l < n ? hs.ncand : 0;
  }
  return FFSRQR_OK;
}

}  // namespace
}  // namespace ffsrqr

namespace ffsrqr {
namespace {
ffsrqr_status sketch_mixed(const float* A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int64_t l, float* B,
                           int64_t ldb, double* anorm2, void* work, size_t work_bytes, const DeviceInfo& d,
                           hipStream_t s) {
  Arena ar{(char*)work, work_bytes, 0};
  const int64_t mp = bf16_ld(m);
  __bf16* Ot = ar.take<__bf16>((size_t)mp * l);
  if (!Ot) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(launch_omega<__bf16>(seed, l, m, Ot, mp, s));
  hipError_t e = gemm_bf16(1, l, n, m, Ot, nullptr, mp, A, lda, B, ldb, anorm2, ar, d.num_cu, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

template <typename T>
ffsrqr_status sketch_impl(const T* A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int64_t l, T* B, int64_t ldb,
                          double* anorm2, void* work, size_t work_bytes, const DeviceInfo& d, hipStream_t s) {
  Arena ar{(char*)work, work_bytes, 0};
  T* Ot = ar.take<T>((size_t)m * l);
  if (!Ot) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(launch_omega<T>(seed, l, m, Ot, m, s));
  hipError_t e = gemm_tn<T>(l, n, m, Ot, m, A, lda, B, ldb, anorm2, ar, d.num_cu, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}
// Algorithm 9, last steps: workspace carving shared by the sizing and the call.
template <typename T>
struct Alg9Layout {
  T *tt, *P, *Qt, *Rt, *UR, *VR;
  double* sg;
  unsigned* err;
  size_t scratch_off;
};

template <typename T>
size_t alg9_scratch(int64_t m, int64_t n, int64_t l, int64_t k, const DeviceInfo& d) {
  size_t s = 0;
  s = std::max(s, gemm_tn_scratch<T>(l, m, n, d.num_cu));
  s = std::max(s, gemm_tn_scratch<T>(k, m, l, d.num_cu));
  s = std::max(s, gemm_tn_scratch<T>(k, n, l, d.num_cu));
  s = std::max(s, tallqr_scratch<T>(m, l, d));
  s = std::max(s, jacobi_scratch<T>(l, d));
  s = std::max(s, swap_scratch<T>(m, l));
  return s + 16 * 256;
}

template <typename T>
bool alg9_carve(Arena& ar, int64_t m, int64_t n, int64_t l, int64_t k, Alg9Layout<T>* o) {
  o->tt = ar.take<T>(std::max((size_t)l * m, (size_t)k * n));  // tmp^T, then U^T, then V_k^T
  o->P = ar.take<T>((size_t)m * l);                             // tmp, factored in place
  o->Qt = ar.take<T>((size_t)m * l);
  o->Rt = ar.take<T>((size_t)l * l);
  o->UR = ar.take<T>((size_t)l * l);
  o->VR = ar.take<T>((size_t)l * l);
  o->sg = ar.take<double>((size_t)k);
  o->err = ar.take<unsigned>(64);
  o->scratch_off = ar.used;
  return o->err != nullptr;
}

template <typename T>
size_t alg9_bytes(int64_t m, int64_t n, int64_t l, int64_t k, const DeviceInfo& d) {
  Arena ar{nullptr, 0, 0};
  Alg9Layout<T> o;
  alg9_carve<T>(ar, m, n, l, k, &o);
  return ar.used + 256 + alg9_scratch<T>(m, n, l, k, d);
}

template <typename T>
ffsrqr_status alg9_impl(const T* A, int64_t m, int64_t n, int64_t lda, const T* V, int64_t ldv, int64_t l, int64_t k,
                        T* U, int64_t ldu, double* sigma, T* Vk, int64_t ldvk, void* work, size_t work_bytes,
                        const DeviceInfo& d, hipStream_t s) {
  const size_t need = alg9_bytes<T>(m, n, l, k, d);
  if (work_bytes < need) return fail(FFSRQR_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  Arena ar{(char*)work, work_bytes, 0};
  Alg9Layout<T> o;
  if (!alg9_carve<T>(ar, m, n, l, k, &o)) return fail(FFSRQR_EWORKSPACE, "workspace carving failed");
  auto scratch = [&]() { return Arena{(char*)work, work_bytes, o.scratch_off}; };
  FF_HIP(zero_words(o.err, 64, s));
  {
    // tmp^T = V^T A^T (l x m): the third pass over A (A read by columns)
    Arena a = scratch();
    FF_HIP(gemm_tn<T>(l, m, n, V, ldv, A, lda, o.tt, l, nullptr, a, d.num_cu, s, true));
  }
  FF_HIP(transpose<T>(o.tt, l, m, l, o.P, m, s));
  {
    // thin SVD of tmp: Householder QR, then Jacobi with vectors on R
    Arena a = scratch();
    FF_HIP(tall_qr<T>(o.P, m, l, m, o.Qt, m, o.Rt, l, false, a, o.err, d, s));
  }
  {
    Arena a = scratch();
    FF_HIP(jacobi_svd_vectors<T>(o.Rt, l, l, sigma, o.UR, l, o.VR, l, a, o.err, d, s));
  }
  {
    // U = Qt UR(:, 1:k) and V_k = V VR(:, 1:k), both through their transposes
    Arena a = scratch();
    FF_HIP(gemm_tn<T>(k, m, l, o.UR, l, o.Qt, m, o.tt, k, nullptr, a, d.num_cu, s, true));
    FF_HIP(transpose<T>(o.tt, k, m, k, U, ldu, s));
    Arena b = scratch();
    FF_HIP(gemm_tn<T>(k, n, l, o.VR, l, V, ldv, o.tt, k, nullptr, b, d.num_cu, s, true));
    FF_HIP(transpose<T>(o.tt, k, n, k, Vk, ldvk, s));
  }
  FF_HIP(normalize_pair_signs<T>(U, m, ldu, Vk, n, ldvk, k, o.sg, s));
  unsigned herr = 0;
  FF_HIP(hipMemcpyAsync(&herr, o.err, sizeof(herr), hipMemcpyDeviceToHost, s));
  FF_HIP(hipStreamSynchronize(s));
  if (herr) return fail(FFSRQR_EHIP, "a device-wide wait exceeded its spin limit; the outputs are incomplete");
  return FFSRQR_OK;
}

// ----------------------------------------------------------------- ST-HOSVD
// The ST-HOSVD loop (Section 2, the ST-HOSVD algorithm) with Flip-Flop SRQR
// and Algorithm 9's completion as the rank-k SVD of each unfolding.  Step j
// processes mode r = order[j]: its unfolding G_(r) is m x n with m = the
// current n_r and n = the product of the other current dimensions (the
// modes already processed reduced to their ranks); l = min(k_r + p, m, n).
struct HosvdPlan {
  int d = 0;
  int64_t dims[kMaxTensorOrder] = {}, ranks[kMaxTensorOrder] = {};
  int order[kMaxTensorOrder] = {};
  int64_t m[kMaxTensorOrder] = {}, n[kMaxTensorOrder] = {}, l[kMaxTensorOrder] = {};
  int64_t total = 0, m_max = 0, n_max = 0, l_max = 0, k_max = 0;
};

ffsrqr_status hosvd_plan(int32_t d, const int64_t* dims, const int64_t* ranks, const int32_t* order, int64_t p,
                         const DeviceInfo& dev, HosvdPlan* pl) {
  if (d < 1 || d > kMaxTensorOrder) return fail(FFSRQR_EINVAL, "tensor order must be between 1 and 8");
  if (!dims || !ranks) return fail(FFSRQR_EINVAL, "NULL dims or ranks");
  if (p < 0) return fail(FFSRQR_EINVAL, "p must be >= 0");
  pl->d = d;
  pl->total = 1;
  bool seen[kMaxTensorOrder] = {};
  for (int j = 0; j < d; ++j) {
    if (dims[j] < 1 || ranks[j] < 1 || ranks[j] > dims[j])
      return fail(FFSRQR_EINVAL, "need 1 <= ranks[j] <= dims[j] for every mode");
    if (pl->total > (int64_t(1) << 40) / dims[j]) return fail(FFSRQR_EINVAL, "tensor too large");
    pl->total *= dims[j];
    pl->dims[j] = dims[j];
    pl->ranks[j] = ranks[j];
    const int o = order ? order[j] : j;
    if (o < 0 || o >= d || seen[o]) return fail(FFSRQR_EINVAL, "order must be a permutation of 0..d-1");
    seen[o] = true;
    pl->order[j] = o;
  }
  int64_t cur[kMaxTensorOrder];
  int64_t size = pl->total;
  for (int j = 0; j < d; ++j) cur[j] = dims[j];
  for (int j = 0; j < d; ++j) {
    const int r = pl->order[j];
    const int64_t m = cur[r], n = size / m, k = ranks[r];
    ffsrqr_status st = check_dims(m, n, k, p);
    if (st != FFSRQR_OK) return fail(FFSRQR_EINVAL, "mode " + std::to_string(r) + ": " + ffsrqr_last_error());
    const int64_t l = std::min(k + p, std::min(m, n));
    st = check_limits(m, n, l, dev);
    if (st != FFSRQR_OK) return fail(FFSRQR_EINVAL, "mode " + std::to_string(r) + ": " + ffsrqr_last_error());
    pl->m[j] = m;
    pl->n[j] = n;
    pl->l[j] = l;
    pl->m_max = std::max(pl->m_max, m);
    pl->n_max = std::max(pl->n_max, n);
    pl->l_max = std::max(pl->l_max, l);
    pl->k_max = std::max(pl->k_max, k);
    size = size / m * k;
    cur[r] = k;
  }
  return FFSRQR_OK;
}

// Two tensor buffers (each the input's size), the factor outputs of the
// largest step, then one region shared by the steps' workspaces.
template <typename T>
size_t hosvd_fixed_bytes(const HosvdPlan& pl) {
  return 2 * align256((size_t)pl.total * sizeof(T)) + align256((size_t)pl.n_max * sizeof(int64_t)) +
         align256((size_t)pl.m_max * pl.l_max * sizeof(T)) + align256((size_t)pl.l_max * pl.l_max * sizeof(T)) +
         align256((size_t)pl.n_max * pl.l_max * sizeof(T)) + align256((size_t)pl.l_max * sizeof(double)) +
         align256((size_t)pl.n_max * pl.k_max * sizeof(T)) + 256;
}
template <typename T>
size_t hosvd_bytes(const HosvdPlan& pl, const DeviceInfo& d) {
  size_t w = 0;
  for (int j = 0; j < pl.d; ++j) {
    const int64_t m = pl.m[j], n = pl.n[j], l = pl.l[j], k = pl.ranks[pl.order[j]];
    w = std::max(w, total_bytes<T>(m, n, l, d));
    w = std::max(w, alg9_bytes<T>(m, n, l, k, d));
    w = std::max(w, gemm_tn_scratch<T>(k, n, m, d.num_cu) + 256);
  }
  return hosvd_fixed_bytes<T>(pl) + w + 1024;
}

template <typename T>
ffsrqr_status hosvd_impl(const T* X, const HosvdPlan& pl, int64_t p, uint64_t seed, T* core, T* const* U,
                         const int64_t* ldu, void* work, size_t work_bytes, const ffsrqr_opts* opts,
                         const DeviceInfo& d, hipStream_t s) {
  const size_t need = hosvd_bytes<T>(pl, d);
  if (work_bytes < need) return fail(FFSRQR_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  Arena ar{(char*)work, work_bytes, 0};
  T* buf[2] = {ar.take<T>((size_t)pl.total), ar.take<T>((size_t)pl.total)};
  int64_t* perm = ar.take<int64_t>((size_t)pl.n_max);
  T* Q = ar.take<T>((size_t)pl.m_max * pl.l_max);
  T* L = ar.take<T>((size_t)pl.l_max * pl.l_max);
  T* V = ar.take<T>((size_t)pl.n_max * pl.l_max);
  double* sigma = ar.take<double>((size_t)pl.l_max);
  T* Vk = ar.take<T>((size_t)pl.n_max * pl.k_max);
  if (!buf[0] || !buf[1] || !perm || !Q || !L || !V || !sigma || !Vk)
    return fail(FFSRQR_EWORKSPACE, "workspace carving failed");
  const size_t off = align256(ar.used);
  char* fwork = (char*)work + off;
  const size_t fbytes = work_bytes - off;
  int64_t cur[kMaxTensorOrder];
  for (int j = 0; j < pl.d; ++j) cur[j] = pl.dims[j];
  const T* G = X;  // the current tensor, held as its mode-gmode unfolding
  int gmode = 0, nb = 0;
  for (int j = 0; j < pl.d; ++j) {
    const int r = pl.order[j];
    const int64_t m = pl.m[j], n = pl.n[j], l = pl.l[j], k = pl.ranks[r];
    const T* Gr = G;
    if (gmode != r) {
      FF_HIP(reunfold<T>(G, gmode, buf[nb], r, pl.d, cur, s));
      Gr = buf[nb];
      nb ^= 1;
    }
    // rank-k_r SVD of G_(r): Flip-Flop SRQR, then Algorithm 9's completion
    const ffsrqr_opts op = resolve(opts, l);
    ffsrqr_status st = factor_impl<T>(Gr, m, n, m, k, p, seed, perm, Q, m, L, l, V, n, sigma, nullptr, fwork, fbytes,
                                      op, d, s);
    if (st != FFSRQR_OK) return st;
    st = alg9_impl<T>(Gr, m, n, m, V, n, l, k, U[r], ldu[r], sigma, Vk, n, fwork, fbytes, d, s);
    if (st != FFSRQR_OK) return st;
    // G_(r) <- U_r^T G_(r), the mode-r unfolding of the reduced tensor
    T* W = buf[nb];
    nb ^= 1;
    Arena a{fwork, fbytes, 0};
    FF_HIP(gemm_tn<T>(k, n, m, U[r], ldu[r], Gr, m, W, k, nullptr, a, d.num_cu, s));
    cur[r] = k;
    G = W;
    gmode = r;
  }
  // the core in Fortran order, i.e. its mode-0 unfolding
  FF_HIP(reunfold<T>(G, gmode, core, 0, pl.d, cur, s));
  FF_HIP(hipStreamSynchronize(s));
  return FFSRQR_OK;
}

// ---------------------------------------------------------------- robust PCA
// Robust PCA by IALM (Section 2, the robust PCA algorithm) with the whole
// path plus Algorithm 9 as the rank-sv SVD of each iteration.  sv is capped
// at `cap` (min(m, n), 1024 - p, and the caller's max_rank), so that
// l = min(sv + p, m, n) stays within the path's limit.
struct RpcaSizes {
  int64_t r = 0, cap = 0, lmax = 0;
};

RpcaSizes rpca_sizes(int64_t m, int64_t n, int64_t p, int64_t max_rank) {
  RpcaSizes z;
  z.r = std::min(m, n);
  z.cap = std::min(z.r, 1024 - p);
  if (max_rank > 0) z.cap = std::min(z.cap, max_rank);
  z.lmax = std::min(z.cap + p, z.r);
  return z;
}

template <typename T>
size_t rpca_fixed_bytes(int64_t m, int64_t n, const RpcaSizes& z) {
  const size_t mn = (size_t)m * n;
  return 3 * align256(mn * sizeof(T)) + align256((size_t)z.cap * m * sizeof(T)) +
         align256((size_t)z.cap * n * sizeof(T)) + align256((size_t)n * sizeof(int64_t)) +
         align256((size_t)m * z.lmax * sizeof(T)) + align256((size_t)z.lmax * z.lmax * sizeof(T)) +
         align256((size_t)n * z.lmax * sizeof(T)) + align256((size_t)z.lmax * sizeof(double)) +
         align256((size_t)m * z.cap * sizeof(T)) + align256((size_t)n * z.cap * sizeof(T)) +
         align256((size_t)(2 * kIalmBlocks + 8) * sizeof(double)) + 256;
}
template <typename T>
size_t rpca_bytes(int64_t m, int64_t n, const RpcaSizes& z, const DeviceInfo& d) {
  size_t w = total_bytes<T>(m, n, z.lmax, d);
  w = std::max(w, alg9_bytes<T>(m, n, z.lmax, z.cap, d));
  w = std::max(w, gemm_tn_scratch<T>(m, n, z.cap, d.num_cu) + 256);
  return rpca_fixed_bytes<T>(m, n, z) + w + 1024;
}

template <typename T>
ffsrqr_status rpca_impl(const T* M, int64_t m, int64_t n, int64_t ldm, double lam, double tol, int32_t max_iter,
                        int64_t p, uint64_t seed, const RpcaSizes& z, T* X, int64_t ldx, T* E, int64_t lde,
                        ffsrqr_rpca_info* info, void* work, size_t work_bytes, const ffsrqr_opts* opts,
                        const DeviceInfo& d, hipStream_t s) {
  const size_t need = rpca_bytes<T>(m, n, z, d);
  if (work_bytes < need) return fail(FFSRQR_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  Arena ar{(char*)work, work_bytes, 0};
  const size_t mn = (size_t)m * n;
  T* D = ar.take<T>(mn);
  T* Y = ar.take<T>(mn);
  T* Ei = ar.take<T>(mn);
  T* Ut = ar.take<T>((size_t)z.cap * m);
  T* Vt = ar.take<T>((size_t)z.cap * n);
  int64_t* perm = ar.take<int64_t>((size_t)n);
  T* Q = ar.take<T>((size_t)m * z.lmax);
  T* L = ar.take<T>((size_t)z.lmax * z.lmax);
  T* V = ar.take<T>((size_t)n * z.lmax);
  double* sigma = ar.take<double>((size_t)z.lmax);
  T* U = ar.take<T>((size_t)m * z.cap);
  T* Vk = ar.take<T>((size_t)n * z.cap);
  double* part = ar.take<double>((size_t)2 * kIalmBlocks + 8);
  if (!D || !Y || !Ei || !Ut || !Vt || !perm || !Q || !L || !V || !sigma || !U || !Vk || !part)
    return fail(FFSRQR_EWORKSPACE, "workspace carving failed");
  double* out = part + 2 * kIalmBlocks;
  const size_t off = align256(ar.used);
  char* fwork = (char*)work + off;
  const size_t fbytes = work_bytes - off;
  double hout[2];
  auto read_out = [&]() -> ffsrqr_status {
    FF_HIP(hipMemcpyAsync(hout, out, sizeof(hout), hipMemcpyDeviceToHost, s));
    FF_HIP(hipStreamSynchronize(s));
    return FFSRQR_OK;
  };
  // ||M||_F and max |M_ij|
  FF_HIP(matrix_norms<T>(M, ldm, m, n, part, out, s));
  ffsrqr_status st = read_out();
  if (st != FFSRQR_OK) return st;
  const double fro = std::sqrt(hout[0]), amax = hout[1];
  // ||M||_2 estimate: sigma_1 of the flip-flop factor L of M (k = 1)
  double norm2 = 0.0;
  {
    const int64_t l1 = std::min<int64_t>(1 + p, z.r);
    st = factor_impl<T>(M, m, n, ldm, 1, p, seed, perm, Q, m, L, l1, V, n, sigma, nullptr, fwork, fbytes,
                        resolve(opts, l1), d, s);
    if (st != FFSRQR_OK) return st;
    FF_HIP(hipMemcpy(&norm2, sigma, sizeof(double), hipMemcpyDeviceToHost));
  }
  ffsrqr_rpca_info inf{};
  inf.norm2 = norm2;
  if (!(norm2 > 0.0) || !(fro > 0.0)) {
    // M = 0: X = E = 0
    FF_HIP(zero_matrix<T>(X, ldx, m, n, s));
    FF_HIP(zero_matrix<T>(E, lde, m, n, s));
    FF_HIP(hipStreamSynchronize(s));
    inf.converged = 1;
    if (info) *info = inf;
    return FFSRQR_OK;
  }
  const double J = std::max(norm2, amax);
  FF_HIP(ialm_init<T>(M, ldm, m, n, 1.0 / J, Y, Ei, s));
  double mu = 1.25 / norm2;
  const double mu_bar = 1e7 * mu, rho = 1.5;
  int64_t sv = std::min<int64_t>(10, z.cap);
  int64_t svp = 0;
  int32_t it = 0;
  double res = HUGE_VAL;
  bool capped = false;
  std::vector<double> hs((size_t)z.lmax);
  while (it < max_iter) {
    ++it;
    FF_HIP(ialm_shift<T>(M, ldm, Ei, Y, m, n, 1.0 / mu, D, s));
    // rank-sv SVD of D: Flip-Flop SRQR, then Algorithm 9's completion
    const int64_t l = std::min(sv + p, z.r);
    st = factor_impl<T>(D, m, n, m, sv, p, seed, perm, Q, m, L, l, V, n, sigma, nullptr, fwork, fbytes,
                        resolve(opts, l), d, s);
    if (st != FFSRQR_OK) return st;
    st = alg9_impl<T>(D, m, n, m, V, n, l, sv, U, m, sigma, Vk, n, fwork, fbytes, d, s);
    if (st != FFSRQR_OK) return st;
    FF_HIP(hipMemcpy(hs.data(), sigma, (size_t)sv * sizeof(double), hipMemcpyDeviceToHost));
    svp = 0;
    for (int64_t j = 0; j < sv; ++j)
      if (hs[(size_t)j] > 1.0 / mu) ++svp;
    // X = U(:, 0:svp) S_{1/mu}(Sigma) V_k(:, 0:svp)^T
    if (svp > 0) {
      FF_HIP(scaled_transpose<T>(U, m, svp, m, sigma, 1.0 / mu, Ut, svp, s));
      FF_HIP(transpose<T>(Vk, n, svp, n, Vt, svp, s));
      Arena a{fwork, fbytes, 0};
      FF_HIP(gemm_tn<T>(m, n, svp, Ut, svp, Vt, svp, X, ldx, nullptr, a, d.num_cu, s));
    } else {
      FF_HIP(zero_matrix<T>(X, ldx, m, n, s));
    }
    // E, Y and the residual
    FF_HIP(ialm_update<T>(M, ldm, X, ldx, m, n, mu, lam / mu, Ei, Y, part, out, s));
    st = read_out();
    if (st != FFSRQR_OK) return st;
    res = std::sqrt(hout[0]) / fro;
    sv = svp < sv ? std::min(svp + 1, z.r) : std::min(svp + (int64_t)std::llround(0.05 * (double)n), z.r);
    if (sv > z.cap) {
      sv = z.cap;
      capped = true;
    }
    if (sv < 1) sv = 1;
    mu = std::min(mu * rho, mu_bar);
    if (res < tol) break;
  }
  FF_HIP(hipMemcpy2DAsync(E, (size_t)lde * sizeof(T), Ei, (size_t)m * sizeof(T), (size_t)m * sizeof(T), (size_t)n,
                          hipMemcpyDeviceToDevice, s));
  FF_HIP(hipStreamSynchronize(s));
  inf.iterations = it;
  inf.rank = (int32_t)svp;
  inf.residual = res;
  inf.mu = mu;
  inf.converged = res < tol ? 1 : 0;
  inf.rank_capped = capped ? 1 : 0;
  if (info) *info = inf;
  return FFSRQR_OK;
}

ffsrqr_status alg9_check(int64_t m, int64_t n, int64_t l, int64_t k, int32_t precision, const DeviceInfo& d) {
  if (m < 1 || n < 1 || l < 1 || l > std::min(m, n) || k < 1 || k > l)
    return fail(FFSRQR_EINVAL, "need 1 <= k <= l <= min(m, n)");
  if (precision != FFSRQR_FP64 && precision != FFSRQR_FP32 && precision != FFSRQR_MIXED)
    return fail(FFSRQR_EINVAL, "unknown precision");
  return check_limits(m, n, l, d);
}

}  // namespace
}  // namespace ffsrqr

using namespace ffsrqr;

extern "C" {

void ffsrqr_default_opts(ffsrqr_opts* o) {
  if (!o) return;
  o->precision = FFSRQR_FP64;
  o->max_swaps = -1;
  o->g = 2.0;
  o->block = 0;
  o->g2_probe = 0;
  o->est_norms = 0;
  o->reserved = 0;
}

const char* ffsrqr_status_string(ffsrqr_status s) {
  switch (s) {
    case FFSRQR_OK: return "ok";
    case FFSRQR_EINVAL: return "invalid argument";
    case FFSRQR_EWORKSPACE: return "workspace too small";
    case FFSRQR_EHIP: return "HIP runtime error";
    case FFSRQR_ENODEV: return "no usable gfx950 device";
    case FFSRQR_EBUSY: return "request ended unrun";
  }
  return "unknown status";
}

const char* ffsrqr_last_error(void) { return g_last_error.c_str(); }

void ffsrqr_release(void) {
  for (int i = 0; i < 64; ++i) {
    SideStream& ss = g_side[i];
    if (!ss.stream) continue;
    (void)hipEventDestroy(ss.fork);
    (void)hipEventDestroy(ss.join);
    (void)hipStreamDestroy(ss.stream);
    ss = SideStream{};
  }
}

void ffsrqr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  for (int i = 0; i < FFSRQR_NUM_STEPS; ++i) {
    g_prof.ms[i] = 0.0;
    g_prof.launches[i] = 0;
  }
}

int ffsrqr_profile_read(double* ms, int64_t* launches, int nsteps) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (int i = 0; i < nsteps && i < FFSRQR_NUM_STEPS; ++i) {
    if (ms) ms[i] = g_prof.ms[i];
    if (launches) launches[i] = g_prof.launches[i];
  }
  return FFSRQR_NUM_STEPS;
}

ffsrqr_status ffsrqr_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, const ffsrqr_opts* opts,
                                    size_t* bytes) {
  if (!bytes) return fail(FFSRQR_EINVAL, "bytes is NULL");
  ffsrqr_status st = check_dims(m, n, k, p);
  if (st != FFSRQR_OK) return st;
  const int32_t prec = opts ? opts->precision : FFSRQR_FP64;
  if (!valid_precision(prec)) return fail(FFSRQR_EINVAL, "unknown precision");
  const int64_t l = std::min(k + p, std::min(m, n));
  st = check_limits(m, n, l, limits_device());
  if (st != FFSRQR_OK) return st;
  const DeviceInfo d = sizing_device();
  const int64_t blk = opts && opts->block > 0 ? std::min<int64_t>(opts->block, k) : 0;
  if (opts && (opts->g2_probe < 0 || opts->g2_probe > kMaxProbe))
    return fail(FFSRQR_EINVAL, "g2_probe must be 0 (exact) or 1..64");
  if (opts && opts->est_norms != 0 && opts->est_norms != 1) return fail(FFSRQR_EINVAL, "est_norms must be 0 or 1");
  if (opts && opts->block != 0) {
    st = check_block(m, n, k, p, l, opts->block);
    if (st != FFSRQR_OK) return st;
  }
  const bool est = opts && opts->est_norms == 1;
  *bytes = prec == FFSRQR_FP64 ? total_bytes<double>(m, n, l, d, blk, p, est)
                               : total_bytes<float>(m, n, l, d, blk, p, est);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_factor(const void* A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p, uint64_t seed,
                            int64_t* perm, void* Q, int64_t ldq, void* L, int64_t ldl, void* V, int64_t ldv,
                            double* sigma, ffsrqr_info* info, void* work, size_t work_bytes,
                            const ffsrqr_opts* opts, ffsrqr_stream_t stream) {
  ffsrqr_status st = check_dims(m, n, k, p);
  if (st != FFSRQR_OK) return st;
  const int64_t l = std::min(k + p, std::min(m, n));
  const ffsrqr_opts op = resolve(opts, l);
  if (!valid_precision(op.precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  if (!(op.g > 1.0)) return fail(FFSRQR_EINVAL, "g must be > 1");
  if (lda < m || ldq < m || ldl < l || ldv < n) return fail(FFSRQR_EINVAL, "leading dimension too small");
  if (!A || !perm || !Q || !L || !V || !sigma || !work) return fail(FFSRQR_EINVAL, "NULL pointer argument");
  st = check_block(m, n, k, p, l, op.block);
  if (st != FFSRQR_OK) return st;
  const DeviceInfo* d = nullptr;
  st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  st = check_limits(m, n, l, *d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (op.precision == FFSRQR_MIXED && ((uintptr_t)A & 3) != 0) return fail(FFSRQR_EINVAL, "A must be 4-byte aligned");
  if (op.precision == FFSRQR_FP64)
    return factor_impl<double>((const double*)A, m, n, lda, k, p, seed, perm, (double*)Q, ldq, (double*)L, ldl,
                               (double*)V, ldv, sigma, info, work, work_bytes, op, *d, s);
  return factor_impl<float>((const float*)A, m, n, lda, k, p, seed, perm, (float*)Q, ldq, (float*)L, ldl,
                            (float*)V, ldv, sigma, info, work, work_bytes, op, *d, s);
}

ffsrqr_status ffsrqr_omega(uint64_t seed, int64_t l, int64_t m, void* omega_t, int64_t ldo, int32_t precision,
                           ffsrqr_stream_t stream) {
  if (l < 1 || m < 1 || ldo < m || !omega_t) return fail(FFSRQR_EINVAL, "bad omega arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (precision == FFSRQR_FP64) FF_HIP(launch_omega<double>(seed, l, m, (double*)omega_t, ldo, s));
  else FF_HIP(launch_omega<float>(seed, l, m, (float*)omega_t, ldo, s));
  return FFSRQR_OK;
}


ffsrqr_status ffsrqr_sketch(const void* A, int64_t m, int64_t n, int64_t lda, uint64_t seed, int64_t l, void* B,
                            int64_t ldb, double* anorm2, void* work, size_t work_bytes, int32_t precision,
                            ffsrqr_stream_t stream) {
  if (m < 1 || n < 1 || l < 1 || lda < m || ldb < l || !A || !B || !anorm2 || !work)
    return fail(FFSRQR_EINVAL, "bad sketch arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (precision == FFSRQR_MIXED)
    return sketch_mixed((const float*)A, m, n, lda, seed, l, (float*)B, ldb, anorm2, work, work_bytes, *d, s);
  if (precision == FFSRQR_FP64)
    return sketch_impl<double>((const double*)A, m, n, lda, seed, l, (double*)B, ldb, anorm2, work, work_bytes, *d, s);
  return sketch_impl<float>((const float*)A, m, n, lda, seed, l, (float*)B, ldb, anorm2, work, work_bytes, *d, s);
}

ffsrqr_status ffsrqr_qrcp(const void* B, int64_t l, int64_t n, int64_t ldb, int64_t* piv, double* margins, void* work,
                          size_t work_bytes, int32_t precision, ffsrqr_stream_t stream) {
  if (l < 1 || n < l || ldb < l || !B || !piv || !margins || !work) return fail(FFSRQR_EINVAL, "bad qrcp arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  unsigned* err = ar.take<unsigned>(64);
  if (!err) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(zero_words(err, 64, s));
  hipError_t e = precision == FFSRQR_FP64
                     ? qrcp<double>((const double*)B, l, n, ldb, piv, margins, ar, err, *d, s)
                     : qrcp<float>((const float*)B, l, n, ldb, piv, margins, ar, err, *d, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_panel_qr(const void* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols, int64_t c,
                              void* Q, int64_t ldq, void* R, int64_t ldr, void* work, size_t work_bytes,
                              int32_t precision, ffsrqr_stream_t stream) {
  if (m < 1 || n < 1 || c < 1 || c > m || lda < m || ldq < m || ldr < c || !A || !cols || !Q || !R || !work)
    return fail(FFSRQR_EINVAL, "bad panel_qr arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  unsigned* err = ar.take<unsigned>(64);
  const size_t es = elem_size(precision);
  char* P = ar.take<char>((size_t)m * c * es);
  if (!err || !P) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(zero_words(err, 64, s));
  hipError_t e;
  if (precision == FFSRQR_FP64) {
    FF_HIP(gather_cols<double>((const double*)A, m, n, lda, cols, c, (double*)P, m, s));
    e = tall_qr<double>((double*)P, m, c, m, (double*)Q, ldq, (double*)R, ldr, false, ar, err, *d, s);
  } else {
    FF_HIP(gather_cols<float>((const float*)A, m, n, lda, cols, c, (float*)P, m, s));
    e = tall_qr<float>((float*)P, m, c, m, (float*)Q, ldq, (float*)R, ldr, false, ar, err, *d, s);
  }
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_project(const void* Q, int64_t m, int64_t c, int64_t ldq, const void* A, int64_t n, int64_t lda,
                             void* W, int64_t ldw, const double* anorm2, double* gamma2, void* work,
                             size_t work_bytes, int32_t precision, ffsrqr_stream_t stream) {
  if (m < 1 || n < 1 || c < 1 || ldq < m || lda < m || ldw < c || !Q || !A || !W || !anorm2 || !gamma2 || !work)
    return fail(FFSRQR_EINVAL, "bad project arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  hipError_t e;
  if (precision == FFSRQR_MIXED) {
    const int64_t mp = bf16_ld(m);
    __bf16* qh = ar.take<__bf16>((size_t)mp * c);
    __bf16* ql = ar.take<__bf16>((size_t)mp * c);
    if (!qh || !ql) return fail(FFSRQR_EWORKSPACE, "workspace too small");
    e = split_bf16((const float*)Q, m, c, ldq, qh, ql, mp, s);
    if (e == hipSuccess)
      e = gemm_bf16(3, c, n, m, qh, ql, mp, (const float*)A, lda, (float*)W, ldw, nullptr, ar, d->num_cu, s);
    if (e == hipSuccess) e = residual_norms<float>((const float*)W, c, n, ldw, anorm2, gamma2, s);
  } else if (precision == FFSRQR_FP64) {
    e = gemm_tn<double>(c, n, m, (const double*)Q, ldq, (const double*)A, lda, (double*)W, ldw, nullptr, ar,
                        d->num_cu, s);
    if (e == hipSuccess) e = residual_norms<double>((const double*)W, c, n, ldw, anorm2, gamma2, s);
  } else {
    e = gemm_tn<float>(c, n, m, (const float*)Q, ldq, (const float*)A, lda, (float*)W, ldw, nullptr, ar,
                       d->num_cu, s);
    if (e == hipSuccess) e = residual_norms<float>((const float*)W, c, n, ldw, anorm2, gamma2, s);
  }
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_srqr_rho(const void* R11, int64_t l, int64_t ldr, const void* a, double alpha, double* rho,
                              void* work, size_t work_bytes, int32_t precision, ffsrqr_stream_t stream) {
  if (l < 1 || ldr < l || !R11 || !a || !rho || !work || !(alpha > 0.0))
    return fail(FFSRQR_EINVAL, "bad srqr_rho arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  hipError_t e = precision == FFSRQR_FP64
                     ? srqr_rho<double>((const double*)R11, ldr, (const double*)a, 0, nullptr, alpha, l, rho, nullptr,
                                        ar, s)
                     : srqr_rho<float>((const float*)R11, ldr, (const float*)a, 0, nullptr, alpha, l, rho, nullptr,
                                       ar, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_srqr_probe(const void* R11, int64_t l, int64_t ldr, const void* a, double alpha, int32_t d,
                                uint64_t seed, uint64_t q, double* est, void* work, size_t work_bytes,
                                int32_t precision, ffsrqr_stream_t stream) {
  if (l < 1 || ldr < l || !R11 || !a || !est || !work || !(alpha > 0.0) || d < 1 || d > kMaxProbe || q < 1)
    return fail(FFSRQR_EINVAL, "bad srqr_probe arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* dev = nullptr;
  ffsrqr_status st = get_device(&dev);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  hipError_t e = precision == FFSRQR_FP64
                     ? srqr_probe<double>((const double*)R11, ldr, (const double*)a, 0, nullptr, alpha, l, d, seed, q,
                                          est, nullptr, ar, s)
                     : srqr_probe<float>((const float*)R11, ldr, (const float*)a, 0, nullptr, alpha, l, d, seed, q,
                                         est, nullptr, ar, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_lq(const void* R, int64_t l, int64_t n, int64_t ldr, const int64_t* perm, void* L, int64_t ldl,
                        void* V, int64_t ldv, void* work, size_t work_bytes, int32_t precision,
                        ffsrqr_stream_t stream) {
  if (l < 1 || n < l || ldr < l || ldl < l || ldv < n || !R || !perm || !L || !V || !work)
    return fail(FFSRQR_EINVAL, "bad lq arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  unsigned* err = ar.take<unsigned>(64);
  const size_t es = elem_size(precision);
  char* Rt = ar.take<char>((size_t)n * l * es);
  char* Qh = ar.take<char>((size_t)n * l * es);
  if (!err || !Rt || !Qh) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(zero_words(err, 64, s));
  hipError_t e;
  if (precision == FFSRQR_FP64) {
    FF_HIP(assemble_rt<double>((const double*)R, ldr, (const double*)R, ldr, nullptr, l, n, (double*)Rt, n, s));
    e = tall_qr<double>((double*)Rt, n, l, n, (double*)Qh, n, (double*)L, ldl, true, ar, err, *d, s);
    if (e == hipSuccess) e = scatter_rows<double>((const double*)Qh, n, l, n, perm, (double*)V, ldv, s);
  } else {
    FF_HIP(assemble_rt<float>((const float*)R, ldr, (const float*)R, ldr, nullptr, l, n, (float*)Rt, n, s));
    e = tall_qr<float>((float*)Rt, n, l, n, (float*)Qh, n, (float*)L, ldl, true, ar, err, *d, s);
    if (e == hipSuccess) e = scatter_rows<float>((const float*)Qh, n, l, n, perm, (float*)V, ldv, s);
  }
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_svd_small(const void* L, int64_t l, int64_t ldl, double* sigma, void* work, size_t work_bytes,
                               int32_t precision, ffsrqr_stream_t stream) {
  if (l < 1 || ldl < l || !L || !sigma || !work) return fail(FFSRQR_EINVAL, "bad svd_small arguments");
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{(char*)work, work_bytes, 0};
  unsigned* err = ar.take<unsigned>(64);
  if (!err) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(zero_words(err, 64, s));
  hipError_t e = precision == FFSRQR_FP64
                     ? jacobi_sigma<double>((const double*)L, l, ldl, sigma, ar, err, *d, s)
                     : jacobi_sigma<float>((const float*)L, l, ldl, sigma, ar, err, *d, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "workspace too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_alg9_workspace_size(int64_t m, int64_t n, int64_t l, int64_t k, int32_t precision,
                                         size_t* bytes) {
  if (!bytes) return fail(FFSRQR_EINVAL, "bytes is NULL");
  ffsrqr_status st = alg9_check(m, n, l, k, precision, limits_device());
  if (st != FFSRQR_OK) return st;
  const DeviceInfo d = sizing_device();
  *bytes = precision == FFSRQR_FP64 ? alg9_bytes<double>(m, n, l, k, d) : alg9_bytes<float>(m, n, l, k, d);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_alg9_svd(const void* A, int64_t m, int64_t n, int64_t lda, const void* V, int64_t ldv, int64_t l,
                              int64_t k, void* U, int64_t ldu, double* sigma, void* Vk, int64_t ldvk, void* work,
                              size_t work_bytes, int32_t precision, ffsrqr_stream_t stream) {
  const DeviceInfo lim = limits_device();
  ffsrqr_status st = alg9_check(m, n, l, k, precision, lim);
  if (st != FFSRQR_OK) return st;
  if (lda < m || ldv < n || ldu < m || ldvk < n) return fail(FFSRQR_EINVAL, "leading dimension too small");
  if (!A || !V || !U || !sigma || !Vk || !work) return fail(FFSRQR_EINVAL, "NULL pointer argument");
  const DeviceInfo* d = nullptr;
  st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  st = check_limits(m, n, l, *d);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (precision == FFSRQR_FP64)
    return alg9_impl<double>((const double*)A, m, n, lda, (const double*)V, ldv, l, k, (double*)U, ldu, sigma,
                             (double*)Vk, ldvk, work, work_bytes, *d, s);
  return alg9_impl<float>((const float*)A, m, n, lda, (const float*)V, ldv, l, k, (float*)U, ldu, sigma,
                          (float*)Vk, ldvk, work, work_bytes, *d, s);
}

ffsrqr_status ffsrqr_st_hosvd_workspace_size(int32_t d, const int64_t* dims, const int64_t* ranks,
                                             const int32_t* order, int64_t p, const ffsrqr_opts* opts,
                                             size_t* bytes) {
  if (!bytes) return fail(FFSRQR_EINVAL, "bytes is NULL");
  const int32_t prec = opts ? opts->precision : FFSRQR_FP64;
  if (!valid_precision(prec)) return fail(FFSRQR_EINVAL, "unknown precision");
  ffsrqr_status st = check_driver_opts(opts);
  if (st != FFSRQR_OK) return st;
  HosvdPlan pl;
  st = hosvd_plan(d, dims, ranks, order, p, limits_device(), &pl);
  if (st != FFSRQR_OK) return st;
  const DeviceInfo dv = sizing_device();
  *bytes = prec == FFSRQR_FP64 ? hosvd_bytes<double>(pl, dv) : hosvd_bytes<float>(pl, dv);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_st_hosvd(const void* X, int32_t d, const int64_t* dims, const int64_t* ranks,
                              const int32_t* order, int64_t p, uint64_t seed, void* core, void* const* U,
                              const int64_t* ldu, void* work, size_t work_bytes, const ffsrqr_opts* opts,
                              ffsrqr_stream_t stream) {
  const int32_t prec = opts ? opts->precision : FFSRQR_FP64;
  if (!valid_precision(prec)) return fail(FFSRQR_EINVAL, "unknown precision");
  if (opts && !(opts->g == 0.0 || opts->g > 1.0)) return fail(FFSRQR_EINVAL, "g must be > 1");
  if (!X || !core || !U || !ldu || !work) return fail(FFSRQR_EINVAL, "NULL pointer argument");
  ffsrqr_status st = check_driver_opts(opts);
  if (st != FFSRQR_OK) return st;
  const DeviceInfo* dv = nullptr;
  st = get_device(&dv);
  if (st != FFSRQR_OK) return st;
  HosvdPlan pl;
  st = hosvd_plan(d, dims, ranks, order, p, *dv, &pl);
  if (st != FFSRQR_OK) return st;
  for (int j = 0; j < d; ++j)
    if (!U[j] || ldu[j] < dims[j]) return fail(FFSRQR_EINVAL, "U[j] NULL or ldu[j] < dims[j]");
  if (prec == FFSRQR_MIXED && ((uintptr_t)X & 3) != 0) return fail(FFSRQR_EINVAL, "X must be 4-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (prec == FFSRQR_FP64)
    return hosvd_impl<double>((const double*)X, pl, p, seed, (double*)core, (double* const*)U, ldu, work, work_bytes,
                              opts, *dv, s);
  return hosvd_impl<float>((const float*)X, pl, p, seed, (float*)core, (float* const*)U, ldu, work, work_bytes, opts,
                           *dv, s);
}

ffsrqr_status ffsrqr_batched_workspace_size(int32_t count, const ffsrqr_problem* probs, const ffsrqr_opts* opts,
                                            size_t* bytes) {
  if (!bytes || !probs || count < 1) return fail(FFSRQR_EINVAL, "need count >= 1, probs and bytes");
  size_t best = 0;
  for (int32_t i = 0; i < count; ++i) {
    size_t b = 0;
    const ffsrqr_problem& q = probs[i];
    ffsrqr_status st = ffsrqr_workspace_size(q.m, q.n, q.k, q.p, opts, &b);
    if (st != FFSRQR_OK) return fail(st, "problem " + std::to_string(i) + ": " + ffsrqr_last_error());
    best = std::max(best, b);
  }
  *bytes = best;
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_factor_batched(int32_t count, const ffsrqr_problem* probs, void* work, size_t work_bytes,
                                    const ffsrqr_opts* opts, ffsrqr_stream_t stream) {
  if (!probs || count < 1) return fail(FFSRQR_EINVAL, "need count >= 1 and probs");
  if (!work) return fail(FFSRQR_EINVAL, "NULL pointer argument");
  // every problem is checked before any work is enqueued
  for (int32_t i = 0; i < count; ++i) {
    const ffsrqr_problem& q = probs[i];
    ffsrqr_status st = check_dims(q.m, q.n, q.k, q.p);
    if (st != FFSRQR_OK) return fail(st, "problem " + std::to_string(i) + ": " + ffsrqr_last_error());
    const int64_t l = std::min(q.k + q.p, std::min(q.m, q.n));
    if (q.lda < q.m || q.ldq < q.m || q.ldl < l || q.ldv < q.n)
      return fail(FFSRQR_EINVAL, "problem " + std::to_string(i) + ": leading dimension too small");
    if (!q.A || !q.perm || !q.Q || !q.L || !q.V || !q.sigma)
      return fail(FFSRQR_EINVAL, "problem " + std::to_string(i) + ": NULL pointer argument");
    size_t b = 0;
    st = ffsrqr_workspace_size(q.m, q.n, q.k, q.p, opts, &b);
    if (st != FFSRQR_OK) return fail(st, "problem " + std::to_string(i) + ": " + ffsrqr_last_error());
    if (b > work_bytes) return fail(FFSRQR_EWORKSPACE, "problem " + std::to_string(i) + ": workspace too small");
  }
  for (int32_t i = 0; i < count; ++i) {
    const ffsrqr_problem& q = probs[i];
    ffsrqr_status st = ffsrqr_factor(q.A, q.m, q.n, q.lda, q.k, q.p, q.seed, q.perm, q.Q, q.ldq, q.L, q.ldl, q.V,
                                     q.ldv, q.sigma, q.info, work, work_bytes, opts, stream);
    if (st != FFSRQR_OK) return fail(st, "problem " + std::to_string(i) + ": " + ffsrqr_last_error());
  }
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_rpca_workspace_size(int64_t m, int64_t n, int64_t p, int64_t max_rank,
                                         const ffsrqr_opts* opts, size_t* bytes) {
  if (!bytes) return fail(FFSRQR_EINVAL, "bytes is NULL");
  const int32_t prec = opts ? opts->precision : FFSRQR_FP64;
  if (!valid_precision(prec)) return fail(FFSRQR_EINVAL, "unknown precision");
  if (m < 1 || n < 1 || p < 0 || p > 1023) return fail(FFSRQR_EINVAL, "need m, n >= 1 and 0 <= p <= 1023");
  const RpcaSizes z = rpca_sizes(m, n, p, max_rank);
  ffsrqr_status st = check_dims(m, n, 1, p);
  if (st != FFSRQR_OK) return st;
  st = check_driver_opts(opts);
  if (st != FFSRQR_OK) return st;
  st = check_limits(m, n, z.lmax, limits_device());
  if (st != FFSRQR_OK) return st;
  const DeviceInfo dv = sizing_device();
  *bytes = prec == FFSRQR_FP64 ? rpca_bytes<double>(m, n, z, dv) : rpca_bytes<float>(m, n, z, dv);
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_rpca_ialm(const void* M, int64_t m, int64_t n, int64_t ldm, double lambda, double tol,
                               int32_t max_iter, int64_t p, uint64_t seed, int64_t max_rank, void* X, int64_t ldx,
                               void* E, int64_t lde, ffsrqr_rpca_info* info, void* work, size_t work_bytes,
                               const ffsrqr_opts* opts, ffsrqr_stream_t stream) {
  const int32_t prec = opts ? opts->precision : FFSRQR_FP64;
  if (!valid_precision(prec)) return fail(FFSRQR_EINVAL, "unknown precision");
  if (opts && !(opts->g == 0.0 || opts->g > 1.0)) return fail(FFSRQR_EINVAL, "g must be > 1");
  if (m < 1 || n < 1 || p < 0 || p > 1023) return fail(FFSRQR_EINVAL, "need m, n >= 1 and 0 <= p <= 1023");
  if (ldm < m || ldx < m || lde < m) return fail(FFSRQR_EINVAL, "leading dimension too small");
  if (!M || !X || !E || !work) return fail(FFSRQR_EINVAL, "NULL pointer argument");
  if (!(tol > 0.0) || max_iter < 1) return fail(FFSRQR_EINVAL, "need tol > 0 and max_iter >= 1");
  const double lam = lambda > 0.0 ? lambda : 1.0 / std::sqrt((double)std::max(m, n));
  const RpcaSizes z = rpca_sizes(m, n, p, max_rank);
  ffsrqr_status st = check_dims(m, n, 1, p);
  if (st != FFSRQR_OK) return st;
  st = check_driver_opts(opts);
  if (st != FFSRQR_OK) return st;
  const DeviceInfo* dv = nullptr;
  st = get_device(&dv);
  if (st != FFSRQR_OK) return st;
  st = check_limits(m, n, z.lmax, *dv);
  if (st != FFSRQR_OK) return st;
  if (prec == FFSRQR_MIXED && ((uintptr_t)M & 3) != 0) return fail(FFSRQR_EINVAL, "M must be 4-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (prec == FFSRQR_FP64)
    return rpca_impl<double>((const double*)M, m, n, ldm, lam, tol, max_iter, p, seed, z, (double*)X, ldx,
                             (double*)E, lde, info, work, work_bytes, opts, *dv, s);
  return rpca_impl<float>((const float*)M, m, n, ldm, lam, tol, max_iter, p, seed, z, (float*)X, ldx, (float*)E, lde,
                          info, work, work_bytes, opts, *dv, s);
}

ffsrqr_status ffsrqr_svd_small_noalloc(const void* L, int64_t l, int64_t ldl, double* sigma, int32_t precision,
                                       ffsrqr_stream_t stream) {
  if (l < 1 || ldl < l || !L || !sigma) return fail(FFSRQR_EINVAL, "bad svd_small_noalloc arguments");
  if (l > kNoAllocMaxL)
    return fail(FFSRQR_EINVAL, "svd_small_noalloc supports l <= " + std::to_string(kNoAllocMaxL));
  if (!valid_precision(precision)) return fail(FFSRQR_EINVAL, "unknown precision");
  const DeviceInfo* d = nullptr;
  ffsrqr_status st = get_device(&d);
  if (st != FFSRQR_OK) return st;
  void* base = nullptr;
  st = scratch_for(d->id, &base);
  if (st != FFSRQR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the same carving and kernels as ffsrqr_svd_small, over the static scratch
  Arena ar{(char*)base, kNoAllocBytes, 0};
  unsigned* err = ar.take<unsigned>(64);
  if (!err) return fail(FFSRQR_EWORKSPACE, "static scratch too small");
  FF_HIP(zero_words(err, 64, s));
  hipError_t e = precision == FFSRQR_FP64
                     ? jacobi_sigma<double>((const double*)L, l, ldl, sigma, ar, err, *d, s)
                     : jacobi_sigma<float>((const float*)L, l, ldl, sigma, ar, err, *d, s);
  if (e == hipErrorOutOfMemory) return fail(FFSRQR_EWORKSPACE, "static scratch too small");
  FF_HIP(e);
  return FFSRQR_OK;
}

}  // extern "C"
