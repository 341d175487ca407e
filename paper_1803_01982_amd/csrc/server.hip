// A serving loop over the path: requests (one ffsrqr_problem each, A and
// the outputs device-resident and owned by the caller) are queued and
// admitted in arrival order as soon as a worker slot is free and the
// request's workspace fits the server's device pool; each admitted request
// runs the whole path on its worker's stream with a workspace carved from
// the pool, and the pool space returns when it completes.  Requests that
// arrive while others run are admitted as slots and memory free up
// (continuous batching); on the device their kernels overlap except the
// cooperative ones, which the runtime serialises.
//
// Host side only: a fixed set of worker threads (one stream each, default
// priority), a first-fit allocator over one device allocation made at
// creation, and a ticket table for polling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ffsrqr.h"

namespace {

constexpr size_t kAlign = 256;

// First-fit allocator of [0, size) in kAlign units, with coalescing.
class Pool {
 public:
  explicit Pool(size_t size) { free_[0] = size; }
  bool take(size_t bytes, size_t* off) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
  uint64_t ticket;
  ffsrqr_problem prob;
  size_t bytes;
};

struct Result {
  bool done = false;
  ffsrqr_status status = FFSRQR_OK;
  ffsrqr_info info{};
  std::string error;
};

}  // namespace

struct ffsrqr_server {
  int device = 0;
  ffsrqr_opts opts{};
  size_t budget = 0;
  char* base = nullptr;
  Pool* pool = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::map<uint64_t, Result> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;

  void work() {
    hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (;;) {
      Request r;
      size_t off = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        // arrival order: the oldest request runs as soon as it fits
        cv.wait(lk, [&] { return stop || (!pending.empty() && pool->take(pending.front().bytes, &off)); });
        if (stop && pending.empty()) break;
        if (stop) {
          // shutting down: the queued requests end without running
          Result& res = results[pending.front().ticket];
          res.done = true;
          res.status = FFSRQR_EBUSY;
          res.error = "server destroyed before the request ran";
          pending.pop_front();
          cv.notify_all();
          continue;
        }
        r = pending.front();
        pending.pop_front();
      }
      ffsrqr_info info{};
      const ffsrqr_problem& q = r.prob;
      const ffsrqr_status st =
          ffsrqr_factor(q.A, q.m, q.n, q.lda, q.k, q.p, q.seed, q.perm, q.Q, q.ldq, q.L, q.ldl, q.V, q.ldv, q.sigma,
                        &info, base + off, r.bytes, &opts, (ffsrqr_stream_t)s);
      const std::string err = st == FFSRQR_OK ? std::string() : std::string(ffsrqr_last_error());
      {
        std::lock_guard<std::mutex> lk(mu);
        pool->give(off, r.bytes);
        Result& res = results[r.ticket];
        res.done = true;
        res.status = st;
        res.info = info;
        res.error = err;
      }
      cv.notify_all();
    }
    ffsrqr_release();
    if (s) hipStreamDestroy(s);
  }
};

extern "C" {

ffsrqr_server* ffsrqr_server_create(const ffsrqr_server_cfg* cfg) {
  if (!cfg || cfg->hbm_budget < (1u << 20) || cfg->slots < 1 || cfg->slots > 16) return nullptr;
  if (cfg->precision != FFSRQR_FP64 && cfg->precision != FFSRQR_FP32 && cfg->precision != FFSRQR_MIXED) return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  void* base = nullptr;
  if (hipMalloc(&base, cfg->hbm_budget) != hipSuccess) return nullptr;
  ffsrqr_server* sv = new ffsrqr_server;
  sv->device = dev;
  ffsrqr_default_opts(&sv->opts);
  sv->opts.precision = cfg->precision;
  sv->budget = cfg->hbm_budget;
  sv->base = (char*)base;
  sv->pool = new Pool(cfg->hbm_budget);
  for (int i = 0; i < cfg->slots; ++i) sv->workers.emplace_back([sv] { sv->work(); });
  return sv;
}

ffsrqr_status ffsrqr_submit(ffsrqr_server* sv, const ffsrqr_problem* prob, uint64_t* ticket) {
  if (!sv || !prob || !ticket) return FFSRQR_EINVAL;
  size_t bytes = 0;
  ffsrqr_status st = ffsrqr_workspace_size(prob->m, prob->n, prob->k, prob->p, &sv->opts, &bytes);
  if (st != FFSRQR_OK) return st;
  if (bytes > sv->budget) return FFSRQR_EWORKSPACE;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return FFSRQR_EBUSY;
    *ticket = sv->next_ticket++;
    sv->results[*ticket] = Result{};
    sv->pending.push_back(Request{*ticket, *prob, bytes});
  }
  sv->cv.notify_all();
  return FFSRQR_OK;
}

ffsrqr_status ffsrqr_poll(ffsrqr_server* sv, uint64_t ticket, ffsrqr_info* out, int32_t* done) {
  if (!sv || !done) return FFSRQR_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) return FFSRQR_EINVAL;
  *done = it->second.done ? 1 : 0;
  if (!it->second.done) return FFSRQR_OK;
  if (out) *out = it->second.info;
  const ffsrqr_status st = it->second.status;
  sv->results.erase(it);
  return st;
}

void ffsrqr_server_destroy(ffsrqr_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  for (auto& t : sv->workers) t.join();
  hipFree(sv->base);
  delete sv->pool;
  delete sv;
}

}  // extern "C"
