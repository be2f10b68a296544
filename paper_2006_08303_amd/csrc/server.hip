// Request server: continuous batching of independent reconstructions on one
// GPU, built on the public plan API of this library.
//
// * Memory: one device arena of hbm_budget_bytes is allocated when the server
//   is created; operators (plans: tables resident for the server's lifetime)
//   and in-flight requests (solve state + measurements + result) are carved
//   from it by a first-fit allocator with coalescing, so admission is decided
//   by HBM footprint and the hot loop never calls the device allocator.
// * Concurrency: n_slots worker threads, each owning one HIP stream (default
//   priority). A worker admits the oldest queued request whose footprint fits
//   in the free memory (a request may be overtaken by smaller ones at most
//   MAX_BYPASS times, after which only it can be admitted), attaches a solve
//   state to the operator's shared tables (cip_plan_attach), copies y in,
//   runs cip_solve, copies x out and frees the memory. Requests that arrive
//   while others run are admitted as soon as a slot and memory are free; their
//   kernels overlap on the device.
// * Latency of a request = completion time - submit time (host steady clock).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cip.h"
#include "errors.hpp"

using cip::fail;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t ALIGN = 256;
constexpr int MAX_BYPASS = 16;
constexpr int MAX_SLOTS = 16;

size_t round_up(size_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over [0, capacity) with coalescing of free blocks.
class Arena {
 public:
  explicit Arena(size_t capacity) : capacity_(capacity) {
    if (capacity) free_[0] = capacity;
  }
  // Offset of a block of `bytes` (rounded up to ALIGN), or SIZE_MAX.
  size_t alloc(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
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
  size_t capacity() const { return capacity_; }

 private:
  size_t capacity_;
  std::map<size_t, size_t> free_;
};

struct Operator {
  cip_plan_t plan = nullptr;
  int K = 0, S = 0, N1 = 0, N2 = 0;
  size_t ws_off = 0, ws_bytes = 0, state_bytes = 0;
};

struct Request {
  int op = 0, iters = 0;
  const float* y = nullptr;
  float* x = nullptr;
  size_t bytes = 0;          // footprint: state + y + x
  int bypassed = 0;
  int status = 1;            // 1 queued, 2 running, 0 done, < 0 failed
  std::string error;
  Clock::time_point submit, start, end;
};

}  // namespace

struct cip_server_s {
  int device = 0;
  bool autotune = false;
  void* base = nullptr;
  std::unique_ptr<Arena> arena;
  size_t reserved_ops = 0;   // bytes held by operators
  std::deque<Operator> ops;   // stable element addresses while workers read them
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable work_cv;   // queue changed or memory freed
  std::condition_variable done_cv;   // a request finished
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  hipStream_t op_stream = nullptr;   // operator registration (plan build, autotuning)
  std::mutex op_mu;                  // one registration at a time

  // Pick and reserve memory for the next admissible request (lock held).
  bool pick(uint64_t* ticket, size_t* off) {
    for (size_t i = 0; i < queue.size(); ++i) {
      Request& r = reqs[queue[i]];
      const size_t o = arena->alloc(r.bytes);
      if (o != SIZE_MAX) {
        if (i > 0) reqs[queue[0]].bypassed++;
        *ticket = queue[i];
        *off = o;
        queue.erase(queue.begin() + (long)i);
        return true;
      }
      if (i == 0 && r.bypassed >= MAX_BYPASS) return false;   // the head waits for memory
    }
    return false;
  }

  // `op` is a copy taken under the lock (ops may grow meanwhile).
  int run(const Request& r, const Operator& op, size_t off, hipStream_t st) {
    unsigned char* mem = static_cast<unsigned char*>(base) + off;
    float* dy = reinterpret_cast<float*>(mem + round_up(op.state_bytes));
    const size_t ybytes = (size_t)op.K * op.N1 * op.N2 * 4;
    float* dx = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(dy) + round_up(ybytes));
    const size_t xbytes = (size_t)op.S * op.N1 * op.N2 * 4;
    cip_plan_t pl = nullptr;
    int rc = cip_plan_attach(op.plan, mem, op.state_bytes, &pl);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(dy, r.y, ybytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      rc = cip_solve(pl, dy, r.iters, dx, st);
      if (!rc) e = hipMemcpyAsync(r.x, dx, xbytes, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cip_plan_destroy(pl);
    if (e != hipSuccess) return fail(CIP_EHIP, std::string("request: ") + hipGetErrorString(e));
    return rc;
  }

  void worker(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[slot];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      uint64_t t = 0;
      size_t off = 0;
      work_cv.wait(lk, [&] { return pick(&t, &off) || (stop && queue.empty()); });
      if (t == 0) break;
      Request& r = reqs[t];
      r.status = 2;
      r.start = Clock::now();
      const Operator op = ops[r.op];
      lk.unlock();
      const int rc = run(r, op, off, st);
      const std::string msg = rc ? cip::g_last_error : std::string();
      lk.lock();
      arena->release(off, r.bytes);
      r.end = Clock::now();
      r.status = rc ? rc : 0;
      r.error = msg;
      work_cv.notify_all();
      done_cv.notify_all();
    }
  }
};

extern "C" {

int cip_server_create(const cip_server_config* cfg, cip_server_t* out) {
  if (!cfg || !out) return fail(CIP_EINVAL, "NULL argument");
  if (cfg->n_slots < 1 || cfg->n_slots > MAX_SLOTS)
    return fail(CIP_EINVAL, "n_slots must be in [1, 16]");
  if (cfg->hbm_budget_bytes < (1u << 20)) return fail(CIP_EINVAL, "budget below 1 MiB");
  auto s = std::make_unique<cip_server_s>();
  if (hipGetDevice(&s->device) != hipSuccess) return fail(CIP_EHIP, "hipGetDevice failed");
  const size_t cap = cfg->hbm_budget_bytes & ~(ALIGN - 1);
  if (hipMalloc(&s->base, cap) != hipSuccess)
    return fail(CIP_EHIP, "hipMalloc of the server arena failed");
  s->arena = std::make_unique<Arena>(cap);
  s->autotune = cfg->autotune != 0;
  for (int i = 0; i < cfg->n_slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto q : s->streams) (void)hipStreamDestroy(q);
      (void)hipFree(s->base);
      return fail(CIP_EHIP, "hipStreamCreate failed");
    }
    s->streams.push_back(st);
  }
  if (hipStreamCreateWithFlags(&s->op_stream, hipStreamNonBlocking) != hipSuccess) {
    for (auto q : s->streams) (void)hipStreamDestroy(q);
    (void)hipFree(s->base);
    return fail(CIP_EHIP, "hipStreamCreate failed");
  }
  cip_server_s* raw = s.get();
  for (int i = 0; i < cfg->n_slots; ++i) raw->workers.emplace_back([raw, i] { raw->worker(i); });
  *out = s.release();
  return CIP_OK;
}

int cip_server_add_operator(cip_server_t s, int K, int S, int N1, int N2, const float* d_psf,
                            const cip_prior_desc* prior, double rho, double lambda, int* op_id) {
  if (!s || !op_id) return fail(CIP_EINVAL, "NULL argument");
  size_t ws = 0;
  int rc = cip_plan_workspace_bytes(K, S, N1, N2, prior, &ws);
  if (rc) return rc;
  std::lock_guard<std::mutex> reg(s->op_mu);
  auto release = [&](size_t off, size_t bytes, bool op_bytes) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->arena->release(off, bytes);
    if (op_bytes) s->reserved_ops -= round_up(bytes);
    s->work_cv.notify_all();   // a queued request may fit now
  };
  size_t off;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    off = s->arena->alloc(ws);
    if (off == SIZE_MAX) return fail(CIP_ENOSPC, "operator does not fit in the server budget");
    s->reserved_ops += round_up(ws);
  }
  // plan build and autotuning on the registration stream, without the lock
  hipStream_t st = s->op_stream;
  cip_plan_t plan = nullptr;
  rc = cip_plan_create(K, S, N1, N2, d_psf, prior, rho, lambda,
                       static_cast<unsigned char*>(s->base) + off, ws, st, &plan);
  if (rc) {
    release(off, ws, true);
    return rc;
  }
  if (s->autotune && prior->kind != CIP_PRIOR_PATCH && prior->kind != CIP_PRIOR_CONV2D) {
    // one short solve on zero measurements (the tuner times the row pass on
    // the plan's own buffers), with y and x carved from the arena meanwhile
    const size_t yb = round_up((size_t)K * N1 * N2 * 4), xb = (size_t)S * N1 * N2 * 4;
    size_t toff;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      toff = s->arena->alloc(yb + xb);
    }
    if (toff != SIZE_MAX) {
      unsigned char* t = static_cast<unsigned char*>(s->base) + toff;
      int trc = hipMemsetAsync(t, 0, yb, st) == hipSuccess ? CIP_OK : CIP_EHIP;
      if (!trc) trc = cip_solve(plan, reinterpret_cast<float*>(t), 2,
                                reinterpret_cast<float*>(t + yb), st);
      if (!trc) {
        trc = cip_plan_autotune(plan, 10, st, nullptr);
        if (trc == CIP_EUNSUPPORTED) trc = CIP_OK;   // this prior has one row-pass shape
      }
      if (!trc && hipStreamSynchronize(st) != hipSuccess) trc = CIP_EHIP;
      release(toff, yb + xb, false);
      if (trc) {
        const std::string msg = cip::g_last_error;
        cip_plan_destroy(plan);
        release(off, ws, true);
        return fail(trc, "operator autotuning failed: " + msg);
      }
    }
  }
  Operator op;
  op.plan = plan;
  op.K = K;
  op.S = S;
  op.N1 = N1;
  op.N2 = N2;
  op.ws_off = off;
  op.ws_bytes = ws;
  cip_plan_state_bytes(plan, &op.state_bytes);
  std::lock_guard<std::mutex> lk(s->mu);
  s->ops.push_back(op);
  *op_id = (int)s->ops.size() - 1;
  return CIP_OK;
}

int cip_server_submit(cip_server_t s, const cip_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(CIP_EINVAL, "NULL argument");
  if (!req->y || !req->x || req->iters < 1) return fail(CIP_EINVAL, "bad request");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(CIP_EINVAL, "server is shutting down");
  if (req->op < 0 || req->op >= (int)s->ops.size()) return fail(CIP_EINVAL, "unknown operator");
  const Operator& op = s->ops[req->op];
  Request r;
  r.op = req->op;
  r.iters = req->iters;
  r.y = req->y;
  r.x = req->x;
  r.bytes = round_up(op.state_bytes) + round_up((size_t)op.K * op.N1 * op.N2 * 4) +
            (size_t)op.S * op.N1 * op.N2 * 4;
  if (round_up(r.bytes) > s->arena->capacity() - s->reserved_ops)
    return fail(CIP_ENOSPC, "request can never fit in the server budget");
  r.submit = Clock::now();
  const uint64_t t = s->next_ticket++;
  s->reqs.emplace(t, r);
  s->queue.push_back(t);
  s->work_cv.notify_one();
  *ticket = t;
  return CIP_OK;
}

int cip_server_poll(cip_server_t s, uint64_t ticket, int* done, double* latency_s) {
  if (!s || !done) return fail(CIP_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CIP_EINVAL, "unknown ticket");
  const Request& r = it->second;
  if (r.status > 0) {
    *done = 0;
    return CIP_OK;
  }
  *done = 1;
  if (latency_s) *latency_s = std::chrono::duration<double>(r.end - r.submit).count();
  if (r.status < 0) return fail(r.status, r.error);
  return CIP_OK;
}

int cip_server_wait(cip_server_t s, uint64_t ticket, double* latency_s, double* queue_s) {
  if (!s) return fail(CIP_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CIP_EINVAL, "unknown ticket");
  const Request& r = it->second;   // element addresses survive rehashing
  s->done_cv.wait(lk, [&] { return r.status <= 0; });
  if (latency_s) *latency_s = std::chrono::duration<double>(r.end - r.submit).count();
  if (queue_s) *queue_s = std::chrono::duration<double>(r.start - r.submit).count();
  if (r.status < 0) return fail(r.status, r.error);
  return CIP_OK;
}

int cip_server_destroy(cip_server_t s) {
  if (!s) return CIP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  for (auto& w : s->workers) w.join();
  for (auto& op : s->ops) cip_plan_destroy(op.plan);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->op_stream) (void)hipStreamDestroy(s->op_stream);
  (void)hipFree(s->base);
  delete s;
  return CIP_OK;
}

}  // extern "C"
