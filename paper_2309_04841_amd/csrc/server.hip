// server.hip -- continuous-batching request loop over the QAOA entry points.
//
// An outer optimiser (Section 2: the angles are tuned by repeated objective
// evaluations) submits objective and gradient requests for problems whose cost
// vectors stay resident on the device.  A scheduler thread admits requests in
// arrival order whenever their device footprint (state(s) + workspace + output)
// fits the arena and an in-flight slot is free, enqueues them on a pool of
// streams so independent requests overlap on the GPU, and retires them as their
// completion events fire, which frees memory for the next admissions.  Every
// request owns its buffers and the kernels reduce in a fixed order, so a
// request's result does not depend on what else is in flight.  Cost vectors sit
// at the top of the arena and requests at the bottom (arena.hpp); a request
// that cannot be placed while nothing is in flight fails with QAOA_ERR_NOMEM
// instead of waiting for memory that no finishing request will free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "qaoa.h"

// Shared with qaoa.hip: sets the calling thread's qaoa_last_error() message.
int qaoa_internal_set_error(int code, const char* msg);

namespace {

int sfail(int code, const char* msg) { return qaoa_internal_set_error(code, msg); }

using Clock = std::chrono::steady_clock;

// One device allocation carved by qaoa_arena::ArenaMap.
class Arena {
 public:
  bool init(size_t bytes) {
    map_.reset(bytes);
    if (hipMalloc(&base_, map_.size()) != hipSuccess) { base_ = nullptr; return false; }
    return true;
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  size_t alloc_request(size_t bytes) { return map_.alloc_low(bytes); }
  size_t alloc_resident(size_t bytes) { return map_.alloc_high(bytes); }
  void release(size_t off, size_t bytes) { map_.release(off, bytes); }
  char* ptr(size_t off) const { return base_ + off; }
  size_t size() const { return map_.size(); }
  size_t used() const { return map_.used(); }
  size_t peak() const { return map_.peak(); }
  void reset_peak() { map_.reset_peak(); }

 private:
  char* base_ = nullptr;
  qaoa_arena::ArenaMap map_;
};

struct Problem {
  int n;
  int diag_dtype;
  double offset;
  size_t off, bytes;
};

struct Request {
  int64_t ticket;
  int problem;
  int kind;  // 0 objective, 1 gradient
  int state_dtype;
  int p;
  std::vector<double> gamma, beta;
  size_t off = SIZE_MAX, bytes = 0;  // arena block: [out][state][adj][work]
  size_t out_len = 0;
  int slot = -1, stream = -1;
  hipEvent_t done_ev = nullptr;  // the slot's event while in flight
  Clock::time_point t_submit, t_done;
  int status = QAOA_OK;
  std::string error;
  std::vector<double> result;
  bool finished = false;
};

constexpr int kMaxServerLayers = 256;
constexpr size_t kSlotDoubles = 1 + 2 * kMaxServerLayers;

size_t state_bytes(int n, int sdt) { return ((size_t)1 << n) * (sdt == QAOA_C128 ? 16 : 8); }
size_t diag_elem(int ddt) { return ddt == QAOA_DIAG_F64 ? 8 : ddt == QAOA_DIAG_I32 ? 4 : 2; }

}  // namespace

struct qaoa_server {
  Arena arena;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  int max_in_flight = 0;
  double* pinned = nullptr;  // max_in_flight slots of kSlotDoubles
  std::vector<hipEvent_t> slot_events;  // one completion event per slot, reused
  std::vector<int> free_slots;
  std::vector<Problem> problems;
  size_t problem_bytes = 0;  // arena bytes held by resident cost vectors

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> in_flight;
  std::unordered_map<int64_t, std::shared_ptr<Request>> by_ticket;
  int64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;

  // Device resources (the worker thread has ended or was never started).
  ~qaoa_server() {
    for (auto st : streams) (void)hipStreamDestroy(st);
    for (auto ev : slot_events) (void)hipEventDestroy(ev);
    if (pinned) (void)hipHostFree(pinned);
  }

  // stats
  uint64_t submitted = 0, completed = 0, failed = 0;
  std::vector<double> latencies;
  Clock::time_point first_submit, last_done;
  bool any_submit = false;

  size_t footprint(const Request& r, size_t* work_bytes) const {
    const Problem& pr = problems[r.problem];
    size_t wb = 0;
    if (r.kind == 0) qaoa_workspace_bytes(QAOA_OP_EVOLVE, pr.n, r.state_dtype, pr.diag_dtype, &wb);
    else qaoa_grad_workspace_bytes(pr.n, r.p, r.state_dtype, pr.diag_dtype, &wb);
    *work_bytes = wb;
    const size_t sb = (state_bytes(pr.n, r.state_dtype) + 255) & ~(size_t)255;
    return 256 + sb * (r.kind == 0 ? 1 : 2) + wb;
  }

  // Enqueue an admitted request (mu held).
  void launch(const std::shared_ptr<Request>& r, size_t work_bytes) {
    const Problem& pr = problems[r->problem];
    char* blk = arena.ptr(r->off);
    double* d_out = reinterpret_cast<double*>(blk);
    const size_t sb = (state_bytes(pr.n, r->state_dtype) + 255) & ~(size_t)255;
    void* st_a = blk + 256;
    void* st_b = blk + 256 + sb;
    void* work = blk + 256 + sb * (r->kind == 0 ? 1 : 2);
    r->stream = next_stream;
    next_stream = (next_stream + 1) % (int)streams.size();
    hipStream_t st = streams[r->stream];
    const void* diag = arena.ptr(pr.off);
    int rc;
    if (r->kind == 0)
      rc = qaoa_evolve(pr.n, r->p, r->gamma.data(), r->beta.data(), diag, pr.diag_dtype, pr.offset, pr.bytes, st_a,
                       r->state_dtype, state_bytes(pr.n, r->state_dtype), 1, d_out, work, work_bytes, st);
    else
      rc = qaoa_grad(pr.n, r->p, r->gamma.data(), r->beta.data(), diag, pr.diag_dtype, pr.offset, pr.bytes, st_a, st_b,
                     r->state_dtype, state_bytes(pr.n, r->state_dtype), d_out, work, work_bytes, st);
    if (rc == QAOA_OK) {
      r->done_ev = slot_events[r->slot];
      if (hipMemcpyAsync(pinned + (size_t)r->slot * kSlotDoubles, d_out, r->out_len * sizeof(double),
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipEventRecord(r->done_ev, st) != hipSuccess) {
        rc = QAOA_ERR_DEVICE;
        qaoa_internal_set_error(rc, "hipMemcpyAsync/hipEventRecord of a request failed");
      }
    }
    if (rc != QAOA_OK) {
      r->status = rc;
      r->error = qaoa_last_error();
      r->done_ev = nullptr;
    }
    in_flight.push_back(r);
  }

  void retire(const std::shared_ptr<Request>& r) {
    if (r->status == QAOA_OK) {
      const double* src = pinned + (size_t)r->slot * kSlotDoubles;
      r->result.assign(src, src + r->out_len);
      ++completed;
    } else {
      ++failed;
    }
    r->done_ev = nullptr;
    if (r->off != SIZE_MAX) arena.release(r->off, r->bytes);
    if (r->slot >= 0) free_slots.push_back(r->slot);
    r->t_done = Clock::now();
    latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
    last_done = r->t_done;
    r->finished = true;
  }

  void run() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      // retire finished requests
      bool retired = false;
      for (size_t i = 0; i < in_flight.size();) {
        auto& r = in_flight[i];
        bool done = (r->status != QAOA_OK);
        if (!done) {
          const hipError_t qe = hipEventQuery(r->done_ev);
          if (qe == hipSuccess) {
            done = true;
          } else if (qe != hipErrorNotReady) {  // a device error retires the request instead of stalling it
            r->status = QAOA_ERR_DEVICE;
            r->error = hipGetErrorString(qe);
            done = true;
          }
        }
        if (done) {
          retire(r);
          in_flight[i] = in_flight.back();
          in_flight.pop_back();
          retired = true;
        } else {
          ++i;
        }
      }
      if (retired) cv_done.notify_all();
      // requests not yet admitted when the server is destroyed are dropped
      if (stop && !queue.empty()) {
        while (!queue.empty()) {
          auto r = queue.front();
          queue.pop_front();
          r->status = QAOA_ERR_INVALID;
          r->error = "server destroyed before the request was admitted";
          retire(r);
        }
        cv_done.notify_all();
      }
      // admit in arrival order while memory and slots allow
      while (!queue.empty() && (int)in_flight.size() < max_in_flight) {
        auto r = queue.front();
        size_t wb = 0;
        const size_t need = footprint(*r, &wb);
        const size_t off = arena.alloc_request(need);
        if (off == SIZE_MAX) {
          if (qaoa_arena::head_blocked(in_flight.size()) == qaoa_arena::HeadAction::kWait) break;
          // nothing in flight will free memory: fail the request rather than stall the queue
          queue.pop_front();
          r->status = QAOA_ERR_NOMEM;
          r->error = "no contiguous arena block for the request (" + std::to_string(need) +
                     " bytes) with no request in flight";
          retire(r);
          cv_done.notify_all();
          continue;
        }
        queue.pop_front();
        r->off = off;
        r->bytes = need;
        r->slot = free_slots.back();
        free_slots.pop_back();
        launch(r, wb);
      }
      if (stop && queue.empty() && in_flight.empty()) break;
      if (in_flight.empty() && queue.empty()) {
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      } else {
        // poll completions without holding the lock
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
  }
};

extern "C" {

int qaoa_server_create(size_t arena_bytes, int num_streams, int max_in_flight, qaoa_server** out) {
  if (!out) return sfail(QAOA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (arena_bytes < ((size_t)1 << 20)) return sfail(QAOA_ERR_INVALID, "arena_bytes must be >= 1 MiB");
  if (num_streams < 1 || num_streams > 64) return sfail(QAOA_ERR_INVALID, "num_streams must be in [1, 64]");
  if (max_in_flight < 1 || max_in_flight > 4096) return sfail(QAOA_ERR_INVALID, "max_in_flight must be in [1, 4096]");
  std::unique_ptr<qaoa_server> s(new qaoa_server());
  if (!s->arena.init(arena_bytes)) return sfail(QAOA_ERR_NOMEM, "hipMalloc of the arena failed");
  if (hipHostMalloc(reinterpret_cast<void**>(&s->pinned), sizeof(double) * kSlotDoubles * max_in_flight) != hipSuccess)
    return sfail(QAOA_ERR_DEVICE, "hipHostMalloc of the result slots failed");
  for (int i = 0; i < num_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return sfail(QAOA_ERR_DEVICE, "hipStreamCreate failed");
    s->streams.push_back(st);
  }
  for (int i = 0; i < max_in_flight; ++i) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
      return sfail(QAOA_ERR_DEVICE, "hipEventCreate failed");
    s->slot_events.push_back(ev);
  }
  s->max_in_flight = max_in_flight;
  for (int i = max_in_flight - 1; i >= 0; --i) s->free_slots.push_back(i);
  qaoa_server* raw = s.release();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
  return QAOA_OK;
}

int qaoa_server_destroy(qaoa_server* s) {
  if (!s) return sfail(QAOA_ERR_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  delete s;
  return QAOA_OK;
}

int qaoa_server_add_problem(qaoa_server* s, int n, int64_t num_terms, const double* w, const int64_t* term_ptr,
                            const int32_t* term_idx, int diag_dtype, int* problem_id) {
  if (!s || !problem_id) return sfail(QAOA_ERR_INVALID, "server/problem_id is NULL");
  if (n < 1 || n > QAOA_MAX_QUBITS) return sfail(QAOA_ERR_INVALID, "n out of range");
  if (diag_dtype != QAOA_DIAG_F64 && diag_dtype != QAOA_DIAG_I32 && diag_dtype != QAOA_DIAG_U16)
    return sfail(QAOA_ERR_INVALID, "bad diag dtype");
  size_t wb = 0;
  int rc = qaoa_workspace_bytes(QAOA_OP_PRECOMPUTE, n, QAOA_C64, diag_dtype, &wb);
  if (rc) return sfail(rc, qaoa_last_error());
  const size_t dbytes = ((size_t)1 << n) * diag_elem(diag_dtype);
  std::lock_guard<std::mutex> lk(s->mu);
  const size_t off = s->arena.alloc_resident(dbytes);
  if (off == SIZE_MAX) return sfail(QAOA_ERR_NOMEM, "arena has no room for the cost vector");
  size_t woff = SIZE_MAX;
  if (wb) {
    woff = s->arena.alloc_resident(wb);
    if (woff == SIZE_MAX) {
      s->arena.release(off, dbytes);
      return sfail(QAOA_ERR_NOMEM, "arena has no room for the precompute workspace");
    }
  }
  double offset = 0.0;
  hipStream_t st = s->streams[0];
  rc = qaoa_precompute_diag(n, num_terms, w, term_ptr, term_idx, diag_dtype, s->arena.ptr(off), dbytes, &offset,
                            wb ? s->arena.ptr(woff) : nullptr, wb, st);
  if (rc == QAOA_OK && hipStreamSynchronize(st) != hipSuccess) rc = QAOA_ERR_DEVICE;
  if (wb) s->arena.release(woff, wb);
  if (rc != QAOA_OK) {
    std::string m = qaoa_last_error();
    s->arena.release(off, dbytes);
    return sfail(rc, m.c_str());
  }
  s->problems.push_back(Problem{n, diag_dtype, offset, off, dbytes});
  s->problem_bytes += (dbytes + 255) & ~(size_t)255;
  *problem_id = (int)s->problems.size() - 1;
  return QAOA_OK;
}

int qaoa_server_submit(qaoa_server* s, int problem_id, int kind, int state_dtype, int p, const double* gamma,
                       const double* beta, int64_t* ticket) {
  if (!s || !ticket) return sfail(QAOA_ERR_INVALID, "server/ticket is NULL");
  if (kind != 0 && kind != 1) return sfail(QAOA_ERR_INVALID, "kind must be 0 (objective) or 1 (gradient)");
  if (state_dtype != QAOA_C64 && state_dtype != QAOA_C128) return sfail(QAOA_ERR_INVALID, "bad state dtype");
  if (p < 1 || p > kMaxServerLayers) return sfail(QAOA_ERR_INVALID, "p must be in [1, 256]");
  if (!gamma || !beta) return sfail(QAOA_ERR_INVALID, "gamma/beta is NULL");
  auto r = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (problem_id < 0 || problem_id >= (int)s->problems.size()) return sfail(QAOA_ERR_INVALID, "unknown problem");
    r->problem = problem_id;
    r->kind = kind;
    r->state_dtype = state_dtype;
    r->p = p;
    r->gamma.assign(gamma, gamma + p);
    r->beta.assign(beta, beta + p);
    r->out_len = kind == 0 ? 2 : (size_t)(1 + 2 * p);
    size_t wb = 0;
    if (s->footprint(*r, &wb) > s->arena.size() - s->problem_bytes)
      return sfail(QAOA_ERR_NOMEM, "request needs more device memory than the arena has besides the cost vectors");
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    if (!s->any_submit) { s->first_submit = r->t_submit; s->any_submit = true; }
    ++s->submitted;
    s->by_ticket[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
  }
  s->cv_work.notify_all();
  return QAOA_OK;
}

int qaoa_server_wait(qaoa_server* s, int64_t ticket, double* out, int out_len, double* latency_s) {
  if (!s) return sfail(QAOA_ERR_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return sfail(QAOA_ERR_INVALID, "unknown ticket");
  auto r = it->second;
  s->cv_done.wait(lk, [&] { return r->finished; });
  s->by_ticket.erase(it);
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (r->status != QAOA_OK) return sfail(r->status, r->error.c_str());
  if (out) {
    if (out_len < (int)r->out_len) return sfail(QAOA_ERR_NOMEM, "out buffer too small");
    std::memcpy(out, r->result.data(), r->out_len * sizeof(double));
  }
  return QAOA_OK;
}

int qaoa_server_stats_get(qaoa_server* s, qaoa_server_stats* out) {
  if (!s || !out) return sfail(QAOA_ERR_INVALID, "server/out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = s->queue.size();
  out->in_flight = s->in_flight.size();
  out->arena_bytes = s->arena.size();
  out->peak_bytes = s->arena.peak();
  std::vector<double> l = s->latencies;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)(f * (l.size() - 1) + 0.5))]; };
    out->p50_s = q(0.50);
    out->p99_s = q(0.99);
    out->max_s = l.back();
    double sum = 0.0;
    for (double v : l) sum += v;
    out->mean_s = sum / l.size();
    out->busy_s = std::chrono::duration<double>(s->last_done - s->first_submit).count();
    out->requests_per_s = out->busy_s > 0 ? (double)l.size() / out->busy_s : 0.0;
  }
  return QAOA_OK;
}

int qaoa_server_reset_stats(qaoa_server* s) {
  if (!s) return sfail(QAOA_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->latencies.clear();
  s->submitted = s->completed = s->failed = 0;
  s->any_submit = false;
  s->arena.reset_peak();
  return QAOA_OK;
}

}  // extern "C"
