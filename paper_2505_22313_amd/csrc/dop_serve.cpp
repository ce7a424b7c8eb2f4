// Continuous-batching PSF server.
//
// Requests are queued FIFO.  A scheduler thread admits the head of the queue
// as soon as a slot is free and its workspace fits in the caller's device
// arena (first-fit sub-allocator, no hipMalloc per request), enqueues the
// request's passes on that slot's stream and records an event.  Completed
// events release the slot and the arena range, which admits the next
// requests while others are still running, so the passes of several requests
// overlap on the device.  Results do not depend on what runs beside them:
// every kernel is deterministic and each request has its own workspace.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dop.h"
#include "dop_host.h"

namespace dop {

using Clock = std::chrono::steady_clock;

static double now_s() {
  return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  dop_problem prob{};
  std::vector<double> lam, nidx;
  std::vector<float> weight;
  const float *h = nullptr, *amp = nullptr;
  float *psf = nullptr;
  size_t need = 0;
  double t_submit = 0, t_done = 0;
  dop_status status = DOP_NOT_READY;
  int slot = -1;
  size_t off = 0;
};

// First-fit sub-allocator over [0, size) with coalescing free ranges.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  static constexpr size_t kAlign = 256;
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    used_ -= bytes;
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
  size_t size() const { return size_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

// Executes admitted requests.  start() enqueues without blocking; done()
// polls without blocking and, once true, result() gives the status.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual void thread_init() {}
  virtual dop_status start(int slot, Request &r, void *ws, size_t ws_bytes) = 0;
  virtual bool done(int slot, dop_status *st) = 0;
};

class GpuExecutor : public Executor {
 public:
  GpuExecutor(dop_context *ctx, int slots) : ctx_(ctx), streams_(slots), events_(slots) {}
  dop_status init() {
    (void)hipSetDevice(context_device(ctx_));
    for (size_t i = 0; i < streams_.size(); ++i) {
      if (hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking) != hipSuccess)
        return fail(DOP_ERR_DEVICE, "hipStreamCreate failed");
      if (hipEventCreateWithFlags(&events_[i], hipEventDisableTiming) != hipSuccess)
        return fail(DOP_ERR_DEVICE, "hipEventCreate failed");
    }
    return DOP_OK;
  }
  ~GpuExecutor() override {
    for (auto s : streams_)
      if (s) (void)hipStreamSynchronize(s);
    for (auto e : events_)
      if (e) (void)hipEventDestroy(e);
    for (auto s : streams_)
      if (s) (void)hipStreamDestroy(s);
  }
  void thread_init() override { (void)hipSetDevice(context_device(ctx_)); }
  dop_status start(int slot, Request &r, void *ws, size_t ws_bytes) override {
    dop_status s =
        enqueue_psf(ctx_, &r.prob, r.h, r.amp, r.psf, nullptr, ws, ws_bytes, streams_[slot]);
    if (s != DOP_OK) return s;
    if (hipEventRecord(events_[slot], streams_[slot]) != hipSuccess)
      return fail(DOP_ERR_DEVICE, "hipEventRecord failed");
    return DOP_OK;
  }
  bool done(int slot, dop_status *st) override {
    const hipError_t e = hipEventQuery(events_[slot]);
    if (e == hipErrorNotReady) return false;
    *st = (e == hipSuccess) ? DOP_OK : DOP_ERR_DEVICE;
    return true;
  }

 private:
  dop_context *ctx_;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
};

// Host-only stand-in: a request occupies its slot for a wall time
// proportional to K * M^2.
class MockExecutor : public Executor {
 public:
  MockExecutor(int slots, double us_per_mpix) : end_(slots, 0.0), us_per_mpix_(us_per_mpix) {}
  dop_status start(int slot, Request &r, void *, size_t) override {
    const double mpix =
        (double)r.prob.n_lambda * grid_cols(&r.prob) * (double)grid_rows(&r.prob) / 1e6;
    end_[slot] = now_s() + us_per_mpix_ * mpix * 1e-6;
    return DOP_OK;
  }
  bool done(int slot, dop_status *st) override {
    if (now_s() < end_[slot]) return false;
    *st = DOP_OK;
    return true;
  }

 private:
  std::vector<double> end_;
  double us_per_mpix_;
};

}  // namespace dop

using namespace dop;

struct dop_server {
  std::unique_ptr<Executor> ex;
  char *arena_base = nullptr;
  Arena arena;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<Request *> slots;
  std::vector<double> latencies_ms;
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0, failed = 0;
  bool stopping = false;
  int policy = DOP_SERVE_FIFO;
  double share_ratio = 0.25;
  std::thread sched;

  dop_server(char *base, size_t bytes, int n) : arena_base(base), arena(bytes), max_slots(n),
                                                slots(n, nullptr) {}

  // padded pixels x wavelengths: the request's share of GPU time
  static double work(const Request &r) {
    return (double)r.prob.n_lambda * (double)grid_cols(&r.prob) * (double)grid_rows(&r.prob);
  }

  void finish(Request *r, dop_status st) {
    r->status = st;
    r->t_done = now_s();
    latencies_ms.push_back((r->t_done - r->t_submit) * 1e3);
    ++completed;
    if (st != DOP_OK) ++failed;
  }

  void loop() {
    ex->thread_init();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool any_done = false;
      int running = 0;
      for (int s = 0; s < max_slots; ++s) {
        Request *r = slots[s];
        if (!r) continue;
        dop_status st;
        if (ex->done(s, &st)) {
          arena.release(r->off, r->need);
          slots[s] = nullptr;
          finish(r, st);
          any_done = true;
        } else {
          ++running;
        }
      }
      while (!stopping && !queue.empty()) {
        Request *r = queue.front();
        int free_slot = -1;
        for (int s = 0; s < max_slots; ++s)
          if (!slots[s]) { free_slot = s; break; }
        if (free_slot < 0) break;
        if (policy == DOP_SERVE_SIZE_AWARE && running > 0) {
          // the head shares the GPU only if it is small next to what runs
          double wmax = 0.0;
          for (Request *q : slots)
            if (q) wmax = std::max(wmax, work(*q));
          if (work(*r) > share_ratio * wmax) break;
        }
        size_t off = 0;
        if (!arena.alloc(r->need, &off)) break;  // FIFO: the head waits for memory
        queue.pop_front();
        r->slot = free_slot;
        r->off = off;
        const dop_status st = ex->start(free_slot, *r, arena_base + off, r->need);
        if (st != DOP_OK) {
          arena.release(off, r->need);
          finish(r, st);
          any_done = true;
        } else {
          slots[free_slot] = r;
          ++running;
        }
      }
      if (any_done) cv_done.notify_all();
      if (stopping && running == 0) break;
      if (running == 0 && queue.empty()) {
        cv_work.wait(lk);
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
  }
};

static dop_status make_server(std::unique_ptr<Executor> ex, void *arena, size_t bytes, int slots,
                              dop_server **out) {
  dop_server *srv = new dop_server(static_cast<char *>(arena), bytes, slots);
  srv->ex = std::move(ex);
  srv->sched = std::thread([srv] { srv->loop(); });
  *out = srv;
  return DOP_OK;
}

extern "C" {

dop_status dop_serve_create(dop_context *ctx, void *arena, size_t arena_bytes, int max_slots,
                            dop_server **out) {
  clear_error();
  if (!out) return fail(DOP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(DOP_ERR_INVALID_ARG, "context is NULL");
  if (!arena || arena_bytes == 0) return fail(DOP_ERR_INVALID_ARG, "arena is empty");
  if (reinterpret_cast<uintptr_t>(arena) % Arena::kAlign != 0)
    return fail(DOP_ERR_INVALID_ARG, "arena must be %zu-byte aligned", Arena::kAlign);
  if (max_slots < 1 || max_slots > 64) return fail(DOP_ERR_INVALID_ARG, "max_slots must be 1..64");
  auto ex = std::make_unique<GpuExecutor>(ctx, max_slots);
  const dop_status s = ex->init();
  if (s != DOP_OK) return s;
  return make_server(std::move(ex), arena, arena_bytes, max_slots, out);
}

dop_status dop_serve_create_mock(void *arena, size_t arena_bytes, int max_slots,
                                 double service_us_per_mpix, dop_server **out) {
  clear_error();
  if (!out) return fail(DOP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!arena || arena_bytes == 0) return fail(DOP_ERR_INVALID_ARG, "arena is empty");
  if (max_slots < 1 || max_slots > 64) return fail(DOP_ERR_INVALID_ARG, "max_slots must be 1..64");
  if (!(service_us_per_mpix >= 0.0)) return fail(DOP_ERR_INVALID_ARG, "service time must be >= 0");
  return make_server(std::make_unique<MockExecutor>(max_slots, service_us_per_mpix), arena,
                     arena_bytes, max_slots, out);
}

dop_status dop_serve_submit(dop_server *srv, const dop_problem *prob, const float *h,
                            const float *amp, float *psf, uint64_t *ticket) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  if (!ticket) return fail(DOP_ERR_INVALID_ARG, "ticket is NULL");
  dop_status s = validate_problem(prob);
  if (s != DOP_OK) return s;
  if (!h || !psf) return fail(DOP_ERR_INVALID_ARG, "h / psf must not be NULL");
  auto misaligned = [](const void *q) { return reinterpret_cast<uintptr_t>(q) % 4 != 0; };
  if (misaligned(h) || misaligned(psf) || (amp && misaligned(amp)))
    return fail(DOP_ERR_INVALID_ARG, "float arrays must be 4-byte aligned");
  auto r = std::make_unique<Request>();
  r->prob = *prob;
  r->lam.assign(prob->lambda, prob->lambda + prob->n_lambda);
  r->nidx.assign(prob->n_index, prob->n_index + prob->n_lambda);
  r->prob.lambda = r->lam.data();
  r->prob.n_index = r->nidx.data();
  if (prob->weight) {
    r->weight.assign(prob->weight, prob->weight + prob->n_lambda);
    r->prob.weight = r->weight.data();
  }
  r->h = h;
  r->amp = amp;
  r->psf = psf;
  r->need = workspace_bytes(prob);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return fail(DOP_ERR_SHUTDOWN, "server is shutting down");
    if ((r->need + Arena::kAlign - 1) / Arena::kAlign * Arena::kAlign > srv->arena.size())
      return fail(DOP_ERR_BUDGET, "request needs %zu bytes, arena holds %zu", r->need,
                  srv->arena.size());
    r->ticket = srv->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->all.emplace(r->ticket, std::move(r));
    ++srv->submitted;
  }
  srv->cv_work.notify_one();
  return DOP_OK;
}

dop_status dop_serve_set_policy(dop_server *srv, int policy, double share_ratio) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  if (policy != DOP_SERVE_FIFO && policy != DOP_SERVE_SIZE_AWARE)
    return fail(DOP_ERR_INVALID_ARG, "unknown policy %d", policy);
  if (!(share_ratio >= 0.0) || !std::isfinite(share_ratio))
    return fail(DOP_ERR_INVALID_ARG, "share_ratio must be finite and >= 0");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->policy = policy;
    srv->share_ratio = share_ratio;
  }
  srv->cv_work.notify_one();
  return DOP_OK;
}

dop_status dop_serve_poll(dop_server *srv, uint64_t ticket) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(DOP_ERR_NOT_FOUND, "unknown ticket %llu",
                                        (unsigned long long)ticket);
  return it->second->status;
}

dop_status dop_serve_wait(dop_server *srv, uint64_t ticket, double timeout_s) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(DOP_ERR_NOT_FOUND, "unknown ticket %llu",
                                        (unsigned long long)ticket);
  Request *r = it->second.get();
  auto ready = [r] { return r->status != DOP_NOT_READY; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return fail(DOP_ERR_TIMEOUT, "ticket %llu not done after %.3f s", (unsigned long long)ticket,
                timeout_s);
  }
  return r->status;
}

dop_status dop_serve_latency(dop_server *srv, uint64_t ticket, double *ms) {
  clear_error();
  if (!srv || !ms) return fail(DOP_ERR_INVALID_ARG, "server / ms is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(DOP_ERR_NOT_FOUND, "unknown ticket");
  if (it->second->status == DOP_NOT_READY) return DOP_NOT_READY;
  *ms = (it->second->t_done - it->second->t_submit) * 1e3;
  return DOP_OK;
}

dop_status dop_serve_stats_get(dop_server *srv, dop_serve_stats *out) {
  clear_error();
  if (!srv || !out) return fail(DOP_ERR_INVALID_ARG, "server / out is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  dop_serve_stats st{};
  st.submitted = srv->submitted;
  st.completed = srv->completed;
  st.failed = srv->failed;
  st.queued = (uint32_t)srv->queue.size();
  uint32_t running = 0;
  for (auto r : srv->slots)
    if (r) ++running;
  st.running = running;
  st.arena_bytes = srv->arena.size();
  st.arena_peak = srv->arena.peak();
  if (!srv->latencies_ms.empty()) {
    std::vector<double> v = srv->latencies_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&v](double q) {
      const double pos = q * (double)(v.size() - 1);
      const size_t i = (size_t)pos;
      const double f = pos - (double)i;
      return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
    };
    st.p50_ms = pct(0.50);
    st.p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    st.mean_ms = sum / (double)v.size();
  }
  *out = st;
  return DOP_OK;
}

dop_status dop_serve_destroy(dop_server *srv) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    for (Request *r : srv->queue) srv->finish(r, DOP_ERR_SHUTDOWN);
    srv->queue.clear();
  }
  srv->cv_work.notify_all();
  srv->cv_done.notify_all();
  if (srv->sched.joinable()) srv->sched.join();
  srv->cv_done.notify_all();
  delete srv;
  return DOP_OK;
}

}  // extern "C"
