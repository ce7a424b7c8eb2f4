// Continuous-batching PSF server.
//
// Requests are queued in submission order.  A scheduler thread admits them
// as request slots and arena memory free up (each admitted request holds its
// own workspace, sub-allocated first-fit from the caller's device arena: no
// hipMalloc per request) and feeds their work to the GPU under one of three
// policies:
//
//  - DOP_SERVE_CHUNKED (default): a request's wavelengths run in chunks of
//    one wavelength group (up to four wavelengths that share one read of the
//    heights and one read-modify-write of the PSF).  Chunks of all admitted
//    requests go through one in-order stream, two enqueued at a time (more
//    while they hold under about a millisecond of work).  Each time a chunk
//    completes, the next one is taken from the admitted request with the
//    least work left (shortest remaining processing time), unless requests
//    have waited longer than the age bound: then the oldest of those goes
//    first.  A request that arrives while a large one runs waits for the
//    chunks already enqueued instead of the whole large request, and the
//    large one is never slowed by sharing the GPU: it only pauses.
//    Admission takes the head of the queue first; a request behind a head
//    that does not fit yet may go ahead of it unless the head has passed the
//    age bound.  An admitted request gets a workspace of up to one group of
//    fields, at most half the arena, and as many as fit at admission.
//  - DOP_SERVE_FIFO and DOP_SERVE_SIZE_AWARE: a request's whole PSF is
//    enqueued at admission on the stream of its slot, so admitted requests
//    run side by side (processor sharing); admission is strictly in order.
//
// Results do not depend on the schedule: every kernel is deterministic, each
// request has its own workspace and output, its chunks run in wavelength
// order on one stream, and a chunk adds its wavelengths to the PSF in the
// order and rounding of one dop_psf call.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
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

// Chunks enqueued ahead on the chunked policy's stream: at least two (one
// running, one waiting behind it, so the GPU does not idle while the
// scheduler picks), and more, up to kMaxDepth, while the enqueued chunks hold
// less than kMinQueued padded pixels x wavelengths (about 1 ms of work):
// short chunks of small grids finish faster than the scheduler thread reacts.
constexpr int kDepth = 2;
constexpr int kMaxDepth = 8;
constexpr double kMinQueued = 1e8;
// Queue entries the chunked policy's admission looks at past a head that
// does not fit yet.
constexpr int kAdmitLookahead = 32;
// Default age bound of the chunked policy (seconds).
constexpr double kDefaultAgeBound = 0.25;

struct Request {
  uint64_t ticket = 0;
  dop_problem prob{};
  std::vector<double> lam, nidx;
  std::vector<float> weight;
  const float *h = nullptr, *amp = nullptr;
  float *psf = nullptr;
  size_t field = 0;      // bytes of one workspace field
  size_t need = 0;       // workspace bytes held while admitted
  int group = 1;         // wavelengths per chunk (fields in the workspace)
  bool chunked = false;  // admitted under DOP_SERVE_CHUNKED
  double t_submit = 0, t_done = 0;
  dop_status status = DOP_NOT_READY;
  int slot = -1;         // whole-request policies: the slot (and stream) it runs on
  size_t off = 0;
  int k_next = 0;        // first wavelength not yet enqueued
  int inflight = 0;      // chunks enqueued and not yet complete
  dop_status err = DOP_OK;  // first chunk error (no further chunks after one)
};

// First-fit sub-allocator over [0, size) with coalescing free ranges.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  static constexpr size_t kAlign = 256;
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = round(bytes);
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
    bytes = round(bytes);
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

// Executes chunks (wavelengths [k0, k1) of a request) on lanes (in-order
// streams).  start() enqueues without blocking and names the chunk by a
// token; done() polls without blocking; release() returns the token.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual void thread_init() {}
  virtual dop_status start(int lane, Request &r, int k0, int k1, void *ws, size_t ws_bytes,
                           int *token) = 0;
  virtual bool done(int token, dop_status *st) = 0;
  virtual void release(int token) = 0;
};

// Tokens 0..n-1 handed out and returned.
class TokenPool {
 public:
  explicit TokenPool(int n) {
    for (int i = n - 1; i >= 0; --i) free_.push_back(i);
  }
  bool take(int *t) {
    if (free_.empty()) return false;
    *t = free_.back();
    free_.pop_back();
    return true;
  }
  void give(int t) { free_.push_back(t); }

 private:
  std::vector<int> free_;
};

class GpuExecutor : public Executor {
 public:
  // lanes streams; at most `tokens` chunks in flight (one completion event each)
  GpuExecutor(dop_context *ctx, int lanes, int tokens)
      : ctx_(ctx), streams_(lanes), events_(tokens), pool_(tokens) {}
  dop_status init() {
    (void)hipSetDevice(context_device(ctx_));
    for (auto &s : streams_)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return fail(DOP_ERR_DEVICE, "hipStreamCreate failed");
    for (auto &e : events_)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(DOP_ERR_DEVICE, "hipEventCreate failed");
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
  dop_status start(int lane, Request &r, int k0, int k1, void *ws, size_t ws_bytes,
                   int *token) override {
    int t = 0;
    if (!pool_.take(&t)) return fail(DOP_ERR_DEVICE, "no completion event free");
    dop_status s = enqueue_psf_range(ctx_, &r.prob, k0, k1, r.h, r.amp, r.psf, nullptr, ws,
                                     ws_bytes, streams_[lane]);
    if (s == DOP_OK && hipEventRecord(events_[t], streams_[lane]) != hipSuccess)
      s = fail(DOP_ERR_DEVICE, "hipEventRecord failed");
    if (s != DOP_OK) {
      // work enqueued before the failure still runs: wait for it before the
      // workspace can be handed to another request
      (void)hipStreamSynchronize(streams_[lane]);
      pool_.give(t);
      return s;
    }
    *token = t;
    return DOP_OK;
  }
  bool done(int token, dop_status *st) override {
    const hipError_t e = hipEventQuery(events_[token]);
    if (e == hipErrorNotReady) return false;
    *st = (e == hipSuccess) ? DOP_OK : DOP_ERR_DEVICE;
    return true;
  }
  void release(int token) override { pool_.give(token); }

 private:
  dop_context *ctx_;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  TokenPool pool_;
};

// Host-only stand-in: each lane is an in-order queue whose chunks occupy it
// for service_us_per_mpix * (chunk wavelengths * M^2 / 1e6) microseconds of
// wall time; nothing is written.
class MockExecutor : public Executor {
 public:
  MockExecutor(int lanes, int tokens, double us_per_mpix)
      : lane_end_(lanes, 0.0), tok_end_(tokens, 0.0), pool_(tokens), us_per_mpix_(us_per_mpix) {}
  dop_status start(int lane, Request &r, int k0, int k1, void *, size_t, int *token) override {
    int t = 0;
    if (!pool_.take(&t)) return fail(DOP_ERR_DEVICE, "no completion token free");
    const double mpix = (double)(k1 - k0) * grid_cols(&r.prob) * (double)grid_rows(&r.prob) / 1e6;
    lane_end_[lane] = std::max(now_s(), lane_end_[lane]) + us_per_mpix_ * mpix * 1e-6;
    tok_end_[t] = lane_end_[lane];
    *token = t;
    return DOP_OK;
  }
  bool done(int token, dop_status *st) override {
    if (now_s() < tok_end_[token]) return false;
    *st = DOP_OK;
    return true;
  }
  void release(int token) override { pool_.give(token); }

 private:
  std::vector<double> lane_end_, tok_end_;
  TokenPool pool_;
  double us_per_mpix_;
};

}  // namespace dop

using namespace dop;

struct dop_server {
  struct Chunk {
    int token;
    Request *r;
    int k_end;
    int lane;
    double work = 0.0;  // padded pixels x wavelengths
  };

  std::unique_ptr<Executor> ex;
  char *arena_base = nullptr;
  Arena arena;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<Request *> slots;  // admitted requests by slot (whole-request lanes)
  std::list<Chunk> chunks;       // enqueued, not yet complete, in enqueue order
  std::vector<double> latencies_ms;
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0, failed = 0;
  bool stopping = false;
  int policy = DOP_SERVE_CHUNKED;
  double share_ratio = 0.25;            // DOP_SERVE_SIZE_AWARE
  double age_bound = kDefaultAgeBound;  // DOP_SERVE_CHUNKED, seconds
  std::thread sched;

  dop_server(char *base, size_t bytes, int n) : arena_base(base), arena(bytes), max_slots(n),
                                                slots(n, nullptr) {}

  // padded pixels x wavelengths: the request's share of GPU time
  static double work(const Request &r) {
    return (double)r.prob.n_lambda * (double)grid_cols(&r.prob) * (double)grid_rows(&r.prob);
  }
  static double work_left(const Request &r) {
    return (double)(r.prob.n_lambda - r.k_next) * (double)grid_cols(&r.prob) *
           (double)grid_rows(&r.prob);
  }

  void finish(Request *r, dop_status st) {
    r->status = st;
    r->t_done = now_s();
    latencies_ms.push_back((r->t_done - r->t_submit) * 1e3);
    ++completed;
    if (st != DOP_OK) ++failed;
  }

  int running() const {
    int n = 0;
    for (Request *r : slots)
      if (r) ++n;
    return n;
  }

  int free_slot() const {
    for (int s = 0; s < max_slots; ++s)
      if (!slots[s]) return s;
    return -1;
  }

  // Finished or failed with nothing in flight: release its slot and memory.
  void retire_if_done(Request *r) {
    if (r->inflight > 0) return;
    if (r->err == DOP_OK && r->k_next < r->prob.n_lambda) return;
    arena.release(r->off, r->need);
    slots[r->slot] = nullptr;
    finish(r, r->err);
  }

  // Enqueue wavelengths [k_next, k1) of r on `lane`.
  void start_chunk(Request *r, int k1, int lane) {
    int tok = 0;
    const dop_status st = ex->start(lane, *r, r->k_next, k1, arena_base + r->off, r->need, &tok);
    if (st != DOP_OK) {
      r->err = st;
      retire_if_done(r);
      return;
    }
    r->k_next = k1;
    ++r->inflight;
    chunks.push_back({tok, r, k1, lane});
  }

  // Reserve a slot and workspace for r and admit it under the current policy.
  bool try_admit(Request *r) {
    const int s = free_slot();
    if (s < 0) return false;
    const bool ch = policy == DOP_SERVE_CHUNKED;
    // whole-request policies run one wavelength at a time in one field; the
    // chunked policy gives a request up to a wavelength group of fields, at
    // most half the arena, or as many fields as fit now (at least one)
    int g = 1;
    if (ch) {
      g = psf_group(&r->prob, nullptr, (size_t)-1);
      while (g > 1 && Arena::round((size_t)g * r->field) > arena.size() / 2) --g;
    }
    size_t off = 0;
    while (!arena.alloc((size_t)g * r->field, &off)) {
      if (g == 1) return false;
      --g;
    }
    r->group = g;
    r->need = (size_t)g * r->field;
    r->off = off;
    r->slot = s;
    r->chunked = ch;
    slots[s] = r;
    if (!ch) start_chunk(r, r->prob.n_lambda, s);
    return true;
  }

  void admit(double now) {
    while (!stopping && !queue.empty() && free_slot() >= 0) {
      Request *head = queue.front();
      if (policy == DOP_SERVE_SIZE_AWARE && running() > 0) {
        // the head shares the GPU only if it is small next to what runs
        double wmax = 0.0;
        for (Request *q : slots)
          if (q) wmax = std::max(wmax, work(*q));
        if (work(*head) > share_ratio * wmax) return;
      }
      if (try_admit(head)) {
        queue.pop_front();
        continue;
      }
      // the head does not fit yet: in order for the whole-request policies,
      // and under the chunked policy while the head has passed the age bound
      if (policy != DOP_SERVE_CHUNKED || now - head->t_submit > age_bound) return;
      bool admitted = false;
      int seen = 0;
      for (auto it = std::next(queue.begin()); it != queue.end() && seen < kAdmitLookahead;
           ++it, ++seen) {
        if (try_admit(*it)) {
          queue.erase(it);
          admitted = true;
          break;
        }
      }
      if (!admitted) return;
    }
  }

  // The chunked request whose next chunk goes next, or NULL.
  Request *pick(double now) const {
    Request *best = nullptr;
    bool best_aged = false;
    for (Request *r : slots) {
      if (!r || !r->chunked || r->err != DOP_OK || r->k_next >= r->prob.n_lambda) continue;
      const bool aged = now - r->t_submit > age_bound;
      if (!best) {
        best = r;
        best_aged = aged;
        continue;
      }
      if (aged != best_aged) {
        if (aged) {
          best = r;
          best_aged = true;
        }
        continue;
      }
      const bool better = aged ? r->ticket < best->ticket
                               : (work_left(*r) < work_left(*best) ||
                                  (work_left(*r) == work_left(*best) && r->ticket < best->ticket));
      if (better) best = r;
    }
    return best;
  }

  void feed(double now) {
    int on_lane0 = 0;
    double queued = 0.0;
    for (const Chunk &c : chunks) {
      if (!c.r->chunked) continue;
      ++on_lane0;
      queued += c.work;
    }
    while (on_lane0 < kDepth || (on_lane0 < kMaxDepth && queued < kMinQueued)) {
      Request *r = pick(now);
      if (!r) return;
      const int k1 = std::min(r->prob.n_lambda, r->k_next + r->group);
      const double w = (double)(k1 - r->k_next) * grid_cols(&r->prob) * (double)grid_rows(&r->prob);
      const size_t before = chunks.size();
      start_chunk(r, k1, 0);
      if (chunks.size() > before) {
        chunks.back().work = w;
        ++on_lane0;
        queued += w;
      }
    }
  }

  void loop() {
    ex->thread_init();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool any_done = false;
      for (auto it = chunks.begin(); it != chunks.end();) {
        dop_status st;
        if (!ex->done(it->token, &st)) {
          ++it;
          continue;
        }
        Request *r = it->r;
        ex->release(it->token);
        --r->inflight;
        if (st != DOP_OK && r->err == DOP_OK) r->err = st;
        it = chunks.erase(it);
        const uint64_t before = completed;
        retire_if_done(r);
        any_done = any_done || completed != before;
      }
      const double now = now_s();
      const uint64_t before = completed;
      admit(now);
      feed(now);
      any_done = any_done || completed != before;
      if (any_done) cv_done.notify_all();
      const bool idle = chunks.empty() && running() == 0;
      if (stopping && idle) break;
      if (idle && queue.empty()) {
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
  auto ex = std::make_unique<GpuExecutor>(ctx, max_slots, max_slots + kMaxDepth);
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
  return make_server(std::make_unique<MockExecutor>(max_slots, max_slots + kMaxDepth,
                                                    service_us_per_mpix),
                     arena, arena_bytes, max_slots, out);
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
  r->field = workspace_bytes(prob);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return fail(DOP_ERR_SHUTDOWN, "server is shutting down");
    if (Arena::round(r->field) > srv->arena.size())
      return fail(DOP_ERR_BUDGET, "request needs %zu bytes, arena holds %zu", r->field,
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

dop_status dop_serve_set_policy(dop_server *srv, int policy, double param) {
  clear_error();
  if (!srv) return fail(DOP_ERR_INVALID_ARG, "server is NULL");
  if (policy != DOP_SERVE_FIFO && policy != DOP_SERVE_SIZE_AWARE && policy != DOP_SERVE_CHUNKED)
    return fail(DOP_ERR_INVALID_ARG, "unknown policy %d", policy);
  if (!(param >= 0.0) || !std::isfinite(param))
    return fail(DOP_ERR_INVALID_ARG, "the policy parameter must be finite and >= 0");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->policy = policy;
    if (policy == DOP_SERVE_SIZE_AWARE) srv->share_ratio = param;
    if (policy == DOP_SERVE_CHUNKED) srv->age_bound = param;
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
  st.running = (uint32_t)srv->running();
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
