// Concurrency stress of the serving engine's scheduler through its C ABI,
// with the host-side mock executor (no GPU).  Built and run under the
// thread sanitizer and under the address + undefined-behaviour sanitizers
// by tests/test_serve_sanitizers_cpu.py; any report fails the run.
//
// Scenarios:
//  1. four submitter threads, each with its own waiter thread (poll, wait,
//     latency), a statistics reader and a policy switcher cycling through
//     the chunked, size-aware and FIFO policies, all at once, against a
//     4-slot server whose arena admits only a few requests (requests of
//     several policies are admitted and run side by side);
//  2. requests that can never fit the arena (budget error) and invalid
//     arguments, from several threads;
//  3. shutdown with requests still queued and running.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../include/dop.h"

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, \
                   #c, dop_last_error());                                 \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

static const double kLam[3] = {0.45, 0.55, 0.65};
static const double kIdx[3] = {1.46, 1.46, 1.46};

static dop_problem make_problem(int m, int k) {
  dop_problem p{};
  p.n = m / 2;
  p.m = m;
  p.dx = 1.0;
  p.z = 1000.0;
  p.n_lambda = k;
  p.lambda = kLam;
  p.n_index = kIdx;
  return p;
}

static size_t field_bytes(int m) { return (size_t)m * (m + 16) * 8; }

static void scenario_concurrent() {
  const size_t arena = 3 * field_bytes(1024);  // a few requests at a time
  dop_server *srv = nullptr;
  // 2 us per Mpix: a 1024^2 request with three wavelengths takes ~6 us
  CHECK(dop_serve_create_mock(reinterpret_cast<void *>(256), arena, 4, 2.0, &srv) == DOP_OK);
  constexpr int kThreads = 4, kPer = 300;
  std::atomic<int> submitted_done{0};
  std::atomic<bool> stop{false};
  std::vector<std::thread> th;
  std::vector<std::vector<uint64_t>> tickets(kThreads);
  std::vector<std::mutex> mus(kThreads);
  for (int t = 0; t < kThreads; ++t) {
    th.emplace_back([&, t] {  // submitter
      std::mt19937 rng(100 + t);
      const int sizes[4] = {64, 256, 512, 1024};
      for (int i = 0; i < kPer; ++i) {
        const dop_problem p = make_problem(sizes[rng() % 4], 1 + (int)(rng() % 3));
        uint64_t tk = 0;
        CHECK(dop_serve_submit(srv, &p, reinterpret_cast<const float *>(4096),
                               nullptr, reinterpret_cast<float *>(8192), &tk) == DOP_OK);
        std::lock_guard<std::mutex> lk(mus[t]);
        tickets[t].push_back(tk);
      }
      submitted_done.fetch_add(1);
    });
    th.emplace_back([&, t] {  // waiter
      size_t next = 0;
      while (next < (size_t)kPer) {
        uint64_t tk = 0;
        {
          std::lock_guard<std::mutex> lk(mus[t]);
          if (next < tickets[t].size()) tk = tickets[t][next];
        }
        if (!tk) {
          std::this_thread::yield();
          continue;
        }
        const dop_status st = dop_serve_poll(srv, tk);
        CHECK(st == DOP_OK || st == DOP_NOT_READY);
        CHECK(dop_serve_wait(srv, tk, 30.0) == DOP_OK);
        double ms = -1;
        CHECK(dop_serve_latency(srv, tk, &ms) == DOP_OK && ms >= 0);
        ++next;
      }
    });
  }
  th.emplace_back([&] {  // statistics reader
    while (!stop.load()) {
      dop_serve_stats s{};
      CHECK(dop_serve_stats_get(srv, &s) == DOP_OK);
      CHECK(s.completed <= s.submitted && s.arena_peak <= s.arena_bytes);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  });
  th.emplace_back([&] {  // policy switcher
    int i = 0;
    while (!stop.load()) {
      const int pols[3] = {DOP_SERVE_CHUNKED, DOP_SERVE_SIZE_AWARE, DOP_SERVE_FIFO};
      const int pol = pols[i++ % 3];
      CHECK(dop_serve_set_policy(srv, pol, pol == DOP_SERVE_CHUNKED ? 0.001 : 0.25) == DOP_OK);
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  for (int t = 0; t < 2 * kThreads; ++t) th[t].join();
  stop.store(true);
  for (size_t t = 2 * kThreads; t < th.size(); ++t) th[t].join();
  dop_serve_stats s{};
  CHECK(dop_serve_stats_get(srv, &s) == DOP_OK);
  CHECK(s.submitted == (uint64_t)kThreads * kPer && s.completed == s.submitted);
  CHECK(s.failed == 0 && s.queued == 0 && s.running == 0);
  CHECK(s.p50_ms <= s.p99_ms && s.arena_peak <= arena);
  CHECK(dop_serve_destroy(srv) == DOP_OK);
}

static void scenario_errors() {
  dop_server *srv = nullptr;
  CHECK(dop_serve_create_mock(reinterpret_cast<void *>(256), field_bytes(256), 2, 1.0, &srv) ==
        DOP_OK);
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) {
    th.emplace_back([&] {
      for (int i = 0; i < 200; ++i) {
        const dop_problem big = make_problem(512, 1);  // never fits the arena
        uint64_t tk = 0;
        CHECK(dop_serve_submit(srv, &big, reinterpret_cast<const float *>(4096), nullptr,
                               reinterpret_cast<float *>(8192), &tk) == DOP_ERR_BUDGET);
        dop_problem bad = make_problem(256, 1);
        bad.n_lambda = 0;
        CHECK(dop_serve_submit(srv, &bad, reinterpret_cast<const float *>(4096), nullptr,
                               reinterpret_cast<float *>(8192), &tk) == DOP_ERR_INVALID_ARG);
        CHECK(dop_serve_poll(srv, 1u << 30) == DOP_ERR_NOT_FOUND);
        const dop_problem ok = make_problem(256, 2);
        CHECK(dop_serve_submit(srv, &ok, reinterpret_cast<const float *>(4096), nullptr,
                               reinterpret_cast<float *>(8192), &tk) == DOP_OK);
        CHECK(dop_serve_wait(srv, tk, 30.0) == DOP_OK);
      }
    });
  }
  for (auto &t : th) t.join();
  CHECK(dop_serve_destroy(srv) == DOP_OK);
}

static void scenario_shutdown() {
  for (int round = 0; round < 20; ++round) {
    dop_server *srv = nullptr;
    // 1 slot, slow service: most requests are still queued at shutdown
    CHECK(dop_serve_create_mock(reinterpret_cast<void *>(256), field_bytes(1024), 1, 500.0,
                                &srv) == DOP_OK);
    std::vector<uint64_t> tk(16);
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t) {
      th.emplace_back([&, t] {
        for (int i = 0; i < 4; ++i) {
          const dop_problem p = make_problem(1024, 1);
          CHECK(dop_serve_submit(srv, &p, reinterpret_cast<const float *>(4096), nullptr,
                                 reinterpret_cast<float *>(8192), &tk[4 * t + i]) == DOP_OK);
        }
      });
    }
    for (auto &t : th) t.join();
    const dop_status first = dop_serve_wait(srv, tk[0], 0.0);
    CHECK(first == DOP_OK || first == DOP_ERR_TIMEOUT);
    CHECK(dop_serve_destroy(srv) == DOP_OK);
  }
}

int main() {
  scenario_concurrent();
  scenario_errors();
  scenario_shutdown();
  std::printf("serve stress: ok\n");
  return 0;
}
