// host_checks.cpp -- host-side checks of the library built with a plain C++
// compiler (no device): the planner's scheduler against fake executors, and
// the host functions (argument checks, pair counts, plate inverses, the
// perturbation sampler). Built and run by tests/test_host_sanitizers.py under
// AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer.
// Prints "ok <check>" per check and "ALL OK" at the end; exits 1 on failure.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host_common.h"
#include "planner_core.h"

namespace {

#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      std::exit(1);                                                         \
    }                                                                       \
  } while (0)

using Clock = std::chrono::steady_clock;

// A request of the fake service: its work takes `work_us` of simulated device
// time; its result is a pure function of its inputs.
struct FakeJob : vpm::Job {
  int a = 0, b = 0;
  int work_us = 0;
  bool fail_launch = false, fail_query = false;
  long result = 0;
  std::atomic<int> *released = nullptr;
};

// Simulated device: a launch arms the slot's deadline; query reports done
// once it has passed. Tracks the largest number of slots busy at once.
class FakeExec : public vpm::Executor {
 public:
  explicit FakeExec(int n_slots) : slots_(static_cast<size_t>(n_slots)) {}
  int launch(int slot, vpm::Job &job) override {
    auto &f = static_cast<FakeJob &>(job);
    if (f.fail_launch) return VPM_EDEVICE;
    Slot &s = slots_[slot];
    CHECK(!s.busy);  // the scheduler never launches on a busy slot
    s.busy = true;
    s.deadline = Clock::now() + std::chrono::microseconds(f.work_us);
    s.inputs[0] = f.a;
    s.inputs[1] = f.b;
    const int now_busy = ++busy_;
    int prev = max_busy_.load();
    while (now_busy > prev && !max_busy_.compare_exchange_weak(prev, now_busy)) {
    }
    return VPM_OK;
  }
  int query(int slot) override {
    Slot &s = slots_[slot];
    CHECK(s.busy);
    if (Clock::now() < s.deadline) return VPM_PENDING;
    s.busy = false;
    --busy_;
    return s.fail_next ? VPM_EDEVICE : VPM_OK;
  }
  int collect(int slot, vpm::Job &job) override {
    auto &f = static_cast<FakeJob &>(job);
    const Slot &s = slots_[slot];
    f.result = 1000L * s.inputs[0] + s.inputs[1];
    return VPM_OK;
  }
  void release(vpm::Job &job) override {
    auto &f = static_cast<FakeJob &>(job);
    if (f.released) ++*f.released;
  }
  // query() of the job launched next on any slot fails (set before submit)
  void arm_query_failure(int slot) { slots_[slot].fail_next = true; }
  int max_busy() const { return max_busy_.load(); }

 private:
  struct Slot {
    bool busy = false, fail_next = false;
    Clock::time_point deadline;
    int inputs[2] = {0, 0};
  };
  std::vector<Slot> slots_;
  std::atomic<int> busy_{0}, max_busy_{0};
};

std::unique_ptr<FakeJob> make_job(vpm::Scheduler &s, int a, int b, int work_us, size_t fp,
                                  std::atomic<int> *released = nullptr) {
  auto j = std::make_unique<FakeJob>();
  j->a = a;
  j->b = b;
  j->work_us = work_us;
  j->footprint = fp;
  j->released = released;
  j->t_arrive = s.now_us();
  return j;
}

std::unique_ptr<FakeJob> take(vpm::Scheduler &s, uint64_t t) {
  std::unique_ptr<vpm::Job> j;
  CHECK(s.poll(t, &j, -1) == VPM_OK);
  return std::unique_ptr<FakeJob>(static_cast<FakeJob *>(j.release()));
}

// Results are the same served one at a time and concurrently; with several
// slots, work overlaps; every job's timestamps are ordered.
void check_serial_and_concurrent() {
  std::vector<long> serial, concurrent;
  int overlap_1 = 0, overlap_4 = 0;
  for (int slots : {1, 4}) {
    FakeExec ex(slots);
    std::atomic<int> released{0};
    std::vector<uint64_t> tickets;
    std::vector<std::pair<double, double>> iv;
    {
      vpm::Scheduler s(slots, 1 << 30, &ex);
      for (int i = 0; i < 12; ++i) {
        uint64_t t = 0;
        CHECK(s.submit(make_job(s, i, 7 * i % 5, 2000 + 500 * (i % 3), 1000, &released), &t) ==
              VPM_OK);
        tickets.push_back(t);
      }
      for (uint64_t t : tickets) {
        auto j = take(s, t);
        CHECK(j->status == VPM_OK);
        CHECK(j->t_arrive <= j->t_admit && j->t_admit <= j->t_done);
        (slots == 1 ? serial : concurrent).push_back(j->result);
        iv.push_back({j->t_admit, j->t_done});
      }
    }
    CHECK(released.load() == 12);
    std::sort(iv.begin(), iv.end());
    int ov = 0;
    for (size_t i = 0; i + 1 < iv.size(); ++i) ov += iv[i + 1].first < iv[i].second;
    (slots == 1 ? overlap_1 : overlap_4) = ov;
    CHECK(ex.max_busy() <= slots);
    if (slots == 4) CHECK(ex.max_busy() >= 2);
  }
  CHECK(serial == concurrent);
  CHECK(overlap_1 == 0 && overlap_4 > 0);
  for (int i = 0; i < 12; ++i) CHECK(serial[i] == 1000L * i + 7 * i % 5);
  std::puts("ok serial_and_concurrent");
}

// A budget that holds one job at a time admits them one by one; a job larger
// than the budget is refused before it queues.
void check_budget() {
  FakeExec ex(4);
  vpm::Scheduler s(4, 1500, &ex);
  std::vector<uint64_t> t(6);
  for (int i = 0; i < 6; ++i) CHECK(s.submit(make_job(s, i, 0, 1500, 1000), &t[i]) == VPM_OK);
  std::vector<std::pair<double, double>> iv;
  for (uint64_t x : t) {
    auto j = take(s, x);
    iv.push_back({j->t_admit, j->t_done});
  }
  std::sort(iv.begin(), iv.end());
  for (size_t i = 0; i + 1 < iv.size(); ++i) CHECK(iv[i + 1].first >= iv[i].second);
  CHECK(ex.max_busy() == 1);
  uint64_t big = 0;
  CHECK(s.submit(make_job(s, 0, 0, 10, 1501), &big) == VPM_EBUDGET);
  std::puts("ok budget");
}

// Tickets: pending with a zero timeout while queued or running, returned
// once, unknown afterwards; unknown tickets are reported.
void check_ticket_life_cycle() {
  FakeExec ex(1);
  vpm::Scheduler s(1, 1 << 20, &ex);
  uint64_t t1 = 0, t2 = 0;
  CHECK(s.submit(make_job(s, 1, 1, 30000, 10), &t1) == VPM_OK);
  CHECK(s.submit(make_job(s, 2, 2, 1000, 10), &t2) == VPM_OK);
  std::unique_ptr<vpm::Job> j;
  CHECK(s.poll(t2, &j, 0) == VPM_PENDING);  // queued behind t1
  CHECK(s.poll(t1, &j, 100) == VPM_PENDING);
  CHECK(s.poll(t1, &j, -1) == VPM_OK && j && j->status == VPM_OK);
  CHECK(s.poll(t1, &j, 0) == VPM_ENOTFOUND);
  CHECK(s.poll(t2, &j, -1) == VPM_OK);
  CHECK(s.poll(999, &j, 0) == VPM_ENOTFOUND);
  std::puts("ok ticket_life_cycle");
}

// p50 / p99 bookkeeping: latencies from the job timestamps of a serial
// service with equal jobs grow with queue position.
void check_latency_bookkeeping() {
  FakeExec ex(1);
  std::vector<double> lat;
  {
    vpm::Scheduler s(1, 1 << 20, &ex);
    std::vector<uint64_t> t(8);
    for (int i = 0; i < 8; ++i) CHECK(s.submit(make_job(s, i, 0, 2000, 1), &t[i]) == VPM_OK);
    for (uint64_t x : t) {
      auto j = take(s, x);
      lat.push_back(j->t_done - j->t_arrive);
    }
  }
  for (size_t i = 0; i + 1 < lat.size(); ++i) CHECK(lat[i + 1] > lat[i]);
  CHECK(lat.back() >= 8 * 2000.0 * 0.9);  // the last waited for all the others
  std::vector<double> sorted = lat;
  std::sort(sorted.begin(), sorted.end());
  const double p50 = sorted[sorted.size() / 2], p99 = sorted.back();
  CHECK(p50 < p99);
  std::puts("ok latency_bookkeeping");
}

// A failing executor fails only the affected jobs; the slot is reused and
// the others complete.
void check_failing_executor() {
  FakeExec ex(2);
  std::atomic<int> released{0};
  {
    vpm::Scheduler s(2, 1 << 20, &ex);
    std::vector<uint64_t> t(6);
    for (int i = 0; i < 6; ++i) {
      auto j = make_job(s, i, 0, 500, 1, &released);
      j->fail_launch = (i == 1 || i == 4);
      CHECK(s.submit(std::move(j), &t[i]) == VPM_OK);
    }
    for (int i = 0; i < 6; ++i) {
      auto j = take(s, t[i]);
      CHECK(j->status == ((i == 1 || i == 4) ? VPM_EDEVICE : VPM_OK));
      if (j->status == VPM_OK) CHECK(j->result == 1000L * i);
    }
    // a completion that reports a device error
    ex.arm_query_failure(0);
    ex.arm_query_failure(1);
    uint64_t bad = 0;
    CHECK(s.submit(make_job(s, 9, 9, 200, 1, &released), &bad) == VPM_OK);
    auto j = take(s, bad);
    CHECK(j->status == VPM_EDEVICE);
  }
  CHECK(released.load() == 7);
  std::puts("ok failing_executor");
}

// Several client threads submit and poll at once (the thread sanitizer's
// case); a set-up call runs only when the service is idle.
void check_concurrent_clients() {
  FakeExec ex(4);
  std::atomic<int> released{0};
  std::atomic<long> sum{0};
  {
    vpm::Scheduler s(4, 1 << 20, &ex);
    bool ran = s.when_idle([] {});
    CHECK(ran);
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c)
      clients.emplace_back([&, c] {
        for (int i = 0; i < 10; ++i) {
          uint64_t t = 0;
          CHECK(s.submit(make_job(s, c, i, 100 + 50 * ((c + i) % 4), 10, &released), &t) ==
                VPM_OK);
          std::unique_ptr<vpm::Job> j;
          int rc;
          while ((rc = s.poll(t, &j, 200)) == VPM_PENDING) {
          }
          CHECK(rc == VPM_OK && j->status == VPM_OK);
          sum += static_cast<FakeJob &>(*j).result;
        }
      });
    // a busy service refuses the set-up call (it may also find it idle)
    (void)s.when_idle([] {});
    for (auto &th : clients) th.join();
    CHECK(s.when_idle([] {}));
  }
  long want = 0;
  for (int c = 0; c < 4; ++c)
    for (int i = 0; i < 10; ++i) want += 1000L * c + i;
  CHECK(sum.load() == want && released.load() == 40);
  std::puts("ok concurrent_clients");
}

// Host functions of the library.
void check_host_functions() {
  // plate inverses of every size and mode: A^-1 A = I is checked by the
  // oracle tests; here the sizes and the absence of memory errors
  for (int nb = 1; nb <= 64; ++nb)
    for (int mode : {VPM_SHED_BOTH, VPM_SHED_TE, VPM_SHED_NONE}) {
      if (mode == VPM_SHED_NONE && nb < 2) continue;
      std::vector<double> inv;
      CHECK(vpm::plate_inverse_T(nb, 0.3, 0.02, 0.01, mode, inv) == VPM_OK);
      const size_t S = vpm::system_size(nb, mode);
      CHECK(inv.size() == S * S);
      for (double v : inv) CHECK(std::isfinite(v));
    }
  // sampler: odd sizes, tails of the 4-step blocks
  for (int H : {1, 2, 3, 5, 8, 203}) {
    std::vector<double> e(static_cast<size_t>(3) * H, -7.0);
    CHECK(vpm_sample_eps(42, 1, 3, H, 0.15, e.data()) == VPM_OK);
    for (double v : e) CHECK(std::isfinite(v) && v != -7.0);
  }
  CHECK(vpm_sample_eps(1, 0, 0, 1, 0.1, nullptr) == VPM_EINVAL);
  // argument checks
  vpm_params p{};
  CHECK(vpm_validate_batch(nullptr, nullptr, nullptr) == VPM_EINVAL);
  CHECK(std::strlen(vpm_last_error()) > 0);
  p.n_bound = 32;
  p.chord = 0.3;
  p.shed_frac = 0.02;
  p.r_core = 0.01;
  p.mass = 0.12;
  p.inertia = 0.002;
  CHECK(vpm::check_params(&p) == VPM_OK);
  vpm_batch_in in{};
  vpm_batch_out out{};
  CHECK(vpm_validate_batch(&p, &in, &out) == VPM_EINVAL);  // K = 0
  p.n_bound = 65;
  CHECK(vpm::check_params(&p) == VPM_EINVAL);
  // pair counts: one step of an empty wake sheds two vortices
  CHECK(vpm_pair_count(0, 1, 32, 0) == 2 * 1 + 2 * 32);
  CHECK(vpm_pair_count(10, 3, 16, 12) > 0);
  std::puts("ok host_functions");
}

}  // namespace

int main() {
  check_host_functions();
  check_serial_and_concurrent();
  check_budget();
  check_ticket_life_cycle();
  check_latency_bookkeeping();
  check_failing_executor();
  check_concurrent_clients();
  std::puts("ALL OK");
  return 0;
}
