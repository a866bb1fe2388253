// planner_core.h -- admission and slot scheduling of the replanning service,
// with no device API in it: the device work is behind the Executor interface,
// so the same scheduler runs the HIP executor in the library and fake
// executors in host tests (including thread-sanitizer builds).
//
// Requests wait in arrival order. One worker thread admits the oldest while a
// slot is free and the sum of the in-flight footprints stays within the
// budget (a request that arrives to an idle service is admitted whatever its
// size; requests larger than the budget are refused before they queue),
// launches it on that slot, and watches the slots for completion. Executor
// calls are made without the scheduler's lock, so submissions and polls never
// wait on device work.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "vpm.h"

namespace vpm {

enum class JobState { kPending, kRunning, kDone };

// A request as the scheduler sees it; executors derive their payload.
struct Job {
  uint64_t ticket = 0;
  size_t footprint = 0;
  JobState st = JobState::kPending;
  int status = VPM_OK;
  int slot = -1;
  double t_arrive = 0, t_admit = 0, t_done = 0;  // us since the scheduler started
  virtual ~Job() = default;
};

// The device side. Only the scheduler's worker thread calls launch, query and
// collect, one slot at a time, never with the scheduler's lock held;
// release is called with the lock held, once per admitted or failed job.
class Executor {
 public:
  virtual ~Executor() = default;
  // Enqueue `job` on slot `slot`; VPM_OK or an error (the job then fails and
  // the slot must be reusable on return).
  virtual int launch(int slot, Job &job) = 0;
  // VPM_PENDING while the slot's work runs, VPM_OK when it has finished, or
  // an error.
  virtual int query(int slot) = 0;
  // Move the finished results of the slot into `job`; VPM_OK or an error.
  virtual int collect(int slot, Job &job) = 0;
  // The job has finished with job.status (called for every job that reaches
  // the worker or fails in it, before a poll can return it).
  virtual void release(Job &job) { (void)job; }
};

class Scheduler {
 public:
  Scheduler(int n_slots, size_t budget, Executor *ex)
      : n_slots_(n_slots), budget_(budget), ex_(ex), t0_(std::chrono::steady_clock::now()),
        slot_job_(static_cast<size_t>(n_slots), nullptr) {
    worker_ = std::thread([this] { loop(); });
  }
  Scheduler(const Scheduler &) = delete;
  Scheduler &operator=(const Scheduler &) = delete;
  // Waits for every queued and running job, then stops the worker.
  ~Scheduler() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
  }

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0_)
        .count();
  }
  size_t budget() const { return budget_; }
  int n_slots() const { return n_slots_; }

  // Queue a job whose t_arrive and footprint are set and return its ticket
  // in *ticket: VPM_OK, or VPM_EBUDGET (job not queued) if its footprint
  // alone exceeds the budget.
  int submit(std::unique_ptr<Job> job, uint64_t *ticket) {
    if (job->footprint > budget_) return VPM_EBUDGET;
    std::lock_guard<std::mutex> lk(mu_);
    job->ticket = next_ticket_++;
    job->st = JobState::kPending;
    Job *raw = job.get();
    *ticket = raw->ticket;
    jobs_[raw->ticket] = std::move(job);
    pending_.push_back(raw);
    cv_.notify_all();
    return VPM_OK;
  }

  // Wait up to timeout_us (0: do not wait, < 0: forever). VPM_PENDING, or
  // VPM_OK with the finished job moved to *out (the ticket is released), or
  // VPM_ENOTFOUND.
  int poll(uint64_t ticket, std::unique_ptr<Job> *out, int timeout_us) {
    std::unique_lock<std::mutex> lk(mu_);
    // looked up afresh on every wake-up: another poll of the same ticket may
    // have taken the job meanwhile
    auto done = [&] {
      auto f = jobs_.find(ticket);
      return f == jobs_.end() || f->second->st == JobState::kDone;
    };
    if (jobs_.find(ticket) == jobs_.end()) return VPM_ENOTFOUND;
    if (!done()) {
      if (timeout_us == 0) return VPM_PENDING;
      if (timeout_us < 0) {
        cv_.wait(lk, done);
      } else if (!cv_.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return VPM_PENDING;
      }
    }
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return VPM_ENOTFOUND;
    *out = std::move(it->second);
    jobs_.erase(it);
    return VPM_OK;
  }

  // Run fn() while no job is queued or running and none can be admitted;
  // returns false (fn not run) if the service is busy.
  template <typename Fn>
  bool when_idle(Fn fn) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!pending_.empty() || in_flight_ > 0 || launching_) return false;
    fn();
    return true;
  }

 private:
  void finish(Job *j, int status) {
    j->status = status;
    j->t_done = now_us();
    ex_->release(*j);
    j->st = JobState::kDone;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      bool progress = false;
      for (int i = 0; i < n_slots_; ++i) {
        Job *j = slot_job_[i];
        if (!j) continue;
        lk.unlock();
        int q = ex_->query(i);
        if (q == VPM_OK) q = ex_->collect(i, *j);
        lk.lock();
        if (q == VPM_PENDING) continue;
        finish(j, q);
        slot_job_[i] = nullptr;
        in_flight_--;
        in_flight_bytes_ -= j->footprint;
        progress = true;
      }
      while (!pending_.empty()) {
        Job *j = pending_.front();
        int free_slot = -1;
        for (int i = 0; i < n_slots_ && free_slot < 0; ++i)
          if (!slot_job_[i]) free_slot = i;
        if (free_slot < 0) break;
        if (in_flight_ > 0 && in_flight_bytes_ + j->footprint > budget_) break;
        pending_.pop_front();
        slot_job_[free_slot] = j;
        in_flight_++;
        in_flight_bytes_ += j->footprint;
        j->slot = free_slot;
        j->st = JobState::kRunning;
        j->t_admit = now_us();
        launching_ = true;
        lk.unlock();
        const int rc = ex_->launch(free_slot, *j);
        lk.lock();
        launching_ = false;
        if (rc != VPM_OK) {
          finish(j, rc);
          slot_job_[free_slot] = nullptr;
          in_flight_--;
          in_flight_bytes_ -= j->footprint;
        }
        progress = true;
      }
      if (progress) cv_.notify_all();
      if (stop_ && pending_.empty() && in_flight_ == 0) break;
      if (!progress)
        cv_.wait_for(lk, in_flight_ > 0 ? std::chrono::microseconds(50)
                                         : std::chrono::microseconds(5000));
    }
  }

  const int n_slots_;
  const size_t budget_;
  Executor *const ex_;
  const std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  bool launching_ = false;
  uint64_t next_ticket_ = 1;
  std::map<uint64_t, std::unique_ptr<Job>> jobs_;
  std::deque<Job *> pending_;
  std::vector<Job *> slot_job_;  // worker thread only (and after join)
  int in_flight_ = 0;
  size_t in_flight_bytes_ = 0;
  std::thread worker_;
};

}  // namespace vpm
