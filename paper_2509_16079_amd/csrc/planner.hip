// planner.hip -- replanning service over the rollout engine.
//
// Resident states (wake + glider) live in device memory. A scheduler thread
// admits queued requests in arrival order while a slot is free and the
// in-flight footprint fits the HBM budget; each admitted request runs on its
// slot's own context and stream (inputs from pinned staging, the rollout
// batch, the MPPI update, results back to pinned memory), so requests that
// arrive while others are on the GPU overlap with them. Completion is
// detected with events; planner_poll hands results to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "vpm_internal.h"

namespace vpm {
namespace {

constexpr int kMaxSlots = 16;

__global__ void broadcast_state_kernel(int K, int nb, const double *__restrict__ g7,
                                       const double *__restrict__ gb,
                                       double *__restrict__ g0,
                                       double *__restrict__ gb0,
                                       int32_t *__restrict__ field_of) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  for (int i = 0; i < 7; ++i) g0[(size_t)k * 7 + i] = g7[i];
  for (int j = 0; j < nb; ++j) gb0[(size_t)k * nb + j] = gb[j];
  field_of[k] = 0;
}

struct State {
  int n = 0, nb = 0;
  double *wx = nullptr, *wz = nullptr, *wg = nullptr;  // device
  int64_t *field_off = nullptr;                        // device [2]
  double *g7 = nullptr, *gb = nullptr;                 // device
  int refs = 0;
};

enum class ReqState { kPending, kRunning, kDone };

struct Request {
  uint64_t ticket = 0, state_id = 0;
  vpm_params params{};
  int K = 0, H = 0, iters = 1;
  double dt = 0, lambda = 1;
  double x_goal[7]{}, q_diag[7]{};
  std::vector<double> u_mean, u_eps;  // host copies
  size_t footprint = 0;
  ReqState st = ReqState::kPending;
  int status = VPM_OK;
  int slot = -1;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  // results
  std::vector<double> u_new, w, cost, g_final;
  int argmin = -1;
  double jmin = 0;
  int64_t pairs = 0;
};

// Device and pinned buffers of a slot, grown when a request needs more.
struct Slot {
  vpm_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Request *req = nullptr;
  size_t cap_kh = 0, cap_k = 0, cap_h = 0, cap_kb = 0;
  double *d_u_eps = nullptr, *d_u_mean = nullptr, *d_g0 = nullptr, *d_gb0 = nullptr;
  double *d_g_final = nullptr, *d_cost = nullptr, *d_w = nullptr, *d_u_new = nullptr;
  double *d_jmin = nullptr;
  int32_t *d_field_of = nullptr, *d_status = nullptr, *d_argmin = nullptr;
  int64_t *d_pairs = nullptr;
  double *h_in = nullptr;   // pinned staging: u_eps then u_mean
  double *h_out = nullptr;  // pinned results: cost, w, g_final, u_new, jmin
  int64_t *h_pairs = nullptr;
  int32_t *h_argmin = nullptr;
};

}  // namespace
}  // namespace vpm

struct planner {
  int device = 0;
  int n_slots = 1;
  size_t budget = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1, next_state = 1;
  std::map<uint64_t, vpm::State> states;
  std::map<uint64_t, std::unique_ptr<vpm::Request>> reqs;
  std::deque<vpm::Request *> pending;
  size_t in_flight_bytes = 0;
  int in_flight = 0;
  vpm::Slot slots[vpm::kMaxSlots];
  std::thread worker;
};

namespace vpm {
namespace {

double now_us(const planner *p) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - p->t0)
      .count();
}

template <typename T>
int grow(T **ptr, size_t have, size_t need) {
  if (have >= need && *ptr) return VPM_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(ptr), need * sizeof(T)) != hipSuccess)
    return VPM_ENOMEM;
  return VPM_OK;
}

template <typename T>
int grow_pinned(T **ptr, size_t have, size_t need) {
  if (have >= need && *ptr) return VPM_OK;
  if (*ptr) (void)hipHostFree(*ptr);
  *ptr = nullptr;
  if (hipHostMalloc(reinterpret_cast<void **>(ptr), need * sizeof(T), hipHostMallocDefault) !=
      hipSuccess)
    return VPM_ENOMEM;
  return VPM_OK;
}

// Make the slot's buffers hold a request of `iters` K x H perturbation sets
// with nb bound vortices (capacities grow by at least 1.5x so a stream of
// varied requests settles).
int reserve(Slot &s, size_t K, size_t H, size_t nb, size_t iters) {
  const size_t kh = K * H * iters;
  if (kh <= s.cap_kh && K <= s.cap_k && H <= s.cap_h && K * nb <= s.cap_kb && s.h_in)
    return VPM_OK;
  if (hipStreamSynchronize(s.stream) != hipSuccess) return VPM_EDEVICE;
  auto up = [](size_t have, size_t need) { return std::max(need, have + have / 2); };
  int rc = VPM_OK;
  if (kh > s.cap_kh) {
    s.cap_kh = up(s.cap_kh, kh);
    rc |= grow(&s.d_u_eps, 0, s.cap_kh);
  }
  if (H > s.cap_h) {
    s.cap_h = up(s.cap_h, H);
    rc |= grow(&s.d_u_mean, 0, s.cap_h);
    rc |= grow(&s.d_u_new, 0, s.cap_h);
  }
  if (K > s.cap_k) {
    s.cap_k = up(s.cap_k, K);
    rc |= grow(&s.d_g0, 0, 7 * s.cap_k);
    rc |= grow(&s.d_g_final, 0, 7 * s.cap_k);
    rc |= grow(&s.d_cost, 0, s.cap_k);
    rc |= grow(&s.d_w, 0, s.cap_k);
    rc |= grow(&s.d_field_of, 0, s.cap_k);
    rc |= grow(&s.d_status, 0, s.cap_k);
    rc |= grow(&s.d_pairs, 0, s.cap_k);
  }
  if (K * nb > s.cap_kb) {
    s.cap_kb = up(s.cap_kb, K * nb);
    rc |= grow(&s.d_gb0, 0, s.cap_kb);
  }
  // pinned staging: u_eps then u_mean in; cost, w, g_final, u_new, jmin out
  rc |= grow_pinned(&s.h_in, 0, s.cap_kh + s.cap_h);
  rc |= grow_pinned(&s.h_out, 0, 9 * s.cap_k + s.cap_h + 1);
  rc |= grow_pinned(&s.h_pairs, 0, s.cap_k);
  if (!s.d_jmin) rc |= grow(&s.d_jmin, 0, 1);
  if (!s.d_argmin) rc |= grow(&s.d_argmin, 0, 1);
  if (!s.h_argmin) rc |= grow_pinned(&s.h_argmin, 0, 1);
  return rc ? VPM_ENOMEM : VPM_OK;
}

void finish_request(planner *p, Request *r, int status) {
  r->status = status;
  r->t_done = now_us(p);
  r->st = ReqState::kDone;
  auto it = p->states.find(r->state_id);
  if (it != p->states.end()) it->second.refs--;
}

// Enqueue request r on slot s (called with the planner lock held).
int launch(planner *p, Slot &s, Request *r) {
  const State &st = p->states.at(r->state_id);
  const size_t K = r->K, H = r->H, nb = st.nb, it_n = r->iters;
  int rc = reserve(s, K, H, nb, it_n);
  if (rc != VPM_OK) return fail(rc, "planner slot allocation failed");
  const size_t kh = K * H * it_n;
  std::memcpy(s.h_in, r->u_eps.data(), kh * sizeof(double));
  std::memcpy(s.h_in + kh, r->u_mean.data(), H * sizeof(double));
  VPM_HIP_TRY(hipMemcpyAsync(s.d_u_eps, s.h_in, kh * sizeof(double), hipMemcpyHostToDevice,
                             s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(s.d_u_mean, s.h_in + kh, H * sizeof(double),
                             hipMemcpyHostToDevice, s.stream));
  hipLaunchKernelGGL(broadcast_state_kernel, dim3((K + 255) / 256), dim3(256), 0, s.stream,
                     r->K, st.nb, st.g7, st.gb, s.d_g0, s.d_gb0, s.d_field_of);
  VPM_HIP_TRY(hipGetLastError());
  vpm_batch_in in{};
  in.K = r->K;
  in.H = r->H;
  in.dt = r->dt;
  in.n_fields = 1;
  in.max_wake0 = st.n;
  in.n_pairs = 0;
  in.g0 = s.d_g0;
  in.gb0 = s.d_gb0;
  in.field_off = st.field_off;
  in.field_of = s.d_field_of;
  in.wx = st.wx;
  in.wz = st.wz;
  in.wg = st.wg;
  std::memcpy(in.x_goal, r->x_goal, sizeof(in.x_goal));
  std::memcpy(in.q_diag, r->q_diag, sizeof(in.q_diag));
  vpm_batch_out out{};
  out.g_final = s.d_g_final;
  out.cost = s.d_cost;
  out.status = s.d_status;
  out.pair_count = s.d_pairs;
  // MPPI iterations (Sec. IV-A): each rolls the same initial state out under
  // its own perturbations around the previous iteration's update; the mean
  // alternates between the two device buffers
  double *mean = s.d_u_mean, *next = s.d_u_new;
  for (size_t i = 0; i < it_n; ++i) {
    in.u_mean = mean;
    in.u_eps = s.d_u_eps + i * K * H;
    rc = vpm_rollout_batch(s.ctx, &r->params, &in, &out, s.stream);
    if (rc != VPM_OK) return rc;
    rc = mppi_weights(s.ctx, r->K, r->H, s.d_cost, r->lambda, mean, in.u_eps, s.d_w, next,
                      s.d_argmin, s.d_jmin, s.stream);
    if (rc != VPM_OK) return rc;
    std::swap(mean, next);
  }
  double *h = s.h_out;
  VPM_HIP_TRY(hipMemcpyAsync(h, s.d_cost, K * 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(h + K, s.d_w, K * 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(h + 2 * K, s.d_g_final, 7 * K * 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(h + 9 * K, mean, H * 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(h + 9 * K + H, s.d_jmin, 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(s.h_argmin, s.d_argmin, 4, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(s.h_pairs, s.d_pairs, K * 8, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipEventRecord(s.done, s.stream));
  return VPM_OK;
}

void collect(planner *p, Slot &s) {
  Request *r = s.req;
  const size_t K = r->K, H = r->H;
  const double *h = s.h_out;
  r->cost.assign(h, h + K);
  r->w.assign(h + K, h + 2 * K);
  r->g_final.assign(h + 2 * K, h + 9 * K);
  r->u_new.assign(h + 9 * K, h + 9 * K + H);
  r->jmin = h[9 * K + H];
  r->argmin = *s.h_argmin;
  r->pairs = 0;
  for (size_t k = 0; k < K; ++k) r->pairs += s.h_pairs[k];
  r->pairs *= r->iters;  // the wake-count schedule, so the work, is the same each iteration
}

void worker_loop(planner *p) {
  (void)hipSetDevice(p->device);
  std::unique_lock<std::mutex> lock(p->mu);
  for (;;) {
    bool progress = false;
    for (int i = 0; i < p->n_slots; ++i) {
      Slot &s = p->slots[i];
      if (!s.req) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      Request *r = s.req;
      if (q == hipSuccess) collect(p, s);
      finish_request(p, r, q == hipSuccess ? VPM_OK : VPM_EDEVICE);
      p->in_flight_bytes -= r->footprint;
      p->in_flight--;
      s.req = nullptr;
      progress = true;
    }
    while (!p->pending.empty()) {
      Request *r = p->pending.front();
      int free_slot = -1;
      for (int i = 0; i < p->n_slots; ++i)
        if (!p->slots[i].req) {
          free_slot = i;
          break;
        }
      if (free_slot < 0) break;
      if (p->in_flight > 0 && p->in_flight_bytes + r->footprint > p->budget) break;
      p->pending.pop_front();
      Slot &s = p->slots[free_slot];
      r->t_admit = now_us(p);
      r->st = ReqState::kRunning;
      r->slot = free_slot;
      const int rc = launch(p, s, r);
      if (rc != VPM_OK) {
        finish_request(p, r, rc);
      } else {
        s.req = r;
        p->in_flight_bytes += r->footprint;
        p->in_flight++;
      }
      progress = true;
    }
    if (progress) p->cv.notify_all();
    if (p->stop && p->pending.empty() && p->in_flight == 0) break;
    if (!progress) {
      if (p->in_flight > 0)
        p->cv.wait_for(lock, std::chrono::microseconds(50));
      else
        p->cv.wait_for(lock, std::chrono::milliseconds(5));
    }
  }
}

void free_slot(Slot &s) {
  (void)hipFree(s.d_u_eps);
  (void)hipFree(s.d_u_mean);
  (void)hipFree(s.d_g0);
  (void)hipFree(s.d_gb0);
  (void)hipFree(s.d_g_final);
  (void)hipFree(s.d_cost);
  (void)hipFree(s.d_w);
  (void)hipFree(s.d_u_new);
  (void)hipFree(s.d_jmin);
  (void)hipFree(s.d_field_of);
  (void)hipFree(s.d_status);
  (void)hipFree(s.d_argmin);
  (void)hipFree(s.d_pairs);
  (void)hipHostFree(s.h_in);
  (void)hipHostFree(s.h_out);
  (void)hipHostFree(s.h_pairs);
  (void)hipHostFree(s.h_argmin);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.ctx) vpm_destroy(s.ctx);
  s = Slot{};
}

void free_state(State &st) {
  (void)hipFree(st.wx);
  (void)hipFree(st.wz);
  (void)hipFree(st.wg);
  (void)hipFree(st.field_off);
  (void)hipFree(st.g7);
  (void)hipFree(st.gb);
}

}  // namespace
}  // namespace vpm

using vpm::fail;

extern "C" {

VPM_API size_t planner_footprint(int32_t K, int32_t H, int32_t n0, int32_t n_bound,
                                 int32_t iterations) {
  const size_t k = K > 0 ? K : 0, h = H > 0 ? H : 0, nb = n_bound > 0 ? n_bound : 0;
  const size_t it = iterations > 0 ? iterations : 1;
  size_t bytes = 8 * (it * k * h + 2 * h + 7 * k + k * nb + 7 * k + 3 * k + 1) + 4 * (2 * k + 1);
  // wakes beyond the LDS-resident kernel take a streaming workspace of
  // 24 B per vortex of capacity for each of the GPU's 256 CUs
  const size_t cap = (size_t)(n0 > 0 ? n0 : 0) + 2 * h;
  if (cap > (size_t)vpm::lds_resident_capacity(n_bound > 0 ? n_bound : 1))
    bytes += 256 * cap * 24;
  return bytes;
}

VPM_API int planner_create(planner **out, const planner_opts *opts) {
  if (!out || !opts) return fail(VPM_EINVAL, "out or opts is NULL");
  *out = nullptr;
  if (opts->max_slots < 1 || opts->max_slots > vpm::kMaxSlots)
    return fail(VPM_EINVAL, "max_slots must be in 1..16");
  if (opts->hbm_budget_bytes == 0) return fail(VPM_EINVAL, "budget must be > 0");
  auto *p = new (std::nothrow) planner();
  if (!p) return fail(VPM_ENOMEM, "planner allocation failed");
  p->device = opts->device;
  p->n_slots = opts->max_slots;
  p->budget = opts->hbm_budget_bytes;
  p->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < p->n_slots; ++i) {
    vpm::Slot &s = p->slots[i];
    int rc = vpm_create(&s.ctx, opts->device);
    if (rc == VPM_OK &&
        (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess))
      rc = VPM_EDEVICE;
    if (rc != VPM_OK) {
      for (int j = 0; j <= i; ++j) vpm::free_slot(p->slots[j]);
      delete p;
      return fail(rc, "planner slot creation failed");
    }
  }
  p->worker = std::thread(vpm::worker_loop, p);
  *out = p;
  return VPM_OK;
}

VPM_API void planner_destroy(planner *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lock(p->mu);
    p->stop = true;
  }
  p->cv.notify_all();
  if (p->worker.joinable()) p->worker.join();
  (void)hipSetDevice(p->device);
  for (int i = 0; i < p->n_slots; ++i) vpm::free_slot(p->slots[i]);
  for (auto &kv : p->states) vpm::free_state(kv.second);
  delete p;
}

VPM_API int planner_state_put(planner *p, int32_t n, const double *wx, const double *wz,
                              const double *wg, const double *g7, int32_t n_bound,
                              const double *gb, uint64_t *state_id) {
  if (!p || !state_id || !g7 || (n > 0 && (!wx || !wz || !wg)) || n < 0)
    return fail(VPM_EINVAL, "bad state arguments");
  if (n_bound < 1 || n_bound > vpm::kMaxBound || !gb)
    return fail(VPM_EINVAL, "n_bound must be in 1..64 with gb given");
  VPM_HIP_TRY(hipSetDevice(p->device));
  vpm::State st;
  st.n = n;
  st.nb = n_bound;
  const size_t nn = n > 0 ? n : 1;
  int rc = vpm::grow(&st.wx, 0, nn) | vpm::grow(&st.wz, 0, nn) | vpm::grow(&st.wg, 0, nn) |
           vpm::grow(&st.field_off, 0, 2) | vpm::grow(&st.g7, 0, 7) |
           vpm::grow(&st.gb, 0, (size_t)n_bound);
  if (rc != VPM_OK) {
    vpm::free_state(st);
    return fail(VPM_ENOMEM, "state allocation failed");
  }
  const int64_t off[2] = {0, n};
  hipError_t e = hipSuccess;
  if (n > 0) {
    e = hipMemcpy(st.wx, wx, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.wz, wz, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.wg, wg, n * 8, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(st.field_off, off, 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st.g7, g7, 56, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(st.gb, gb, n_bound * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vpm::free_state(st);
    return fail(VPM_EDEVICE, std::string("state upload: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lock(p->mu);
  *state_id = p->next_state++;
  p->states[*state_id] = st;
  return VPM_OK;
}

VPM_API int planner_state_drop(planner *p, uint64_t state_id) {
  if (!p) return fail(VPM_EINVAL, "planner is NULL");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->states.find(state_id);
  if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
  if (it->second.refs > 0) return fail(VPM_EINVAL, "state is used by queued requests");
  vpm::free_state(it->second);
  p->states.erase(it);
  return VPM_OK;
}

VPM_API int planner_submit(planner *p, const plan_req *req, uint64_t *ticket) {
  if (!p || !req || !ticket) return fail(VPM_EINVAL, "NULL argument");
  if (req->K < 1 || req->H < 1 || !(req->dt > 0) || !(req->lambda > 0) || !req->u_mean ||
      !req->u_eps || req->iterations < 1 || req->iterations > 64)
    return fail(VPM_EINVAL, "bad request sizes, iterations (1..64) or pointers");
  auto r = std::make_unique<vpm::Request>();
  {
    std::lock_guard<std::mutex> lock(p->mu);
    auto it = p->states.find(req->state_id);
    if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
    if (req->params.n_bound != it->second.nb)
      return fail(VPM_EINVAL, "params.n_bound differs from the state's");
    r->footprint =
        planner_footprint(req->K, req->H, it->second.n, it->second.nb, req->iterations);
    if (r->footprint > p->budget) return fail(VPM_EBUDGET, "request exceeds the HBM budget");
  }
  r->state_id = req->state_id;
  r->params = req->params;
  r->K = req->K;
  r->H = req->H;
  r->dt = req->dt;
  r->lambda = req->lambda;
  r->iters = req->iterations;
  std::memcpy(r->x_goal, req->x_goal, sizeof(r->x_goal));
  std::memcpy(r->q_diag, req->q_diag, sizeof(r->q_diag));
  r->u_mean.assign(req->u_mean, req->u_mean + req->H);
  r->u_eps.assign(req->u_eps, req->u_eps + (size_t)req->iterations * req->K * req->H);
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->states.find(req->state_id);
  if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
  it->second.refs++;
  r->ticket = p->next_ticket++;
  r->t_arrive = vpm::now_us(p);
  *ticket = r->ticket;
  p->pending.push_back(r.get());
  p->reqs[r->ticket] = std::move(r);
  p->cv.notify_all();
  return VPM_OK;
}

VPM_API int planner_poll(planner *p, uint64_t ticket, plan_result *res, int32_t timeout_us) {
  if (!p || !res) return fail(VPM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lock(p->mu);
  auto it = p->reqs.find(ticket);
  if (it == p->reqs.end()) return fail(VPM_ENOTFOUND, "unknown ticket");
  vpm::Request *r = it->second.get();
  auto done = [&] { return r->st == vpm::ReqState::kDone; };
  if (!done()) {
    if (timeout_us == 0) return VPM_PENDING;
    if (timeout_us < 0)
      p->cv.wait(lock, done);
    else if (!p->cv.wait_for(lock, std::chrono::microseconds(timeout_us), done))
      return VPM_PENDING;
  }
  res->status = r->status;
  res->argmin = r->argmin;
  res->jmin = r->jmin;
  res->t_arrive_us = r->t_arrive;
  res->t_admit_us = r->t_admit;
  res->t_done_us = r->t_done;
  res->pairs = r->pairs;
  if (r->status == VPM_OK) {
    if (res->u_new) std::memcpy(res->u_new, r->u_new.data(), r->u_new.size() * 8);
    if (res->w) std::memcpy(res->w, r->w.data(), r->w.size() * 8);
    if (res->cost) std::memcpy(res->cost, r->cost.data(), r->cost.size() * 8);
    if (res->g_final) std::memcpy(res->g_final, r->g_final.data(), r->g_final.size() * 8);
  }
  p->reqs.erase(it);
  return VPM_OK;
}

}  // extern "C"
