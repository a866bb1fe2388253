// planner.hip -- replanning service over the rollout engine.
//
// Resident states (wake + glider) live in device memory. The scheduler of
// planner_core.h admits queued requests in arrival order while a slot is
// free and the in-flight footprint fits the HBM budget; each admitted request
// runs on its slot's own context and stream (inputs from pinned staging, the
// rollout batches and MPPI updates of its iterations, optionally the
// advance of its state under the updated controls, results back to pinned
// memory), so requests that arrive while others are on the GPU overlap with
// them. Completion is detected with events; planner_poll hands results to the
// caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "planner_core.h"
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

// off = {0, cap}: the output layout of a one-rollout wake.
__global__ void capacity_layout_kernel(int64_t *off, int64_t cap) {
  if (threadIdx.x == 0) {
    off[0] = 0;
    off[1] = cap;
  }
}

// field_off = {0, n}: the advanced state's wake holds the n_final vortices.
__global__ void state_layout_kernel(const int32_t *__restrict__ n_final,
                                    int64_t *__restrict__ field_off) {
  if (threadIdx.x == 0) {
    field_off[0] = 0;
    field_off[1] = n_final[0];
  }
}

__global__ void zero_kernel(double *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// A resident fluid and vehicle state. Device buffers; wake capacity `cap`
// holds `n` vortices in age order.
struct State {
  int n = 0, nb = 0;
  size_t cap = 0;
  double *wx = nullptr, *wz = nullptr, *wg = nullptr;
  int64_t *field_off = nullptr;  // {0, n}
  double *g7 = nullptr, *gb = nullptr;
  int refs = 0;
};

template <typename T>
int dev_alloc(T **ptr, size_t n) {
  *ptr = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(ptr), std::max<size_t>(n, 1) * sizeof(T)) !=
      hipSuccess) {
    *ptr = nullptr;
    return VPM_ENOMEM;
  }
  return VPM_OK;
}

void free_state(State &st) {
  (void)hipFree(st.wx);
  (void)hipFree(st.wz);
  (void)hipFree(st.wg);
  (void)hipFree(st.field_off);
  (void)hipFree(st.g7);
  (void)hipFree(st.gb);
  st = State{};
}

int alloc_state(State &st, size_t cap, int nb) {
  st.cap = cap;
  st.nb = nb;
  int rc = dev_alloc(&st.wx, cap) | dev_alloc(&st.wz, cap) | dev_alloc(&st.wg, cap) |
           dev_alloc(&st.field_off, 2) | dev_alloc(&st.g7, 7) |
           dev_alloc(&st.gb, (size_t)nb);
  if (rc != VPM_OK) free_state(st);
  return rc != VPM_OK ? VPM_ENOMEM : VPM_OK;
}

// One request: its inputs (copied at submit), the resident state it plans
// from, and its results.
struct PlanJob : Job {
  uint64_t state_id = 0;
  State st;  // copy of the resident state's handles (the state holds a ref)
  vpm_params params{};
  int K = 0, H = 0, iters = 1, advance = 0;
  double dt = 0, lambda = 1;
  double x_goal[7]{}, q_diag[7]{};
  std::vector<double> u_mean, u_eps;
  // results
  std::vector<double> u_new, w, cost, g_final;
  int argmin = -1;
  double jmin = 0;
  int64_t pairs = 0;
  State adv;  // the advanced state while it is being built
  int adv_status = 0;
  uint64_t new_state_id = 0;
};

// Device and pinned buffers of a slot, grown when a request needs more.
struct Slot {
  vpm_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  size_t cap_kh = 0, cap_k = 0, cap_h = 0, cap_kb = 0;
  double *d_u_eps = nullptr, *d_u_mean = nullptr, *d_g0 = nullptr, *d_gb0 = nullptr;
  double *d_g_final = nullptr, *d_cost = nullptr, *d_w = nullptr, *d_u_new = nullptr;
  double *d_jmin = nullptr, *d_zero = nullptr, *d_adv_cost = nullptr;
  int32_t *d_field_of = nullptr, *d_status = nullptr, *d_argmin = nullptr;
  int32_t *d_adv = nullptr;     // advance: n_final, status
  int64_t *d_pairs = nullptr, *d_wake_off = nullptr;
  double *h_in = nullptr;   // pinned staging: u_eps then u_mean
  double *h_out = nullptr;  // pinned results: cost, w, g_final, u_new, jmin
  int64_t *h_pairs = nullptr;
  int32_t *h_small = nullptr;  // argmin, advance n_final, advance status
};

template <typename T>
int regrow(T **ptr, size_t need) {
  if (*ptr) (void)hipFree(*ptr);
  return dev_alloc(ptr, need);
}

template <typename T>
int regrow_pinned(T **ptr, size_t need) {
  if (*ptr) (void)hipHostFree(*ptr);
  *ptr = nullptr;
  if (hipHostMalloc(reinterpret_cast<void **>(ptr), std::max<size_t>(need, 1) * sizeof(T),
                    hipHostMallocDefault) != hipSuccess) {
    *ptr = nullptr;
    return VPM_ENOMEM;
  }
  return VPM_OK;
}

// Make the slot's buffers hold a request of `iters` K x H perturbation sets
// with nb bound vortices. Capacities grow by at least 1.5x so a stream of
// varied requests settles; a growth frees device memory, which synchronises
// the device (planner_reserve sizes the slots up front instead).
int reserve_slot(Slot &s, size_t K, size_t H, size_t nb, size_t iters) {
  const size_t kh = K * H * iters;
  if (kh <= s.cap_kh && K <= s.cap_k && H <= s.cap_h && K * nb <= s.cap_kb && s.h_in)
    return VPM_OK;
  if (hipStreamSynchronize(s.stream) != hipSuccess) return VPM_EDEVICE;
  auto up = [](size_t have, size_t need) { return std::max(need, have + have / 2); };
  int rc = VPM_OK;
  if (kh > s.cap_kh) {
    s.cap_kh = up(s.cap_kh, kh);
    rc |= regrow(&s.d_u_eps, s.cap_kh);
  }
  if (H > s.cap_h || !s.d_zero) {
    s.cap_h = up(s.cap_h, H);
    rc |= regrow(&s.d_u_mean, s.cap_h);
    rc |= regrow(&s.d_u_new, s.cap_h);
    rc |= regrow(&s.d_zero, s.cap_h);
    if (rc == VPM_OK) {
      hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((s.cap_h + 255) / 256)), dim3(256), 0,
                         s.stream, s.d_zero, s.cap_h);
      if (hipGetLastError() != hipSuccess) return VPM_EDEVICE;
    }
  }
  if (K > s.cap_k) {
    s.cap_k = up(s.cap_k, K);
    rc |= regrow(&s.d_g0, 7 * s.cap_k);
    rc |= regrow(&s.d_g_final, 7 * s.cap_k);
    rc |= regrow(&s.d_cost, s.cap_k);
    rc |= regrow(&s.d_w, s.cap_k);
    rc |= regrow(&s.d_field_of, s.cap_k);
    rc |= regrow(&s.d_status, s.cap_k);
    rc |= regrow(&s.d_pairs, s.cap_k);
  }
  if (K * nb > s.cap_kb) {
    s.cap_kb = up(s.cap_kb, K * nb);
    rc |= regrow(&s.d_gb0, s.cap_kb);
  }
  // pinned staging: u_eps then u_mean in; cost, w, g_final, u_new, jmin out
  rc |= regrow_pinned(&s.h_in, s.cap_kh + s.cap_h);
  rc |= regrow_pinned(&s.h_out, 9 * s.cap_k + s.cap_h + 1);
  rc |= regrow_pinned(&s.h_pairs, s.cap_k);
  if (!s.d_jmin) rc |= dev_alloc(&s.d_jmin, 1);
  if (!s.d_argmin) rc |= dev_alloc(&s.d_argmin, 1);
  if (!s.d_adv_cost) rc |= dev_alloc(&s.d_adv_cost, 1);
  if (!s.d_adv) rc |= dev_alloc(&s.d_adv, 2);
  if (!s.d_wake_off) rc |= dev_alloc(&s.d_wake_off, 2);
  if (!s.h_small) rc |= regrow_pinned(&s.h_small, 3);
  if (rc != VPM_OK) {
    s.cap_kh = s.cap_k = s.cap_h = s.cap_kb = 0;  // regrow everything next time
    return VPM_ENOMEM;
  }
  return hipStreamSynchronize(s.stream) == hipSuccess ? VPM_OK : VPM_EDEVICE;
}

void free_slot(Slot &s) {
  for (double *p : {s.d_u_eps, s.d_u_mean, s.d_g0, s.d_gb0, s.d_g_final, s.d_cost, s.d_w,
                    s.d_u_new, s.d_jmin, s.d_zero, s.d_adv_cost})
    (void)hipFree(p);
  for (int32_t *p : {s.d_field_of, s.d_status, s.d_argmin, s.d_adv}) (void)hipFree(p);
  (void)hipFree(s.d_pairs);
  (void)hipFree(s.d_wake_off);
  (void)hipHostFree(s.h_in);
  (void)hipHostFree(s.h_out);
  (void)hipHostFree(s.h_pairs);
  (void)hipHostFree(s.h_small);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.ctx) vpm_destroy(s.ctx);
  s = Slot{};
}

// Wake vortices a rollout of `steps` steps can add per shedding mode.
int shed_per_step(const vpm_params &p) {
  return p.shed_mode == VPM_SHED_BOTH ? 2 : p.shed_mode == VPM_SHED_TE ? 1 : 0;
}

}  // namespace
}  // namespace vpm

// The service: resident states, slots and the scheduler that drives them.
struct planner : vpm::Executor {
  int device = 0;
  int n_slots = 1;
  std::mutex st_mu;  // states and next_state (lock order: scheduler, then st_mu)
  std::map<uint64_t, vpm::State> states;
  uint64_t next_state = 1;
  std::mutex exec_mu;  // slot buffers: the worker's launches against planner_reserve
  vpm::Slot slots[vpm::kMaxSlots];
  std::unique_ptr<vpm::Scheduler> sched;

  int launch(int slot, vpm::Job &job) override;
  int query(int slot) override;
  int collect(int slot, vpm::Job &job) override;
  void release(vpm::Job &job) override;

 private:
  int enqueue(vpm::Slot &s, vpm::PlanJob &r, bool *queued);
};

int planner::enqueue(vpm::Slot &s, vpm::PlanJob &r, bool *queued) {
  using namespace vpm;
  const State &st = r.st;
  const size_t K = r.K, H = r.H, it_n = r.iters;
  const size_t kh = K * H * it_n;
  std::memcpy(s.h_in, r.u_eps.data(), kh * sizeof(double));
  std::memcpy(s.h_in + kh, r.u_mean.data(), H * sizeof(double));
  *queued = true;
  VPM_HIP_TRY(hipMemcpyAsync(s.d_u_eps, s.h_in, kh * sizeof(double), hipMemcpyHostToDevice,
                             s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(s.d_u_mean, s.h_in + kh, H * sizeof(double),
                             hipMemcpyHostToDevice, s.stream));
  hipLaunchKernelGGL(broadcast_state_kernel, dim3((K + 255) / 256), dim3(256), 0, s.stream,
                     r.K, st.nb, st.g7, st.gb, s.d_g0, s.d_gb0, s.d_field_of);
  VPM_HIP_TRY(hipGetLastError());
  vpm_batch_in in{};
  in.K = r.K;
  in.H = r.H;
  in.dt = r.dt;
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
  std::memcpy(in.x_goal, r.x_goal, sizeof(in.x_goal));
  std::memcpy(in.q_diag, r.q_diag, sizeof(in.q_diag));
  vpm_batch_out out{};
  out.g_final = s.d_g_final;
  out.cost = s.d_cost;
  out.status = s.d_status;
  out.pair_count = s.d_pairs;
  // MPPI iterations (Sec. IV-A): each rolls the same initial state out under
  // its own perturbations around the previous iteration's update; the mean
  // alternates between the two device buffers
  double *mean = s.d_u_mean, *next = s.d_u_new;
  int rc = VPM_OK;
  for (size_t i = 0; i < it_n; ++i) {
    in.u_mean = mean;
    in.u_eps = s.d_u_eps + i * K * H;
    rc = vpm_rollout_batch(s.ctx, &r.params, &in, &out, s.stream);
    if (rc != VPM_OK) return rc;
    rc = mppi_weights(s.ctx, r.K, r.H, s.d_cost, r.lambda, mean, in.u_eps, s.d_w, next,
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
  VPM_HIP_TRY(hipMemcpyAsync(s.h_small, s.d_argmin, 4, hipMemcpyDeviceToHost, s.stream));
  VPM_HIP_TRY(hipMemcpyAsync(s.h_pairs, s.d_pairs, K * 8, hipMemcpyDeviceToHost, s.stream));
  if (r.advance > 0) {
    // the resident state carried forward: one rollout of `advance` steps from
    // the planned-from state under the updated controls (no perturbation)
    const size_t cap = (size_t)st.n + (size_t)shed_per_step(r.params) * r.advance;
    if (alloc_state(r.adv, cap, st.nb) != VPM_OK)
      return fail(VPM_ENOMEM, "allocation of the advanced state failed");
    hipLaunchKernelGGL(capacity_layout_kernel, dim3(1), dim3(64), 0, s.stream, s.d_wake_off,
                       (int64_t)cap);
    VPM_HIP_TRY(hipGetLastError());
    vpm_batch_in a = in;
    a.K = 1;
    a.H = r.advance;
    a.g0 = st.g7;
    a.gb0 = st.gb;
    a.field_of = nullptr;
    a.u_mean = mean;
    a.u_eps = s.d_zero;
    vpm_batch_out o{};
    o.g_final = r.adv.g7;
    o.cost = s.d_adv_cost;
    o.status = s.d_adv + 1;
    o.wake_off = s.d_wake_off;
    o.wx = r.adv.wx;
    o.wz = r.adv.wz;
    o.wg = r.adv.wg;
    o.n_final = s.d_adv;
    o.gb_final = r.adv.gb;
    rc = vpm_rollout_batch(s.ctx, &r.params, &a, &o, s.stream);
    if (rc != VPM_OK) return rc;
    hipLaunchKernelGGL(state_layout_kernel, dim3(1), dim3(64), 0, s.stream, s.d_adv,
                       r.adv.field_off);
    VPM_HIP_TRY(hipGetLastError());
    VPM_HIP_TRY(hipMemcpyAsync(s.h_small + 1, s.d_adv, 8, hipMemcpyDeviceToHost, s.stream));
  }
  VPM_HIP_TRY(hipEventRecord(s.done, s.stream));
  return VPM_OK;
}

int planner::launch(int slot, vpm::Job &job) {
  using namespace vpm;
  auto &r = static_cast<PlanJob &>(job);
  std::lock_guard<std::mutex> lock(exec_mu);
  Slot &s = slots[slot];
  (void)hipSetDevice(device);
  int rc = reserve_slot(s, r.K, r.H, r.st.nb, r.iters);
  if (rc != VPM_OK) return fail(rc, "planner slot allocation failed");
  bool queued = false;
  rc = enqueue(s, r, &queued);
  if (rc != VPM_OK && queued) {
    // copies from the slot's pinned staging may still be in flight: the slot
    // is reused only once its stream has drained
    (void)hipStreamSynchronize(s.stream);
  }
  return rc;
}

int planner::query(int slot) {
  const hipError_t q = hipEventQuery(slots[slot].done);
  if (q == hipErrorNotReady) return VPM_PENDING;
  return q == hipSuccess ? VPM_OK : vpm::fail(VPM_EDEVICE, hipGetErrorString(q));
}

int planner::collect(int slot, vpm::Job &job) {
  using namespace vpm;
  auto &r = static_cast<PlanJob &>(job);
  std::lock_guard<std::mutex> lock(exec_mu);
  Slot &s = slots[slot];
  const size_t K = r.K, H = r.H;
  const double *h = s.h_out;
  r.cost.assign(h, h + K);
  r.w.assign(h + K, h + 2 * K);
  r.g_final.assign(h + 2 * K, h + 9 * K);
  r.u_new.assign(h + 9 * K, h + 9 * K + H);
  r.jmin = h[9 * K + H];
  r.argmin = s.h_small[0];
  r.pairs = 0;
  for (size_t k = 0; k < K; ++k) r.pairs += s.h_pairs[k];
  r.pairs *= r.iters;  // the wake-count schedule, so the work, is the same each iteration
  if (r.advance > 0) {
    r.adv.n = s.h_small[1];
    r.adv_status = s.h_small[2];
    std::lock_guard<std::mutex> sl(st_mu);
    r.new_state_id = next_state++;
    states[r.new_state_id] = r.adv;
    r.adv = State{};
  }
  return VPM_OK;
}

void planner::release(vpm::Job &job) {
  auto &r = static_cast<vpm::PlanJob &>(job);
  if (r.adv.wx) vpm::free_state(r.adv);  // a failed request's unfinished state
  std::lock_guard<std::mutex> sl(st_mu);
  auto it = states.find(r.state_id);
  if (it != states.end()) it->second.refs--;
}

using vpm::fail;

namespace {

// Bytes of device memory a request occupies while in flight: perturbations
// of every iteration, per-rollout inputs and outputs, the advanced state, and
// for wakes that exceed the LDS-resident kernels the streaming workspace of
// one slot per CU (24 B per vortex of capacity in FP32, 48 B in FP64).
size_t footprint(const vpm_params *p, size_t K, size_t H, size_t n0, size_t it,
                 size_t advance) {
  const size_t nb = p->n_bound;
  size_t bytes = 8 * (it * K * H + 3 * H + 7 * K + K * nb + 7 * K + 3 * K + 1) + 4 * (2 * K + 3);
  const size_t shed = vpm::shed_per_step(*p);
  if (advance > 0) bytes += 8 * (3 * (n0 + shed * advance) + 9 + nb);
  const size_t cap = n0 + shed * H;
  if (cap > (size_t)vpm::lds_resident_capacity(p->n_bound, p->precision))
    bytes += 256 * cap * (p->precision == VPM_FP64 ? 48 : 24);
  return bytes;
}

}  // namespace

extern "C" {

VPM_API size_t planner_footprint(const vpm_params *params, int32_t K, int32_t H, int32_t n0,
                                 int32_t iterations, int32_t advance) {
  if (!params || params->n_bound < 1 || params->n_bound > vpm::kMaxBound) return 0;
  auto nn = [](int32_t v) { return v > 0 ? (size_t)v : (size_t)0; };
  return footprint(params, nn(K), nn(H), nn(n0), iterations > 0 ? (size_t)iterations : 1,
                   nn(advance));
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
  p->sched = std::make_unique<vpm::Scheduler>(p->n_slots, opts->hbm_budget_bytes, p);
  *out = p;
  return VPM_OK;
}

VPM_API void planner_destroy(planner *p) {
  if (!p) return;
  p->sched.reset();  // waits for queued and running requests
  (void)hipSetDevice(p->device);
  for (int i = 0; i < p->n_slots; ++i) vpm::free_slot(p->slots[i]);
  for (auto &kv : p->states) vpm::free_state(kv.second);
  delete p;
}

VPM_API int planner_reserve(planner *p, const vpm_params *params, int32_t K, int32_t H,
                            int32_t n0, int32_t iterations) {
  if (!p) return fail(VPM_EINVAL, "planner is NULL");
  int rc = vpm::check_params(params);
  if (rc != VPM_OK) return rc;
  if (K < 1 || H < 1 || n0 < 0 || iterations < 1 || iterations > 64)
    return fail(VPM_EINVAL, "K, H >= 1, n0 >= 0 and iterations in 1..64");
  VPM_HIP_TRY(hipSetDevice(p->device));
  std::lock_guard<std::mutex> lock(p->exec_mu);
  bool ran = p->sched->when_idle([&] {
    for (int i = 0; i < p->n_slots && rc == VPM_OK; ++i) {
      vpm::Slot &s = p->slots[i];
      rc = vpm::reserve_slot(s, K, H, params->n_bound, iterations);
      if (rc != VPM_OK) {
        rc = fail(rc, "planner slot allocation failed");
        break;
      }
      // plate inverses and the rollout workspaces, for the batch and for the
      // one-rollout advance
      rc = vpm_reserve(s.ctx, params, K, H, n0, 1);
    }
  });
  if (!ran) return fail(VPM_EINVAL, "planner_reserve needs an idle planner (nothing queued)");
  return rc;
}

VPM_API int planner_set_tuning(planner *p, int32_t kernel_class, int32_t targets_per_thread,
                               int32_t tile) {
  if (!p) return fail(VPM_EINVAL, "planner is NULL");
  for (int i = 0; i < p->n_slots; ++i) {
    const int rc = vpm_set_tuning(p->slots[i].ctx, kernel_class, targets_per_thread, tile);
    if (rc != VPM_OK) return rc;
  }
  return VPM_OK;
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
  if (vpm::alloc_state(st, (size_t)n, n_bound) != VPM_OK)
    return fail(VPM_ENOMEM, "state allocation failed");
  st.n = n;
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
  std::lock_guard<std::mutex> lock(p->st_mu);
  *state_id = p->next_state++;
  p->states[*state_id] = st;
  return VPM_OK;
}

VPM_API int planner_state_get(planner *p, uint64_t state_id, int32_t *n, double *wx, double *wz,
                              double *wg, double *g7, double *gb, int32_t capacity) {
  if (!p || !n) return fail(VPM_EINVAL, "NULL argument");
  vpm::State st;
  {
    std::lock_guard<std::mutex> lock(p->st_mu);
    auto it = p->states.find(state_id);
    if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
    st = it->second;
    it->second.refs++;  // held while it is read
  }
  *n = st.n;
  int rc = VPM_OK;
  if (wx || wz || wg || g7 || gb) {
    if (capacity < st.n) {
      rc = fail(VPM_EINVAL, "capacity is smaller than the state's wake");
    } else {
      VPM_HIP_TRY(hipSetDevice(p->device));
      hipError_t e = hipSuccess;
      if (st.n > 0) {
        if (wx) e = hipMemcpy(wx, st.wx, st.n * 8, hipMemcpyDeviceToHost);
        if (wz && e == hipSuccess) e = hipMemcpy(wz, st.wz, st.n * 8, hipMemcpyDeviceToHost);
        if (wg && e == hipSuccess) e = hipMemcpy(wg, st.wg, st.n * 8, hipMemcpyDeviceToHost);
      }
      if (g7 && e == hipSuccess) e = hipMemcpy(g7, st.g7, 56, hipMemcpyDeviceToHost);
      if (gb && e == hipSuccess) e = hipMemcpy(gb, st.gb, st.nb * 8, hipMemcpyDeviceToHost);
      if (e != hipSuccess) rc = fail(VPM_EDEVICE, std::string("state read: ") + hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lock(p->st_mu);
  p->states[state_id].refs--;
  return rc;
}

VPM_API int planner_state_drop(planner *p, uint64_t state_id) {
  if (!p) return fail(VPM_EINVAL, "planner is NULL");
  std::lock_guard<std::mutex> lock(p->st_mu);
  auto it = p->states.find(state_id);
  if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
  if (it->second.refs > 0) return fail(VPM_EINVAL, "state is used by queued requests");
  (void)hipSetDevice(p->device);
  vpm::free_state(it->second);
  p->states.erase(it);
  return VPM_OK;
}

VPM_API int planner_submit(planner *p, const plan_req *req, uint64_t *ticket) {
  if (!p || !req || !ticket) return fail(VPM_EINVAL, "NULL argument");
  auto r = std::make_unique<vpm::PlanJob>();
  r->t_arrive = p->sched->now_us();  // before any lock or copy
  if (req->K < 1 || req->H < 1 || !(req->dt > 0) || !(req->lambda > 0) || !req->u_mean ||
      req->iterations < 1 || req->iterations > 64)
    return fail(VPM_EINVAL, "bad request sizes, iterations (1..64) or pointers");
  if (req->advance < 0 || req->advance > req->H)
    return fail(VPM_EINVAL, "advance must be in 0..H");
  if (!req->u_eps && !(std::isfinite(req->sigma) && req->sigma >= 0.0))
    return fail(VPM_EINVAL, "seeded perturbations need a finite sigma >= 0");
  int rc = vpm::check_params(&req->params);
  if (rc != VPM_OK) return rc;
  {
    std::lock_guard<std::mutex> lock(p->st_mu);
    auto it = p->states.find(req->state_id);
    if (it == p->states.end()) return fail(VPM_ENOTFOUND, "unknown state");
    if (req->params.n_bound != it->second.nb)
      return fail(VPM_EINVAL, "params.n_bound differs from the state's");
    r->footprint = footprint(&req->params, req->K, req->H, it->second.n, req->iterations,
                             req->advance);
    if (r->footprint > p->sched->budget())
      return fail(VPM_EBUDGET, "request exceeds the HBM budget");
    it->second.refs++;
    r->st = it->second;
  }
  r->state_id = req->state_id;
  r->params = req->params;
  r->K = req->K;
  r->H = req->H;
  r->dt = req->dt;
  r->lambda = req->lambda;
  r->iters = req->iterations;
  r->advance = req->advance;
  std::memcpy(r->x_goal, req->x_goal, sizeof(r->x_goal));
  std::memcpy(r->q_diag, req->q_diag, sizeof(r->q_diag));
  r->u_mean.assign(req->u_mean, req->u_mean + req->H);
  const size_t kh = (size_t)req->K * req->H;
  if (req->u_eps) {
    r->u_eps.assign(req->u_eps, req->u_eps + req->iterations * kh);
  } else {
    r->u_eps.resize(req->iterations * kh);
    for (int i = 0; i < req->iterations; ++i)
      vpm::sample_eps(req->seed, i, req->K, req->H, req->sigma, r->u_eps.data() + i * kh);
  }
  const uint64_t sid = r->state_id;
  rc = p->sched->submit(std::move(r), ticket);
  if (rc != VPM_OK) {  // not queued (checked above already; kept for safety)
    std::lock_guard<std::mutex> lock(p->st_mu);
    p->states[sid].refs--;
    return fail(rc, "request exceeds the HBM budget");
  }
  return VPM_OK;
}

VPM_API int planner_poll(planner *p, uint64_t ticket, plan_result *res, int32_t timeout_us) {
  if (!p || !res) return fail(VPM_EINVAL, "NULL argument");
  std::unique_ptr<vpm::Job> job;
  const int rc = p->sched->poll(ticket, &job, timeout_us);
  if (rc == VPM_ENOTFOUND) return fail(rc, "unknown ticket");
  if (rc != VPM_OK) return rc;
  auto &r = static_cast<vpm::PlanJob &>(*job);
  res->status = r.status;
  res->argmin = r.argmin;
  res->jmin = r.jmin;
  res->t_arrive_us = r.t_arrive;
  res->t_admit_us = r.t_admit;
  res->t_done_us = r.t_done;
  res->pairs = r.pairs;
  res->new_state_id = r.new_state_id;
  res->new_state_status = r.adv_status;
  if (r.status == VPM_OK) {
    if (res->u_new) std::memcpy(res->u_new, r.u_new.data(), r.u_new.size() * 8);
    if (res->w) std::memcpy(res->w, r.w.data(), r.w.size() * 8);
    if (res->cost) std::memcpy(res->cost, r.cost.data(), r.cost.size() * 8);
    if (res->g_final) std::memcpy(res->g_final, r.g_final.data(), r.g_final.size() * 8);
  }
  return VPM_OK;
}

}  // extern "C"
