// replan.hip -- one replanning cycle of the nonlinear MPC (Sec. IV-C) on one
// stream: projection of the resident state under the policy in force, MPPI
// iterations from the projected state, then the nominal and perturbed
// rollouts and the local feedback policy (Sec. IV-B). The steps are the
// library's own launches; the small kernels here only shift controls, build
// the batch inputs from the projected state and chain the wake between
// batches, so that no value makes a round trip through the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vpm_internal.h"

namespace vpm {
namespace {

constexpr int kFill = 256;

// u_out[n] = u_plan[min(n + P, H - 1)]: the plan in force, from where the
// new plan takes over, its last control held.
__global__ void shift_kernel(const double *u_plan, int H, int P, double *u_out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < H) u_out[n] = u_plan[n + P < H ? n + P : H - 1];
}

__global__ void fill_kernel(double *x, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// Field offsets of the projection's input and output layouts and, when
// nothing is projected, the wake count the later batches read.
__global__ void init_kernel(int64_t *proj_field_off, int64_t *proj_off, int32_t *proj_n,
                            int n_wake, int P) {
  if (threadIdx.x == 0) {
    proj_field_off[0] = 0;
    proj_field_off[1] = n_wake;
    proj_off[0] = 0;
    proj_off[1] = (int64_t)n_wake + 2 * (int64_t)P;
    if (P == 0) proj_n[0] = n_wake;
  }
}

// Projection outputs -> inputs of a batch sharing the projected wake as one
// field: field_off = {0, n_final}, and per rollout i of the batch the glider
// state g_proj (+ x_eps[i - 1] for i >= 1 when x_eps is given), the bound
// circulations gb_proj, the control perturbation (0 for i = 0, du[i - 1]
// otherwise when du is given, else 0) and the pair indices.
__global__ void batch_inputs_kernel(const double *g_proj, const double *gb_proj,
                                    const int32_t *n_proj, const double *x_eps,
                                    const double *du, const int32_t *pairs, int n_pairs,
                                    int H, int nb, double *g0, double *gb0,
                                    double *u_eps, int32_t *pairs_out, int64_t *field_off,
                                    int32_t *field_of) {
  const int i = blockIdx.x;  // rollout of the batch
  const int t = threadIdx.x;
  if (i == 0 && t == 0) {
    field_off[0] = 0;
    field_off[1] = n_proj[0];
  }
  if (t < 7) g0[(size_t)i * 7 + t] = g_proj[t] + (x_eps && i > 0 ? x_eps[(size_t)(i - 1) * 7 + t] : 0.0);
  for (int j = t; j < nb; j += blockDim.x) gb0[(size_t)i * nb + j] = gb_proj[j];
  if (u_eps)
    for (int n = t; n < H; n += blockDim.x)
      u_eps[(size_t)i * H + n] = du && i > 0 ? du[(size_t)(i - 1) * H + n] : 0.0;
  if (t < 2 * n_pairs) pairs_out[(size_t)i * 2 * n_pairs + t] = pairs[t];
  if (t == 0) field_of[i] = 0;
}

// Bump allocator over the context's cycle workspace (256-byte aligned).
struct Arena {
  char *base;
  size_t off;
  template <typename T> T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(base) + off);
    off += n * sizeof(T);
    return p;
  }
};

struct Layout {
  double *proj_g, *proj_gb, *proj_cost, *proj_wx, *proj_wz, *proj_wg, *u_zero;
  double *u_mean[2], *g0, *gb0, *cost, *g_final, *w, *traj, *u_eps_p;
  int32_t *proj_status, *proj_n, *status, *pairs, *field_of;
  int64_t *proj_off, *proj_field_off, *field_off;
  double *a, *b;
  size_t bytes;
};

Layout plan_layout(char *base, const vpm_replan_in *in, int nb) {
  Arena ar{base, 0};
  Layout L{};
  const int H = in->H, P = in->P, K = in->K, Kb = in->Kp + 1, Kmax = K > Kb ? K : Kb;
  const size_t cap_proj = (size_t)in->n_wake + 2 * (size_t)P;
  L.proj_g = ar.take<double>(7);
  L.proj_gb = ar.take<double>(nb);
  L.proj_cost = ar.take<double>(1);
  L.proj_wx = ar.take<double>(cap_proj + 1);
  L.proj_wz = ar.take<double>(cap_proj + 1);
  L.proj_wg = ar.take<double>(cap_proj + 1);
  L.u_zero = ar.take<double>(H > 0 ? H : 1);
  L.proj_status = ar.take<int32_t>(1);
  L.proj_n = ar.take<int32_t>(1);
  L.proj_off = ar.take<int64_t>(2);
  L.proj_field_off = ar.take<int64_t>(2);
  L.u_mean[0] = ar.take<double>(H);
  L.u_mean[1] = ar.take<double>(H);
  L.g0 = ar.take<double>((size_t)Kmax * 7);
  L.gb0 = ar.take<double>((size_t)Kmax * nb);
  L.cost = ar.take<double>(Kmax);
  L.g_final = ar.take<double>((size_t)Kmax * 7);
  L.w = ar.take<double>(K);
  L.traj = ar.take<double>((size_t)Kb * (H + 1) * 7);
  L.u_eps_p = ar.take<double>((size_t)Kb * H);
  L.status = ar.take<int32_t>(Kmax);
  L.pairs = ar.take<int32_t>((size_t)Kmax * 2 * (in->n_pairs > 0 ? in->n_pairs : 1));
  L.field_of = ar.take<int32_t>(Kmax);
  L.field_off = ar.take<int64_t>(2);
  L.a = ar.take<double>((size_t)H * 49);
  L.b = ar.take<double>((size_t)H * 7);
  L.bytes = ar.off + 256;
  return L;
}


}  // namespace

int check_replan(const vpm_params *p, const vpm_replan_in *in, const vpm_replan_out *out) {
  if (!p || !in || !out) return fail(VPM_EINVAL, "params, in or out is NULL");
  if (!(std::isfinite(in->dt) && in->dt > 0.0)) return fail(VPM_EINVAL, "dt must be > 0");
  if (in->H < 1 || in->P < 0 || in->P > in->H) return fail(VPM_EINVAL, "need H >= 1, 0 <= P <= H");
  if (in->K < 1 || in->iterations < 1) return fail(VPM_EINVAL, "K and iterations must be >= 1");
  if (in->Kp < 1) return fail(VPM_EINVAL, "Kp must be >= 1");
  if (in->n_wake < 0) return fail(VPM_EINVAL, "n_wake must be >= 0");
  if (in->n_pairs < 0 || in->n_pairs > kMaxPairs) return fail(VPM_EINVAL, "n_pairs must be 0..4");
  if (in->n_pairs > 0) {
    if (!in->pairs) return fail(VPM_EINVAL, "pairs is NULL with n_pairs > 0");
    const long long most = (long long)in->n_wake + 2LL * (in->P + in->H);
    if (p->n_wake_max > 0 && most > p->n_wake_max)
      return fail(VPM_EINVAL, "disturbance pairs need a wake that cannot merge within P + H steps");
  }
  if (!(std::isfinite(in->lambda) && in->lambda > 0.0)) return fail(VPM_EINVAL, "lambda must be > 0");
  if (!in->g || !in->gb || !in->u_plan || !in->u_eps || !in->x_eps || !in->du)
    return fail(VPM_EINVAL, "a required input pointer is NULL");
  if (in->n_wake > 0 && (!in->wx || !in->wz || !in->wg))
    return fail(VPM_EINVAL, "wake pointers are NULL");
  if ((in->gain_plan == nullptr) != (in->x_plan == nullptr))
    return fail(VPM_EINVAL, "gain_plan and x_plan go together");
  if (!out->g_proj || !out->u_new || !out->x_new || !out->gain || !out->jmin || !out->argmin ||
      !out->status)
    return fail(VPM_EINVAL, "a required output pointer is NULL");
  return VPM_OK;
}

int run_replan(vpm_ctx *ctx, const vpm_params *p, const vpm_replan_in *in, vpm_replan_out *out,
               hipStream_t stream) {
  int rc = check_replan(p, in, out);
  if (rc != VPM_OK) return rc;
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const int nb = p->n_bound, H = in->H, P = in->P, K = in->K, Kb = in->Kp + 1;
  std::lock_guard<std::mutex> lock(ctx->replan_mu);
  Layout L = plan_layout(nullptr, in, nb);
  rc = ensure_buffer(&ctx->replan, &ctx->replan_bytes, L.bytes, "replanning workspace",
                     stream_capturing(stream));
  if (rc != VPM_OK) return rc;
  L = plan_layout(static_cast<char *>(ctx->replan), in, nb);
  void *sv = stream;
  auto fill = [&](double *x, size_t n, double v) {
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + kFill - 1) / kFill)), dim3(kFill), 0,
                       stream, x, n, v);
  };
  auto copy_goal = [&](vpm_batch_in &b) {
    for (int i = 0; i < 7; ++i) {
      b.x_goal[i] = in->x_goal[i];
      b.q_diag[i] = in->q_diag[i];
    }
  };
  fill(L.u_zero, H, 0.0);
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, stream, L.proj_field_off, L.proj_off,
                     L.proj_n, in->n_wake, P);

  // 1. projection: P steps of the resident state under the policy in force
  const double *g_start = in->g, *gb_start = in->gb;
  const double *wx = in->wx, *wz = in->wz, *wg = in->wg;
  int n_wake = in->n_wake;
  if (P > 0) {
    vpm_batch_in b{};
    b.K = 1;
    b.H = P;
    b.dt = in->dt;
    b.n_fields = 1;
    b.max_wake0 = in->n_wake;
    b.n_pairs = in->n_pairs;
    b.g0 = in->g;
    b.gb0 = in->gb;
    b.field_off = L.proj_field_off;
    b.field_of = nullptr;
    b.wx = in->n_wake > 0 ? in->wx : L.u_zero;
    b.wz = in->n_wake > 0 ? in->wz : L.u_zero;
    b.wg = in->n_wake > 0 ? in->wg : L.u_zero;
    b.pairs = in->n_pairs > 0 ? in->pairs : nullptr;
    b.u_mean = in->u_plan;
    b.u_eps = L.u_zero;
    b.fb_gain = in->gain_plan;
    b.fb_xref = in->x_plan;
    copy_goal(b);
    vpm_batch_out o{};
    o.g_final = L.proj_g;
    o.cost = L.proj_cost;
    o.status = L.proj_status;
    o.wake_off = L.proj_off;
    o.wx = L.proj_wx;
    o.wz = L.proj_wz;
    o.wg = L.proj_wg;
    o.n_final = L.proj_n;
    o.gb_final = L.proj_gb;
    rc = vpm_rollout_batch(ctx, p, &b, &o, sv);
    if (rc != VPM_OK) return rc;
    g_start = L.proj_g;
    gb_start = L.proj_gb;
    wx = L.proj_wx;
    wz = L.proj_wz;
    wg = L.proj_wg;
    n_wake = in->n_wake + 2 * P;  // an upper bound; the count is on the device
  } else if (in->n_wake == 0) {
    wx = wz = wg = L.u_zero;  // never read: the field is empty
  }
  VPM_HIP_TRY(hipMemcpyAsync(out->g_proj, g_start, 7 * sizeof(double), hipMemcpyDeviceToDevice,
                             stream));

  // 2. MPPI iterations from the projected state
  hipLaunchKernelGGL(shift_kernel, dim3((H + kFill - 1) / kFill), dim3(kFill), 0, stream,
                     in->u_plan, H, P, L.u_mean[0]);
  hipLaunchKernelGGL(batch_inputs_kernel, dim3(K), dim3(64), 0, stream, g_start, gb_start,
                     L.proj_n, nullptr, nullptr, in->pairs, in->n_pairs, H, nb, L.g0, L.gb0,
                     nullptr, L.pairs, L.field_off, L.field_of);
  VPM_HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int it = 0; it < in->iterations; ++it) {
    vpm_batch_in b{};
    b.K = K;
    b.H = H;
    b.dt = in->dt;
    b.n_fields = 1;
    b.max_wake0 = n_wake;
    b.n_pairs = in->n_pairs;
    b.g0 = L.g0;
    b.gb0 = L.gb0;
    b.field_off = L.field_off;
    b.field_of = L.field_of;
    b.wx = wx;
    b.wz = wz;
    b.wg = wg;
    b.pairs = in->n_pairs > 0 ? L.pairs : nullptr;
    b.u_mean = L.u_mean[cur];
    b.u_eps = in->u_eps + (size_t)it * K * H;
    copy_goal(b);
    vpm_batch_out o{};
    o.g_final = L.g_final;
    o.cost = L.cost;
    o.status = L.status;
    rc = vpm_rollout_batch(ctx, p, &b, &o, sv);
    if (rc != VPM_OK) return rc;
    rc = launch_mppi(K, H, L.cost, in->lambda, L.u_mean[cur], b.u_eps, L.w, L.u_mean[1 - cur],
                     out->argmin + it, out->jmin + it, stream);
    if (rc != VPM_OK) return rc;
    cur = 1 - cur;
  }
  VPM_HIP_TRY(hipMemcpyAsync(out->u_new, L.u_mean[cur], H * sizeof(double),
                             hipMemcpyDeviceToDevice, stream));

  // 3. nominal + perturbed rollouts under the new mean, then the policy
  hipLaunchKernelGGL(batch_inputs_kernel, dim3(Kb), dim3(64), 0, stream, g_start, gb_start,
                     L.proj_n, in->x_eps, in->du, in->pairs, in->n_pairs, H, nb, L.g0, L.gb0,
                     L.u_eps_p, L.pairs, L.field_off, L.field_of);
  VPM_HIP_TRY(hipGetLastError());
  {
    vpm_batch_in b{};
    b.K = Kb;
    b.H = H;
    b.dt = in->dt;
    b.n_fields = 1;
    b.max_wake0 = n_wake;
    b.n_pairs = in->n_pairs;
    b.g0 = L.g0;
    b.gb0 = L.gb0;
    b.field_off = L.field_off;
    b.field_of = L.field_of;
    b.wx = wx;
    b.wz = wz;
    b.wg = wg;
    b.pairs = in->n_pairs > 0 ? L.pairs : nullptr;
    b.u_mean = L.u_mean[cur];
    b.u_eps = L.u_eps_p;
    copy_goal(b);
    vpm_batch_out o{};
    o.g_final = L.g_final;
    o.cost = L.cost;
    o.status = L.status;
    o.traj = L.traj;
    // FP64 whatever the planning precision: the regression differences
    // trajectories 1e-2 apart, which binary32 state storage would blur
    vpm_params p64 = *p;
    p64.precision = VPM_FP64;
    rc = vpm_rollout_batch(ctx, &p64, &b, &o, sv);
    if (rc != VPM_OK) return rc;
  }
  VPM_HIP_TRY(hipMemcpyAsync(out->x_new, L.traj, (size_t)(H + 1) * 7 * sizeof(double),
                             hipMemcpyDeviceToDevice, stream));
  vpm_policy_in pin{};
  pin.K = in->Kp;
  pin.H = H;
  pin.dt = in->dt;
  pin.traj_nom = L.traj;
  pin.traj = L.traj + (size_t)(H + 1) * 7;
  pin.du = in->du;
  for (int i = 0; i < 7; ++i) {
    pin.q_f[i] = in->q_f[i];
    pin.q_c[i] = in->q_c[i];
  }
  pin.r_c = in->r_c;
  vpm_policy_out pout{};
  pout.a = L.a;
  pout.b = L.b;
  pout.gain = out->gain;
  pout.s = nullptr;
  pout.status = out->status;
  return launch_policy(&pin, &pout, stream);
}

}  // namespace vpm

// ------------------------------------------- finite-difference Jacobians

namespace vpm {
namespace {

constexpr int kFdRows = 13;  // nominal, +-h for 5 states, +-h for u

struct FdSteps {
  double hx[5], hu;
};

// The 13 one-step rollouts of step k from the current nominal state: row 0
// unperturbed, rows 1 + 2j / 2 + 2j with +h_j / -h_j on state 2 + j
// (theta, phi, x_dot, z_dot, theta_dot), rows 11 / 12 with +h_u / -h_u on u.
__global__ void fd_inputs_kernel(const double *g_cur, const double *gb_cur, const int32_t *n_cur,
                                 FdSteps h, const int32_t *pairs, int n_pairs, int nb,
                                 double *g0, double *gb0, double *u_eps, int32_t *pairs_out,
                                 int64_t *field_off, int32_t *field_of) {
  const int i = blockIdx.x, t = threadIdx.x;
  if (i == 0 && t == 0) {
    field_off[0] = 0;
    field_off[1] = n_cur[0];
  }
  if (t < 7) {
    double v = g_cur[t];
    if (i >= 1 && i <= 10 && t == 2 + (i - 1) / 2) v += (i % 2 == 1 ? 1.0 : -1.0) * h.hx[(i - 1) / 2];
    g0[i * 7 + t] = v;
  }
  for (int j = t; j < nb; j += blockDim.x) gb0[(size_t)i * nb + j] = gb_cur[j];
  if (t == 0) {
    u_eps[i] = i == 11 ? h.hu : i == 12 ? -h.hu : 0.0;
    field_of[i] = 0;
  }
  if (t < 2 * n_pairs) pairs_out[(size_t)i * 2 * n_pairs + t] = pairs[t];
}

// Central differences of the one-step accelerations (x_{k+1} - x_k)/dt of
// rows x_dot, z_dot, theta_dot, and the explicit Euler map of Eq. 28's form.
__global__ void fd_jacobian_kernel(const double *g0, const double *g1, double dt, FdSteps h,
                                   double *A, double *B, double *x_nom) {
  if (threadIdx.x != 0) return;
  auto acc = [&](int i, int r) { return (g1[i * 7 + 4 + r] - g0[i * 7 + 4 + r]) / dt; };
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) A[r * 7 + c] = r == c ? 1.0 : 0.0;
  A[0 * 7 + 4] = A[1 * 7 + 5] = A[2 * 7 + 6] = dt;
  for (int r = 0; r < 7; ++r) B[r] = 0.0;
  B[3] = dt;
  for (int r = 0; r < 3; ++r) {
    for (int j = 0; j < 5; ++j)
      A[(4 + r) * 7 + 2 + j] += dt * (acc(1 + 2 * j, r) - acc(2 + 2 * j, r)) / (2.0 * h.hx[j]);
    B[4 + r] = dt * (acc(11, r) - acc(12, r)) / (2.0 * h.hu);
  }
  if (x_nom)
    for (int c = 0; c < 7; ++c) x_nom[c] = g0[c];
}

// Start state into the first of the two state buffers; field offsets of the
// wake output layout.
__global__ void fd_init_kernel(int32_t *n_cur, int n_wake, int64_t *wake_off, int64_t cap) {
  if (threadIdx.x == 0) {
    n_cur[0] = n_wake;
    wake_off[0] = 0;
    wake_off[1] = cap;
  }
}

struct FdLayout {
  double *g[2], *gb[2], *wx[2], *wz[2], *wg[2];
  int32_t *n[2];
  int64_t *wake_off, *field_off;
  double *g0, *gb0, *u_eps, *g1, *cost, *zero, *cost1;
  int32_t *status, *status1, *pairs, *field_of;
  size_t bytes;
};

FdLayout fd_layout(char *base, const vpm_fd_in *in, int nb) {
  Arena ar{base, 0};
  FdLayout L{};
  const size_t cap = (size_t)in->n_wake + 2 * (size_t)in->H + 2;
  for (int s = 0; s < 2; ++s) {
    L.g[s] = ar.take<double>(7);
    L.gb[s] = ar.take<double>(nb);
    L.wx[s] = ar.take<double>(cap);
    L.wz[s] = ar.take<double>(cap);
    L.wg[s] = ar.take<double>(cap);
    L.n[s] = ar.take<int32_t>(1);
  }
  L.wake_off = ar.take<int64_t>(2);
  L.field_off = ar.take<int64_t>(2);
  L.g0 = ar.take<double>(kFdRows * 7);
  L.gb0 = ar.take<double>((size_t)kFdRows * nb);
  L.u_eps = ar.take<double>(kFdRows);
  L.g1 = ar.take<double>(kFdRows * 7);
  L.cost = ar.take<double>(kFdRows);
  L.zero = ar.take<double>(1);
  L.cost1 = ar.take<double>(1);
  L.status = ar.take<int32_t>(kFdRows);
  L.status1 = ar.take<int32_t>(1);
  L.pairs = ar.take<int32_t>((size_t)kFdRows * 2 * (in->n_pairs > 0 ? in->n_pairs : 1));
  L.field_of = ar.take<int32_t>(kFdRows);
  L.bytes = ar.off + 256;
  return L;
}

}  // namespace

int check_fd(const vpm_params *p, const vpm_fd_in *in, const vpm_fd_out *out) {
  if (!p || !in || !out) return fail(VPM_EINVAL, "params, in or out is NULL");
  if (!(std::isfinite(in->dt) && in->dt > 0.0)) return fail(VPM_EINVAL, "dt must be > 0");
  if (in->H < 1) return fail(VPM_EINVAL, "H must be >= 1");
  if (in->n_wake < 0) return fail(VPM_EINVAL, "n_wake must be >= 0");
  if (in->n_pairs < 0 || in->n_pairs > kMaxPairs) return fail(VPM_EINVAL, "n_pairs must be 0..4");
  if (in->n_pairs > 0) {
    if (!in->pairs) return fail(VPM_EINVAL, "pairs is NULL with n_pairs > 0");
    if (p->n_wake_max > 0 && (long long)in->n_wake + 2LL * in->H > p->n_wake_max)
      return fail(VPM_EINVAL, "disturbance pairs need a wake that cannot merge within H steps");
  }
  for (double h : in->h_x)
    if (!(std::isfinite(h) && h > 0.0)) return fail(VPM_EINVAL, "h_x must be > 0");
  if (!(std::isfinite(in->h_u) && in->h_u > 0.0)) return fail(VPM_EINVAL, "h_u must be > 0");
  if (!in->g || !in->gb || !in->u_nom) return fail(VPM_EINVAL, "a required input pointer is NULL");
  if (in->n_wake > 0 && (!in->wx || !in->wz || !in->wg))
    return fail(VPM_EINVAL, "wake pointers are NULL");
  if (!out->a || !out->b) return fail(VPM_EINVAL, "a required output pointer is NULL");
  return VPM_OK;
}

int run_fd(vpm_ctx *ctx, const vpm_params *p, const vpm_fd_in *in, vpm_fd_out *out,
           hipStream_t stream) {
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const int nb = p->n_bound, H = in->H;
  std::lock_guard<std::mutex> lock(ctx->replan_mu);
  FdLayout L = fd_layout(nullptr, in, nb);
  int rc = ensure_buffer(&ctx->fd, &ctx->fd_bytes, L.bytes, "finite-difference workspace",
                         stream_capturing(stream));
  if (rc != VPM_OK) return rc;
  L = fd_layout(static_cast<char *>(ctx->fd), in, nb);
  vpm_params p64 = *p;
  p64.precision = VPM_FP64;
  void *sv = stream;
  const int64_t cap = (int64_t)in->n_wake + 2 * (int64_t)H + 2;
  FdSteps h{};
  for (int j = 0; j < 5; ++j) h.hx[j] = in->h_x[j];
  h.hu = in->h_u;
  // the start state into buffer 0
  hipLaunchKernelGGL(fd_init_kernel, dim3(1), dim3(64), 0, stream, L.n[0], in->n_wake, L.wake_off,
                     cap);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(kFill), 0, stream, L.zero, (size_t)1, 0.0);
  VPM_HIP_TRY(hipMemcpyAsync(L.g[0], in->g, 7 * sizeof(double), hipMemcpyDeviceToDevice, stream));
  VPM_HIP_TRY(hipMemcpyAsync(L.gb[0], in->gb, nb * sizeof(double), hipMemcpyDeviceToDevice,
                             stream));
  if (in->n_wake > 0) {
    const size_t nw = (size_t)in->n_wake * sizeof(double);
    VPM_HIP_TRY(hipMemcpyAsync(L.wx[0], in->wx, nw, hipMemcpyDeviceToDevice, stream));
    VPM_HIP_TRY(hipMemcpyAsync(L.wz[0], in->wz, nw, hipMemcpyDeviceToDevice, stream));
    VPM_HIP_TRY(hipMemcpyAsync(L.wg[0], in->wg, nw, hipMemcpyDeviceToDevice, stream));
  }
  auto batch = [&](int cur, int K, const double *g0, const double *gb0, const double *u_mean,
                   const double *u_eps, int max_wake0) {
    vpm_batch_in b{};
    b.K = K;
    b.H = 1;
    b.dt = in->dt;
    b.n_fields = 1;
    b.max_wake0 = max_wake0;
    b.n_pairs = in->n_pairs;
    b.g0 = g0;
    b.gb0 = gb0;
    b.field_off = L.field_off;
    b.field_of = L.field_of;
    b.wx = L.wx[cur];
    b.wz = L.wz[cur];
    b.wg = L.wg[cur];
    b.pairs = in->n_pairs > 0 ? L.pairs : nullptr;
    b.u_mean = u_mean;
    b.u_eps = u_eps;
    for (int i = 0; i < 7; ++i) b.q_diag[i] = 0.0;
    return b;
  };
  int cur = 0;
  for (int k = 0; k < H; ++k) {
    const int max_wake0 = in->n_wake + 2 * k;
    hipLaunchKernelGGL(fd_inputs_kernel, dim3(kFdRows), dim3(64), 0, stream, L.g[cur], L.gb[cur],
                       L.n[cur], h, in->pairs, in->n_pairs, nb, L.g0, L.gb0, L.u_eps, L.pairs,
                       L.field_off, L.field_of);
    VPM_HIP_TRY(hipGetLastError());
    // the 13 perturbed one-step rollouts, then their differences
    vpm_batch_in b = batch(cur, kFdRows, L.g0, L.gb0, in->u_nom + k, L.u_eps, max_wake0);
    vpm_batch_out o{};
    o.g_final = L.g1;
    o.cost = L.cost;
    o.status = L.status;
    rc = vpm_rollout_batch(ctx, &p64, &b, &o, sv);
    if (rc != VPM_OK) return rc;
    hipLaunchKernelGGL(fd_jacobian_kernel, dim3(1), dim3(64), 0, stream, L.g0, L.g1, in->dt, h,
                       out->a + (size_t)k * 49, out->b + (size_t)k * 7,
                       out->x_nom ? out->x_nom + (size_t)k * 7 : nullptr);
    VPM_HIP_TRY(hipGetLastError());
    // advance the nominal one step (same inputs as row 0) into the other buffer
    vpm_batch_in bn = batch(cur, 1, L.g[cur], L.gb[cur], in->u_nom + k, L.zero, max_wake0);
    vpm_batch_out on{};
    on.g_final = L.g[1 - cur];
    on.cost = L.cost1;
    on.status = L.status1;
    on.wake_off = L.wake_off;
    on.wx = L.wx[1 - cur];
    on.wz = L.wz[1 - cur];
    on.wg = L.wg[1 - cur];
    on.n_final = L.n[1 - cur];
    on.gb_final = L.gb[1 - cur];
    rc = vpm_rollout_batch(ctx, &p64, &bn, &on, sv);
    if (rc != VPM_OK) return rc;
    cur = 1 - cur;
  }
  if (out->x_nom)
    VPM_HIP_TRY(hipMemcpyAsync(out->x_nom + (size_t)H * 7, L.g[cur], 7 * sizeof(double),
                               hipMemcpyDeviceToDevice, stream));
  return VPM_OK;
}

}  // namespace vpm
