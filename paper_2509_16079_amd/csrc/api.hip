// api.hip -- the C ABI declared in include/vpm.h: context management, the
// device copy of the plate inverse and dispatch (argument checks are in
// host.cpp).
#include <cmath>
#include <cstring>
#include <string>

#include "vpm_internal.h"

namespace vpm {

int plate_inverse_device(vpm_ctx *ctx, const vpm_params *p, int mode,
                         const double **out, bool capturing) {
  PlateKey key{p->n_bound, mode, p->chord, p->shed_frac, p->r_core};
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto it = ctx->plate_cache.find(key);
  if (it != ctx->plate_cache.end()) {
    *out = it->second;
    return VPM_OK;
  }
  if (capturing)
    return fail(VPM_EINVAL, "the plate inverse of this geometry must be built by an "
                            "eager call before graph capture");
  std::vector<double> inv_t;
  int rc = plate_inverse_T(p->n_bound, p->chord, p->shed_frac, p->r_core, mode,
                           inv_t);
  if (rc != VPM_OK) return fail(rc, "plate system is singular");
  double *d = nullptr;
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  if (hipMalloc(&d, inv_t.size() * sizeof(double)) != hipSuccess)
    return fail(VPM_ENOMEM, "hipMalloc of the plate inverse failed");
  hipError_t e = hipMemcpy(d, inv_t.data(), inv_t.size() * sizeof(double),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(VPM_EDEVICE, std::string("plate inverse upload: ") +
                                 hipGetErrorString(e));
  }
  ctx->plate_cache[key] = d;
  *out = d;
  return VPM_OK;
}

// The cached inverse only (calls that must not allocate).
int plate_inverse_cached(vpm_ctx *ctx, const vpm_params *p, int mode, const double **out) {
  PlateKey key{p->n_bound, mode, p->chord, p->shed_frac, p->r_core};
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto it = ctx->plate_cache.find(key);
  if (it == ctx->plate_cache.end())
    return fail(VPM_EINVAL, "the plate inverse of this geometry is not built: call vpm_reserve "
                            "(or vpm_rollout_batch) with these params first");
  *out = it->second;
  return VPM_OK;
}

bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

}  // namespace vpm

using vpm::fail;

extern "C" {

VPM_API int vpm_create(vpm_ctx **out, int device) {
  if (!out) return fail(VPM_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1)
    return fail(VPM_EDEVICE, "no HIP device");
  if (device < 0 || device >= n) return fail(VPM_EDEVICE, "no such device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(VPM_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(VPM_EDEVICE, std::string("device is ") + prop.gcnArchName +
                                 ", this library is built for gfx950");
  vpm_ctx *c = new (std::nothrow) vpm_ctx();
  if (!c) return fail(VPM_ENOMEM, "context allocation failed");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  int lds = 0, optin = 0;
  (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  (void)hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device);
  c->max_lds = lds > optin ? lds : optin;
  if (c->max_lds <= 0) c->max_lds = 65536;
  // the side streams of uneven batches are created on first use: a context
  // that never runs one (as each planner slot's) holds no idle streams, which
  // would otherwise share the process's hardware queues with busy ones
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->fork_event, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    vpm_destroy(c);
    return fail(VPM_EDEVICE, "stream or event creation failed");
  }
  const int rc = vpm::static_scratch_address(device, &c->scratch);
  if (rc != VPM_OK) {
    vpm_destroy(c);
    return rc;
  }
  *out = c;
  return VPM_OK;
}

VPM_API int vpm_set_path(vpm_ctx *ctx, int path) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  if (path < VPM_PATH_AUTO || path > VPM_PATH_STREAM)
    return fail(VPM_EINVAL, "unknown path");
  ctx->path = path;
  return VPM_OK;
}

VPM_API void vpm_destroy(vpm_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto &kv : ctx->plate_cache) (void)hipFree(kv.second);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->plan) (void)hipFree(ctx->plan);
  if (ctx->replan) (void)hipFree(ctx->replan);
  if (ctx->fd) (void)hipFree(ctx->fd);
  if (ctx->ws_event) (void)hipEventDestroy(ctx->ws_event);
  if (ctx->fork_event) (void)hipEventDestroy(ctx->fork_event);
  for (int i = 0; i < 3; ++i) {
    if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
    if (ctx->join_event[i]) (void)hipEventDestroy(ctx->join_event[i]);
  }
  delete ctx;
}

VPM_API int vpm_rollout_batch(vpm_ctx *ctx, const vpm_params *params,
                              const vpm_batch_in *in, vpm_batch_out *out,
                              void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm_validate_batch(params, in, out);
  if (rc != VPM_OK) return rc;
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const bool capturing = vpm::stream_capturing(static_cast<hipStream_t>(stream));
  const double *kinv = nullptr, *kinv_te = nullptr;
  rc = vpm::plate_inverse_device(ctx, params, params->shed_mode, &kinv, capturing);
  if (rc == VPM_OK && params->gate)
    rc = vpm::plate_inverse_device(ctx, params, VPM_SHED_TE, &kinv_te, capturing);
  if (rc != VPM_OK) return rc;
  return vpm::launch_rollout(ctx, params, in, out, kinv, kinv_te,
                             static_cast<hipStream_t>(stream), false);
}

VPM_API int vpm_rollout_batch_noalloc(vpm_ctx *ctx, const vpm_params *params,
                                      const vpm_batch_in *in, vpm_batch_out *out,
                                      void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm_validate_batch(params, in, out);
  if (rc != VPM_OK) return rc;
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const double *kinv = nullptr, *kinv_te = nullptr;
  rc = vpm::plate_inverse_cached(ctx, params, params->shed_mode, &kinv);
  if (rc == VPM_OK && params->gate)
    rc = vpm::plate_inverse_cached(ctx, params, VPM_SHED_TE, &kinv_te);
  if (rc != VPM_OK) return rc;
  return vpm::launch_rollout(ctx, params, in, out, kinv, kinv_te,
                             static_cast<hipStream_t>(stream), true);
}

VPM_API int vpm_set_tuning(vpm_ctx *ctx, int32_t kernel_class, int32_t targets_per_thread,
                           int32_t tile) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  if (kernel_class < VPM_CLASS_SMALL || kernel_class > VPM_CLASS_STREAM)
    return fail(VPM_EINVAL, "unknown kernel class");
  if (targets_per_thread != 1 && targets_per_thread != 2 && targets_per_thread != 4)
    return fail(VPM_EINVAL, "targets_per_thread must be 1, 2 or 4");
  if (tile != 64 && tile != 128 && tile != 256)
    return fail(VPM_EINVAL, "tile must be 64, 128 or 256");
  std::lock_guard<std::mutex> lock(ctx->ws_mu);
  ctx->tune[kernel_class] = vpm::Tune{targets_per_thread, tile};
  return VPM_OK;
}

VPM_API int vpm_get_tuning(const vpm_ctx *ctx, int32_t kernel_class,
                           int32_t *targets_per_thread, int32_t *tile) {
  if (!ctx || !targets_per_thread || !tile) return fail(VPM_EINVAL, "NULL argument");
  if (kernel_class < VPM_CLASS_SMALL || kernel_class > VPM_CLASS_STREAM)
    return fail(VPM_EINVAL, "unknown kernel class");
  *targets_per_thread = ctx->tune[kernel_class].tmax;
  *tile = ctx->tune[kernel_class].tile;
  return VPM_OK;
}

VPM_API int vpm_reserve(vpm_ctx *ctx, const vpm_params *params, int32_t K, int32_t H,
                        int32_t max_wake0, int32_t n_fields) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm::check_params(params);
  if (rc != VPM_OK) return rc;
  if (K < 1 || H < 1 || max_wake0 < 0 || n_fields < 1)
    return fail(VPM_EINVAL, "K, H, n_fields must be >= 1 and max_wake0 >= 0");
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const double *kinv = nullptr;
  rc = vpm::plate_inverse_device(ctx, params, params->shed_mode, &kinv, false);
  if (rc == VPM_OK && params->gate)
    rc = vpm::plate_inverse_device(ctx, params, VPM_SHED_TE, &kinv, false);
  if (rc != VPM_OK) return rc;
  return vpm::reserve_rollout(ctx, params, K, H, max_wake0, n_fields);
}

VPM_API int vpm_plate_solve(vpm_ctx *ctx, const vpm_params *params, int32_t B,
                            const double *pose, const double *vw_c,
                            const double *sum_gw, int32_t shed_mode,
                            double *gamma_s, void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm::check_params(params);
  if (rc != VPM_OK) return rc;
  if (shed_mode < VPM_SHED_BOTH || shed_mode > VPM_SHED_NONE)
    return fail(VPM_EINVAL, "unknown shed_mode");
  if (shed_mode == VPM_SHED_NONE && params->n_bound < 2)
    return fail(VPM_EINVAL, "shed_mode NONE needs n_bound >= 2");
  if (B < 0) return fail(VPM_EINVAL, "B must be >= 0");
  if (B == 0) return VPM_OK;
  if (!pose || !vw_c || !sum_gw || !gamma_s)
    return fail(VPM_EINVAL, "a pointer is NULL");
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  const double *kinv = nullptr;
  rc = vpm::plate_inverse_device(ctx, params, shed_mode, &kinv,
                                 vpm::stream_capturing(static_cast<hipStream_t>(stream)));
  if (rc != VPM_OK) return rc;
  return vpm::launch_plate_solve(params, B, pose, vw_c, sum_gw, shed_mode, kinv,
                                 gamma_s, static_cast<hipStream_t>(stream));
}

VPM_API int mppi_weights(vpm_ctx *ctx, int32_t K, int32_t H, const double *cost,
                         double lambda, const double *u_mean,
                         const double *u_eps, double *w_out, double *u_new,
                         int32_t *argmin, double *jmin, void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  if (K < 1 || H < 1) return fail(VPM_EINVAL, "K and H must be >= 1");
  if (!vpm::finite_pos(lambda)) return fail(VPM_EINVAL, "lambda must be > 0");
  if (!cost || !u_mean || !u_eps || !w_out || !u_new || !argmin || !jmin)
    return fail(VPM_EINVAL, "a pointer is NULL");
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  return vpm::launch_mppi(K, H, cost, lambda, u_mean, u_eps, w_out, u_new,
                          argmin, jmin, static_cast<hipStream_t>(stream));
}

VPM_API int vpm_policy(vpm_ctx *ctx, const vpm_policy_in *in, vpm_policy_out *out,
                       void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  if (!in || !out) return fail(VPM_EINVAL, "in or out is NULL");
  if (in->K < 1 || in->H < 1) return fail(VPM_EINVAL, "K and H must be >= 1");
  if (!vpm::finite_pos(in->dt)) return fail(VPM_EINVAL, "dt must be > 0");
  if (!vpm::finite_pos(in->r_c)) return fail(VPM_EINVAL, "r_c must be > 0");
  for (int i = 0; i < 7; ++i)
    if (!(std::isfinite(in->q_f[i]) && in->q_f[i] >= 0.0 && std::isfinite(in->q_c[i]) &&
          in->q_c[i] >= 0.0))
      return fail(VPM_EINVAL, "q_f and q_c must be finite and >= 0");
  if (!in->traj_nom || !in->traj || !in->du)
    return fail(VPM_EINVAL, "a required input pointer is NULL");
  if (!out->a || !out->b || !out->gain || !out->status)
    return fail(VPM_EINVAL, "a required output pointer is NULL");
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  return vpm::launch_policy(in, out, static_cast<hipStream_t>(stream));
}

VPM_API int vpm_replan(vpm_ctx *ctx, const vpm_params *params, const vpm_replan_in *in,
                       vpm_replan_out *out, void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm::check_params(params);
  if (rc == VPM_OK) rc = vpm::check_replan(params, in, out);
  if (rc != VPM_OK) return rc;
  return vpm::run_replan(ctx, params, in, out, static_cast<hipStream_t>(stream));
}

VPM_API int vpm_tvlqr(vpm_ctx *ctx, int32_t H, const double *a, const double *b,
                      const double q_f[7], const double q_c[7], double r_c, double *gain,
                      double *s, void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  if (H < 1) return fail(VPM_EINVAL, "H must be >= 1");
  if (!a || !b || !gain || !q_f || !q_c) return fail(VPM_EINVAL, "a pointer is NULL");
  if (!vpm::finite_pos(r_c)) return fail(VPM_EINVAL, "r_c must be > 0");
  for (int i = 0; i < 7; ++i)
    if (!(std::isfinite(q_f[i]) && q_f[i] >= 0.0 && std::isfinite(q_c[i]) && q_c[i] >= 0.0))
      return fail(VPM_EINVAL, "q_f and q_c must be finite and >= 0");
  VPM_HIP_TRY(hipSetDevice(ctx->device));
  return vpm::launch_tvlqr(H, a, b, q_f, q_c, r_c, gain, s, static_cast<hipStream_t>(stream));
}

VPM_API int vpm_fd_jacobians(vpm_ctx *ctx, const vpm_params *params, const vpm_fd_in *in,
                             vpm_fd_out *out, void *stream) {
  if (!ctx) return fail(VPM_EINVAL, "ctx is NULL");
  int rc = vpm::check_params(params);
  if (rc == VPM_OK) rc = vpm::check_fd(params, in, out);
  if (rc != VPM_OK) return rc;
  return vpm::run_fd(ctx, params, in, out, static_cast<hipStream_t>(stream));
}

}  // extern "C"
