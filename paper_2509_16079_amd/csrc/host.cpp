// host.cpp -- host-only parts of the C ABI declared in include/vpm.h: the
// per-thread error message, the argument checks (pure host code, run before
// any HIP call) and the exact pair-interaction count.
#include <cmath>
#include <string>

#include "host_common.h"

namespace vpm {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }
int fail(int code, const std::string &msg) {
  g_error = msg;
  return code;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_params(const vpm_params *p) {
  if (!p) return fail(VPM_EINVAL, "params is NULL");
  if (p->n_bound < 1 || p->n_bound > kMaxBound)
    return fail(VPM_EINVAL, "n_bound must be in 1..64");
  if (p->shed_mode < VPM_SHED_BOTH || p->shed_mode > VPM_SHED_NONE)
    return fail(VPM_EINVAL, "unknown shed_mode");
  if (p->precision != VPM_FP32C && p->precision != VPM_FP64)
    return fail(VPM_EINVAL, "unknown precision");
  if (!finite_pos(p->chord)) return fail(VPM_EINVAL, "chord must be > 0");
  if (!(std::isfinite(p->shed_frac) && p->shed_frac >= 0.0))
    return fail(VPM_EINVAL, "shed_frac must be >= 0");
  if (!(std::isfinite(p->r_core) && p->r_core >= 1e-6))
    return fail(VPM_EINVAL, "r_core must be >= 1e-6 m");
  if (!(std::isfinite(p->decay) && p->decay >= 0.0))
    return fail(VPM_EINVAL, "decay must be >= 0");
  if (!finite_pos(p->mass) || !finite_pos(p->inertia))
    return fail(VPM_EINVAL, "mass and inertia must be > 0");
  const double f[] = {p->rho, p->span, p->grav, p->l_body, p->l_wing,
                      p->l_elev, p->s_elev};
  for (double v : f)
    if (!std::isfinite(v)) return fail(VPM_EINVAL, "non-finite parameter");
  if (p->gate != 0 && p->gate != 1) return fail(VPM_EINVAL, "gate must be 0 or 1");
  if (p->gate && (p->shed_mode != VPM_SHED_BOTH || !std::isfinite(p->alpha_crit)))
    return fail(VPM_EINVAL, "the separation gate needs shed_mode BOTH and a finite alpha_crit");
  if (p->shed_mode == VPM_SHED_NONE && p->n_bound < 2)
    return fail(VPM_EINVAL, "shed_mode NONE needs n_bound >= 2");
  return VPM_OK;
}

}  // namespace vpm

using vpm::fail;

extern "C" {

VPM_API const char *vpm_last_error(void) { return vpm::g_error.c_str(); }

VPM_API int vpm_validate_batch(const vpm_params *p, const vpm_batch_in *in,
                               const vpm_batch_out *out) {
  int rc = vpm::check_params(p);
  if (rc != VPM_OK) return rc;
  if (!in || !out) return fail(VPM_EINVAL, "in or out is NULL");
  if (in->K < 1 || in->H < 1) return fail(VPM_EINVAL, "K and H must be >= 1");
  if (!vpm::finite_pos(in->dt)) return fail(VPM_EINVAL, "dt must be > 0");
  if (in->n_fields < 1) return fail(VPM_EINVAL, "n_fields must be >= 1");
  if (in->max_wake0 < 0) return fail(VPM_EINVAL, "max_wake0 must be >= 0");
  if ((long long)in->max_wake0 + 2LL * in->H > (1LL << 30))
    return fail(VPM_EINVAL, "max_wake0 + 2H too large");
  if (in->n_pairs < 0 || in->n_pairs > vpm::kMaxPairs)
    return fail(VPM_EINVAL, "n_pairs must be in 0..4");
  if (in->n_pairs > 0 && !in->pairs)
    return fail(VPM_EINVAL, "pairs is NULL with n_pairs > 0");
  if (!in->g0 || !in->gb0 || !in->field_off || !in->wx || !in->wz ||
      !in->wg || !in->u_mean || !in->u_eps)
    return fail(VPM_EINVAL, "a required input pointer is NULL");
  if (!in->field_of && in->n_fields < in->K)
    return fail(VPM_EINVAL, "field_of is NULL but n_fields < K");
  if ((in->fb_gain == nullptr) != (in->fb_xref == nullptr))
    return fail(VPM_EINVAL, "fb_gain and fb_xref go together");
  for (int i = 0; i < 7; ++i)
    if (!std::isfinite(in->x_goal[i]) || !std::isfinite(in->q_diag[i]))
      return fail(VPM_EINVAL, "non-finite x_goal or q_diag");
  if (!out->g_final || !out->cost || !out->status)
    return fail(VPM_EINVAL, "g_final, cost and status are required");
  const bool any_wake = out->wx || out->wz || out->wg || out->vel_last;
  if (any_wake && (!out->wake_off || !out->n_final))
    return fail(VPM_EINVAL, "wake outputs need wake_off and n_final");
  return VPM_OK;
}

VPM_API int64_t vpm_pair_count(int32_t n0, int32_t H, int32_t n_bound,
                               int32_t n_wake_max) {
  int64_t total = 0, n = n0;
  for (int32_t s = 0; s < H; ++s) {
    const int64_t m = n + 2;
    total += n * (2 * n_bound + 1) + m * (m - 1) + m * n_bound;
    n = m;
    if (n_wake_max > 0 && n > n_wake_max) n = n_wake_max;
  }
  return total;
}

}  // extern "C"
