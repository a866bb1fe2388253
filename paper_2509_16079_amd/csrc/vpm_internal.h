// vpm_internal.h -- private declarations of the gfx950 rollout library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host_common.h"
#include "vpm.h"

namespace vpm {

#define VPM_HIP_TRY(expr)                                                   \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess)                                                   \
      return ::vpm::fail(VPM_EDEVICE, std::string(#expr ": ") +             \
                                          hipGetErrorString(_e));           \
  } while (0)

// FP32 kernel shape of one class: targets per thread (pass-A register
// blocking) and sources per compensated tile.
struct Tune {
  int tmax, tile;
};

struct PlateKey {
  int nb, mode;
  double chord, shed_frac, r_core;
  bool operator<(const PlateKey &o) const {
    return std::tie(nb, mode, chord, shed_frac, r_core) <
           std::tie(o.nb, o.mode, o.chord, o.shed_frac, o.r_core);
  }
};

}  // namespace vpm

struct vpm_ctx {
  int device = 0;
  int max_lds = 65536;      // dynamic LDS bytes one workgroup may use
  int n_cu = 0;
  int path = VPM_PATH_AUTO; // kernel variant selection (vpm_set_path)
  // FP32 shape per kernel class (vpm_set_tuning): small, large, streamed
  vpm::Tune tune[3] = {{4, 64}, {2, 64}, {4, 64}};
  std::mutex mu;
  std::map<vpm::PlateKey, double *> plate_cache;  // device inverses
  // streaming-kernel workspace, shared by calls on this context; each launch
  // that uses it waits for the previous one (ws_event) whatever the stream
  std::mutex ws_mu;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  void *plan = nullptr;  // uneven-batch order and class cursors
  size_t plan_bytes = 0;
  hipEvent_t ws_event = nullptr;
  bool ws_event_valid = false;
  // forked streams for the class kernels of an uneven batch (default
  // priority) and the events that fork and join them
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork_event = nullptr;
  hipEvent_t join_event[3] = {nullptr, nullptr, nullptr};
  // replanning-cycle and finite-difference workspaces, grown on demand
  std::mutex replan_mu;
  void *replan = nullptr;
  size_t replan_bytes = 0;
  void *fd = nullptr;
  size_t fd_bytes = 0;
  void *scratch = nullptr;  // this device's static scratch (noalloc calls)
};

namespace vpm {

// Device inverse for a plate (cached in the context; building one is
// refused while the caller's stream is captured into a graph).
int plate_inverse_device(vpm_ctx *ctx, const vpm_params *p, int mode,
                         const double **out, bool capturing);

// True if `stream` is being captured into a graph.
bool stream_capturing(hipStream_t stream);

// Largest wake capacity (N_0 + 2H) the LDS-resident kernel holds on a gfx950
// workgroup (160 KB of LDS) in a precision (VPM_FP32C or VPM_FP64, with the
// large class's default 2 targets per thread); larger wakes take the
// streaming kernel.
int lds_resident_capacity(int nb, int precision);

// Create the context's side streams for the class kernels of uneven batches
// (on first use, so that contexts that never run one hold no idle streams).
int ensure_side_streams(vpm_ctx *ctx, bool capturing);

// Grow the context's workspace and plan buffers for later batches of these
// sizes (vpm_reserve).
int reserve_rollout(vpm_ctx *ctx, const vpm_params *p, int K, int H, int max_wake0,
                    int n_fields);

// kinv_t: inverse of the plate system of p->shed_mode; kinv_te: of the
// trailing-edge-only system when the separation gate is on (else NULL).
// noalloc: the scratch comes from the library's static device array
// (vpm_rollout_batch_noalloc) instead of the context's buffers.
int launch_rollout(vpm_ctx *ctx, const vpm_params *p, const vpm_batch_in *in,
                   vpm_batch_out *out, const double *kinv_t, const double *kinv_te,
                   hipStream_t stream, bool noalloc);

// Size of the static scratch of vpm_rollout_batch_noalloc.
constexpr size_t kScratchBytes = VPM_NOALLOC_SCRATCH_BYTES;

// Device address of this device's copy of the static scratch (looked up once
// per device, which must be current).
int static_scratch_address(int device, void **out);
int launch_plate_solve(const vpm_params *p, int B, const double *pose,
                       const double *vw_c, const double *sum_gw, int mode,
                       const double *kinv_t, double *gamma_s,
                       hipStream_t stream);
int launch_policy(const vpm_policy_in *in, vpm_policy_out *out, hipStream_t stream);
int launch_tvlqr(int H, const double *a, const double *b, const double *q_f, const double *q_c,
                 double r_c, double *gain, double *s, hipStream_t stream);
// Host-only argument checks (no device access) and drivers of vpm_fd_jacobians.
int check_fd(const vpm_params *p, const vpm_fd_in *in, const vpm_fd_out *out);
int run_fd(vpm_ctx *ctx, const vpm_params *p, const vpm_fd_in *in, vpm_fd_out *out,
           hipStream_t stream);
// Host-only argument check of vpm_replan (no device access).
int check_replan(const vpm_params *p, const vpm_replan_in *in, const vpm_replan_out *out);
int run_replan(vpm_ctx *ctx, const vpm_params *p, const vpm_replan_in *in, vpm_replan_out *out,
               hipStream_t stream);
// Grow *buf to at least `bytes` (device-synchronises before freeing).
int ensure_buffer(void **buf, size_t *have, size_t bytes, const char *what, bool capturing);
int launch_mppi(int K, int H, const double *cost, double lambda,
                const double *u_mean, const double *u_eps, double *w_out,
                double *u_new, int32_t *argmin, double *jmin,
                hipStream_t stream);

}  // namespace vpm
