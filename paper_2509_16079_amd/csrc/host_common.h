// host_common.h -- host-only declarations of the library (no HIP types), so
// that the argument checks, the plate system, the perturbation sampler and the
// planner's scheduler also build with a plain C++ compiler for host tests.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "vpm.h"

namespace vpm {

// Per-thread error message and a helper that records it.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

constexpr int kMaxPairs = 4;
constexpr int kMaxBound = 64;

// Shared by host code and kernels; a plain inline function for host-only
// compilers.
#ifdef __HIP__
#define VPM_HD __host__ __device__
#else
#define VPM_HD
#endif

// System size per shedding mode (bound unknowns, then LEV, then TEV).
VPM_HD inline int system_size(int nb, int mode) {
  return mode == VPM_SHED_BOTH ? nb + 2 : mode == VPM_SHED_TE ? nb + 1 : nb;
}
// First collocation row of the system per mode (LE row dropped unless BOTH).
VPM_HD inline int first_row(int mode) { return mode == VPM_SHED_BOTH ? 0 : 1; }

bool finite_pos(double v);

// Model parameter checks shared by every entry point (VPM_OK or VPM_EINVAL).
int check_params(const vpm_params *p);

// FP64 inverse of the surface matrix in the plate's body frame, returned
// transposed (column j of the inverse is contiguous) so that lane i of a wave
// reading entry (i, j) touches consecutive addresses. VPM_OK or VPM_ESINGULAR.
int plate_inverse_T(int nb, double chord, double shed_frac, double r_core, int mode,
                    std::vector<double> &inv_t);

// MPPI perturbations of one iteration from a seed (vpm_sample_eps).
void sample_eps(uint64_t seed, int iteration, int K, int H, double sigma, double *out);

}  // namespace vpm
