// solve_mppi.hip -- the standalone FP64 surface solve and the MPPI
// reweighting kernels.
#include <cmath>

#include "vpm_internal.h"

namespace vpm {
namespace {

constexpr int kThreads = 256;

// One wave per pose: lane r assembles row r of b (Eqs. 10 and 12) and row r
// of Gamma_S = K^-1 b (Eq. 11).
__global__ __launch_bounds__(kThreads) void plate_solve_kernel(
    int B, int nb, int S, int r0, double chord, const double *__restrict__ pose,
    const double *__restrict__ vw_c, const double *__restrict__ sum_gw,
    const double *__restrict__ kinv_t, double *__restrict__ gamma_s) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (b >= B) return;  // uniform per wave
  const double *ps = pose + 6 * (size_t)b;
  const double xw = ps[0], zw = ps[1], th = ps[2], xwd = ps[3], zwd = ps[4],
               thd = ps[5];
  const double ct = cos(th), st = sin(th), lb = chord / nb;
  const double lex = xw + 0.5 * chord * ct, lez = zw + 0.5 * chord * st;
  const double etx = -ct, etz = -st, enx = -st, enz = ct;
  auto rhs = [&](int r) -> double {
    if (r >= S) return 0.0;
    if (r == S - 1) return -sum_gw[b];
    const int i = r0 + r;
    const double px = lex + i * lb * etx, pz = lez + i * lb * etz;
    const double *v = vw_c + ((size_t)b * (nb + 1) + i) * 2;
    const double vx = v[0] - xwd + thd * (pz - zw);
    const double vz = v[1] - zwd - thd * (px - xw);
    return -(vx * enx + vz * enz);
  };
  const double b0 = rhs(lane), b1 = rhs(lane + 64);
  double g0 = 0.0, g1 = 0.0;
  for (int j = 0; j < S; ++j) {
    const double bj = j < 64 ? __shfl(b0, j, 64) : __shfl(b1, j - 64, 64);
    if (lane < S) g0 += kinv_t[j * S + lane] * bj;
    if (lane + 64 < S) g1 += kinv_t[j * S + lane + 64] * bj;
  }
  if (lane < S) gamma_s[(size_t)b * S + lane] = g0;
  if (lane + 64 < S) gamma_s[(size_t)b * S + lane + 64] = g1;
}

// MPPI step 1 (one workgroup): J_min and argmin over finite costs (lowest
// index on ties), then w_i = exp(-(J_i - J_min)/lambda) / sum (Eq. 25) with
// an FP64 normaliser reduced in a fixed tree order.
constexpr int kMppiThreads = 1024;

__global__ __launch_bounds__(kMppiThreads) void mppi_weights_kernel(
    int K, const double *__restrict__ cost, double lambda,
    double *__restrict__ w, int32_t *__restrict__ argmin,
    double *__restrict__ jmin) {
  __shared__ double sj[kMppiThreads];
  __shared__ int si[kMppiThreads];
  const int t = threadIdx.x;
  double best = INFINITY;
  int bi = -1;
  for (int i = t; i < K; i += kMppiThreads) {
    const double c = cost[i];
    if (isfinite(c) && c < best) {  // i increases: first minimum kept
      best = c;
      bi = i;
    }
  }
  sj[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int o = kMppiThreads / 2; o > 0; o >>= 1) {
    if (t < o) {
      const double c2 = sj[t + o];
      const int i2 = si[t + o];
      if (i2 >= 0 && (si[t] < 0 || c2 < sj[t] || (c2 == sj[t] && i2 < si[t]))) {
        sj[t] = c2;
        si[t] = i2;
      }
    }
    __syncthreads();
  }
  const double jm = sj[0];
  const int am = si[0];
  __syncthreads();
  double part = 0.0;
  if (am >= 0)
    for (int i = t; i < K; i += kMppiThreads) {
      const double c = cost[i];
      if (isfinite(c)) part += exp(-(c - jm) / lambda);
    }
  sj[t] = part;
  __syncthreads();
  for (int o = kMppiThreads / 2; o > 0; o >>= 1) {
    if (t < o) sj[t] += sj[t + o];
    __syncthreads();
  }
  const double eta = am >= 0 ? 1.0 / sj[0] : 0.0;
  for (int i = t; i < K; i += kMppiThreads) {
    const double c = cost[i];
    w[i] = (am >= 0 && isfinite(c)) ? exp(-(c - jm) / lambda) * eta : 0.0;
  }
  if (t == 0) {
    *argmin = am;
    *jmin = am >= 0 ? jm : INFINITY;
  }
}

// MPPI step 2: u_new[h] = u_mean[h] + sum_i w_i eps[i][h]. Each workgroup
// owns 64 consecutive h (lane = h, coalesced rows of eps); its 16 waves take
// contiguous slices of the samples and are combined in wave order.
constexpr int kUpdWaves = 16;

__global__ __launch_bounds__(64 * kUpdWaves) void mppi_update_kernel(
    int K, int H, const double *__restrict__ w, const double *__restrict__ u_mean,
    const double *__restrict__ u_eps, double *__restrict__ u_new) {
  __shared__ double part[kUpdWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = blockIdx.x * 64 + lane;
  const int i0 = (int)((long long)K * wave / kUpdWaves);
  const int i1 = (int)((long long)K * (wave + 1) / kUpdWaves);
  double acc = 0.0;
  if (h < H) {
#pragma unroll 4
    for (int i = i0; i < i1; ++i) acc += w[i] * u_eps[(size_t)i * H + h];
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && h < H) {
    double s = 0.0;
    for (int q = 0; q < kUpdWaves; ++q) s += part[q][lane];
    u_new[h] = u_mean[h] + s;
  }
}

}  // namespace

int launch_plate_solve(const vpm_params *p, int B, const double *pose,
                       const double *vw_c, const double *sum_gw, int mode,
                       const double *kinv_t, double *gamma_s,
                       hipStream_t stream) {
  const int nb = p->n_bound, S = system_size(nb, mode);
  const int waves_per_block = kThreads / 64;
  const int grid = (B + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(plate_solve_kernel, dim3(grid), dim3(kThreads), 0, stream,
                     B, nb, S, first_row(mode), p->chord, pose, vw_c, sum_gw,
                     kinv_t, gamma_s);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}

int launch_mppi(int K, int H, const double *cost, double lambda,
                const double *u_mean, const double *u_eps, double *w_out,
                double *u_new, int32_t *argmin, double *jmin,
                hipStream_t stream) {
  hipLaunchKernelGGL(mppi_weights_kernel, dim3(1), dim3(kMppiThreads), 0,
                     stream, K, cost, lambda, w_out, argmin, jmin);
  VPM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(mppi_update_kernel, dim3((H + 63) / 64), dim3(64 * kUpdWaves),
                     0, stream, K, H, w_out, u_mean, u_eps, u_new);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}

}  // namespace vpm
