// policy.hip -- local feedback policy from rollouts on gfx950 (Sec. IV-B).
//
//   synthesis_kernel  one workgroup per step k: FP64 normal equations of the
//                     least-squares problem of Eq. 27 over the K perturbed
//                     rollouts (21 + 18 sums, wave reductions then LDS), and a
//                     column-scaled Cholesky solve for the 3 x 5 and 3 x 1
//                     unknown blocks of Eq. 28; writes the explicit Euler
//                     A_k, B_k.
//   riccati_kernel    one wavefront: the TVLQR recursion of Eqs. 29-30
//                     backwards over the steps, S in LDS, lane (r, c) owns
//                     entry (r, c) of the 7 x 7 products.
//
// The work is small (tens of KB per step) and latency-bound: the synthesis
// reads each rollout's two state rows of step k once (one thread per
// rollout, rows contiguous), the recursion is serial in k.
#include <hip/hip_runtime.h>

#include <cmath>

#include "vpm_internal.h"
#include "wave_ops.h"

namespace vpm {
namespace {

constexpr int kNx = 7;
constexpr int kReg = 6;     // regressors: theta, phi, x_dot, z_dot, theta_dot, u
constexpr int kAcc = 3;     // unknown rows: x_ddot, z_ddot, theta_ddot
constexpr int kGram = 21;   // upper triangle of the 6 x 6 normal matrix
constexpr int kSums = kGram + kReg * kAcc;
constexpr int kSynThreads = 256;
constexpr double kPivotTol = 1e-14;

// Order of this wave's LDS writes before its later LDS reads (one-wave
// kernel: no workgroup barrier, so no wait for outstanding global stores).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct PolicyArgs {
  int K, H;
  double dt;
  const double *traj_nom, *traj, *du;
  double q_f[kNx], q_c[kNx], r_c;
  double *a, *b, *gain, *s;
  int32_t *status;
};

__global__ __launch_bounds__(kSynThreads) void synthesis_kernel(PolicyArgs p) {
  __shared__ double part[kSynThreads / 64][kSums];
  __shared__ double tot[kSums];
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t row = (size_t)(p.H + 1) * kNx;  // doubles per rollout
  const double *n0 = p.traj_nom + (size_t)k * kNx, *n1 = n0 + kNx;
  const double inv_dt = 1.0 / p.dt;
  double acc[kSums];
#pragma unroll
  for (int q = 0; q < kSums; ++q) acc[q] = 0.0;
  for (int i = tid; i < p.K; i += kSynThreads) {
    const double *x0 = p.traj + i * row + (size_t)k * kNx, *x1 = x0 + kNx;
    double z[kReg], y[kAcc];
#pragma unroll
    for (int c = 0; c < 5; ++c) z[c] = x0[2 + c] - n0[2 + c];
    z[5] = p.du[(size_t)i * p.H + k];
    // rate deviations of the accelerations: (x_{k+1} - x_k)/dt of the
    // rollout minus that of the nominal
#pragma unroll
    for (int r = 0; r < kAcc; ++r)
      y[r] = (x1[4 + r] - x0[4 + r]) * inv_dt - (n1[4 + r] - n0[4 + r]) * inv_dt;
    int q = 0;
#pragma unroll
    for (int r = 0; r < kReg; ++r)
#pragma unroll
      for (int c = r; c < kReg; ++c) acc[q++] += z[r] * z[c];
#pragma unroll
    for (int r = 0; r < kReg; ++r)
#pragma unroll
      for (int c = 0; c < kAcc; ++c) acc[q++] += z[r] * y[c];
  }
#pragma unroll
  for (int q = 0; q < kSums; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) part[wave][q] = v;
  }
  __syncthreads();
  if (tid < kSums) {
    double v = 0.0;
    for (int w = 0; w < kSynThreads / 64; ++w) v += part[w][tid];
    tot[tid] = v;
  }
  __syncthreads();
  if (tid != 0) return;

  // normal equations G w = R (G = Z'Z, R = Z'Y), scaled to unit diagonal
  double G[kReg][kReg], R[kReg][kAcc];
  int q = 0;
#pragma unroll
  for (int r = 0; r < kReg; ++r)
#pragma unroll
    for (int c = r; c < kReg; ++c) G[r][c] = G[c][r] = tot[q++];
#pragma unroll
  for (int r = 0; r < kReg; ++r)
#pragma unroll
    for (int c = 0; c < kAcc; ++c) R[r][c] = tot[q++];
  bool ok = p.K >= kReg;
  double dinv[kReg];  // D^-1: column scales to unit diagonal
#pragma unroll
  for (int r = 0; r < kReg; ++r) {
    ok = ok && G[r][r] > 0.0;
    dinv[r] = G[r][r] > 0.0 ? 1.0 / sqrt(G[r][r]) : 1.0;
  }
  // Cholesky of D^-1 G D^-1 (a failed pivot leaves ok false and L finite);
  // the reciprocal of each pivot is kept, so the solves only multiply
  double L[kReg][kReg] = {}, linv[kReg];
#pragma unroll
  for (int j = 0; j < kReg; ++j) {
    double sjj = G[j][j] * dinv[j] * dinv[j];
#pragma unroll
    for (int m = 0; m < j; ++m) sjj -= L[j][m] * L[j][m];
    ok = ok && sjj > kPivotTol;
    L[j][j] = sjj > kPivotTol ? sqrt(sjj) : 1.0;
    linv[j] = 1.0 / L[j][j];
#pragma unroll
    for (int i = j + 1; i < kReg; ++i) {
      double v = G[i][j] * dinv[i] * dinv[j];
#pragma unroll
      for (int m = 0; m < j; ++m) v -= L[i][m] * L[j][m];
      L[i][j] = v * linv[j];
    }
  }
  double W[kReg][kAcc] = {};  // rows: theta, phi, x_dot, z_dot, theta_dot, u
#pragma unroll
  for (int c = 0; c < kAcc; ++c) {
    double t[kReg];
#pragma unroll
    for (int i = 0; i < kReg; ++i) {  // L t = D^-1 R
      double v = R[i][c] * dinv[i];
#pragma unroll
      for (int m = 0; m < i; ++m) v -= L[i][m] * t[m];
      t[i] = v * linv[i];
    }
#pragma unroll
    for (int i = kReg - 1; i >= 0; --i) {  // L' w = t
      double v = t[i];
#pragma unroll
      for (int m = i + 1; m < kReg; ++m) v -= L[m][i] * W[m][c];
      W[i][c] = v * linv[i];
    }
#pragma unroll
    for (int i = 0; i < kReg; ++i) W[i][c] = ok ? W[i][c] * dinv[i] : 0.0;
  }
  // Eq. 28 and the explicit Euler map: A = I + dt A_c, B = dt B_c
  double *A = p.a + (size_t)k * kNx * kNx, *B = p.b + (size_t)k * kNx;
  for (int r = 0; r < kNx; ++r)
    for (int c = 0; c < kNx; ++c) A[r * kNx + c] = r == c ? 1.0 : 0.0;
  A[0 * kNx + 4] = A[1 * kNx + 5] = A[2 * kNx + 6] = p.dt;
  for (int r = 0; r < kNx; ++r) B[r] = 0.0;
  B[3] = p.dt;
  for (int r = 0; r < kAcc; ++r) {
    for (int c = 0; c < 5; ++c) A[(4 + r) * kNx + 2 + c] += p.dt * W[c][r];
    B[4 + r] = p.dt * W[5][r];
  }
  p.status[k] = ok ? 0 : 1;
}

// One wavefront; lane l < 49 owns entry (r, c) = (l / 7, l % 7), lanes
// 49..55 own row j = l - 49 of B'S (= (S B)' as S is symmetric). Two phases
// per step: (1) SA = S A and B'S; (2) every lane forms B'SA at r and at c,
// B'SB and its own entry of S_k (Eq. 29); lanes 0..6 also the gain (Eq. 30).
// A_{k-1}, B_{k-1} are loaded into registers while step k computes; the
// phases exchange data through LDS with wave-scope ordering only.
__global__ __launch_bounds__(64) void riccati_kernel(PolicyArgs p) {
  __shared__ double S[kNx * kNx], A[kNx * kNx], SA[kNx * kNx], B[kNx], BS[kNx];
  const int l = threadIdx.x, r = l / kNx, c = l % kNx, j7 = l - kNx * kNx;
  const bool on = l < kNx * kNx, bs_lane = j7 >= 0 && j7 < kNx;
  const double s_init = on && r == c ? p.q_f[r] : 0.0;
  if (on) S[l] = s_init;
  if (on && p.s) p.s[(size_t)p.H * kNx * kNx + l] = s_init;
  const double q = on && r == c ? p.q_c[r] : 0.0;
  const int k0 = p.H - 1;
  double a_next = on ? p.a[(size_t)k0 * kNx * kNx + l] : 0.0;
  double b_next = l < kNx ? p.b[(size_t)k0 * kNx + l] : 0.0;
  for (int k = k0; k >= 0; --k) {
    if (on) A[l] = a_next;
    if (l < kNx) B[l] = b_next;
    if (k > 0) {
      a_next = on ? p.a[(size_t)(k - 1) * kNx * kNx + l] : 0.0;
      b_next = l < kNx ? p.b[(size_t)(k - 1) * kNx + l] : 0.0;
    }
    wave_sync();
    if (on) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < kNx; ++j) v += S[r * kNx + j] * A[j * kNx + c];
      SA[l] = v;
    } else if (bs_lane) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < kNx; ++i) v += B[i] * S[i * kNx + j7];
      BS[j7] = v;
    }
    wave_sync();
    double s_new = 0.0, bsa_c = 0.0, inv = 0.0;
    if (on) {
      double bsa_r = 0.0, bsb = 0.0, v = 0.0, vt = 0.0;
#pragma unroll
      for (int j = 0; j < kNx; ++j) {
        const double bs = BS[j];
        bsa_r += bs * A[j * kNx + r];
        bsa_c += bs * A[j * kNx + c];
        bsb += bs * B[j];
        // A'SA at (r, c) and (c, r), averaged: S stays symmetric
        v += A[j * kNx + r] * SA[j * kNx + c];
        vt += A[j * kNx + c] * SA[j * kNx + r];
      }
      inv = 1.0 / (p.r_c + bsb);
      s_new = 0.5 * (v + vt) - bsa_r * bsa_c * inv + q;
    }
    wave_sync();  // every lane is done reading this step's S
    if (on) {
      S[l] = s_new;
      if (p.s) p.s[(size_t)k * kNx * kNx + l] = s_new;
      if (r == 0) p.gain[(size_t)k * kNx + c] = bsa_c * inv;
    }
    wave_sync();
  }
}

}  // namespace

int launch_policy(const vpm_policy_in *in, vpm_policy_out *out, hipStream_t stream) {
  PolicyArgs p{};
  p.K = in->K;
  p.H = in->H;
  p.dt = in->dt;
  p.traj_nom = in->traj_nom;
  p.traj = in->traj;
  p.du = in->du;
  for (int i = 0; i < kNx; ++i) {
    p.q_f[i] = in->q_f[i];
    p.q_c[i] = in->q_c[i];
  }
  p.r_c = in->r_c;
  p.a = out->a;
  p.b = out->b;
  p.gain = out->gain;
  p.s = out->s;
  p.status = out->status;
  hipLaunchKernelGGL(synthesis_kernel, dim3(p.H), dim3(kSynThreads), 0, stream, p);
  VPM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(riccati_kernel, dim3(1), dim3(64), 0, stream, p);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}

int launch_tvlqr(int H, const double *a, const double *b, const double *q_f, const double *q_c,
                 double r_c, double *gain, double *s, hipStream_t stream) {
  PolicyArgs p{};
  p.H = H;
  for (int i = 0; i < kNx; ++i) {
    p.q_f[i] = q_f[i];
    p.q_c[i] = q_c[i];
  }
  p.r_c = r_c;
  p.a = const_cast<double *>(a);  // the recursion only reads A and B
  p.b = const_cast<double *>(b);
  p.gain = gain;
  p.s = s;
  hipLaunchKernelGGL(riccati_kernel, dim3(1), dim3(64), 0, stream, p);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}

}  // namespace vpm
