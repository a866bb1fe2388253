/*
 * oracle_checks.c -- drives the CPU oracle through every output and mode on
 * small inputs so that tests/test_host_sanitizers.py can run it under
 * AddressSanitizer + UndefinedBehaviorSanitizer (memory errors, overflow,
 * invalid shifts, misaligned or null accesses). It checks only that results
 * are finite and the wake counts consistent: the oracle's values are pinned
 * by the Python tests. Prints "ALL OK" and exits 0, or exits 1.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vpm_oracle.h"

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);  \
      exit(1);                                                        \
    }                                                                 \
  } while (0)

static unsigned long long lcg_state = 88172645463325252ULL;
static double uniform(double lo, double hi) {
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return lo + (hi - lo) * (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static orc_params params(int nb, int mode, int gate, int n_max) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.n_bound = nb;
  p.n_wake_max = n_max;
  p.shed_mode = mode;
  p.chord = 0.3;
  p.shed_frac = 0.02;
  p.r_core = 0.01;
  p.decay = 0.1;
  p.rho = 1.225;
  p.span = 0.5;
  p.grav = 9.81;
  p.mass = 0.12;
  p.inertia = 0.002;
  p.l_body = 0.35;
  p.l_wing = 0.08;
  p.l_elev = 0.03;
  p.s_elev = 0.02;
  p.gate = gate;
  p.alpha_crit = 0.0;
  return p;
}

/* K rollouts of H steps from two wake fields with a disturbance pair each. */
static void run_case(int nb, int mode, int gate, int n_max, int reverse, int with_feedback) {
  enum { K = 3, H = 6, NP = 1 };
  const int n0[2] = {7, 0};
  int64_t field_off[3] = {0, n0[0], n0[0] + n0[1]};
  int32_t field_of[K] = {0, 1, 0};
  double wx[8], wz[8], wg[8];
  for (int i = 0; i < n0[0]; ++i) {
    wx[i] = uniform(0.2, 1.0);
    wz[i] = uniform(-0.3, 0.3);
    wg[i] = uniform(-0.05, 0.05);
  }
  wx[0] = 0.4, wz[0] = 0.1, wg[0] = -0.3;  /* the pair */
  wx[1] = 0.4, wz[1] = -0.1, wg[1] = 0.3;
  int32_t pairs[K * 2 * NP] = {0, 1, -1, -1, 0, 1};
  double g0[K * 7], gb0[K * 64], u[K * H], x_goal[7], q_diag[7];
  for (int k = 0; k < K; ++k) {
    double g[7] = {0, 0, 0.05 * k, 0, 6.0, 0, 0};
    memcpy(g0 + 7 * k, g, sizeof g);
    for (int j = 0; j < nb; ++j) gb0[k * nb + j] = 0.0;
    for (int n = 0; n < H; ++n) u[k * H + n] = uniform(-0.2, 0.2);
  }
  for (int i = 0; i < 7; ++i) x_goal[i] = i < 3 ? 1.0 : 0.0, q_diag[i] = i < 3 ? 1.0 : 0.0;
  double fb_gain[H * 7], fb_xref[H * 7];
  for (int i = 0; i < H * 7; ++i) fb_gain[i] = uniform(-0.1, 0.1), fb_xref[i] = 0.0;
  const int S = orc_system_size(nb, mode);
  int64_t out_off[K + 1];
  out_off[0] = 0;
  for (int k = 0; k < K; ++k) out_off[k + 1] = out_off[k] + n0[field_of[k]] + 2 * H;
  const int64_t cap = out_off[K];
  double *traj = malloc(sizeof(double) * K * (H + 1) * 7);
  double *gs = malloc(sizeof(double) * K * H * S);
  double *force = malloc(sizeof(double) * K * H * 3);
  double *ox = malloc(sizeof(double) * cap), *oz = malloc(sizeof(double) * cap);
  double *og = malloc(sizeof(double) * cap), *vel = malloc(sizeof(double) * 2 * cap);
  double g_final[K * 7], cost[K], gb_final[K * 64];
  int32_t status[K], n_final[K], n_vel[K];
  orc_params p = params(nb, mode, gate, n_max);
  CHECK(orc_rollout_batch(&p, K, H, 0.005, g0, gb0, field_off, field_of, wx, wz, wg, pairs, NP,
                          u, x_goal, q_diag, reverse, 1, g_final, cost, status, traj, gs, force,
                          out_off, ox, oz, og, n_final, vel, n_vel,
                          with_feedback ? fb_gain : NULL, with_feedback ? fb_xref : NULL,
                          gb_final) == 0);
  for (int k = 0; k < K; ++k) {
    CHECK(status[k] == ORC_OK);
    CHECK(isfinite(cost[k]));
    CHECK(n_final[k] >= 0 && n_final[k] <= out_off[k + 1] - out_off[k]);
    if (n_max > 0) CHECK(n_final[k] <= n_max);
    for (int i = 0; i < 7; ++i) CHECK(isfinite(g_final[7 * k + i]));
  }
  double w[K], xs[H], jmin;
  int32_t am;
  double mu[H];
  for (int n = 0; n < H; ++n) mu[n] = 0.0;
  orc_mppi(K, H, cost, 1.0, mu, u, w, xs, &am, &jmin);
  CHECK(am >= 0 && am < K);
  free(traj), free(gs), free(force), free(ox), free(oz), free(og), free(vel);
}

int main(void) {
  const int modes[3] = {ORC_SHED_BOTH, ORC_SHED_TE, ORC_SHED_NONE};
  for (int m = 0; m < 3; ++m)
    for (int nb = 2; nb <= 64; nb *= 2) run_case(nb, modes[m], 0, 0, 0, 0);
  run_case(16, ORC_SHED_BOTH, 1, 0, 0, 0);      /* separation gate */
  run_case(16, ORC_SHED_BOTH, 0, 10, 1, 0);     /* merging at a cap, reverse sums */
  run_case(32, ORC_SHED_BOTH, 0, 0, 0, 1);      /* feedback policy */
  /* plate solve at a pose, the surface matrix, elevator, segment test */
  orc_params p = params(8, ORC_SHED_BOTH, 0, 0);
  const int S = orc_system_size(8, ORC_SHED_BOTH);
  double pose[6] = {0.1, 0.2, 0.05, 6.0, 0.1, 0.3}, vw[9 * 2], gsol[10];
  for (int i = 0; i < 18; ++i) vw[i] = uniform(-0.1, 0.1);
  CHECK(orc_plate_solve_pose(&p, pose, vw, 0.01, ORC_SHED_BOTH, gsol) == 0);
  double *a = malloc(sizeof(double) * S * S), g7[7] = {0, 0, 0.1, 0, 6, 0, 0};
  orc_surface_matrix(&p, g7, ORC_SHED_BOTH, a);
  free(a);
  double xe[2], fe[2];
  CHECK(isfinite(orc_elevator(&p, g7, 0.1, xe, fe)));
  double sa[2] = {0.0, 0.1}, sb[2] = {0.0, -0.1};
  (void)orc_segment_hits_plate(&p, g7, sa, sb);
  puts("ALL OK");
  return 0;
}
