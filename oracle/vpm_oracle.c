/*
 * vpm_oracle.c -- plain, slow, FP64 CPU oracle of the paper's rollout:
 * a 2D vortex particle model (VPM) coupled to a flat-plate glider, stepped
 * with explicit Euler, followed by the MPPI terminal cost and softmin
 * reweighting.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no code, header,
 * table or helper with the GPU library. Every sum is a direct loop in index
 * (FIFO) order; there is no blocking, fusion, compensation or fast-math.
 *
 * Method: Gupta, Wolfe, Perrotta, Moore, arXiv 2509.16079.
 *   Sec. III-A  "Vortex Particle Model"   Eqs. 4-17
 *   Sec. III-B  "Glider Dynamics"         kinematics, elevator, rigid body
 *   Sec. IV-A   "Trajectory Optimization" Eqs. 24-25 (cost, MPPI)
 *   Sec. V      disturbance pair and its termination at the wing
 * Readings where the paper is silent or garbled are marked READING and are
 * listed, with the pins that ground them, in the design notes.
 *
 * Built with -DORC_F32_STATE, the oracle also models binary32 storage of the
 * state: after every step the wake positions and strengths and the glider
 * state are rounded to the nearest float (all arithmetic stays FP64). That
 * variant measures how much of an FP32 path's error comes from storing the
 * state in FP32 alone.
 */
#include "vpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI (2.0 * M_PI)

/* ---------------------------------------------------------------- kernels */

/* Eq. 4: K_v(r) = -1/(2 pi r^2) [[0, 1], [-1, 0]] (r - r_v), i.e. the
 * velocity per unit circulation is (-dz, dx) / (2 pi r^2). The term of a
 * coincident point is taken as zero (READING: no guard is given). */
void orc_kernel_sing(double dx, double dz, double *kx, double *kz) {
  double r2 = dx * dx + dz * dz;
  if (r2 == 0.0) {
    *kx = 0.0;
    *kz = 0.0;
    return;
  }
  double f = -1.0 / (TWO_PI * r2);
  /* [[0, 1], [-1, 0]] * (dx, dz) = (dz, -dx) */
  *kx = f * dz;
  *kz = f * (-dx);
}

/* Eq. 5: K'_v = (r/r_core)^2 / sqrt(1 + (r/r_core)^4) * K_v. At r = 0 the
 * factor vanishes and K'_v(0) = 0 (the limit). */
void orc_kernel_reg(double dx, double dz, double r_core, double *kx,
                    double *kz) {
  double r2 = dx * dx + dz * dz;
  if (r2 == 0.0) {
    *kx = 0.0;
    *kz = 0.0;
    return;
  }
  double q = r2 / (r_core * r_core); /* (r / r_core)^2 */
  double scale = q / sqrt(1.0 + q * q);
  double sx, sz;
  orc_kernel_sing(dx, dz, &sx, &sz);
  *kx = scale * sx;
  *kz = scale * sz;
}

/* ------------------------------------------------------- wake dynamics */

/* Eq. 16: the velocity of wake vortex i is the regularised sum over all
 * other wake vortices plus the singular sum over the bound vortices. */
void orc_wake_velocities(int32_t n_w, const double *wx, const double *wz,
                         const double *wg, int32_t n_b, const double *bx,
                         const double *bz, const double *bg, double r_core,
                         int32_t reverse, double *vx, double *vz) {
  for (int32_t i = 0; i < n_w; ++i) {
    double sx = 0.0, sz = 0.0;
    for (int32_t jj = 0; jj < n_w; ++jj) {
      int32_t j = reverse ? (n_w - 1 - jj) : jj;
      if (j == i) continue; /* the sum runs over W - w_i */
      double kx, kz;
      orc_kernel_reg(wx[i] - wx[j], wz[i] - wz[j], r_core, &kx, &kz);
      sx += kx * wg[j];
      sz += kz * wg[j];
    }
    for (int32_t bb = 0; bb < n_b; ++bb) {
      int32_t b = reverse ? (n_b - 1 - bb) : bb;
      double kx, kz;
      orc_kernel_sing(wx[i] - bx[b], wz[i] - bz[b], &kx, &kz);
      sx += kx * bg[b];
      sz += kz * bg[b];
    }
    vx[i] = sx;
    vz[i] = sz;
  }
}

/* Eq. 16 integrated by explicit Euler from the step's velocity snapshot, and
 * Eq. 17 (dGamma/dt = -gamma Gamma) by explicit Euler (READING: the paper
 * names no integrator). */
void orc_advect(int32_t n_w, double *wx, double *wz, double *wg,
                const double *vx, const double *vz, double dt, double decay) {
  for (int32_t i = 0; i < n_w; ++i) {
    wx[i] += dt * vx[i];
    wz[i] += dt * vz[i];
    wg[i] -= dt * decay * wg[i];
  }
}

/* ------------------------------------------------------- plate geometry */

/* Sec. III-B kinematics and Sec. III-A discretisation.
 * Body axis e_f = (cos th, sin th); wing point x_w = (x - l_w c_th,
 * z - l_w s_th) with velocity (xd + l_w thd s_th, zd - l_w thd c_th).
 * READING: x_w is the mid-chord; the leading edge (LE) is x_w + (c/2) e_f;
 * the tangent e_t points from LE to TE (e_t = -e_f); the normal is
 * n = (-s_th, c_th). N_c = N_b + 1 collocation points are equally spaced from
 * LE to TE inclusive; bound vortex j sits midway between collocation points
 * j and j+1. The LEV and TEV are released delta_s = shed_frac * c outside the
 * LE and TE along the tangent. */
void orc_plate_geometry(const orc_params *p, const double *g, double *x_w,
                        double *xw_dot, double *rc, double *rb, double *r_lev,
                        double *r_tev, double *n_hat, double *t_hat) {
  const double x = g[0], z = g[1], th = g[2];
  const double xd = g[4], zd = g[5], thd = g[6];
  const double c = p->chord, lw = p->l_wing;
  const int32_t nb = p->n_bound;
  const double lb = c / nb;
  const double ct = cos(th), st = sin(th);
  double xw[2] = {x - lw * ct, z - lw * st};
  double et[2] = {-ct, -st};
  double en[2] = {-st, ct};
  double le[2] = {xw[0] + 0.5 * c * ct, xw[1] + 0.5 * c * st};
  double ds = p->shed_frac * c;
  if (x_w) {
    x_w[0] = xw[0];
    x_w[1] = xw[1];
  }
  if (xw_dot) {
    xw_dot[0] = xd + lw * thd * st;
    xw_dot[1] = zd - lw * thd * ct;
  }
  if (rc) {
    for (int32_t i = 0; i <= nb; ++i) {
      double s = i * lb;
      rc[2 * i] = le[0] + s * et[0];
      rc[2 * i + 1] = le[1] + s * et[1];
    }
  }
  if (rb) {
    for (int32_t j = 0; j < nb; ++j) {
      double s = (j + 0.5) * lb;
      rb[2 * j] = le[0] + s * et[0];
      rb[2 * j + 1] = le[1] + s * et[1];
    }
  }
  if (r_lev) {
    r_lev[0] = le[0] - ds * et[0];
    r_lev[1] = le[1] - ds * et[1];
  }
  if (r_tev) {
    r_tev[0] = le[0] + (c + ds) * et[0];
    r_tev[1] = le[1] + (c + ds) * et[1];
  }
  if (n_hat) {
    n_hat[0] = en[0];
    n_hat[1] = en[1];
  }
  if (t_hat) {
    t_hat[0] = et[0];
    t_hat[1] = et[1];
  }
}

/* --------------------------------------------------- the surface system */

/* Rows and columns used per shedding mode (READING: the paper states only
 * the both-edges system). BOTH: all N_c collocation rows, columns
 * [bound..., LEV, TEV]. TE: drop the LE row and the LEV column. NONE: drop
 * both edge rows and both edge columns. The Kelvin row closes each system. */
int32_t orc_system_size(int32_t n_bound, int32_t shed_mode) {
  if (shed_mode == ORC_SHED_BOTH) return n_bound + 2;
  if (shed_mode == ORC_SHED_TE) return n_bound + 1;
  return n_bound;
}

static int32_t first_colloc_row(int32_t shed_mode) {
  return shed_mode == ORC_SHED_BOTH ? 0 : 1;
}

/* Eq. 8: row i (collocation point i) holds K_b(r_ci).n for the bound columns
 * and K'_e(r_ci).n for the shed-vortex columns; the last row is all ones
 * (Kelvin, Eq. 7). */
void orc_surface_matrix(const orc_params *p, const double *g, int32_t shed_mode,
                        double *a) {
  const int32_t nb = p->n_bound;
  const int32_t S = orc_system_size(nb, shed_mode);
  double *rc = (double *)malloc(sizeof(double) * 2 * (nb + 1));
  double *rb = (double *)malloc(sizeof(double) * 2 * nb);
  double rlev[2], rtev[2], en[2];
  orc_plate_geometry(p, g, NULL, NULL, rc, rb, rlev, rtev, en, NULL);
  int32_t i0 = first_colloc_row(shed_mode);
  for (int32_t r = 0; r < S - 1; ++r) {
    int32_t i = i0 + r; /* collocation index */
    double px = rc[2 * i], pz = rc[2 * i + 1];
    int32_t col = 0;
    for (int32_t j = 0; j < nb; ++j) {
      double kx, kz;
      orc_kernel_sing(px - rb[2 * j], pz - rb[2 * j + 1], &kx, &kz);
      a[r * S + col++] = kx * en[0] + kz * en[1];
    }
    if (shed_mode == ORC_SHED_BOTH) {
      double kx, kz;
      orc_kernel_reg(px - rlev[0], pz - rlev[1], p->r_core, &kx, &kz);
      a[r * S + col++] = kx * en[0] + kz * en[1];
    }
    if (shed_mode != ORC_SHED_NONE) {
      double kx, kz;
      orc_kernel_reg(px - rtev[0], pz - rtev[1], p->r_core, &kx, &kz);
      a[r * S + col++] = kx * en[0] + kz * en[1];
    }
  }
  for (int32_t col = 0; col < S; ++col) a[(S - 1) * S + col] = 1.0;
  free(rc);
  free(rb);
}

/* Gaussian elimination with partial pivoting and back substitution (the
 * textbook algorithm, e.g. Golub and Van Loan, Sec. 3.4). */
int32_t orc_solve(int32_t n, double *a, double *b, double *x) {
  for (int32_t k = 0; k < n; ++k) {
    int32_t piv = k;
    double best = fabs(a[k * n + k]);
    for (int32_t i = k + 1; i < n; ++i) {
      if (fabs(a[i * n + k]) > best) {
        best = fabs(a[i * n + k]);
        piv = i;
      }
    }
    if (best == 0.0) return -1;
    if (piv != k) {
      for (int32_t j = 0; j < n; ++j) {
        double t = a[k * n + j];
        a[k * n + j] = a[piv * n + j];
        a[piv * n + j] = t;
      }
      double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (int32_t i = k + 1; i < n; ++i) {
      double m = a[i * n + k] / a[k * n + k];
      for (int32_t j = k; j < n; ++j) a[i * n + j] -= m * a[k * n + j];
      b[i] -= m * b[k];
    }
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int32_t j = i + 1; j < n; ++j) s -= a[i * n + j] * x[j];
    x[i] = s / a[i * n + i];
  }
  return 0;
}

/* Eq. 12: relative velocity at a surface point r,
 *   v~(r) = v_W(r) - v - omega x (r - r_g),
 * READING: the rigid-motion term is the velocity of the surface point,
 * xw_dot + thd * J (r - x_w) with J(a) = (-a_z, a_x), so that v~ is the flow
 * velocity relative to the moving plate. */
static void relative_velocity(const double *vw, const double *xw,
                              const double *xw_dot, double thd, const double *r,
                              double *out) {
  double ax = r[0] - xw[0], az = r[1] - xw[1];
  out[0] = vw[0] - xw_dot[0] - thd * (-az);
  out[1] = vw[1] - xw_dot[1] - thd * ax;
}

/* Eqs. 10-11: assemble b (b_i = -v~(r_ci).n, b_S = -sum Gamma_w) and solve
 * K Gamma_S = b at the given glider pose. vw_c holds v_W at all N_c
 * collocation points. */
static int32_t surface_solve(const orc_params *p, const double *g,
                             const double *vw_c, double sum_gw,
                             int32_t shed_mode, double *gamma_s) {
  const int32_t nb = p->n_bound;
  const int32_t S = orc_system_size(nb, shed_mode);
  double *a = (double *)malloc(sizeof(double) * S * S);
  double *b = (double *)malloc(sizeof(double) * S);
  double *rc = (double *)malloc(sizeof(double) * 2 * (nb + 1));
  double xw[2], xwd[2], en[2];
  orc_plate_geometry(p, g, xw, xwd, rc, NULL, NULL, NULL, en, NULL);
  orc_surface_matrix(p, g, shed_mode, a);
  int32_t i0 = first_colloc_row(shed_mode);
  for (int32_t r = 0; r < S - 1; ++r) {
    int32_t i = i0 + r;
    double vt[2];
    relative_velocity(&vw_c[2 * i], xw, xwd, g[6], &rc[2 * i], vt);
    b[r] = -(vt[0] * en[0] + vt[1] * en[1]);
  }
  b[S - 1] = -sum_gw;
  int32_t rcode = orc_solve(S, a, b, gamma_s);
  free(a);
  free(b);
  free(rc);
  return rcode;
}

int32_t orc_plate_solve_pose(const orc_params *p, const double *pose6,
                             const double *vw_c, double sum_gw,
                             int32_t shed_mode, double *gamma_s) {
  /* A glider state whose wing point and wing velocity equal the pose:
   * with l_w = 0 the wing point is the glider position itself. */
  orc_params q = *p;
  q.l_wing = 0.0;
  double g[7] = {pose6[0], pose6[1], pose6[2], 0.0, pose6[3], pose6[4],
                 pose6[5]};
  return surface_solve(&q, g, vw_c, sum_gw, shed_mode, gamma_s);
}

/* ------------------------------------------------------------ elevator */

/* Sec. III-B: elevator position and velocity, alpha_e = th + phi -
 * atan2(zd_e, xd_e), F_e = 1/2 rho |xd_e|^2 S_e C_n n_e with C_n = 2 sin
 * alpha_e and n_e = (-s_{th+phi}, c_{th+phi}). u is the elevator rate. */
double orc_elevator(const orc_params *p, const double *g, double u,
                    double *x_e, double *f_e) {
  const double x = g[0], z = g[1], th = g[2], ph = g[3];
  const double xd = g[4], zd = g[5], thd = g[6];
  const double l = p->l_body, le = p->l_elev;
  double ctp = cos(th + ph), stp = sin(th + ph);
  double xe = x - l * cos(th) - le * ctp;
  double ze = z - l * sin(th) - le * stp;
  double xed = xd + l * thd * sin(th) + le * (thd + u) * stp;
  double zed = zd - l * thd * cos(th) - le * (thd + u) * ctp;
  double alpha = th + ph - atan2(zed, xed);
  double cn = 2.0 * sin(alpha);
  double qdyn = 0.5 * p->rho * (xed * xed + zed * zed) * p->s_elev * cn;
  if (x_e) {
    x_e[0] = xe;
    x_e[1] = ze;
  }
  if (f_e) {
    f_e[0] = qdyn * (-stp);
    f_e[1] = qdyn * ctp;
  }
  return alpha;
}

/* ------------------------------------------- disturbance termination */

/* Orientation of (p, q, r): sign of the cross product (q - p) x (r - p). */
static double orient(const double *p, const double *q, const double *r) {
  return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0]);
}

static int32_t on_segment(const double *p, const double *q, const double *r) {
  /* r collinear with p-q: is r inside the bounding box of p-q? */
  return fmin(p[0], q[0]) <= r[0] && r[0] <= fmax(p[0], q[0]) &&
         fmin(p[1], q[1]) <= r[1] && r[1] <= fmax(p[1], q[1]);
}

/* Closed-segment intersection (CLRS, Sec. 33.1, SEGMENTS-INTERSECT). */
static int32_t segments_intersect(const double *p1, const double *p2,
                                  const double *p3, const double *p4) {
  double d1 = orient(p3, p4, p1), d2 = orient(p3, p4, p2);
  double d3 = orient(p1, p2, p3), d4 = orient(p1, p2, p4);
  if (((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) &&
      ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0)))
    return 1;
  if (d1 == 0 && on_segment(p3, p4, p1)) return 1;
  if (d2 == 0 && on_segment(p3, p4, p2)) return 1;
  if (d3 == 0 && on_segment(p1, p2, p3)) return 1;
  if (d4 == 0 && on_segment(p1, p2, p4)) return 1;
  return 0;
}

/* Point inside or on a convex quadrilateral q[0..3] (either winding). */
static int32_t in_convex_quad(const double q[4][2], const double *pt) {
  int32_t pos = 0, neg = 0;
  for (int32_t e = 0; e < 4; ++e) {
    double o = orient(q[e], q[(e + 1) % 4], pt);
    if (o > 0) pos = 1;
    if (o < 0) neg = 1;
  }
  return !(pos && neg);
}

/* Sec. V: the chord line, inflated by 2 % of chord in the direction opposite
 * to the normal, is checked against the segment joining the two disturbance
 * vortices. READING: the inflated chord is the closed rectangle LE, TE,
 * TE - 0.02 c n, LE - 0.02 c n; a hit is any common point. */
int32_t orc_segment_hits_plate(const orc_params *p, const double *g,
                               const double *a, const double *b) {
  double rc_le[2], rc_te[2], en[2];
  const int32_t nb = p->n_bound;
  double *rc = (double *)malloc(sizeof(double) * 2 * (nb + 1));
  orc_plate_geometry(p, g, NULL, NULL, rc, NULL, NULL, NULL, en, NULL);
  rc_le[0] = rc[0];
  rc_le[1] = rc[1];
  rc_te[0] = rc[2 * nb];
  rc_te[1] = rc[2 * nb + 1];
  free(rc);
  double h = 0.02 * p->chord;
  double quad[4][2] = {{rc_le[0], rc_le[1]},
                       {rc_te[0], rc_te[1]},
                       {rc_te[0] - h * en[0], rc_te[1] - h * en[1]},
                       {rc_le[0] - h * en[0], rc_le[1] - h * en[1]}};
  if (in_convex_quad(quad, a) || in_convex_quad(quad, b)) return 1;
  for (int32_t e = 0; e < 4; ++e)
    if (segments_intersect(a, b, quad[e], quad[(e + 1) % 4])) return 1;
  return 0;
}

/* ------------------------------------------------------------- rollout */

typedef struct {
  double g[7];
  double *gb_prev;  /* bound circulations of the previous step           */
  double glev_prev; /* LEV strength of the previous step (lev_literal)   */
  int32_t n_w, cap;
  double *wx, *wz, *wg; /* wake FIFO, index 0 is the oldest                 */
  int32_t *tag;         /* disturbance pair id (q + 1) or 0                   */
  int32_t status;
} orc_state;

/* Merge the two oldest wake vortices (Sec. III-A): one vortex at their
 * average position carrying the sum of their strengths, kept as the oldest.
 * A merged disturbance vortex takes its pair out of termination tracking. */
static void merge_oldest(orc_state *s) {
  for (int32_t m = 0; m < 2; ++m) {
    int32_t t = s->tag[m];
    if (t != 0)
      for (int32_t i = 0; i < s->n_w; ++i)
        if (s->tag[i] == t) s->tag[i] = 0;
  }
  double mx = 0.5 * (s->wx[0] + s->wx[1]);
  double mz = 0.5 * (s->wz[0] + s->wz[1]);
  double mg = s->wg[0] + s->wg[1];
  for (int32_t i = 1; i < s->n_w - 1; ++i) {
    s->wx[i] = s->wx[i + 1];
    s->wz[i] = s->wz[i + 1];
    s->wg[i] = s->wg[i + 1];
    s->tag[i] = s->tag[i + 1];
  }
  s->wx[0] = mx;
  s->wz[0] = mz;
  s->wg[0] = mg;
  s->tag[0] = 0;
  s->n_w -= 1;
}

/* Sec. V termination: for each tracked pair whose connecting segment meets
 * the inflated chord, both strengths are set to zero and tracking ends. */
static void terminate_pairs(const orc_params *p, orc_state *s) {
  for (int32_t i = 0; i < s->n_w; ++i) {
    int32_t t = s->tag[i];
    if (t == 0) continue;
    int32_t j = -1;
    for (int32_t k = i + 1; k < s->n_w; ++k)
      if (s->tag[k] == t) {
        j = k;
        break;
      }
    if (j < 0) continue;
    double a[2] = {s->wx[i], s->wz[i]}, b[2] = {s->wx[j], s->wz[j]};
    if (orc_segment_hits_plate(p, s->g, a, b)) {
      s->wg[i] = 0.0;
      s->wg[j] = 0.0;
      s->tag[i] = 0;
      s->tag[j] = 0;
    }
  }
}

typedef struct {
  double fx, fz, m;
} orc_loads;

/* One time step of one rollout, in the order of Sec. III-A/B:
 * termination, surface velocities, surface solve, loads, elevator, rigid
 * body accelerations, shedding, wake velocities, advection and decay,
 * merging, glider Euler step. gamma_s_out (S values) and vel (2 * (n_w + 2)
 * values) may be NULL. */
double orc_wing_aoa(const orc_params *p, const double *g) {
  /* wing point x_w = x - l_w e_f; its velocity, differentiated in time */
  const double xd_w = g[4] + p->l_wing * g[6] * sin(g[2]);
  const double zd_w = g[5] - p->l_wing * g[6] * cos(g[2]);
  return g[2] - atan2(zd_w, xd_w);
}

static void orc_step(const orc_params *p, orc_state *s, double dt, double u,
                     int32_t reverse, double *gamma_s_out, orc_loads *ld,
                     double *vel, int32_t *n_vel) {
  const int32_t nb = p->n_bound;
  /* Sec. III-A: with the separation gate the leading edge sheds only while
   * the wing is beyond the critical angle; the trailing edge always does. */
  const int32_t mode = !p->gate ? p->shed_mode
                       : orc_wing_aoa(p, s->g) > p->alpha_crit ? ORC_SHED_BOTH
                                                                : ORC_SHED_TE;
  const int32_t S = orc_system_size(nb, mode);
  const double lb = p->chord / nb;
  double *g = s->g;

  /* kinematics at the start of the step */
  double xw[2], xwd[2], en[2], et[2], rlev[2], rtev[2];
  double *rc = (double *)malloc(sizeof(double) * 2 * (nb + 1));
  double *rb = (double *)malloc(sizeof(double) * 2 * nb);
  orc_plate_geometry(p, g, xw, xwd, rc, rb, rlev, rtev, en, et);

  terminate_pairs(p, s);

  /* Eq. 12: wake-induced velocity at the collocation and bound points */
  double *vw_c = (double *)malloc(sizeof(double) * 2 * (nb + 1));
  double *vt_b = (double *)malloc(sizeof(double) * 2 * nb);
  for (int32_t i = 0; i < 2 * nb + 1; ++i) {
    const double *r = i <= nb ? &rc[2 * i] : &rb[2 * (i - nb - 1)];
    double sx = 0.0, sz = 0.0;
    for (int32_t ww = 0; ww < s->n_w; ++ww) {
      int32_t w = reverse ? s->n_w - 1 - ww : ww;
      double kx, kz;
      orc_kernel_reg(r[0] - s->wx[w], r[1] - s->wz[w], p->r_core, &kx, &kz);
      sx += kx * s->wg[w];
      sz += kz * s->wg[w];
    }
    if (i <= nb) {
      vw_c[2 * i] = sx;
      vw_c[2 * i + 1] = sz;
    } else {
      double vw[2] = {sx, sz};
      relative_velocity(vw, xw, xwd, g[6], r, &vt_b[2 * (i - nb - 1)]);
    }
  }

  /* Eqs. 10-11: Kelvin right-hand side and the surface solve */
  double sum_gw = 0.0;
  for (int32_t ww = 0; ww < s->n_w; ++ww)
    sum_gw += s->wg[reverse ? s->n_w - 1 - ww : ww];
  double *gs = (double *)malloc(sizeof(double) * S);
  if (surface_solve(p, g, vw_c, sum_gw, mode, gs) != 0) {
    s->status |= ORC_SINGULAR;
    for (int32_t i = 0; i < S; ++i) gs[i] = NAN;
  }
  double *gb = gs; /* bound circulations are the first N_b unknowns */
  double glev = mode == ORC_SHED_BOTH ? gs[nb] : 0.0;
  double gtev = mode == ORC_SHED_BOTH ? gs[nb + 1]
                : mode == ORC_SHED_TE ? gs[nb]
                                      : 0.0;
  if (gamma_s_out) memcpy(gamma_s_out, gs, sizeof(double) * S);

  /* Eqs. 13-15: unsteady Bernoulli pressure jump, wing force and moment.
   * READING: d/dt of the bound prefix sums is the backward difference over
   * one step against the state-carried previous values; d/dt Gamma_LEV is
   * the rate at which circulation leaves the leading edge, Gamma_LEV / dt
   * (the potential jump at a panel includes all circulation shed from the
   * LE); the moment arm is (r_bj - x_w).e_f, the moment of the panel forces
   * about the wing point. */
  double sum_dp = 0.0, sum_dp_arm = 0.0;
  double pre = 0.0, pre_prev = 0.0;
  for (int32_t j = 0; j < nb; ++j) {
    pre += gb[j];
    pre_prev += s->gb_prev[j];
    double q = vt_b[2 * j] * et[0] + vt_b[2 * j + 1] * et[1];
    double lev_rate = p->lev_literal ? (glev - s->glev_prev) / dt : glev / dt;
    double dp = p->rho * ((gb[j] / lb) * q + (pre - pre_prev) / dt + lev_rate);
    double arm = (rb[2 * j] - xw[0]) * cos(g[2]) +
                 (rb[2 * j + 1] - xw[1]) * sin(g[2]);
    sum_dp += dp;
    sum_dp_arm += dp * arm;
  }
  double fw[2] = {lb * p->span * sum_dp * en[0], lb * p->span * sum_dp * en[1]};
  double mw = lb * p->span * sum_dp_arm;
  if (ld) {
    ld->fx = fw[0];
    ld->fz = fw[1];
    ld->m = mw;
  }

  /* Sec. III-B: elevator force and the rigid-body equations of motion.
   * READING: the moment arms are the world-frame vectors from the CG to the
   * wing point and to the elevator point, a x b = a_x b_z - a_z b_x. */
  double xe[2], fe[2];
  orc_elevator(p, g, u, xe, fe);
  double acc[3];
  acc[0] = (fw[0] + fe[0]) / p->mass;
  acc[1] = (fw[1] + fe[1]) / p->mass - p->grav;
  double arm_w[2] = {xw[0] - g[0], xw[1] - g[1]};
  double arm_e[2] = {xe[0] - g[0], xe[1] - g[1]};
  acc[2] = (arm_w[0] * fw[1] - arm_w[1] * fw[0] + arm_e[0] * fe[1] -
            arm_e[1] * fe[0] + mw) /
           p->inertia;

  /* Sec. III-A shedding: the new LEV and TEV join the wake (at the tail). */
  if (mode == ORC_SHED_BOTH) {
    int32_t k = s->n_w;
    if (k + 2 > s->cap) {
      s->status |= ORC_CAPACITY;
    } else {
      s->wx[k] = rlev[0];
      s->wz[k] = rlev[1];
      s->wg[k] = glev;
      s->tag[k] = 0;
      s->wx[k + 1] = rtev[0];
      s->wz[k + 1] = rtev[1];
      s->wg[k + 1] = gtev;
      s->tag[k + 1] = 0;
      s->n_w += 2;
    }
  } else if (mode == ORC_SHED_TE) {
    int32_t k = s->n_w;
    if (k + 1 > s->cap) {
      s->status |= ORC_CAPACITY;
    } else {
      s->wx[k] = rtev[0];
      s->wz[k] = rtev[1];
      s->wg[k] = gtev;
      s->tag[k] = 0;
      s->n_w += 1;
    }
  }

  /* Eq. 16 (bound vortices carry the circulations just solved) and Eq. 17 */
  double *bxz = (double *)malloc(sizeof(double) * 2 * nb);
  double *bx = bxz, *bz = bxz + nb;
  for (int32_t j = 0; j < nb; ++j) {
    bx[j] = rb[2 * j];
    bz[j] = rb[2 * j + 1];
  }
  double *vx = (double *)malloc(sizeof(double) * (s->n_w + 1));
  double *vz = (double *)malloc(sizeof(double) * (s->n_w + 1));
  orc_wake_velocities(s->n_w, s->wx, s->wz, s->wg, nb, bx, bz, gb, p->r_core,
                      reverse, vx, vz);
  if (vel) {
    for (int32_t i = 0; i < s->n_w; ++i) {
      vel[2 * i] = vx[i];
      vel[2 * i + 1] = vz[i];
    }
    *n_vel = s->n_w;
  }
  orc_advect(s->n_w, s->wx, s->wz, s->wg, vx, vz, dt, p->decay);

  /* Sec. III-A merging above N_w,max */
  if (p->n_wake_max > 0)
    while (s->n_w > p->n_wake_max && s->n_w >= 2) merge_oldest(s);

  /* explicit Euler step of the glider state; u = phi_dot (Sec. III-B) */
  double gn[7];
  gn[0] = g[0] + dt * g[4];
  gn[1] = g[1] + dt * g[5];
  gn[2] = g[2] + dt * g[6];
  gn[3] = g[3] + dt * u;
  if (p->prescribed) {
    gn[4] = g[4];
    gn[5] = g[5];
    gn[6] = g[6];
  } else {
    gn[4] = g[4] + dt * acc[0];
    gn[5] = g[5] + dt * acc[1];
    gn[6] = g[6] + dt * acc[2];
  }
  memcpy(g, gn, sizeof(gn));
#ifdef ORC_F32_STATE
  for (int32_t i = 0; i < s->n_w; ++i) {
    s->wx[i] = (float)s->wx[i];
    s->wz[i] = (float)s->wz[i];
    s->wg[i] = (float)s->wg[i];
  }
  for (int32_t i = 0; i < 7; ++i) g[i] = (float)g[i];
#endif
  for (int32_t j = 0; j < nb; ++j) s->gb_prev[j] = gb[j];
  s->glev_prev = glev;

  free(rc);
  free(rb);
  free(vw_c);
  free(vt_b);
  free(gs);
  free(bxz);
  free(vx);
  free(vz);
}

double orc_cost(const double *g_final, const double *x_goal,
                const double *q_diag) {
  double j = 0.0;
  for (int32_t k = 0; k < 7; ++k) {
    double d = g_final[k] - x_goal[k];
    j += q_diag[k] * d * d;
  }
  return j;
}

static int32_t shed_per_step(int32_t mode) {
  return mode == ORC_SHED_BOTH ? 2 : mode == ORC_SHED_TE ? 1 : 0;
}

int32_t orc_rollout_batch(
    const orc_params *p, int32_t K, int32_t H, double dt, const double *g0,
    const double *gb0, const int64_t *field_off, const int32_t *field_of,
    const double *wx, const double *wz, const double *wg,
    const int32_t *pairs, int32_t n_pairs, const double *u,
    const double *x_goal, const double *q_diag, int32_t reverse,
    int32_t n_threads, double *g_final, double *cost, int32_t *status,
    double *traj, double *gamma_s, double *force, const int64_t *out_off,
    double *wx_out, double *wz_out, double *wg_out, int32_t *n_final,
    double *vel_last, int32_t *n_vel_last, const double *fb_gain,
    const double *fb_xref, double *gb_final) {
  const int32_t nb = p->n_bound;
  const int32_t S = orc_system_size(nb, p->shed_mode);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int32_t k = 0; k < K; ++k) {
    int32_t fo = field_of ? field_of[k] : k;
    int64_t f0 = field_off[fo], f1 = field_off[fo + 1];
    int32_t n0 = (int32_t)(f1 - f0);
    orc_state s;
    memcpy(s.g, &g0[7 * k], sizeof(s.g));
    s.gb_prev = (double *)malloc(sizeof(double) * nb);
    memcpy(s.gb_prev, &gb0[(int64_t)nb * k], sizeof(double) * nb);
    s.glev_prev = 0.0;
    s.n_w = n0;
    s.cap = n0 + shed_per_step(p->shed_mode) * H;
    s.wx = (double *)malloc(sizeof(double) * (s.cap + 1));
    s.wz = (double *)malloc(sizeof(double) * (s.cap + 1));
    s.wg = (double *)malloc(sizeof(double) * (s.cap + 1));
    s.tag = (int32_t *)calloc(s.cap + 1, sizeof(int32_t));
    s.status = ORC_OK;
    memcpy(s.wx, &wx[f0], sizeof(double) * n0);
    memcpy(s.wz, &wz[f0], sizeof(double) * n0);
    memcpy(s.wg, &wg[f0], sizeof(double) * n0);
    if (pairs)
      for (int32_t q = 0; q < n_pairs; ++q) {
        int32_t a = pairs[(int64_t)k * 2 * n_pairs + 2 * q];
        int32_t b = pairs[(int64_t)k * 2 * n_pairs + 2 * q + 1];
        if (a >= 0 && b >= 0 && a < n0 && b < n0 && a != b) {
          s.tag[a] = q + 1;
          s.tag[b] = q + 1;
        }
      }
    if (traj) memcpy(&traj[(int64_t)k * (H + 1) * 7], s.g, sizeof(s.g));
    for (int32_t n = 0; n < H; ++n) {
      orc_loads ld;
      int32_t last = (n == H - 1);
      double *vel = (last && vel_last) ? &vel_last[2 * out_off[k]] : NULL;
      /* Sec. IV-B feedback policy: u_n = u^d_n - H_n (x_n - x^d_n), with the
       * state at the start of the step (open loop without gains) */
      double un = u[(int64_t)k * H + n];
      if (fb_gain) {
        double fb = 0.0;
        for (int32_t j = 0; j < 7; ++j)
          fb += fb_gain[(int64_t)n * 7 + j] * (s.g[j] - fb_xref[(int64_t)n * 7 + j]);
        un -= fb;
      }
      orc_step(p, &s, dt, un, reverse,
               gamma_s ? &gamma_s[((int64_t)k * H + n) * S] : NULL, &ld, vel,
               (last && n_vel_last) ? &n_vel_last[k] : NULL);
      if (force) {
        double *f = &force[((int64_t)k * H + n) * 3];
        f[0] = ld.fx;
        f[1] = ld.fz;
        f[2] = ld.m;
      }
      if (traj) memcpy(&traj[((int64_t)k * (H + 1) + n + 1) * 7], s.g,
                       sizeof(s.g));
    }
    memcpy(&g_final[7 * k], s.g, sizeof(s.g));
    int32_t finite = 1;
    for (int32_t i = 0; i < 7; ++i)
      if (!isfinite(s.g[i])) finite = 0;
    if (!finite) s.status |= ORC_NONFINITE;
    cost[k] = finite ? orc_cost(s.g, x_goal, q_diag) : INFINITY;
    status[k] = s.status;
    if (gb_final) memcpy(&gb_final[(int64_t)nb * k], s.gb_prev, sizeof(double) * nb);
    if (out_off && n_final) {
      int64_t o = out_off[k];
      int64_t capo = out_off[k + 1] - o;
      int32_t n = s.n_w < capo ? s.n_w : (int32_t)capo;
      if (wx_out) memcpy(&wx_out[o], s.wx, sizeof(double) * n);
      if (wz_out) memcpy(&wz_out[o], s.wz, sizeof(double) * n);
      if (wg_out) memcpy(&wg_out[o], s.wg, sizeof(double) * n);
      n_final[k] = s.n_w;
    }
    free(s.gb_prev);
    free(s.wx);
    free(s.wz);
    free(s.wg);
    free(s.tag);
  }
  return 0;
}

/* ---------------------------------------------------------------- MPPI */

/* Eq. 25: xi* = eta sum_i exp(-(J_i - J_min)/lambda) xi_i, with eta the
 * normaliser making the weights sum to one. */
void orc_mppi(int32_t K, int32_t H, const double *cost, double lambda,
              const double *mu, const double *xi, double *w, double *xi_star,
              int32_t *argmin, double *j_min) {
  int32_t am = -1;
  double jm = INFINITY;
  for (int32_t i = 0; i < K; ++i)
    if (isfinite(cost[i]) && cost[i] < jm) {
      jm = cost[i];
      am = i;
    }
  *argmin = am;
  *j_min = jm;
  if (am < 0) {
    for (int32_t i = 0; i < K; ++i) w[i] = 0.0;
    for (int32_t h = 0; h < H; ++h) xi_star[h] = mu[h];
    return;
  }
  double total = 0.0;
  for (int32_t i = 0; i < K; ++i) {
    w[i] = isfinite(cost[i]) ? exp(-(cost[i] - jm) / lambda) : 0.0;
    total += w[i];
  }
  double eta = 1.0 / total;
  for (int32_t i = 0; i < K; ++i) w[i] *= eta;
  for (int32_t h = 0; h < H; ++h) {
    double acc = 0.0;
    for (int32_t i = 0; i < K; ++i) acc += w[i] * xi[(int64_t)i * H + h];
    xi_star[h] = acc;
  }
}
