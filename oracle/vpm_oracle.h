/*
 * vpm_oracle.h -- declarations of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE. This header belongs to the oracle alone. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load the oracle;
 * the GPU library never includes this file and the oracle never includes the
 * GPU library's headers.
 *
 * Method: Gupta, Wolfe, Perrotta, Moore, "Real-Time Maneuver Planning for
 * Fixed-Wing UAVs in Unsteady Flows Using a GPU-Accelerated Vortex Particle
 * Model" (arXiv 2509.16079). Section and equation numbers below refer to it.
 */
#ifndef VPM_ORACLE_H
#define VPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Shedding modes (which edge vortices are unknowns of the surface system). */
#define ORC_SHED_BOTH 0 /* LEV and TEV every step (Sec. III-A)            */
#define ORC_SHED_TE   1 /* TEV only: drop the LEV column and the LE row    */
#define ORC_SHED_NONE 2 /* no shedding: drop both edge columns and rows    */

/* Per-rollout status bits. */
#define ORC_OK        0
#define ORC_NONFINITE 1 /* a final glider value is NaN or infinite        */
#define ORC_CAPACITY  2 /* the wake outgrew the capacity given            */
#define ORC_SINGULAR  4 /* the surface system had a zero pivot            */

typedef struct {
  int32_t n_bound;     /* N_b bound vortices on the chord (Sec. III-A)      */
  int32_t n_wake_max;  /* N_w,max merge threshold; <= 0 disables merging    */
  int32_t shed_mode;   /* ORC_SHED_*                                        */
  int32_t prescribed;  /* 1: glider rates held fixed (no rigid-body update) */
  double chord;        /* c [m]                                             */
  double shed_frac;    /* delta_s / c (2 % in Sec. III-A)                   */
  double r_core;       /* r_core of the regularised kernel [m]              */
  double decay;        /* gamma of the wake circulation decay [1/s]         */
  double rho;          /* air density [kg/m^3]                              */
  double span;         /* wing span s [m]                                   */
  double grav;         /* g [m/s^2]                                         */
  double mass;         /* m [kg]                                            */
  double inertia;      /* I [kg m^2]                                        */
  double l_body;       /* l, body length to the elevator hinge [m]          */
  double l_wing;       /* l_w, CG to wing mid-chord [m]                     */
  double l_elev;       /* l_e, elevator length [m]                          */
  double s_elev;       /* S_e, elevator area [m^2]                          */
  double alpha_crit;   /* separation gate threshold on the wing AoA [rad]   */
  int32_t gate;        /* 1: shed both edges only while alpha_w > alpha_crit,
                          the trailing edge alone otherwise (shed_mode BOTH) */
  int32_t lev_literal; /* test switch for the LEV term of Eq. 13: 0 (the
                          reading used everywhere) takes dGamma_LEV/dt as the
                          rate Gamma_LEV / dt at which circulation leaves the
                          leading edge; 1 takes the literal backward
                          difference of successive LEV strengths, so that a
                          test can tell the two readings apart              */
} orc_params;

/* Wing angle of attack (the separation criterion of Sec. III-A, measured
 * like the elevator's angle of Sec. III-B): pitch minus the direction of the
 * wing point's velocity, alpha_w = theta - atan2(zd_w, xd_w). */
double orc_wing_aoa(const orc_params *p, const double *g);

/* Kernels (Sec. III-A, Eqs. 4 and 5), per unit circulation. */
void orc_kernel_sing(double dx, double dz, double *kx, double *kz);
void orc_kernel_reg(double dx, double dz, double r_core, double *kx, double *kz);

/* Velocity of every wake vortex (Eq. 16): regularised sum over the other
 * wake vortices in FIFO order, then singular sum over the bound vortices.
 * reverse != 0 sums both lists back to front (self-sensitivity probe). */
void orc_wake_velocities(int32_t n_w, const double *wx, const double *wz,
                         const double *wg, int32_t n_b, const double *bx,
                         const double *bz, const double *bg, double r_core,
                         int32_t reverse, double *vx, double *vz);

/* Explicit Euler advection and circulation decay (Eq. 16, Eq. 17). */
void orc_advect(int32_t n_w, double *wx, double *wz, double *wg,
                const double *vx, const double *vz, double dt, double decay);

/* Plate geometry from the glider state g = (x, z, theta, phi, xd, zd, thd).
 * Outputs (any may be NULL): wing point x_w[2], its velocity xw_dot[2],
 * collocation points rc[(N_b+1)*2], bound points rb[N_b*2], LEV and TEV
 * release points r_lev[2], r_tev[2], unit normal n_hat[2], tangent t_hat[2]. */
void orc_plate_geometry(const orc_params *p, const double *g, double *x_w,
                        double *xw_dot, double *rc, double *rb, double *r_lev,
                        double *r_tev, double *n_hat, double *t_hat);

/* Surface system size for a shedding mode. */
int32_t orc_system_size(int32_t n_bound, int32_t shed_mode);

/* Assemble the surface matrix (Eq. 8) at the given pose: a[S*S], row-major. */
void orc_surface_matrix(const orc_params *p, const double *g, int32_t shed_mode,
                        double *a);

/* Gaussian elimination with partial pivoting; a and b are overwritten.
 * Returns 0, or -1 on a zero pivot. */
int32_t orc_solve(int32_t n, double *a, double *b, double *x);

/* Surface solve from wing pose and wake-induced velocities (Eqs. 10-12):
 * pose6 = (x_w, z_w, theta, xd_w, zd_w, thetad); vw_c[(N_b+1)*2] is the wake
 * velocity at the collocation points; sum_gw = sum of wake circulations.
 * Writes gamma_s[S]; returns 0 or -1 (singular). */
int32_t orc_plate_solve_pose(const orc_params *p, const double *pose6,
                             const double *vw_c, double sum_gw,
                             int32_t shed_mode, double *gamma_s);

/* Elevator force (Sec. III-B): writes x_e[2] and F_e[2]; returns alpha_e. */
double orc_elevator(const orc_params *p, const double *g, double u,
                    double *x_e, double *f_e);

/* Disturbance termination test (Sec. V): 1 if the closed segment a-b meets
 * the chord rectangle inflated by 2 % of chord opposite the normal. */
int32_t orc_segment_hits_plate(const orc_params *p, const double *g,
                               const double *a, const double *b);

/* One rollout batch. Rollout k starts from wake field fo = field_of[k]
 * (field_of NULL: fo = k), i.e. entries [field_off[fo], field_off[fo+1]) of
 * wx/wz/wg, in age order (oldest first). pairs[k*2*n_pairs + 2q + {0,1}] are
 * indices of disturbance pair q in that field, or -1. u[k*H + n] is the full
 * control (mean + perturbation) of step n. Outputs: g_final[K*7], cost[K],
 * status[K]; optional (NULL to skip): traj[K*(H+1)*7], gamma_s[K*H*S],
 * force[K*H*3] (F_w,x, F_w,z, M_w), and the final wake / last-step wake
 * velocities at out_off[k] (capacity out_off[k+1]-out_off[k]) with counts in
 * n_final[k]; vel_last holds (vx, vz) of the N_w + shed vortices advected in
 * the last step, in FIFO order before merging, count n_vel_last[k].
 * n_threads <= 0 uses the OpenMP default. Returns 0. */
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
    const double *fb_xref, double *gb_final);

/* Terminal cost (Eq. 24): J = sum_k q_k (g_k - x_goal_k)^2. */
double orc_cost(const double *g_final, const double *x_goal,
                const double *q_diag);

/* MPPI reweighting (Eq. 25). xi[K*H] are the sampled control sequences and
 * mu[H] their mean; writes w[K], xi_star[H], *argmin (lowest index on ties)
 * and *j_min. Non-finite costs get weight 0; with no finite cost every weight
 * is 0, xi_star = mu, *argmin = -1 and *j_min = +inf. */
void orc_mppi(int32_t K, int32_t H, const double *cost, double lambda,
              const double *mu, const double *xi, double *w, double *xi_star,
              int32_t *argmin, double *j_min);

#ifdef __cplusplus
}
#endif
#endif
