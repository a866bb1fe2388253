/*
 * vpm.h -- C ABI of the MI355X (gfx950) rollout engine for the vortex
 * particle glider planner of Gupta, Wolfe, Perrotta and Moore, "Real-Time
 * Maneuver Planning for Fixed-Wing UAVs in Unsteady Flows Using a
 * GPU-Accelerated Vortex Particle Model" (arXiv 2509.16079).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status (VPM_OK = 0, VPM_PENDING = 1 from
 *    planner_poll only, negative on error) and never throws. On error,
 *    vpm_last_error() returns a message for the calling thread.
 *  - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors
 *    on the context's device) unless marked "host". The caller owns them; the
 *    library only reads inputs and only writes outputs.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream: inputs must stay alive and
 *    outputs must not be read until the stream has been synchronised.
 *  - Floating-point arrays are double in memory whatever the compute
 *    precision; VPM_FP32C computes the interaction sums in FP32 with
 *    compensated per-target accumulation and keeps the surface solve and the
 *    circulation sums in FP64.
 *  - Coordinates: x forward, z up, angles counter-clockwise (nose up), and a
 *    positive circulation turns counter-clockwise.
 */
#ifndef VPM_H
#define VPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VPM_API __attribute__((visibility("default")))

/* ---------------------------------------------------------- status codes */
#define VPM_OK 0
#define VPM_PENDING 1     /* planner_poll: the request has not finished      */
#define VPM_EINVAL (-1)   /* bad argument                                    */
#define VPM_ENOMEM (-2)   /* device or host allocation failed                */
#define VPM_EDEVICE (-3)  /* HIP error (no device, launch failure, ...)      */
#define VPM_ESINGULAR (-4) /* the plate system has a zero pivot              */
#define VPM_EBUDGET (-5)  /* a planner request exceeds the HBM budget alone  */
#define VPM_ECAPACITY (-6) /* a wake does not fit the kernel's limits         */
#define VPM_ENOTFOUND (-7) /* unknown planner ticket or state                */

/* per-rollout status bits written by vpm_rollout_batch */
#define VPM_ROLLOUT_NONFINITE 1 /* a final glider value is NaN or infinite  */
#define VPM_ROLLOUT_CAPACITY 2  /* the initial wake exceeds max_wake0       */
#define VPM_ROLLOUT_BADFIELD 4  /* field_of[k] outside 0..n_fields-1, or its
                                   offsets decrease                          */

/* shedding modes: which edge vortices are unknowns of the surface system */
#define VPM_SHED_BOTH 0 /* an LEV and a TEV every step (Sec. III-A)          */
#define VPM_SHED_TE 1   /* TEV only (Kutta condition at the trailing edge)    */
#define VPM_SHED_NONE 2 /* no shedding                                        */

/* rollout kernel variant (vpm_set_path) */
#define VPM_PATH_AUTO 0   /* LDS-resident wake when it fits, else streaming   */
#define VPM_PATH_LDS 1    /* LDS-resident only (VPM_ECAPACITY if too large)   */
#define VPM_PATH_STREAM 2 /* wake in a device workspace, tiles through LDS    */

/* compute precision */
#define VPM_FP32C 0 /* FP32 interactions, compensated sums; FP64 solve        */
#define VPM_FP64 1  /* FP64 throughout                                        */

/* Model parameters (Sec. III-A and III-B), copied at each call. */
typedef struct {
  int32_t n_bound;    /* N_b bound vortices on the chord, 1..64            */
  int32_t n_wake_max; /* N_w,max: merge the two oldest above it; <= 0: off */
  int32_t shed_mode;  /* VPM_SHED_*: both edges, trailing edge only, none  */
  int32_t precision;  /* VPM_FP32C or VPM_FP64                             */
  double chord;       /* c [m]                                             */
  double shed_frac;   /* delta_s / c; the paper uses 0.02                  */
  double r_core;      /* core radius of the regularised kernel [m], > 0    */
  double decay;       /* gamma of dGamma_w/dt = -gamma Gamma_w [1/s]        */
  double rho;         /* air density [kg/m^3]                              */
  double span;        /* wing span s [m]                                   */
  double grav;        /* g [m/s^2]                                         */
  double mass;        /* m [kg], > 0                                       */
  double inertia;     /* I [kg m^2], > 0                                   */
  double l_body;      /* l: CG to elevator hinge [m]                       */
  double l_wing;      /* l_w: CG to wing mid-chord [m]                     */
  double l_elev;      /* l_e: elevator length [m]                          */
  double s_elev;      /* S_e: elevator area [m^2]                          */
  double alpha_crit;  /* separation threshold on the wing AoA [rad]        */
  int32_t gate;       /* 1 (needs shed_mode BOTH): a step sheds from both
                         edges while the wing's angle of attack, pitch minus
                         the direction of the wing point's velocity, exceeds
                         alpha_crit, from the trailing edge only otherwise
                         (Sec. III-A); 0: shed_mode every step              */
  int32_t reserved;   /* 0                                                 */
} vpm_params;

/* One batch of K independent rollouts of H explicit-Euler steps of the
 * coupled VPM-glider model (Sec. III-A, III-B). Wake fields are stored once
 * and shared: rollout k starts from field fo = field_of[k] (field_of NULL:
 * fo = k), the entries [field_off[fo], field_off[fo+1]) of wx/wz/wg in age
 * order (oldest first). */
typedef struct {
  int32_t K;              /* rollouts, >= 1                                 */
  int32_t H;              /* steps per rollout, >= 1                        */
  double dt;              /* step [s], > 0                                  */
  int32_t n_fields;       /* number of wake fields, >= 1                    */
  int32_t max_wake0;      /* upper bound of every field's size; a rollout
                             whose field is larger gets VPM_ROLLOUT_CAPACITY */
  int32_t n_pairs;        /* disturbance pairs per rollout, 0..4            */
  int32_t reserved;
  const double *g0;       /* [K][7] glider state (x, z, th, phi, xd, zd, thd) */
  const double *gb0;      /* [K][N_b] previous-step bound circulations       */
  const int64_t *field_off; /* [n_fields + 1] nondecreasing, field_off[0]=0 */
  const int32_t *field_of;  /* [K] field index per rollout, or NULL         */
  const double *wx;       /* [field_off[n_fields]] wake x [m]               */
  const double *wz;       /* wake z [m]                                     */
  const double *wg;       /* wake circulation [m^2/s]                       */
  const int32_t *pairs;   /* [K][2 n_pairs] field indices of the two vortices
                             of each disturbance pair (Sec. V), -1 = none;
                             NULL when n_pairs = 0                          */
  const double *u_mean;   /* [H] mean elevator rate (control u = phi_dot)   */
  const double *u_eps;    /* [K][H] perturbation of rollout k; the control of
                             step n is u_mean[n] + u_eps[k][n]              */
  double x_goal[7];       /* host values: goal state of the cost (Eq. 24)   */
  double q_diag[7];       /* host values: diagonal of Q (Eq. 24)            */
  const double *fb_gain;  /* [H][7] feedback gains H_n of the policy of
                             Sec. IV-B, or NULL (open loop); with gains the
                             control of step n is u_mean[n] + u_eps[k][n]
                             - fb_gain[n] . (x_n - fb_xref[n]), x_n the
                             state at the start of the step (FP64)          */
  const double *fb_xref;  /* [H][7] reference states x^d_n (with fb_gain)   */
} vpm_batch_in;

/* Outputs of vpm_rollout_batch. Required: g_final, cost, status. Optional
 * (NULL to skip): traj, gamma_s, pair_count, and the wake block. The wake
 * block (all of wake_off, n_final and at least one of wx/wz/wg/vel_last)
 * uses per-rollout capacity wake_off[k+1] - wake_off[k], which must be at
 * least N_0 + 2H; entries beyond the count are left untouched. */
typedef struct {
  double *g_final;        /* [K][7] state after H steps                     */
  double *cost;           /* [K] J of Eq. 24; +inf when non-finite          */
  int32_t *status;        /* [K] VPM_ROLLOUT_* bits                         */
  double *traj;           /* [K][H+1][7] states, or NULL                    */
  double *gamma_s;        /* [K][H][S] surface circulations per step, or
                             NULL; S = N_b + 2 (bound, LEV, TEV), N_b + 1
                             (bound, TEV) or N_b by shed_mode; a gated step
                             that sheds from the trailing edge only writes
                             (bound, TEV) and a zero                        */
  int64_t *pair_count;    /* [K] pair-interactions the rollout's steps
                             comprise (method count), or NULL               */
  const int64_t *wake_off; /* [K+1] output capacity layout, or NULL         */
  double *wx;             /* final wake x (after merging), or NULL          */
  double *wz;             /* final wake z, or NULL                          */
  double *wg;             /* final wake circulation, or NULL                */
  int32_t *n_final;       /* [K] final wake count                           */
  double *vel_last;       /* [wake_off[K]][2] velocity of each vortex
                             advected in the last step (FIFO order, before
                             merging), or NULL                              */
  int32_t *n_vel_last;    /* [K] count of vel_last entries, or NULL         */
  double *gb_final;       /* [K][N_b] bound circulations of the last step
                             (the gb0 that continues the rollout), or NULL;
                             a rollout with a status bit of its input
                             (capacity, bad field) gets its gb0             */
} vpm_batch_out;

typedef struct vpm_ctx vpm_ctx;

/* Create a context on HIP device `device` (an index as hipSetDevice takes).
 * The context caches the FP64 plate-system inverses and the kernel tuning
 * table. Returns VPM_EDEVICE if the device is absent or is not gfx950. */
VPM_API int vpm_create(vpm_ctx **out, int device);
VPM_API void vpm_destroy(vpm_ctx *ctx);

/* Choose the rollout kernel variant for later calls on this context. Both
 * compute the same steps; AUTO keeps the wake in LDS when it fits (up to a few
 * thousand vortices) and otherwise streams it from a context-owned workspace
 * of (max_wake0 + 2H) x 24 B (FP32) per resident workgroup, grown on demand
 * and serialised across streams. Returns VPM_EINVAL for an unknown value. */
VPM_API int vpm_set_path(vpm_ctx *ctx, int path);

/* Kernel classes of vpm_set_tuning: rollouts whose wake fits a quarter of a
 * CU's LDS run in 4-wave workgroups (several per CU), larger ones in one
 * 16-wave workgroup per CU, and wakes beyond the LDS stream from the
 * workspace. */
#define VPM_CLASS_SMALL 0
#define VPM_CLASS_LARGE 1
#define VPM_CLASS_STREAM 2

/* FP32 kernel shape of one class for later calls on this context (results
 * change only by rounding): targets_per_thread in {1, 2, 4} is how many
 * targets each lane holds in registers against each LDS source read, and
 * tile in {64, 128, 256} how many sources are summed plainly before each
 * compensated (TwoSum) fold. Defaults: small 4/64, large 2/64, streamed
 * 4/64. FP64 keeps 2/64. The project's autotuner (the Python module
 * paper_2509_16079_amd.autotune) picks these by timing. A larger target count
 * in the large class lowers its LDS capacity, moving the streamed-class
 * boundary. Errors: VPM_EINVAL. */
VPM_API int vpm_set_tuning(vpm_ctx *ctx, int32_t kernel_class,
                           int32_t targets_per_thread, int32_t tile);
VPM_API int vpm_get_tuning(const vpm_ctx *ctx, int32_t kernel_class,
                           int32_t *targets_per_thread, int32_t *tile);

/* Message of the calling thread's last error ("" if none). */
VPM_API const char *vpm_last_error(void);

/* Host-only argument check of vpm_rollout_batch (no HIP call): returns
 * VPM_OK or the error vpm_rollout_batch would return for these arguments. */
VPM_API int vpm_validate_batch(const vpm_params *params, const vpm_batch_in *in,
                               const vpm_batch_out *out);

/* Batched rollouts (Sec. III-A/B stepping, Eq. 24 cost). Each step: surface
 * velocities (Eq. 12), the surface solve K Gamma_S = b (Eqs. 8-11) with the
 * Kelvin row, unsteady Bernoulli loads (Eqs. 13-15), elevator force and
 * rigid-body accelerations (Sec. III-B), LEV/TEV shedding, wake velocities
 * (Eq. 16) over the wake and the bound vortices, explicit Euler advection
 * and decay (Eq. 17), merging of the two oldest vortices above N_w,max, the
 * disturbance termination test (Sec. V) and the explicit Euler glider step.
 * Each step sheds per shed_mode, or with the separation gate on per the
 * wing's angle of attack at the start of the step (decided in FP64 from the
 * stored state in both precisions); an edge that does not shed drops its
 * unknown and its collocation row from the system. The wake capacity rule
 * (N_0 + 2H) is the same for every mode.
 * Errors: VPM_EINVAL (bad sizes, NULL required pointers, invalid params; or,
 * during stream capture, a first call that would have to build a plate
 * inverse or grow a context buffer), VPM_ECAPACITY
 * (max_wake0 + 2H beyond the LDS limit when VPM_PATH_LDS is forced),
 * VPM_ENOMEM, VPM_ESINGULAR, VPM_EDEVICE.
 * Graph capture: the call may be captured into a HIP graph once an eager
 * call with the same geometry and no smaller sizes has run on this context;
 * it then allocates nothing, records no memset, and forks its class kernels
 * onto the context's side streams and joins them back. A replayed graph
 * reuses the context's workspace without the cross-stream ordering that
 * eager calls get, so the caller must not run it concurrently with other
 * calls on the same context. */
VPM_API int vpm_rollout_batch(vpm_ctx *ctx, const vpm_params *params,
                              const vpm_batch_in *in, vpm_batch_out *out,
                              void *stream);

/* vpm_rollout_batch for callers that cannot allocate device memory in their
 * hot loop (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, with the kernels' scratch
 * (the uneven-batch plan and the streaming workspace) taken from a static
 * device array of the library of VPM_NOALLOC_SCRATCH_BYTES per GPU (mapped
 * when the library's code is loaded on the GPU, held until the process ends)
 * instead of context buffers. It calls no hipMalloc, hipFree or other
 * allocating routine and creates no stream or event: the class kernels of an
 * uneven batch run one after another on `stream`, and streamed rollouts run
 * on as many workgroups (at most one per CU) as whole slots of
 * (max_wake0 + 2H) x 24 B (FP32) or x 48 B (FP64) fit beside the plan
 * (K x 4 B + 64 B, rounded up to 256 B). The plate inverse of params'
 * geometry must already be cached in the context (vpm_reserve or an earlier
 * vpm_rollout_batch with these params). Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents (the kernels initialise
 * what they read): calls that overlap on one GPU, from any context or
 * stream, race and must be ordered by the caller. Errors: those of
 * vpm_rollout_batch, VPM_EINVAL if the plate inverse is not cached, and
 * VPM_ECAPACITY if the plan or one streaming slot exceeds the array. */
#define VPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
VPM_API int vpm_rollout_batch_noalloc(vpm_ctx *ctx, const vpm_params *params,
                                      const vpm_batch_in *in, vpm_batch_out *out,
                                      void *stream);

/* Prepare the context for later vpm_rollout_batch calls with these or smaller
 * sizes (K rollouts, H steps, initial wakes of at most max_wake0 vortices in
 * n_fields fields, the kernel variant set by vpm_set_path): builds the plate
 * inverse for params' geometry and grows the streaming workspace and the
 * uneven-batch plan buffer as those calls would. Such calls then allocate
 * nothing, so they may be the first calls captured into a HIP graph. Not a
 * step of the method: it serves callers that must not allocate in their hot
 * loop. Synchronises the device when a buffer grows. Errors: VPM_EINVAL,
 * VPM_ENOMEM, VPM_ESINGULAR, VPM_EDEVICE. */
VPM_API int vpm_reserve(vpm_ctx *ctx, const vpm_params *params, int32_t K,
                        int32_t H, int32_t max_wake0, int32_t n_fields);

/* Standalone batched FP64 surface solve (Eqs. 10-12): for B wing poses
 * pose[b] = (x_w, z_w, th, xd_w, zd_w, thd) with wake-induced velocities
 * vw_c[b][i] (i = 0..N_b, collocation points from LE to TE) and wake
 * circulation sums sum_gw[b], writes the surface circulations gamma_s[b][S]
 * (S = N_b + 2 / N_b + 1 / N_b for BOTH / TE / NONE: bound first, then LEV,
 * then TEV). Errors: VPM_EINVAL, VPM_ESINGULAR, VPM_EDEVICE. */
VPM_API int vpm_plate_solve(vpm_ctx *ctx, const vpm_params *params, int32_t B,
                            const double *pose, const double *vw_c,
                            const double *sum_gw, int32_t shed_mode,
                            double *gamma_s, void *stream);

/* MPPI reweighting (Eq. 25). cost[K]; weights w_out[i] = exp(-(J_i -
 * J_min)/lambda) / sum_j exp(-(J_j - J_min)/lambda) (non-finite costs get
 * 0); u_new[h] = u_mean[h] + sum_i w_i u_eps[i][h]; *argmin (device int32,
 * lowest index on ties) and *jmin (device double). With no finite cost:
 * weights 0, u_new = u_mean, argmin = -1, jmin = +inf. Errors: VPM_EINVAL
 * (K < 1, H < 1, lambda <= 0, NULL pointers), VPM_EDEVICE. */
VPM_API int mppi_weights(vpm_ctx *ctx, int32_t K, int32_t H, const double *cost,
                         double lambda, const double *u_mean,
                         const double *u_eps, double *w_out, double *u_new,
                         int32_t *argmin, double *jmin, void *stream);

/* ------------------------------------------------------------ planner
 * A replanning service: fluid and vehicle states stay resident on the
 * device; requests (one MPPI iteration of the planner's hot path, Sec. IV-A:
 * K rollouts of H steps from a resident state, costs and the softmin
 * update) are admitted in arrival order while a slot is free and the sum of
 * in-flight footprints stays within the HBM budget, and admitted requests
 * run concurrently on separate streams, so work that arrives while others
 * are on the GPU overlaps with it. All planner calls are thread-safe. */
typedef struct planner planner;

typedef struct {
  int32_t device;           /* HIP device index                              */
  int32_t max_slots;        /* requests in flight at once, 1..16 (1 = serial) */
  size_t hbm_budget_bytes;  /* admission budget for in-flight footprints      */
} planner_opts;

typedef struct {
  uint64_t state_id;        /* resident state from planner_state_put         */
  vpm_params params;        /* model parameters (n_bound must match the state) */
  int32_t K, H;             /* rollouts and steps                            */
  double dt;                /* step [s]                                      */
  double lambda;            /* MPPI temperature (Eq. 25), > 0                */
  int32_t iterations;       /* MPPI iterations, >= 1: iteration i rolls out
                               the same initial state with the mean updated by
                               iteration i - 1 (the planner's replan runs 3) */
  int32_t advance;          /* 0..H: after the last iteration, carry the
                               resident state `advance` steps forward under the
                               updated controls (no perturbation) and keep
                               the result as a new resident state (the
                               receding-horizon step of Sec. IV-C); 0: none  */
  double x_goal[7];         /* cost goal (Eq. 24)                            */
  double q_diag[7];         /* cost weights (Eq. 24)                         */
  const double *u_mean;     /* host [H]: copied at submit                    */
  const double *u_eps;      /* host [iterations][K][H]: copied at submit; or
                               NULL: drawn at submit from `seed` as
                               vpm_sample_eps(seed, i, K, H, sigma) for
                               iteration i                                   */
  uint64_t seed;            /* with u_eps NULL                               */
  double sigma;             /* with u_eps NULL: perturbation standard
                               deviation (>= 0, the control's units)         */
} plan_req;

typedef struct {
  int32_t status;           /* VPM_OK, or the error the request failed with  */
  int32_t argmin;           /* MPPI argmin (-1 if no finite cost)            */
  double jmin;
  double *u_new;            /* host [H] caller buffer for the update after the
                               last iteration, or NULL                       */
  double *w;                /* host [K] weights of the last iteration, or NULL */
  double *cost;             /* host [K] costs of the last iteration, or NULL  */
  double *g_final;          /* host [K][7] caller buffer, or NULL            */
  double t_arrive_us;       /* submit time (us since planner_create), taken on
                               entry to planner_submit                       */
  double t_admit_us;        /* admission time                               */
  double t_done_us;         /* completion time (results in host memory)     */
  int64_t pairs;            /* pair-interactions of the request (all
                               iterations; the advance not included)         */
  uint64_t new_state_id;    /* the advanced resident state (advance > 0 and
                               status VPM_OK), else 0; the caller drops it   */
  int32_t new_state_status; /* VPM_ROLLOUT_* bits of the advance rollout     */
  int32_t reserved;
} plan_result;

/* Create / destroy a planner (it owns one context and stream per slot).
 * planner_destroy waits for in-flight requests. The HBM budget lives in
 * planner_opts rather than in vpm_create because admission is the planner's
 * job: a bare context allocates only what the calls made on it need. */
VPM_API int planner_create(planner **out, const planner_opts *opts);
VPM_API void planner_destroy(planner *p);

/* Size every slot (staging, per-rollout buffers, plate inverses, rollout
 * workspaces) for requests of up to K rollouts, H steps, resident wakes of
 * n0 vortices and `iterations` iterations with these params, so that serving
 * such requests allocates and frees no device memory (a growth while other
 * slots run would synchronise the device and serialise them). Not a step of
 * the method: a set-up call. Needs an idle planner (nothing queued or
 * running). Errors: VPM_EINVAL (bad sizes, busy planner), VPM_ENOMEM,
 * VPM_ESINGULAR, VPM_EDEVICE. */
VPM_API int planner_reserve(planner *p, const vpm_params *params, int32_t K, int32_t H,
                            int32_t n0, int32_t iterations);

/* vpm_set_tuning for the kernel class on every slot's context. */
VPM_API int planner_set_tuning(planner *p, int32_t kernel_class, int32_t targets_per_thread,
                               int32_t tile);

/* Upload a fluid and vehicle state and keep it resident: n vortices (host
 * arrays, age order), glider state g7 (host [7]) and previous bound
 * circulations gb (host [n_bound]). Returns its id in *state_id. */
VPM_API int planner_state_put(planner *p, int32_t n, const double *wx,
                              const double *wz, const double *wg,
                              const double *g7, int32_t n_bound,
                              const double *gb, uint64_t *state_id);
/* Read a resident state back: *n (its wake count) always; the wake (host
 * arrays of `capacity` >= n entries), g7 [7] and gb [n_bound] for each
 * pointer that is not NULL. Errors: VPM_EINVAL, VPM_ENOTFOUND, VPM_EDEVICE. */
VPM_API int planner_state_get(planner *p, uint64_t state_id, int32_t *n, double *wx,
                              double *wz, double *wg, double *g7, double *gb,
                              int32_t capacity);
VPM_API int planner_state_drop(planner *p, uint64_t state_id);

/* Queue a request; its inputs are copied (seeded perturbations are drawn
 * here, on the caller's thread), so the caller may reuse them on return.
 * Returns a ticket. Errors: VPM_EINVAL, VPM_ENOTFOUND (state), VPM_EBUDGET
 * (the request alone exceeds the budget). */
VPM_API int planner_submit(planner *p, const plan_req *req, uint64_t *ticket);

/* Wait up to timeout_us (0: do not wait, < 0: forever) for a request.
 * Returns VPM_PENDING, or VPM_OK after filling *res (the ticket is then
 * released), or VPM_ENOTFOUND. */
VPM_API int planner_poll(planner *p, uint64_t ticket, plan_result *res,
                         int32_t timeout_us);

/* Device-memory footprint the planner charges a request against its budget
 * (host arithmetic): perturbations of every iteration, per-rollout inputs
 * and outputs, the advanced state, and for wakes beyond the LDS-resident
 * kernel in params' precision the streaming workspace of one slot per CU.
 * Returns 0 for NULL params or n_bound outside 1..64. */
VPM_API size_t planner_footprint(const vpm_params *params, int32_t K, int32_t H, int32_t n0,
                                 int32_t iterations, int32_t advance);

/* MPPI control perturbations from a seed (Sec. IV-A: the K sampled control
 * sequences around the mean), host FP64: out [K][H] (host) receives sigma * z
 * for rollouts k = 0..K-1, steps n = 0..H-1 of MPPI iteration `iteration`,
 * z standard normal from Philox4x64-10 (Salmon et al., SC 2011; key
 * (seed, 0), counter (n / 4, k, iteration, 0)) and the Box-Muller transform
 * of its output words taken in pairs (w0, w1) for steps 4j, 4j+1 and
 * (w2, w3) for 4j+2, 4j+3: with u_a = ((w_a >> 11) + 1) 2^-53 and
 * u_b = (w_b >> 11) 2^-53, r = sqrt(-2 ln u_a), t = 2 pi u_b, the pair is
 * (r cos t, r sin t). Each value depends on (seed, iteration, k, n) only.
 * Errors: VPM_EINVAL (K or H < 1, iteration < 0, sigma < 0 or not finite,
 * out NULL). */
VPM_API int vpm_sample_eps(uint64_t seed, int32_t iteration, int32_t K, int32_t H,
                           double sigma, double *out);

/* Local feedback policy from rollouts (Sec. IV-B). Least-squares Jacobians
 * at every step (Eqs. 26-28): the rates of the K perturbed rollouts minus
 * the nominal's, (x_{k+1} - x_k) / dt exactly for the explicit Euler step,
 * regressed in FP64 on the state deviations of theta, phi, x_dot, z_dot,
 * theta_dot and the control deviation; only the three acceleration rows are
 * unknown (the 3 x 5 block A_hat and 3 x 1 block B_hat of Eq. 28), the
 * kinematic rows are known (rates of x, z, theta are x_dot, z_dot,
 * theta_dot; the rate of phi is u). The discrete system is the explicit
 * Euler map A_k = I + dt dF/dx, B_k = dt dF/du. Then TVLQR (Eqs. 29-30):
 * S_H = diag(q_f), S_k = A_k' S A_k - A_k' S B_k (r_c + B_k' S B_k)^-1
 * B_k' S A_k + diag(q_c) with S = S_{k+1}, kept symmetric each step, and
 * gain_k = (r_c + B_k' S B_k)^-1 B_k' S A_k; the policy is
 * u_k = u_k^d - gain_k . (x_k - x_k^d). */
typedef struct {
  int32_t K;              /* perturbed rollouts (>= 1; fewer than 6 leave
                             every step rank-deficient)                     */
  int32_t H;              /* steps (>= 1)                                   */
  double dt;              /* step of the rollouts (> 0)                     */
  const double *traj_nom; /* device [H+1][7] nominal states                 */
  const double *traj;     /* device [K][H+1][7] perturbed rollouts (the
                             layout of vpm_batch_out.traj)                  */
  const double *du;       /* device [K][H] control deviations u^i_k - u_k   */
  double q_f[7];          /* host: diagonal of the final cost Q_f (>= 0)    */
  double q_c[7];          /* host: diagonal of the running cost Q_c (>= 0)  */
  double r_c;             /* host: control weight R_c (> 0)                 */
} vpm_policy_in;

typedef struct {
  double *a;              /* device [H][7][7] A_k (row-major)               */
  double *b;              /* device [H][7] B_k                              */
  double *gain;           /* device [H][7] gain_k                           */
  double *s;              /* device [H+1][7][7] S_k, or NULL                */
  int32_t *status;        /* device [H]: 1 where the regression is rank-
                             deficient (fewer than 6 samples, a zero
                             column, or a Cholesky pivot of the column-
                             scaled normal matrix <= 1e-14); that step
                             takes A_hat = 0, B_hat = 0                     */
} vpm_policy_out;

/* Runs the synthesis (one workgroup per step) and the Riccati recursion
 * (one wavefront) on `stream`; every buffer is caller-owned device memory,
 * nothing is allocated. Errors: VPM_EINVAL (sizes, NULL required pointers,
 * non-finite or negative weights, r_c <= 0), VPM_EDEVICE. */
VPM_API int vpm_policy(vpm_ctx *ctx, const vpm_policy_in *in, vpm_policy_out *out,
                       void *stream);

/* One replanning cycle of the nonlinear MPC of Sec. IV-C, enqueued on one
 * stream with no host round trip:
 *  1. projection: the resident state (glider, bound circulations, wake) is
 *     stepped P steps forward under the policy in force, u_n = u_plan[n] -
 *     gain_plan[n] . (x_n - x_plan[n]) (open loop when gain_plan is NULL),
 *     to where the new plan will take over;
 *  2. MPPI: `iterations` rounds of K rollouts of H steps from the projected
 *     state around the mean controls, the first mean being u_plan shifted
 *     by P (its last value held), each round followed by the reweighting of
 *     Eq. 25 (perturbations u_eps[iteration][k][n] are inputs);
 *  3. policy: the nominal rollout under the final mean and Kp rollouts from
 *     perturbed projected states (g_proj + x_eps[i]) under perturbed
 *     controls (+ du[i]), then vpm_policy on their trajectories.
 * The projection and MPPI rollouts run in params->precision, the policy
 * rollouts in FP64 (the regression takes differences of trajectories about
 * 1e-2 apart, which binary32 state storage would blur). Disturbance pairs (indices into
 * the resident wake) are only accepted when no merging can occur within
 * P + H steps (n_wake_max = 0 or n_wake + 2 (P + H) <= n_wake_max), so that
 * their indices stay valid in the projected wake. The context keeps a
 * workspace for the cycle, grown on demand (a growth synchronises the
 * device). Errors: VPM_EINVAL, VPM_ENOMEM, VPM_ESINGULAR, VPM_EDEVICE. */
typedef struct {
  double dt;              /* step [s] (> 0)                                  */
  int32_t H;              /* plan horizon in steps (>= 1)                    */
  int32_t P;              /* projection steps (0 <= P <= H)                  */
  int32_t K;              /* MPPI rollouts per iteration (>= 1)              */
  int32_t iterations;     /* MPPI iterations (>= 1)                          */
  int32_t Kp;             /* perturbed rollouts of the policy synthesis      */
  int32_t n_wake;         /* resident wake vortices (>= 0)                   */
  int32_t n_pairs;        /* disturbance pairs (0..4)                        */
  int32_t reserved;
  const double *g;        /* device [7] resident glider state                */
  const double *gb;       /* device [N_b] its previous bound circulations    */
  const double *wx, *wz, *wg; /* device [n_wake] resident wake, oldest first */
  const int32_t *pairs;   /* device [2 n_pairs] or NULL                      */
  const double *u_plan;   /* device [H] controls of the policy in force      */
  const double *x_plan;   /* device [H][7] its nominal states, or NULL       */
  const double *gain_plan; /* device [H][7] its gains, or NULL (open loop)   */
  const double *u_eps;    /* device [iterations][K][H] MPPI perturbations    */
  const double *x_eps;    /* device [Kp][7] initial-state perturbations      */
  const double *du;       /* device [Kp][H] control perturbations            */
  double lambda;          /* MPPI temperature (> 0)                          */
  double x_goal[7], q_diag[7]; /* host: cost of Eq. 24                       */
  double q_f[7], q_c[7], r_c;  /* host: TVLQR weights (vpm_policy)           */
} vpm_replan_in;

typedef struct {
  double *g_proj;         /* device [7] projected glider state               */
  double *u_new;          /* device [H] new nominal controls                 */
  double *x_new;          /* device [H+1][7] new nominal trajectory          */
  double *gain;           /* device [H][7] new TVLQR gains                   */
  double *jmin;           /* device [iterations] best cost of each round     */
  int32_t *argmin;        /* device [iterations] its rollout                 */
  int32_t *status;        /* device [H] rank-deficient steps of the policy   */
} vpm_replan_out;

VPM_API int vpm_replan(vpm_ctx *ctx, const vpm_params *params, const vpm_replan_in *in,
                       vpm_replan_out *out, void *stream);

/* TVLQR alone (Eqs. 29-30 as in vpm_policy) on caller-supplied discrete
 * systems: a [H][7][7] (row-major) and b [H][7] in, gain [H][7] and
 * optionally s [H+1][7][7] out, all device memory. Serves policies whose
 * Jacobians come from elsewhere, such as the finite-difference ones below.
 * Errors: VPM_EINVAL, VPM_EDEVICE. */
VPM_API int vpm_tvlqr(vpm_ctx *ctx, int32_t H, const double *a, const double *b,
                      const double q_f[7], const double q_c[7], double r_c, double *gain,
                      double *s, void *stream);

/* Finite-difference Jacobians through the model (the alternative to the
 * least-squares synthesis that Sec. IV-B compares against): along the
 * nominal trajectory from the given state under controls u_nom, at every
 * step k the one-step accelerations (x_{k+1} - x_k)/dt of rows x_dot,
 * z_dot, theta_dot are differenced centrally in theta, phi, x_dot, z_dot,
 * theta_dot (steps h_x) and in u (step h_u), each perturbed one-step
 * rollout starting from the nominal's full state at step k (glider, bound
 * circulations, wake). The result has the form of vpm_policy's: A_k =
 * I + dt A_c, B_k = dt B_c with the kinematic rows known. FP64 rollouts;
 * the nominal is advanced one step at a time (2 launches per step).
 * Disturbance pairs follow vpm_replan's rule. Errors: VPM_EINVAL,
 * VPM_ENOMEM, VPM_ESINGULAR, VPM_EDEVICE. */
typedef struct {
  double dt;
  int32_t H;              /* steps (>= 1)                                    */
  int32_t n_wake;         /* wake vortices of the start state (>= 0)         */
  int32_t n_pairs;        /* disturbance pairs (0..4)                        */
  int32_t reserved;
  const double *g;        /* device [7] start state                          */
  const double *gb;       /* device [N_b] its previous bound circulations    */
  const double *wx, *wz, *wg; /* device [n_wake] start wake                  */
  const int32_t *pairs;   /* device [2 n_pairs] or NULL                      */
  const double *u_nom;    /* device [H] nominal controls                     */
  double h_x[5];          /* host: steps in theta, phi, x_dot, z_dot,
                             theta_dot (> 0)                                 */
  double h_u;             /* host: step in u (> 0)                           */
} vpm_fd_in;

typedef struct {
  double *a;              /* device [H][7][7]                                */
  double *b;              /* device [H][7]                                   */
  double *x_nom;          /* device [H+1][7] nominal trajectory, or NULL     */
} vpm_fd_out;

VPM_API int vpm_fd_jacobians(vpm_ctx *ctx, const vpm_params *params, const vpm_fd_in *in,
                             vpm_fd_out *out, void *stream);

/* Exact pair-interaction count of one rollout (host arithmetic): per step
 * N_w (2 N_b + 1) surface pairs, N_w' (N_w' - 1) wake pairs and N_w' N_b
 * bound pairs with N_w' = N_w + 2 (both edges shed), merging above
 * n_wake_max (> 0). The pair_count output of vpm_rollout_batch counts the
 * vortices each step actually sheds. */
VPM_API int64_t vpm_pair_count(int32_t n0, int32_t H, int32_t n_bound,
                               int32_t n_wake_max);

#ifdef __cplusplus
}
#endif
#endif /* VPM_H */
