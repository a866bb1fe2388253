// rollout.hip -- fused VPM-glider rollout kernels for gfx950.
//
// A workgroup owns one rollout for all H steps. Per step (Sec. III-A/B of
// the paper):
//
//   prologue (1 thread)  plate kinematics; disturbance termination (Sec. V)
//   pass A   (all waves) sources = the wake at the start of the step;
//                        targets = 2 N_b + 1 surface points (Eq. 12), the
//                        two edge release points and every wake vortex (the
//                        wake part of Eq. 16). FP32 mode sums 64-source tiles
//                        with plain FMAs and folds each tile into a
//                        (sum, error) pair with TwoSum.
//   solve    (wave 0)    Kelvin sum (FP64), RHS, Gamma_S = K^-1 b (Eq. 11)
//                        from a plate inverse built once per geometry,
//                        Bernoulli loads (Eqs. 13-15), elevator and
//                        rigid-body accelerations, shedding.
//   pass B   (all)       each wake vortex adds the new LEV/TEV (regularised)
//                        and bound (singular) terms, completing Eq. 16 in
//                        FIFO order; Euler advection and decay (Eq. 17).
//   epilogue (1 thread)  merge the two oldest above N_w,max; glider Euler.
//
// Two variants differ only in where the wake lives and how pass A walks it:
//  - rollout_lds_kernel (4 waves): the wake is resident in LDS for the whole
//    horizon. Sources are split into 4 contiguous quarters (one per wave);
//    each lane keeps T targets in registers; the quarters are added in FP64
//    in fixed order. A step's last, partly filled chunk is spread over all
//    lanes, each with its targets against one of P equal source parts.
//  - rollout_stream_kernel (NW waves, persistent): the wake lives in a
//    per-workgroup slot of a global workspace; 1024-source tiles are staged
//    cooperatively through LDS and every wave walks all of them for its own
//    targets, in FIFO order; a ragged last round instead gives each group
//    of waves one part of the sources and adds the parts in FP64 in order.
//    It serves wakes too large for LDS (tens of thousands of vortices).
//
// The N^2 work is pure VALU: per regularised pair 7 FP32 ops + 1 v_rsq_f32 on
// sources pre-scaled by 1/Gamma (FP32), 8 + 1 on unscaled sources (FP64, and
// the large FP32 class's ragged tails of fewer than 32 targets),
// no MFMA (the sum is not a dense contraction).
#include <cmath>
#include <type_traits>

#include "vpm_internal.h"
#include "wave_ops.h"

namespace vpm {
namespace {

constexpr int kStreamTile = 1024;  // sources per LDS stage (streaming kernel)
constexpr double kInv2Pi = 0.159154943091895335768883763372514362;
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

struct alignas(16) Src32 {
  float x, z, g, pad;  // position and circulation / (2 pi)
};
struct alignas(32) Src64 {
  double x, z, g, pad;
};
template <typename R> struct SrcOf;
template <> struct SrcOf<float> { using type = Src32; };
template <> struct SrcOf<double> { using type = Src64; };

// Pass-A source of the FP32 kernels, pre-scaled by q = 1/g: with dx' = q dx
// and dz' = q dz, (dx'^2 + dz'^2)^2 + (q rc)^4 = q^4 (r^4 + rc^4), so its
// inverse square root times dz' is g dz / sqrt(r^4 + rc^4), the regularised
// term, for 7 VALU operations and v_rsq_f32 instead of 8 and v_rsq_f32 (the
// multiply by g disappears into the scaling). FP64 sources stay unscaled.
struct alignas(16) Scl32 {
  float px, pz, q, cs;  // q x, q z, q, (q rc)^4
};
template <typename R> struct PassAOf;
template <> struct PassAOf<float> { using type = Scl32; };
template <> struct PassAOf<double> { using type = Src64; };

// Which LDS kernels keep a scaled copy of the wake (16 B more per vortex):
// the FP32 small class. The FP32 large class has no copy: its capacity is
// what LDS holds, and a copy would send rollouts of 3k-5k vortices to the
// streamed class, which runs them slower; each wave scales its sources in
// batches per chunk instead (accumulate_staged). The streamed class scales
// each staged tile.
template <typename R, int NW> constexpr bool lds_scaled() { return sizeof(R) == 4 && NW == 4; }

template <typename R> struct alignas(2 * sizeof(R)) Vec2 { R x, z; };
// A bound vortex as pass B reads it: position and strength / (2 pi).
template <typename R> struct alignas(4 * sizeof(R)) Bound { R x, z, g, pad; };

// Kernel argument block, filled on the host.
struct KArgs {
  int K, H, nb, S, n_wake_max, max_wake0, n_pairs, cap, n_fields;
  int mode, gate, n_inv;  // shedding mode, separation gate, inverse entries staged
  int split_b;            // pass B may split a group's sources over idle waves
  double alpha_crit;
  double dt, chord, shed_frac, r_core, decay, rho, span, grav, mass, inertia;
  double inv_dt, inv_lb, inv_mass, inv_inertia;  // host reciprocals
  double lb;                                      // panel length c / N_b (host)
  double l_body, l_wing, l_elev, s_elev;
  double x_goal[7], q_diag[7];
  const double *g0, *gb0, *wx, *wz, *wg, *u_mean, *u_eps, *kinv_t;
  const double *kinv_te;  // trailing-edge-only inverse (gate on), after kinv_t in LDS
  const double *fb_gain, *fb_xref;  // closed-loop policy [H][7] each, or NULL
  double *gb_final;
  const int64_t *field_off;
  const int32_t *field_of, *pairs;
  double *g_final, *cost, *traj, *gamma_s, *wx_out, *wz_out, *wg_out;
  double *vel_last;
  int32_t *status, *n_final, *n_vel_last;
  int64_t *pair_count;
  const int64_t *wake_off;
  int off_vsurf, off_red, off_vel, off_kinv, off_scl;  // byte offsets into dynamic LDS
  void *ws_src, *ws_vel;  // streaming workspace: one slot of `cap` per block
};

// Per-rollout scalars shared by the workgroup.
template <typename R> struct Shared {
  R g[7], gn[7];
  R le[2], et[2], en[2], xw[2], xwd[2], lev[2], tev[2];
  R ct, st;  // cos and sin of the pitch at the start of the step
  // bound vortices of the step; entries N_b .. (N_b rounded up to 8) - 1
  // are zero, so pass B reads whole blocks of 8 without clamping
  Bound<R> bnd[kMaxBound];
  R shed_g[2];
  double gb_prev[kMaxBound];
  double bvec[kMaxBound + 8];  // b of the solve, zero-padded to a multiple of 8
  int head, n_w, status;
  int claimed;  // rollout claimed from the work queue
  int slot;     // issue-priority slot of this workgroup (see rotate_priority)
  int mode_step, n_shed;  // this step's shedding mode and vortices shed
  double u_fb;            // this step's feedback control term (0 open loop)
  int pa[kMaxPairs], pb[kMaxPairs];
  long long pairs;
};

__device__ inline float rsq(float d) { return __builtin_amdgcn_rsqf(d); }
__device__ inline float rcp(float d) { return __builtin_amdgcn_rcpf(d); }
// FP64: the hardware estimates (v_rsq_f64, v_rcp_f64) refined by two
// Newton-Raphson steps each, which square the relative error twice (from
// below 2^-22 to the last bits of binary64): y <- y + (y/2)(1 - d y^2) for
// 1/sqrt(d), y <- y + y (1 - d y) for 1/d. Arguments here are positive,
// finite and normal (r^4 + r_c^4, r^2 plus the smallest normal). About half
// the instructions of the correctly rounded 1.0 / sqrt(d) and 1.0 / d; the
// results differ from those by a few ulp.
__device__ inline double rsq(double d) {
  double y = __builtin_amdgcn_rsq(d);
  double e = fma(-d * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-d * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ inline double rcp(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = fma(y, fma(-d, y, 1.0), y);
  return fma(y, fma(-d, y, 1.0), y);
}
__device__ inline float tiny(float) { return 1.17549435e-38f; }
__device__ inline double tiny(double) { return 2.2250738585072014e-308; }

// Regularised kernel (Eq. 5) times Gamma, with g = Gamma/(2 pi) folded in:
// g (-dz, dx) / sqrt(rc^4 + r^4).
template <typename R>
__device__ inline void reg_term(R dx, R dz, R g, R rc4, R &vx, R &vz) {
  R r2 = dx * dx + dz * dz;
  R k = g * rsq(r2 * r2 + rc4);
  vx -= dz * k;
  vz += dx * k;
}

// Singular kernel (Eq. 4) times Gamma, g = Gamma/(2 pi): g (-dz, dx) / r^2.
// The smallest normal number is added inside the r^2 FMA chain, so a
// coincident point has a finite k and contributes exactly 0, while any r^2
// above ~1e-30 (FP32) rounds exactly as without it.
template <typename R>
__device__ inline void sing_term(R dx, R dz, R g, R &vx, R &vz) {
  R r2 = fma(dz, dz, fma(dx, dx, tiny(dx)));
  R k = g * rcp(r2);
  vx -= dz * k;
  vz += dx * k;
}

// Scaled form of a source at (x, z) with strength g = Gamma/(2 pi). A source
// with |g| < 1e-30 gets q = 0 and cs = +inf and adds exactly 0 (an exactly
// zero strength, e.g. a terminated disturbance pair, is the case that
// matters; with r_core >= 1e-6 m such a source moves a target by less than
// 1e-24 m/s). Where q^4 (r^4 + rc^4) exceeds the FP32 range the rsq of +inf
// is 0: the term g r / sqrt(r^4 + rc^4) is then below M^(-1/4) = 2.3e-10 m/s
// (M the largest float), since sqrt(r^4 + rc^4) > sqrt(M) g^2 and r^2 is at
// most that root. The floor at the smallest normal number keeps the inverse
// square root finite for coincident points when (q rc)^4 underflows. q = 1/g
// to 1 ulp (v_rcp_f32): the term's strength is 1/q, within 1.2e-7 of g, as
// close as storing g in binary32.
__device__ inline Scl32 scale_source(float x, float z, float g, float rc) {
  if (fabsf(g) < 1e-30f) return Scl32{0.0f, 0.0f, 0.0f, INFINITY};
  const float q = fabsf(g) <= 3.40282347e38f ? __builtin_amdgcn_rcpf(g) : __builtin_nanf("");
  const float rq = rc * q, rq2 = rq * rq;
  return Scl32{x * q, z * q, q, fmaxf(rq2 * rq2, 1.17549435e-38f)};
}

// Regularised term of a scaled source at target (tx, tz): 2 FMA for dx', dz',
// mul + FMA for r'^2, FMA for r'^4 + cs, v_rsq_f32, 2 FMA.
__device__ inline void reg_term_scaled(float tx, float tz, const Scl32 &v, float &vx,
                                       float &vz) {
  const float dx = fmaf(tx, v.q, -v.px), dz = fmaf(tz, v.q, -v.pz);
  const float r2 = fmaf(dz, dz, dx * dx);
  const float k = rsq(fmaf(r2, r2, v.cs));
  vx = fmaf(-dz, k, vx);
  vz = fmaf(dx, k, vz);
}

__device__ inline void pair_term(float tx, float tz, const Scl32 &v, float, float &vx,
                                 float &vz) {
  reg_term_scaled(tx, tz, v, vx, vz);
}
__device__ inline void pair_term(float tx, float tz, const Src32 &v, float rc4, float &vx,
                                 float &vz) {
  reg_term(tx - v.x, tz - v.z, v.g, rc4, vx, vz);
}
__device__ inline void pair_term(double tx, double tz, const Src64 &v, double rc4, double &vx,
                                 double &vz) {
  reg_term(tx - v.x, tz - v.z, v.g, rc4, vx, vz);
}

// A wake vortex is a pass-A target and a source. K'(0) = 0 makes its term on
// itself vanish, but in scaled form dx' = fma(x, q, -RN(q x)) is the rounding
// error of q x, not 0: the self term is of order g |x| 2^-24 / rc^2. It is
// recomputed with the same operations and taken out of the vortex's velocity
// (the streamed class at the end of pass A, the large LDS class in the
// cross-wave combine, the small LDS class in pass B).
__device__ inline void remove_self(float x, float z, const Scl32 &v, double &vx, double &vz) {
  float ax = 0.0f, az = 0.0f;
  reg_term_scaled(x, z, v, ax, az);
  vx -= double(ax);
  vz -= double(az);
}

// Pass-B upkeep of the scaled copy for wake entry p (LDS small class; a
// no-op without a copy), prepared before the pass-B sum so that its loads
// and v_rcp_f32 overlap it: the entry's pass-A self term, when it was a
// pass-A source this step (vortices shed this step were not), and q and cs
// of its decayed strength g_new for the rewritten entry.
struct Upkeep {
  double sx, sz;  // the self term, negated: added to the velocity
  float q, cs;
};
template <typename S>
__device__ inline Upkeep upkeep(const Scl32 *scl, int p, const S &s, bool was_source,
                                float g_new, float rc) {
  Upkeep u{0.0, 0.0, 0.0f, 0.0f};
  if (!scl) return u;
  if (was_source) remove_self(float(s.x), float(s.z), scl[p], u.sx, u.sz);
  const Scl32 n = scale_source(0.0f, 0.0f, g_new, rc);
  u.q = n.q;
  u.cs = n.cs;
  return u;
}

// Pass-A source entry of an FP32 or FP64 wake entry.
__device__ inline Scl32 pass_a_source(const Src32 &s, float rc) {
  return scale_source(s.x, s.z, s.g, rc);
}
__device__ inline Src64 pass_a_source(const Src64 &s, double) { return s; }

// Keep entry p of the scaled copy (FP32 small class; null otherwise) in step
// with the wake entry s just written.
template <typename S>
__device__ inline void rescale(Scl32 *scl, int p, const S &s, float rc) {
  if (scl) scl[p] = scale_source(float(s.x), float(s.z), float(s.g), rc);
}

// Knuth's TwoSum: s + c absorbs t with the rounding error of s + t kept in c.
__device__ inline void two_sum(float &s, float &c, float t) {
  float u = s + t;
  float bp = u - s;
  float err = (s - (u - bp)) + (t - bp);
  s = u;
  c += err;
}

template <typename R, int T>
__device__ inline void fold_tile(R (&sx)[T], R (&sz)[T], R (&cx)[T], R (&cz)[T],
                                 const R (&ax)[T], const R (&az)[T]) {
  if constexpr (sizeof(R) == 4) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      two_sum(sx[j], cx[j], ax[j]);
      two_sum(sz[j], cz[j], az[j]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      sx[j] += ax[j];
      sz[j] += az[j];
    }
  }
}

// Sources [s_lo, s_hi) of `src` onto the T targets of this lane, folded
// every TILE sources. `fresh` (uniform): the sums and their compensations are
// still zero on entry, so the first tile is taken as it is — the fold of a
// tile into zero is exact (TwoSum(0, a) = (a, 0)) and only costs issue slots.
template <typename R, int T, int TILE, typename S>
__device__ inline void accumulate(const S *__restrict__ src,
                                  int s_lo, int s_hi, const R (&tx)[T],
                                  const R (&tz)[T], R rc4, R (&sx)[T], R (&sz)[T],
                                  R (&cx)[T], R (&cz)[T], bool fresh) {
  for (int s0 = s_lo; s0 < s_hi; s0 += TILE) {
    const int s1 = min(s0 + TILE, s_hi);
    R ax[T], az[T];
#pragma unroll
    for (int j = 0; j < T; ++j) ax[j] = az[j] = R(0);
#pragma unroll 4
    for (int q = s0; q < s1; ++q) {
      const S v = src[q];
#pragma unroll
      for (int j = 0; j < T; ++j) pair_term(tx[j], tz[j], v, rc4, ax[j], az[j]);
    }
    if (fresh && s0 == s_lo) {
#pragma unroll
      for (int j = 0; j < T; ++j) {
        sx[j] = ax[j];
        sz[j] = az[j];
      }
    } else {
      fold_tile<R, T>(sx, sz, cx, cz, ax, az);
    }
  }
}

// Sources [s_lo, s_hi), at most one tile of them, onto the T targets of this
// lane: a single tile is never folded, so its plain sums are the totals and
// the compensation terms (all zero) are neither kept nor added.
template <typename R, int T, typename S>
__device__ inline void accumulate_one_tile(const S *__restrict__ src, int s_lo, int s_hi,
                                           const R (&tx)[T], const R (&tz)[T], R rc4,
                                           R (&sx)[T], R (&sz)[T]) {
#pragma unroll
  for (int j = 0; j < T; ++j) sx[j] = sz[j] = R(0);
#pragma unroll 4
  for (int q = s_lo; q < s_hi; ++q) {
    const S v = src[q];
#pragma unroll
    for (int j = 0; j < T; ++j) pair_term(tx[j], tz[j], v, rc4, sx[j], sz[j]);
  }
}

// The thread index, opaque to the compiler at this point: addresses that
// setup and finish derive from it are then computed per rollout instead of
// being hoisted out of the persistent rollout loop, where these per-lane
// 64-bit values would stay live across every step and spill.
__device__ inline int opaque_tid(int tid) {
  asm volatile("" : "+v"(tid));
  return tid;
}

// A 64-bit zero made where it is used: a shared zero register pair
// hoisted out of the rollout loop would be live across every step and spill.
__device__ inline long long opaque_zero64() {
  long long z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// +inf as a double made where it is used, for the same reason.
__device__ inline double opaque_inf64() {
  double v = INFINITY;
  asm volatile("" : "+v"(v));
  return v;
}

// The kernel's arguments (the first kernel argument, at offset 0 of the
// kernarg segment), re-read where this is called: through an address the
// compiler cannot see through, argument loads are not hoisted across the
// rollout and step loops, where the many argument registers would stay live
// and spill to VGPR lanes (every read back costs a VALU issue slot).
__device__ inline const KArgs &fresh_args(const KArgs &) {
  using CK = __attribute__((address_space(4))) const KArgs;
  CK *p = (CK *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const KArgs *)p;
}

// All lanes of a wave: its LDS writes are visible to its own later reads.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP32 large class: the wave's sources [s_lo, s_hi) of the unscaled wake,
// scaled 32 T at a time into `stage` (the wave's own slot of the chunk's
// partial-sum buffer, unused until the chunk's sums are written), so the
// pair costs 8 instructions without a scaled copy of the wake in LDS.
// Conversion: ~12 instructions per source per chunk, under 1 % of the
// 8 T per source it buys back for T = 4.
template <int T, int TILE>
__device__ inline void accumulate_staged(const Src32 *__restrict__ src, Scl32 *stage, int s_lo,
                                         int s_hi, float rc, int lane, const float (&tx)[T],
                                         const float (&tz)[T], float (&sx)[T], float (&sz)[T],
                                         float (&cx)[T], float (&cz)[T]) {
  constexpr int kStage = 32 * T;  // 64 T float2 of partial sums = 32 T Scl32
  for (int b0 = s_lo; b0 < s_hi; b0 += kStage) {
    const int cnt = min(kStage, s_hi - b0);
    for (int q = lane; q < cnt; q += 64) stage[q] = pass_a_source(src[b0 + q], rc);
    wave_lds_sync();
    accumulate<float, T, TILE>(stage, 0, cnt, tx, tz, 0.0f, sx, sz, cx, cz, b0 == s_lo);
    wave_lds_sync();  // every lane done with the batch before it is overwritten
  }
}

// Chord coordinate (from the leading edge) of surface point t: collocation
// points, bound vortices, LEV and TEV release points.
template <typename R>
__device__ inline R surface_s(int t, int nb, R lb, R ds, R c) {
  if (t <= nb) return R(t) * lb;                                  // collocation, LE to TE
  if (t < 2 * nb + 1) return (R(t - nb - 1) + R(0.5)) * lb;       // bound
  if (t == 2 * nb + 1) return -ds;                                // LEV release point
  return c + ds;                                                  // TEV release point
}

template <typename R>
__device__ inline void surface_point(const Shared<R> &sh, int t, int nb, R lb,
                                     R ds, R c, R &px, R &pz) {
  const R s = surface_s(t, nb, lb, ds, c);
  px = sh.le[0] + s * sh.et[0];
  pz = sh.le[1] + s * sh.et[1];
}

// Position of pass-A target t of the LDS kernels: the step's surface points
// sit in the n_surf entries just below the wake (src[head - n_surf ..]), so
// every target is one entry of src.
template <typename R>
__device__ inline void lds_target(const typename SrcOf<R>::type *src, int t, int NT,
                                  int head, int n_surf, R &px, R &pz) {
  px = pz = R(0);
  if (t < NT) {
    const auto v = src[head - n_surf + t];
    px = v.x;
    pz = v.z;
  }
}

// Position of pass-A target t: surface points first, then the wake.
template <typename R>
__device__ inline void target_pos(const KArgs &a, const Shared<R> &sh,
                                  const typename SrcOf<R>::type *src, int t,
                                  int NT, int head, R &px, R &pz) {
  const int n_surf = 2 * a.nb + 3;
  px = pz = R(0);
  if (t >= NT) return;
  if (t < n_surf) {
    surface_point(sh, t, a.nb, R(a.lb), R(a.shed_frac * a.chord),
                  R(a.chord), px, pz);
  } else {
    const auto v = src[head + t - n_surf];
    px = v.x;
    pz = v.z;
  }
}

// Sine and cosine with one argument reduction.
__device__ inline void sin_cos(float x, float &s, float &c) { sincosf(x, &s, &c); }
__device__ inline void sin_cos(double x, double &s, double &c) { sincos(x, &s, &c); }

// Segment a-b against the chord rectangle inflated by 2 % of chord opposite
// the normal (Sec. V), by Liang-Barsky clipping in plate coordinates.
__device__ inline bool clip_slab(double p0, double d, double lo, double hi,
                                 double &u0, double &u1) {
  if (d == 0.0) return p0 >= lo && p0 <= hi;
  const double inv = 1.0 / d;
  double ta = (lo - p0) * inv, tb = (hi - p0) * inv;
  if (ta > tb) {
    double t = ta;
    ta = tb;
    tb = t;
  }
  u0 = fmax(u0, ta);
  u1 = fmin(u1, tb);
  return u0 <= u1;
}

template <typename R>
__device__ bool hits_plate(const Shared<R> &sh, double c, double ax, double az,
                           double bx, double bz) {
  const double lx = sh.le[0], lz = sh.le[1];
  const double tx = sh.et[0], tz = sh.et[1], nx = sh.en[0], nz = sh.en[1];
  double sa = (ax - lx) * tx + (az - lz) * tz, ha = (ax - lx) * nx + (az - lz) * nz;
  double sb = (bx - lx) * tx + (bz - lz) * tz, hb = (bx - lx) * nx + (bz - lz) * nz;
  // both ends on the far side of one slab face: no crossing (the common
  // case, decided without the clipping divisions)
  if ((sa < 0.0 && sb < 0.0) || (sa > c && sb > c) || (ha > 0.0 && hb > 0.0) ||
      (ha < -0.02 * c && hb < -0.02 * c))
    return false;
  double u0 = 0.0, u1 = 1.0;
  if (!clip_slab(sa, sb - sa, 0.0, c, u0, u1)) return false;
  return clip_slab(ha, hb - ha, -0.02 * c, 0.0, u0, u1);
}

template <typename R>
__device__ void geometry(const KArgs &a, Shared<R> &sh) {
  const R th = sh.g[2], thd = sh.g[6], lw = R(a.l_wing);
  R ct, st;
  sin_cos(th, st, ct);
  const R hc = R(0.5 * a.chord), ds = R(a.shed_frac * a.chord);
  sh.ct = ct;
  sh.st = st;
  sh.xw[0] = sh.g[0] - lw * ct;
  sh.xw[1] = sh.g[1] - lw * st;
  sh.xwd[0] = sh.g[4] + lw * thd * st;
  sh.xwd[1] = sh.g[5] - lw * thd * ct;
  sh.et[0] = -ct;
  sh.et[1] = -st;
  sh.en[0] = -st;
  sh.en[1] = ct;
  sh.le[0] = sh.xw[0] + hc * ct;
  sh.le[1] = sh.xw[1] + hc * st;
  sh.lev[0] = sh.le[0] - ds * sh.et[0];
  sh.lev[1] = sh.le[1] - ds * sh.et[1];
  const R s_tev = R(a.chord) + ds;
  sh.tev[0] = sh.le[0] + s_tev * sh.et[0];
  sh.tev[1] = sh.le[1] + s_tev * sh.et[1];
}

// Thread 0 at the start of a step: kinematics and termination.
// Wing angle of attack of the separation gate (Sec. III-A): pitch minus the
// direction of the wing point's velocity, in FP64. Out of line: inlined, its
// sin/cos/atan2 raise the register pressure of the whole kernel, and the FP32
// kernels spill.
__device__ __noinline__ double wing_aoa(double th, double xd, double zd, double thd, double lw) {
  const double xdw = xd + lw * thd * sin(th), zdw = zd - lw * thd * cos(th);
  return th - atan2(zdw, xdw);
}

// EXT: the step's control or shedding mode depends on the state (feedback
// policy or separation gate on). Only those kernel instances contain that
// code: it raises the register pressure of the whole kernel (and the gate's
// out-of-line call alone changes its register allocation), which costs the
// plain open-loop instances a few per cent.
template <typename R, bool EXT>
__device__ __forceinline__ void prologue(const KArgs &a, Shared<R> &sh,
                         typename SrcOf<R>::type *src, Scl32 *scl, int n) {
  geometry(a, sh);
  int mode = a.mode;
  if constexpr (EXT) {
    // Sec. IV-B policy: u_n = u^d_n - H_n (x_n - x^d_n) from the state at
    // the start of the step, in FP64
    double fb = 0.0;
    if (a.fb_gain) {
      const double *hn = a.fb_gain + (size_t)n * 7, *xn = a.fb_xref + (size_t)n * 7;
      for (int j = 0; j < 7; ++j) fb += hn[j] * (double(sh.g[j]) - xn[j]);
    }
    sh.u_fb = -fb;
    // Sec. III-A separation gate: the leading edge sheds only while the
    // wing's angle of attack exceeds the critical angle; decided in FP64 from
    // the stored state
    if (a.gate)
      mode = wing_aoa(sh.g[2], sh.g[4], sh.g[5], sh.g[6], a.l_wing) > a.alpha_crit
                 ? VPM_SHED_BOTH
                 : VPM_SHED_TE;
  }
  sh.mode_step = mode;
  sh.n_shed = mode == VPM_SHED_BOTH ? 2 : mode == VPM_SHED_TE ? 1 : 0;
  for (int q = 0; q < kMaxPairs; ++q) {
    const int pa = sh.pa[q], pb = sh.pb[q];
    if (pa < 0) continue;
    if (hits_plate(sh, a.chord, src[pa].x, src[pa].z, src[pb].x, src[pb].z)) {
      src[pa].g = R(0);
      src[pb].g = R(0);
      rescale(scl, pa, src[pa], float(a.r_core));
      rescale(scl, pb, src[pb], float(a.r_core));
      sh.pa[q] = sh.pb[q] = -1;
    }
  }
}

// Load rollout k's initial state, the wake from entry `base` of src (and
// scl) on. Returns false (after writing the failure outputs) when its field
// is invalid or larger than max_wake0; uniform over the workgroup.
template <typename R>
__device__ bool setup(const KArgs &a, Shared<R> &sh, typename SrcOf<R>::type *src,
                      Scl32 *scl, int k, int tid, int nthr, int base) {
  using Src = typename SrcOf<R>::type;
  const int nb = a.nb;
  const int fo = a.field_of ? a.field_of[k] : k;
  const bool bad_field = fo < 0 || fo >= a.n_fields;
  const int64_t f0 = bad_field ? 0 : a.field_off[fo];
  const int n0 = bad_field ? -1 : static_cast<int>(a.field_off[fo + 1] - f0);
  if (n0 < 0 || n0 > a.max_wake0) {
    if (tid < 7) a.g_final[7 * k + tid] = a.g0[7 * k + tid];
    if (tid == 0) {
      a.cost[k] = opaque_inf64();
      a.status[k] = n0 < 0 ? VPM_ROLLOUT_BADFIELD : VPM_ROLLOUT_CAPACITY;
      if (a.pair_count) a.pair_count[k] = opaque_zero64();
      if (a.n_final) a.n_final[k] = 0;
      if (a.n_vel_last) a.n_vel_last[k] = 0;
      if (a.gb_final)
        for (int j = 0; j < a.nb; ++j) a.gb_final[(size_t)k * a.nb + j] = a.gb0[(size_t)k * a.nb + j];
    }
    return false;
  }
  for (int q = tid; q < n0; q += nthr) {
    src[base + q] = Src{R(a.wx[f0 + q]), R(a.wz[f0 + q]), R(a.wg[f0 + q] * kInv2Pi), R(0)};
    rescale(scl, base + q, src[base + q], float(a.r_core));
  }
  if (tid < 7) {
    sh.g[tid] = R(a.g0[7 * k + tid]);
    if (a.traj) a.traj[(size_t)k * (a.H + 1) * 7 + tid] = a.g0[7 * k + tid];
  }
  if (tid < nb) sh.gb_prev[tid] = a.gb0[(size_t)k * nb + tid];
  if (tid == 0) {
    sh.head = base;
    sh.n_w = n0;
    sh.status = 0;
    sh.pairs = opaque_zero64();
    for (int q = 0; q < kMaxPairs; ++q) {
      int pa = -1, pb = -1;
      if (q < a.n_pairs && a.pairs) {
        pa = a.pairs[(size_t)k * 2 * a.n_pairs + 2 * q];
        pb = a.pairs[(size_t)k * 2 * a.n_pairs + 2 * q + 1];
        if (pa < 0 || pb < 0 || pa >= n0 || pb >= n0 || pa == pb) {
          pa = pb = -1;
        } else {
          pa += base;
          pb += base;
        }
      }
      sh.pa[q] = pa;
      sh.pb[q] = pb;
    }
  }
  return true;
}

// Wave 0: Kelvin sum, surface solve, loads, dynamics, shedding.
template <typename R>
__device__ __forceinline__ void solve_section(
    const KArgs &a, Shared<R> &sh, typename SrcOf<R>::type *src, Vec2<R> *vel,
    const double2 *vsurf, const double *kinv, int k, int n, int head, int n_w,
    int lane, double u_n) {
  using Src = typename SrcOf<R>::type;
  const int nb = a.nb, nc = nb + 1;
  // this step's system (Sec. III-A): BOTH has N_b + 2 unknowns, TE-only
  // drops the LEV column and the LE row, NONE both edges' (the Kelvin row
  // is always last)
  const int mode = __builtin_amdgcn_readfirstlane(sh.mode_step);
  const int S = system_size(nb, mode), c0 = first_row(mode);
  if (a.gate && mode == VPM_SHED_TE) kinv += a.S * a.S;
  const double dt = a.dt, lb = a.lb;
  const R dtr = R(dt);
  // Kelvin sum over the wake, two partial sums in flight
  double sg = 0.0, sg1 = 0.0;
  int qk = lane;
  for (; qk + 64 < n_w; qk += 128) {
    sg += double(src[head + qk].g);
    sg1 += double(src[head + qk + 64].g);
  }
  if (qk < n_w) sg += double(src[head + qk].g);
  const double sum_gw = kTwoPi * wave_sum(sg + sg1);
  const double lex = sh.le[0], lez = sh.le[1], etx = sh.et[0], etz = sh.et[1];
  const double enx = sh.en[0], enz = sh.en[1];
  const double xwx = sh.xw[0], xwz = sh.xw[1], thd = sh.g[6];
  const double xwdx = sh.xwd[0], xwdz = sh.xwd[1];
  // b_i = -v~(r_ci).n with v~ = v_W - xw_dot - thd J(r - x_w) (Eq. 12)
  auto rhs = [&](int r) -> double {
    if (r >= S) return 0.0;
    if (r == S - 1) return -sum_gw;
    const int c = r + c0;  // collocation point of row r
    const double px = lex + c * lb * etx, pz = lez + c * lb * etz;
    const double2 vw = vsurf[c];
    const double vx = vw.x - xwdx + thd * (pz - xwz);
    const double vz = vw.y - xwdz - thd * (px - xwx);
    return -(vx * enx + vz * enz);
  };
  // b goes through LDS (broadcast reads cost no VALU issue slots), zero
  // up to the next multiple of 8; the inverse and b are read 8 entries at a
  // time, into four partial sums so that the FMA chain is a quarter as long
  const int s8 = (S + 7) & ~7;
  if (lane < s8) sh.bvec[lane] = rhs(lane);
  if (lane + 64 < s8) sh.bvec[lane + 64] = rhs(lane + 64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // Gamma_S = K^-1 b (Eq. 11): lane i owns rows i and i + 64
  double p0[4] = {0.0, 0.0, 0.0, 0.0}, gam1 = 0.0;
  const int i0 = lane < S ? lane : 0, i1 = lane + 64 < S ? lane + 64 : 0;
  for (int j0 = 0; j0 < S; j0 += 8) {
    double kv[8], bj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = j0 + q < S ? j0 + q : S - 1;
      kv[q] = kinv[j * S + i0];  // rows past S repeat row S - 1 (times b = 0)
      bj[q] = sh.bvec[j0 + q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) p0[q & 3] += kv[q] * bj[q];
    if (S > 64) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = j0 + q < S ? j0 + q : S - 1;
        gam1 += kinv[j * S + i1] * bj[q];
      }
    }
  }
  const double gam0 = (p0[0] + p0[1]) + (p0[2] + p0[3]);
  auto row = [&](int r) -> double { return r < 64 ? bcast(gam0, r) : bcast(gam1, r - 64); };
  const double r_nb = row(nb), r_nb1 = row(nb + 1);  // both read unconditionally
  const double glev = mode == VPM_SHED_BOTH ? r_nb : 0.0;
  const double gtev = mode == VPM_SHED_BOTH ? r_nb1 : mode == VPM_SHED_TE ? r_nb : 0.0;
  if (a.gamma_s) {  // a.S entries per step; a smaller system pads with zeros
    double *gs = a.gamma_s + ((size_t)k * a.H + n) * a.S;
    if (lane < a.S) gs[lane] = lane < S ? gam0 : 0.0;
    if (lane + 64 < a.S) gs[lane + 64] = lane + 64 < S ? gam1 : 0.0;
  }
  // Eqs. 13-15. With P_j the prefix sums of Gamma_b, the force needs
  // sum_j (P_j - P'_j) = sum_k (N_b - k) dGamma_k and the moment
  // sum_j arm_j (P_j - P'_j) = sum_k A_k dGamma_k, A_k = sum_{j>=k} arm_j
  // = -(N_b - k) k l_b / 2 (arm_j = c/2 - (j + 1/2) l_b): two plain sums.
  const bool on = lane < nb;
  const double gbj = on ? gam0 : 0.0;
  const double dgb = on ? gam0 - sh.gb_prev[lane] : 0.0;
  const double sj = (lane + 0.5) * lb;
  const double bx = lex + sj * etx, bz = lez + sj * etz;
  const double2 vb = on ? vsurf[nc + lane] : make_double2(0.0, 0.0);
  const double vtx = vb.x - xwdx + thd * (bz - xwz);
  const double vtz = vb.y - xwdz - thd * (bx - xwx);
  const double qt = vtx * etx + vtz * etz;
  const double arm = 0.5 * a.chord - sj;
  const double inv_dt = a.inv_dt;
  const double local = gbj * a.inv_lb * qt + glev * inv_dt;
  const double tf = on ? local + (nb - lane) * dgb * inv_dt : 0.0;
  const double tm = on ? arm * local - 0.5 * (nb - lane) * lane * lb * dgb * inv_dt : 0.0;
  const double sdp = a.rho * wave_sum(tf);
  const double sarm = a.rho * wave_sum(tm);
  if (on) {
    sh.gb_prev[lane] = gbj;
    sh.bnd[lane] = Bound<R>{R(bx), R(bz), R(gbj * kInv2Pi), R(0)};
  } else if (lane < ((nb + 7) & ~7)) {
    sh.bnd[lane] = Bound<R>{R(0), R(0), R(0), R(0)};
  }
  if (lane == 0) {
    const double fwx = lb * a.span * sdp * enx, fwz = lb * a.span * sdp * enz;
    const double mw = lb * a.span * sarm;
    // Sec. III-B: elevator force and rigid-body accelerations
    const R x = sh.g[0], z = sh.g[1], th = sh.g[2], ph = sh.g[3];
    const R xd = sh.g[4], zd = sh.g[5], thr = sh.g[6];
    const R u = R(u_n);
    const R l = R(a.l_body), le = R(a.l_elev);
    const R ct = sh.ct, st = sh.st;
    R ctp, stp;
    sin_cos(th + ph, stp, ctp);
    const R xe = x - l * ct - le * ctp, ze = z - l * st - le * stp;
    const R xed = xd + l * thr * st + le * (thr + u) * stp;
    const R zed = zd - l * thr * ct - le * (thr + u) * ctp;
    // f_e = rho S_e V^2 sin(alpha), alpha = th + ph - atan2(zed, xed):
    // V^2 sin(alpha) = V (sin(th + ph) xed - cos(th + ph) zed), no atan2/sin
    const R vel_e = sqrt(xed * xed + zed * zed);
    const R fe = R(a.rho * a.s_elev) * vel_e * (stp * xed - ctp * zed);
    const R fex = -fe * stp, fez = fe * ctp;
    const R fx = R(fwx) + fex, fz = R(fwz) + fez;
    const R ax_ = fx * R(a.inv_mass);
    const R az_ = fz * R(a.inv_mass) - R(a.grav);
    const R mom = (sh.xw[0] - x) * R(fwz) - (sh.xw[1] - z) * R(fwx) +
                  (xe - x) * fez - (ze - z) * fex + R(mw);
    const R ath = mom * R(a.inv_inertia);
    sh.gn[0] = x + dtr * xd;
    sh.gn[1] = z + dtr * zd;
    sh.gn[2] = th + dtr * thr;
    sh.gn[3] = ph + dtr * u;
    sh.gn[4] = xd + dtr * ax_;
    sh.gn[5] = zd + dtr * az_;
    sh.gn[6] = thr + dtr * ath;
    // shedding (Sec. III-A): the LEV, if this step sheds one, then the TEV
    // join the wake tail; an edge that does not shed contributes zero
    // strength to pass B and nothing to the wake
    int p = head + n_w;
    sh.shed_g[0] = R(glev * kInv2Pi);
    sh.shed_g[1] = R(gtev * kInv2Pi);
    const double2 vl = vsurf[2 * nb + 1], vt = vsurf[2 * nb + 2];
    if (mode == VPM_SHED_BOTH) {
      src[p] = Src{sh.lev[0], sh.lev[1], sh.shed_g[0], R(0)};
      vel[p] = Vec2<R>{R(vl.x), R(vl.y)};
      ++p;
    }
    if (mode != VPM_SHED_NONE) {
      src[p] = Src{sh.tev[0], sh.tev[1], sh.shed_g[1], R(0)};
      vel[p] = Vec2<R>{R(vt.x), R(vt.y)};
    }
  }
}

// Pass-B sources [q0, q1) of the list LEV, TEV, bound 0 .. N_b - 1 (FIFO
// order) at (x, z), added to (ex, ez). Bound positions and strengths are read
// from LDS 8 at a time (entries past the range repeat the last position with
// zero strength, which adds exactly nothing).
template <typename R>
__device__ inline void pass_b_sum(const KArgs &a, const Shared<R> &sh, R x, R z, R rc4,
                                  int q0, int q1, R &ex, R &ez) {
  if (q0 <= 0 && q1 > 0) reg_term(x - sh.lev[0], z - sh.lev[1], sh.shed_g[0], rc4, ex, ez);
  if (q0 <= 1 && q1 > 1) reg_term(x - sh.tev[0], z - sh.tev[1], sh.shed_g[1], rc4, ex, ez);
  const int jlo = q0 > 2 ? q0 - 2 : 0, jhi = q1 - 2;
  if (jlo == 0 && jhi == a.nb) {
    // all bound vortices: whole blocks of 8 (zero-strength padding adds
    // exactly nothing), constant LDS offsets, no per-entry selects
    for (int j0 = 0; j0 < jhi; j0 += 8) {
      Bound<R> b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = sh.bnd[j0 + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) sing_term(x - b[q].x, z - b[q].z, b[q].g, ex, ez);
    }
    return;
  }
  for (int j0 = jlo; j0 < jhi; j0 += 8) {
    R bx[8], bz[8], bg[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = j0 + q < jhi ? j0 + q : jhi - 1;
      bx[q] = sh.bnd[j].x;
      bz[q] = sh.bnd[j].z;
      bg[q] = j0 + q < jhi ? sh.bnd[j].g : R(0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) sing_term(x - bx[q], z - bz[q], bg[q], ex, ez);
  }
}

// Wake vortex t of the step: total velocity (pass A + edge and bound terms),
// optional output, Euler advection and decay.
// With a scaled copy, `up` (from upkeep) removes the pass-A self term (sx, sz
// hold its negation) and rewrites the copy's entry as scale_source would.
template <typename R>
__device__ inline void pass_b_finish(const KArgs &a, typename SrcOf<R>::type *src,
                                     Scl32 *scl, const Vec2<R> *vel, int k, bool last,
                                     int head, int t, double ex, double ez, R one_decay,
                                     const Upkeep &up) {
  const int p = head + t;
  auto s = src[p];
  const Vec2<R> v0 = vel[p];
  double vx = double(v0.x) + ex, vz = double(v0.z) + ez;
  if constexpr (sizeof(R) == 4) {
    vx += up.sx;
    vz += up.sz;
  }
  if (last && a.vel_last) {
    double *o = a.vel_last + 2 * (a.wake_off[k] + t);
    o[0] = vx;
    o[1] = vz;
  }
  const R dtr = R(a.dt);
  s.x = s.x + dtr * R(vx);
  s.z = s.z + dtr * R(vz);
  s.g = s.g * one_decay;
  src[p] = s;
  if constexpr (sizeof(R) == 4)
    if (scl) scl[p] = Scl32{s.x * up.q, s.z * up.q, up.q, up.cs};
}

// All waves: the m wake vortices in groups of 64 (group i to wave i mod NW),
// each lane one vortex against every pass-B source. A last group of r < 32
// vortices goes to one wave whose lanes split the sources into 64 / r parts,
// added in FP64 in part order through `scratch` (64 double2 per wave).
template <typename R>
__device__ __forceinline__ void pass_b(const KArgs &a, const Shared<R> &sh,
                                       typename SrcOf<R>::type *src, Scl32 *scl,
                                       const Vec2<R> *vel, int k, bool last,
                                       int head, int m, int n_src, int tid, int nthr,
                                       double2 *scratch) {
  const R rc = R(a.r_core), rc4 = rc * rc * rc * rc;
  const float rcf = float(a.r_core);
  const R one_decay = R(1.0 - a.decay * a.dt);
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = nthr >> 6, ns = a.nb + 2;
  const int r = m & 63, tail = r < 32 ? r : 0;
  const int n_groups = (m >> 6) + (r >= 32 ? 1 : 0);
  // fewer groups than waves and no tail, in a launch of at most one rollout
  // per CU (latency-bound: the idle waves are not covered by other
  // workgroups): each group's sources are split over nw / n_groups waves,
  // partial sums added in FP64 in part order by the group's first wave
  const int parts =
      a.split_b && tail == 0 && n_groups > 0 && n_groups < nw ? nw / n_groups : 1;
  if (parts > 1) {
    const int gi = wave / parts, part = wave % parts, t = gi * 64 + lane;
    R ex = R(0), ez = R(0);
    Upkeep up{};
    if (gi < n_groups && t < m) {
      const auto s = src[head + t];
      if (part == 0) up = upkeep(scl, head + t, s, t < n_src, s.g * one_decay, rcf);
      pass_b_sum(a, sh, s.x, s.z, rc4, (ns * part) / parts, (ns * (part + 1)) / parts, ex, ez);
    }
    scratch[wave * 64 + lane] = make_double2(double(ex), double(ez));
    __syncthreads();
    if (gi < n_groups && part == 0 && t < m) {
      double sx = 0.0, sz = 0.0;
      for (int q = 0; q < parts; ++q) {
        const double2 d = scratch[(wave + q) * 64 + lane];
        sx += d.x;
        sz += d.y;
      }
      pass_b_finish(a, src, scl, vel, k, last, head, t, sx, sz, one_decay, up);
    }
    return;
  }
  for (int gi = wave; gi < n_groups; gi += nw) {
    const int t = gi * 64 + lane;
    if (t < m) {
      const auto s = src[head + t];
      const Upkeep up = upkeep(scl, head + t, s, t < n_src, s.g * one_decay, rcf);
      R ex = R(0), ez = R(0);
      pass_b_sum(a, sh, s.x, s.z, rc4, 0, ns, ex, ez);
      pass_b_finish(a, src, scl, vel, k, last, head, t, double(ex), double(ez), one_decay, up);
    }
  }
  if (tail > 0 && wave == n_groups % nw) {
    const int t0 = n_groups * 64, g = 64 / tail, tt = lane % tail, part = lane / tail;
    R ex = R(0), ez = R(0);
    Upkeep up{};
    if (part < g) {
      const auto s = src[head + t0 + tt];
      if (part == 0) up = upkeep(scl, head + t0 + tt, s, t0 + tt < n_src, s.g * one_decay, rcf);
      pass_b_sum(a, sh, s.x, s.z, rc4, (ns * part) / g, (ns * (part + 1)) / g, ex, ez);
    }
    double2 *sc = scratch + wave * 64;
    sc[lane] = make_double2(double(ex), double(ez));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < tail) {
      double sx = 0.0, sz = 0.0;
      for (int q = 0; q < g; ++q) {
        const double2 d = sc[q * tail + lane];
        sx += d.x;
        sz += d.y;
      }
      pass_b_finish(a, src, scl, vel, k, last, head, t0 + lane, sx, sz, one_decay, up);
    }
  }
}

// Thread 0 at the end of a step: merging and the glider step; then, unless
// it is the last step, the next step's prologue.
template <typename R, bool EXT>
__device__ __forceinline__ void epilogue(const KArgs &a, Shared<R> &sh,
                         typename SrcOf<R>::type *src, Scl32 *scl, int k, int n, int n_w) {
  using Src = typename SrcOf<R>::type;
  const int nb = a.nb, m = n_w + sh.n_shed;
  const bool last = (n == a.H - 1);
  sh.pairs += (long long)n_w * (2 * nb + 1) + (long long)m * (m - 1) + (long long)m * nb;
  int h = sh.head, cnt = m;
  while (a.n_wake_max > 0 && cnt > a.n_wake_max && cnt >= 2) {
    const Src s0 = src[h], s1 = src[h + 1];
    src[h + 1] = Src{R(0.5) * (s0.x + s1.x), R(0.5) * (s0.z + s1.z), s0.g + s1.g, R(0)};
    rescale(scl, h + 1, src[h + 1], float(a.r_core));
    for (int q = 0; q < kMaxPairs; ++q)
      if (sh.pa[q] == h || sh.pa[q] == h + 1 || sh.pb[q] == h || sh.pb[q] == h + 1)
        sh.pa[q] = sh.pb[q] = -1;
    ++h;
    --cnt;
  }
  sh.head = h;
  sh.n_w = cnt;
  for (int i = 0; i < 7; ++i) sh.g[i] = sh.gn[i];
  if (a.traj)
    for (int i = 0; i < 7; ++i)
      a.traj[((size_t)k * (a.H + 1) + n + 1) * 7 + i] = double(sh.gn[i]);
  if (last && a.n_vel_last) a.n_vel_last[k] = m;
  if (!last) prologue<R, EXT>(a, sh, src, scl, n + 1);
}

// Final outputs of rollout k.
template <typename R>
__device__ void finish(const KArgs &a, const Shared<R> &sh,
                       const typename SrcOf<R>::type *src, int k, int tid,
                       int nthr) {
  if (tid == 0) {
    bool finite = true;
    double j = 0.0;
    for (int i = 0; i < 7; ++i) {
      const double gi = double(sh.g[i]);
      a.g_final[7 * k + i] = gi;
      if (!isfinite(gi)) finite = false;
      const double d = gi - a.x_goal[i];
      j += a.q_diag[i] * d * d;
    }
    a.cost[k] = finite ? j : opaque_inf64();
    a.status[k] = sh.status | (finite ? 0 : VPM_ROLLOUT_NONFINITE);
    if (a.pair_count) a.pair_count[k] = sh.pairs;
    if (a.n_final) a.n_final[k] = sh.n_w;
  }
  if (a.gb_final && tid < a.nb) a.gb_final[(size_t)k * a.nb + tid] = sh.gb_prev[tid];
  if (a.wake_off) {
    const int64_t o = a.wake_off[k];
    const int capo = static_cast<int>(a.wake_off[k + 1] - o);
    const int cnt = min(sh.n_w, capo);
    for (int t = tid; t < cnt; t += nthr) {
      const auto s = src[sh.head + t];
      if (a.wx_out) a.wx_out[o + t] = double(s.x);
      if (a.wz_out) a.wz_out[o + t] = double(s.z);
      if (a.wg_out) a.wg_out[o + t] = double(s.g) * kTwoPi;
    }
  }
}

// --------------------------------------------------------- work queues

// A persistent workgroup claims its next rollout: list[next[cls]++] while
// below range[cls].y (the class's slice of the planned order). With no list
// it takes rollout `fallback` once.
struct Queue {
  const int32_t *list;  // rollout order (classes contiguous, longest first)
  int32_t *next;        // per-class cursor into `list`
  const int2 *range;    // per-class [begin, end) of `list`
  int cls;
};

template <typename R>
__device__ inline int claim(const Queue &q, Shared<R> &sh, int tid,
                            int &fallback) {
  if (!q.list) {
    const int k = fallback;
    fallback = -1;
    return k;
  }
  __syncthreads();
  if (tid == 0) {
    const int idx = atomicAdd(&q.next[q.cls], 1);
    sh.claimed = idx < q.range[q.cls].y ? q.list[idx] : -1;
  }
  __syncthreads();
  return sh.claimed;
}

// ---------------------------------------------------------------- LDS path

template <typename R, int T, int NW, int TILE, typename S>
__device__ void lds_pass_a_chunk(const KArgs &a, const Shared<R> &sh,
                                 const typename SrcOf<R>::type *src, const S *pa, Vec2<R> *red,
                                 int c0, int NT, int head, int s_lo, int s_hi,
                                 int lane, int wave) {
  const R rc = R(a.r_core), rc4 = rc * rc * rc * rc;
  R tx[T], tz[T], sx[T], sz[T], cx[T], cz[T];
#pragma unroll
  for (int j = 0; j < T; ++j) lds_target(src, c0 + lane + 64 * j, NT, head, 2 * a.nb + 3, tx[j], tz[j]);
  Vec2<R> *out = red + wave * 64 * T;
  if constexpr (!std::is_same_v<S, Src32>) {
    if (s_hi - s_lo <= TILE) {  // uniform: one tile
      accumulate_one_tile<R, T>(pa, s_lo, s_hi, tx, tz, rc4, sx, sz);
#pragma unroll
      for (int j = 0; j < T; ++j) out[lane + 64 * j] = Vec2<R>{sx[j], sz[j]};
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < T; ++j) sx[j] = sz[j] = cx[j] = cz[j] = R(0);
  if constexpr (std::is_same_v<S, Src32>)
    accumulate_staged<T, TILE>(pa, reinterpret_cast<Scl32 *>(red + wave * 64 * T), s_lo, s_hi,
                               rc, lane, tx, tz, sx, sz, cx, cz);
  else
    accumulate<R, T, TILE>(pa, s_lo, s_hi, tx, tz, rc4, sx, sz, cx, cz, true);
#pragma unroll
  for (int j = 0; j < T; ++j) out[lane + 64 * j] = Vec2<R>{sx[j] + cx[j], sz[j] + cz[j]};
}

// Tail of r < 64 targets: lane l takes target c0 + l mod r and the part
// l / r of g = 64 / r equal parts of this wave's sources, so g r lanes work
// instead of r. The partials land where a T = 1 chunk puts them, lane l at
// red[wave 64 + l], and are added per target over waves, then parts.
template <typename R, int NW, int TILE, typename S>
__device__ void lds_pass_a_tail(const KArgs &a, const Shared<R> &sh,
                                const typename SrcOf<R>::type *src, const S *pa, Vec2<R> *red,
                                int c0, int NT, int head, int s_lo, int s_hi,
                                int r, int lane, int wave) {
  const R rc = R(a.r_core), rc4 = rc * rc * rc * rc;
  const int g = 64 / r, t = lane % r, q = lane / r;
  R tx[1], tz[1], sx[1] = {R(0)}, sz[1] = {R(0)}, cx[1] = {R(0)}, cz[1] = {R(0)};
  lds_target(src, c0 + t, NT, head, 2 * a.nb + 3, tx[0], tz[0]);
  if (q < g) {
    const int len = s_hi - s_lo;
    accumulate<R, 1, TILE>(pa, s_lo + (len * q) / g, s_lo + (len * (q + 1)) / g, tx, tz, rc4,
                     sx, sz, cx, cz, true);
  }
  red[wave * 64 + lane] = Vec2<R>{sx[0] + cx[0], sz[0] + cz[0]};
}

// x / d for x < 2^24 and 1 <= d <= 256 as mulhi(x, ceil(2^32 / d)): the
// multiplier exceeds 2^32 / d by e / d with e < d, so the product's excess
// x e / 2^32 stays below 1 / d and cannot carry the quotient past an integer.
__device__ inline uint32_t mulhi(uint32_t x, uint32_t m) {
  return static_cast<uint32_t>((static_cast<uint64_t>(x) * m) >> 32);
}

// Spread chunks of the FP32 small class. A step's last pass-A chunk holds
// r < 64 TMAX targets; instead of 64 T target slots per wave against a
// quarter of the sources each (up to 3/4 of the slots idle), every one of
// the 256 lanes takes T targets against one of P equal source parts, with
// G = ceil(r / T) target groups and P = floor(256 / G) parts. plan[ti][r]
// holds, for TMAX = 1 << ti, the T <= TMAX with the smallest lane share T / P
// (ties: the smaller T), packed T | G << 3 | P << 12; magic[d] = ceil(2^32 / d)
// for the divisions by G and P (d >= 2; d = 1 is taken apart).
struct SpreadTables {
  uint32_t plan[3][256];
  uint32_t magic[257];
};
constexpr SpreadTables make_spread_tables() {
  SpreadTables t{};
  for (int ti = 0; ti < 3; ++ti) {
    const int tmax = 1 << ti;
    for (int r = 1; r < 64 * tmax; ++r) {
      int bt = 0, bg = 0, bp = 0;
      for (int T = 1; T <= tmax; ++T) {
        const int G = (r + T - 1) / T, P = 256 / G;
        if (P >= 1 && (bt == 0 || T * bp < bt * P)) {
          bt = T;
          bg = G;
          bp = P;
        }
      }
      t.plan[ti][r] = uint32_t(bt) | uint32_t(bg) << 3 | uint32_t(bp) << 12;
    }
  }
  for (int d = 2; d <= 256; ++d) t.magic[d] = uint32_t(((uint64_t(1) << 32) + d - 1) / d);
  return t;
}
__constant__ SpreadTables kSpread = make_spread_tables();

// The spread plan of a step's last chunk: T targets per lane, G groups, P
// parts of L sources; the parts end at the wake's end, so the first starts
// `pads` (< P) entries below it. P = 0: no spread chunk this step (no partial
// chunk, or fewer than P - 1 entries below the wake to hold the pads).
struct Spread {
  int T, G, P, L, pads;
  uint32_t mg;  // magic[G]
};
template <int TMAX>
__device__ inline Spread spread_plan(int NT, int n_w, int head) {
  Spread s{0, 0, 0, 0, 0, 0u};
  constexpr int ti = TMAX >= 4 ? 2 : TMAX == 2 ? 1 : 0;
  const int r = NT & (64 * TMAX - 1);
  if (r == 0) return s;
  const uint32_t e = kSpread.plan[ti][r];
  const int P = static_cast<int>(e >> 12);
  if (P - 1 > head) return s;
  s.T = static_cast<int>(e & 7u);
  s.G = static_cast<int>((e >> 3) & 511u);
  s.P = P;
  s.L = P == 1 ? n_w : static_cast<int>(mulhi(static_cast<uint32_t>(n_w + P - 1), kSpread.magic[P]));
  s.pads = P * s.L - n_w;
  s.mg = kSpread.magic[s.G];
  return s;
}

// The spread chunk at c0: lane gl takes the targets c0 + g + G j (j < T) of
// group g = gl mod G and the sources of part p = gl / G, [end - (P - p) L,
// end - (P - p - 1) L) with end = head + n_w; the pads below the wake are
// zero-strength entries (adding exactly nothing), so every lane runs the same
// L sources. Lanes past P G keep part 0's range and write nothing. Partials
// land at red[(p T + j) G + g].
template <int T, int TILE>
__device__ void lds_pass_a_spread(const Src32 *src, const Scl32 *pa, Vec2<float> *red,
                                  int c0, int NT, int head, int n_w, int n_surf,
                                  const Spread &sp, int gl) {
  const int pq = sp.G == 1 ? gl : static_cast<int>(mulhi(static_cast<uint32_t>(gl), sp.mg));
  const int g = gl - pq * sp.G;
  const bool on = pq < sp.P;
  const int p = on ? pq : 0;
  float tx[T], tz[T], sx[T], sz[T], cx[T], cz[T];
#pragma unroll
  for (int j = 0; j < T; ++j) lds_target<float>(src, c0 + g + sp.G * j, NT, head, n_surf, tx[j], tz[j]);
  const Scl32 *part = pa + (head + n_w - (sp.P - p) * sp.L);
  if (sp.L <= TILE) {  // uniform: one tile
    accumulate_one_tile<float, T>(part, 0, sp.L, tx, tz, 0.0f, sx, sz);
    if (on) {
#pragma unroll
      for (int j = 0; j < T; ++j) red[(p * T + j) * sp.G + g] = Vec2<float>{sx[j], sz[j]};
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < T; ++j) sx[j] = sz[j] = cx[j] = cz[j] = 0.0f;
  accumulate<float, T, TILE>(part, 0, sp.L, tx, tz, 0.0f, sx, sz, cx, cz, true);
  if (on) {
#pragma unroll
    for (int j = 0; j < T; ++j)
      red[(p * T + j) * sp.G + g] = Vec2<float>{sx[j] + cx[j], sz[j] + cz[j]};
  }
}

// Issue priority of this wave for step n. Several rollouts share a CU, and
// the sequencer issues from the oldest wave first, so with equal priorities
// the first-dispatched workgroup runs at almost solo speed and the last one
// finishes long after, alone on an idle CU. Rotating the priority by step
// over four slots makes co-resident workgroups progress at the same rate.
// The slot is the SIMD of the workgroup's first wave (hardware register
// HW_ID), which the dispatcher gives to co-resident workgroups in turn.
__device__ inline void rotate_priority(int slot, int n) {
  switch ((slot + n) & 3) {
    case 0: __builtin_amdgcn_s_setprio(3); break;
    case 1: __builtin_amdgcn_s_setprio(2); break;
    case 2: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
  }
}

__device__ inline int simd_id() {
  // HW_ID bits [5:4]: SIMD of this wave
  return static_cast<int>((__builtin_amdgcn_s_getreg((4 << 0) | (0 << 6) | (31 << 11)) >> 4) & 3u);
}

// Copy the plate inverse into LDS: the shedding mode's S x S system, then
// (separation gate on) the trailing-edge-only system right after it.
__device__ inline void stage_inverses(const KArgs &a, double *kinv, int tid, int nthr) {
  const int n_main = a.S * a.S;
  for (int q = tid; q < a.n_inv; q += nthr)
    kinv[q] = q < n_main ? a.kinv_t[q] : a.kinv_te[q - n_main];
}

// LDS-resident rollout kernel, NW waves per workgroup. Pass A splits the
// sources into NW contiguous slices (one per wave) and adds the slices in
// FP64 in wave order. MINW: waves per SIMD the register budget must allow.
template <typename R, int TMAX, int MINW, int NW, int TILE, bool EXT>
__global__ __launch_bounds__(64 * NW, MINW) void rollout_lds_kernel(KArgs args, Queue qu) {
  const KArgs &a = args;
  using Src = typename SrcOf<R>::type;
  constexpr int kThr = 64 * NW;
  extern __shared__ __align__(32) unsigned char lds[];
  __shared__ Shared<R> sh;
  Src *src = reinterpret_cast<Src *>(lds);
  double2 *vsurf = reinterpret_cast<double2 *>(lds + a.off_vsurf);
  Vec2<R> *red = reinterpret_cast<Vec2<R> *>(lds + a.off_red);
  Vec2<R> *vel = reinterpret_cast<Vec2<R> *>(lds + a.off_vel);
  double *kinv = reinterpret_cast<double *>(lds + a.off_kinv);
  // the scaled copy of the wake that pass A reads, or the wake itself
  constexpr bool SCL = lds_scaled<R, NW>();
  using PA = std::conditional_t<SCL, Scl32, Src>;
  Scl32 *scl = SCL ? reinterpret_cast<Scl32 *>(lds + a.off_scl) : nullptr;
  const PA *pa = reinterpret_cast<const PA *>(SCL ? lds + a.off_scl : lds);

  const int tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar (every lane is active here), so loops bounded by
  // it are counted in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n_surf = 2 * a.nb + 3;
  // this thread's surface point's chord coordinate (threads below n_surf)
  const R s_surf = surface_s(tid, a.nb, R(a.lb), R(a.shed_frac * a.chord), R(a.chord));
  stage_inverses(a, kinv, tid, kThr);
  if (tid == 0) sh.slot = simd_id();
  int fallback = blockIdx.x;
  for (;;) {
    const int k = claim(qu, sh, tid, fallback);
    if (k < 0) break;
    __syncthreads();
    if (!setup(fresh_args(args), sh, src, scl, k, opaque_tid(tid), kThr, n_surf)) continue;
    __syncthreads();

    const int H = a.H;
    for (int n = 0; n < H; ++n) {
      // the arguments as this step reads them (see fresh_args); each section
      // below takes its own copy
      const KArgs &a = fresh_args(args);
      if (n == 0) {
        if (tid == 0) prologue<R, EXT>(fresh_args(args), sh, src, scl, 0);
        __syncthreads();
      }
      rotate_priority(sh.slot, n);
      const int head = sh.head, n_w = sh.n_w, n_shed = sh.n_shed;
      const int NT = n_surf + n_w;
      // the step's surface points (collocation, bound, release) as pass-A
      // targets in the n_surf entries below the wake, which hold no live
      // vortex (the wake starts at n_surf and only moves up as it merges)
      if (tid < n_surf)
        src[head - n_surf + tid] =
            Src{sh.le[0] + s_surf * sh.et[0], sh.le[1] + s_surf * sh.et[1], R(0), R(0)};
      // the plan of this step's last chunk if it is spread, and its pads:
      // zero-strength entries of the scaled copy just below the wake (dead
      // entries: the wake only moves up)
      Spread sp{0, 0, 0, 0, 0, 0u};
      if constexpr (SCL) {
        sp = spread_plan<TMAX>(__builtin_amdgcn_readfirstlane(NT),
                               __builtin_amdgcn_readfirstlane(n_w),
                               __builtin_amdgcn_readfirstlane(head));
        if (tid < sp.pads) scl[head - sp.pads + tid] = Scl32{0.0f, 0.0f, 0.0f, INFINITY};
      }
      __syncthreads();
      // this step's control, loaded now so its latency hides behind pass A
      double u_m = 0.0, u_e = 0.0;
      if (tid == 0) {
        u_m = a.u_mean[n];
        u_e = a.u_eps[(size_t)k * a.H + n];
      }

      const int s_lo = head + (n_w * wave) / NW;
      const int s_hi = head + (n_w * (wave + 1)) / NW;
      // pass-A velocity of target tt (surface point, or wake entry)
      auto store_velocity = [&](int tt, double vx, double vz) {
        if (tt < n_surf) {
          vsurf[tt] = make_double2(vx, vz);
        } else {
          const int i = head + tt - n_surf;
          // the self term of a scaled pair: the small class removes it in
          // pass B; staged chunks of the large class here (tails are unscaled)
          if constexpr (sizeof(R) == 4 && !SCL)
            remove_self(src[i].x, src[i].z, pass_a_source(src[i], float(a.r_core)), vx, vz);
          vel[i] = Vec2<R>{R(vx), R(vz)};
        }
      };
      for (int c0 = 0; c0 < NT;) {
        const int rem = NT - c0;
        if constexpr (SCL) {
          if (sp.P > 0 && rem < 64 * TMAX) {
            // the last chunk, spread over every lane
            switch (sp.T) {
              case 1: lds_pass_a_spread<1, TILE>(src, pa, red, c0, NT, head, n_w, n_surf, sp, tid); break;
              case 2: if constexpr (TMAX >= 2) lds_pass_a_spread<2, TILE>(src, pa, red, c0, NT, head, n_w, n_surf, sp, tid); break;
              case 3: if constexpr (TMAX >= 4) lds_pass_a_spread<3, TILE>(src, pa, red, c0, NT, head, n_w, n_surf, sp, tid); break;
              default: if constexpr (TMAX >= 4) lds_pass_a_spread<4, TILE>(src, pa, red, c0, NT, head, n_w, n_surf, sp, tid); break;
            }
            __syncthreads();
            // lane g adds its groups' parts in FP64 in part order
            if (tid < sp.G) {
              for (int j = 0; j < sp.T; ++j) {
                const int i = tid + sp.G * j;
                if (i < rem) {
                  const Vec2<R> r0 = red[j * sp.G + tid];
                  double vx = double(r0.x), vz = double(r0.z);
                  for (int p = 1; p < sp.P; ++p) {
                    const Vec2<R> r = red[(p * sp.T + j) * sp.G + tid];
                    vx += double(r.x);
                    vz += double(r.z);
                  }
                  store_velocity(c0 + i, vx, vz);
                }
              }
            }
            __syncthreads();
            break;
          }
        }
        // largest chunk of 4, 3, 2 or 1 targets per lane that is at least 3/4
        // full (fewer chunks, barriers and cross-wave combines for a few idle
        // target slots; the 3-target chunk keeps the last chunk of a step
        // fuller than powers of two alone); a tail below 64 takes T=1
        int T = 1;
        if (TMAX >= 4 && 48 * 4 <= rem) T = 4;
        else if (TMAX >= 4 && 48 * 3 <= rem) T = 3;
        else if (TMAX >= 2 && 48 * 2 <= rem) T = 2;
        const int tail = rem < 32 ? rem : 0;  // tails of 32..63 keep a lane each
        if (tail) {
          lds_pass_a_tail<R, NW, TILE>(fresh_args(args), sh, src, pa, red, c0, NT, head, s_lo, s_hi, tail, lane, wave);
        } else {
          switch (T) {
            case 1: lds_pass_a_chunk<R, 1, NW, TILE>(fresh_args(args), sh, src, pa, red, c0, NT, head, s_lo, s_hi, lane, wave); break;
            case 2: if constexpr (TMAX >= 2) lds_pass_a_chunk<R, 2, NW, TILE>(fresh_args(args), sh, src, pa, red, c0, NT, head, s_lo, s_hi, lane, wave); break;
            case 3: if constexpr (TMAX >= 4) lds_pass_a_chunk<R, 3, NW, TILE>(fresh_args(args), sh, src, pa, red, c0, NT, head, s_lo, s_hi, lane, wave); break;
            default: if constexpr (TMAX >= 4) lds_pass_a_chunk<R, 4, NW, TILE>(fresh_args(args), sh, src, pa, red, c0, NT, head, s_lo, s_hi, lane, wave); break;
          }
        }
        __syncthreads();
        const int span = 64 * T;
        const int parts = tail ? 64 / tail : 1;
        for (int t = tid; t < span && c0 + t < NT; t += kThr) {
          // wave 0's first part starts the sum (adding it to zero is exact)
          const Vec2<R> r0 = red[t];
          double vx = double(r0.x), vz = double(r0.z);
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            for (int q = (w == 0 ? 1 : 0); q < parts; ++q) {
              const Vec2<R> r = red[w * span + q * tail + t];
              vx += double(r.x);
              vz += double(r.z);
            }
          }
          const int tt = c0 + t;
          if (tail && tt >= n_surf && sizeof(R) == 4 && !SCL) {
            vel[head + tt - n_surf] = Vec2<R>{R(vx), R(vz)};  // unscaled: no self term
          } else {
            store_velocity(tt, vx, vz);
          }
        }
        __syncthreads();
        c0 += span;
      }

      if (wave == 0)
        solve_section(fresh_args(args), sh, src, vel, vsurf, kinv, k, n, head, n_w, lane,
                      EXT ? u_m + u_e + sh.u_fb : u_m + u_e);
      __syncthreads();
      pass_b(fresh_args(args), sh, src, scl, vel, k, n == H - 1, head, n_w + n_shed, n_w, tid, kThr,
             reinterpret_cast<double2 *>(lds + a.off_red));
      __syncthreads();
      if (tid == 0) epilogue<R, EXT>(fresh_args(args), sh, src, scl, k, n, n_w);
      __syncthreads();
    }
    finish(fresh_args(args), sh, src, k, opaque_tid(tid), kThr);
  }
}

// ---------------------------------------------------------- streaming path

template <typename R, int T, int NW, int TILE>
__device__ void stream_pass_a_round(const KArgs &a, const Shared<R> &sh,
                                    const typename SrcOf<R>::type *src,
                                    typename PassAOf<R>::type *tile, Vec2<R> *vel,
                                    double2 *vsurf, int c0, int NT, int head,
                                    int n_w, int tid, int lane, int wave) {
  const int n_surf = 2 * a.nb + 3;
  const R rc = R(a.r_core), rc4 = rc * rc * rc * rc;
  R tx[T], tz[T], sx[T], sz[T], cx[T], cz[T];
  const int t0 = c0 + wave * 64 + lane;  // target j of this lane: t0 + j 64 NW
#pragma unroll
  for (int j = 0; j < T; ++j) {
    target_pos(a, sh, src, t0 + j * 64 * NW, NT, head, tx[j], tz[j]);
    sx[j] = sz[j] = cx[j] = cz[j] = R(0);
  }
  for (int s0 = 0; s0 < n_w; s0 += kStreamTile) {
    const int cnt = min(kStreamTile, n_w - s0);
    for (int q = tid; q < cnt; q += 64 * NW) tile[q] = pass_a_source(src[head + s0 + q], rc);
    __syncthreads();
    accumulate<R, T, TILE>(tile, 0, cnt, tx, tz, rc4, sx, sz, cx, cz, s0 == 0);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const int t = t0 + j * 64 * NW;
    if (t >= NT) continue;
    double vx = double(sx[j]) + double(cx[j]), vz = double(sz[j]) + double(cz[j]);
    if (t < n_surf) {
      vsurf[t] = make_double2(vx, vz);
    } else {
      const int i = head + t - n_surf;
      if constexpr (sizeof(R) == 4) remove_self(tx[j], tz[j], pass_a_source(src[i], rc), vx, vz);
      vel[i] = Vec2<R>{R(vx), R(vz)};
    }
  }
}

// A source that adds exactly nothing (zero strength) in pass-A form.
__device__ inline Scl32 zero_pass_a(Scl32) { return Scl32{0.0f, 0.0f, 0.0f, INFINITY}; }
__device__ inline Src64 zero_pass_a(Src64) { return Src64{0.0, 0.0, 0.0, 0.0}; }

// The last round of a step when it holds r < 64 NW targets: W = ceil(r / 64)
// waves hold one target per lane, and the P = NW / W groups of W waves take
// one of P equal source parts of L = ceil(n_w / P) each. Every tile step
// stages P slices of kStreamTile / P sources, slice i from part i (entries
// past the wake are zero sources), and each wave sums only its part's slice,
// so the round costs 1 / P of a full pass over the sources instead of a
// whole pass for a partly idle set of lanes. The part sums are added in FP64
// in part order by the first group, through the tile buffer.
template <typename R, int NW, int TILE>
__device__ void stream_pass_a_spread(const KArgs &a, const Shared<R> &sh,
                                     const typename SrcOf<R>::type *src,
                                     typename PassAOf<R>::type *tile, Vec2<R> *vel,
                                     double2 *vsurf, int c0, int NT, int head, int n_w,
                                     int tid, int lane, int wave, int W, int P) {
  using PA = typename PassAOf<R>::type;
  const int n_surf = 2 * a.nb + 3;
  const R rc = R(a.r_core), rc4 = rc * rc * rc * rc;
  const int TS = kStreamTile / P;     // sources of one part per tile step
  const int L = (n_w + P - 1) / P;    // sources per part (the last may run past the wake)
  const int p = wave / W;             // this wave's part (p == P: an idle wave)
  const int slot = (wave - p * W) * 64 + lane;
  const int t = c0 + slot;
  R tx[1], tz[1], sx[1] = {R(0)}, sz[1] = {R(0)}, cx[1] = {R(0)}, cz[1] = {R(0)};
  target_pos(a, sh, src, t, NT, head, tx[0], tz[0]);
  for (int s0 = 0; s0 < L; s0 += TS) {
    const int cnt = min(TS, L - s0);
    for (int q = tid; q < P * TS; q += 64 * NW) {
      const int pp = q / TS, i = q - pp * TS;
      const int g = pp * L + s0 + i;  // source index (part pp, this step's slice)
      tile[q] = i < cnt && g < n_w ? pass_a_source(src[head + g], rc) : zero_pass_a(PA{});
    }
    __syncthreads();
    if (p < P) accumulate<R, 1, TILE>(tile + p * TS, 0, cnt, tx, tz, rc4, sx, sz, cx, cz, s0 == 0);
    __syncthreads();
  }
  double2 *part = reinterpret_cast<double2 *>(tile);  // P W 64 entries fit the tile
  if (p < P)
    part[p * W * 64 + slot] =
        make_double2(double(sx[0]) + double(cx[0]), double(sz[0]) + double(cz[0]));
  __syncthreads();
  if (p == 0 && t < NT) {
    double vx = part[slot].x, vz = part[slot].y;
    for (int q = 1; q < P; ++q) {
      const double2 d = part[q * W * 64 + slot];
      vx += d.x;
      vz += d.y;
    }
    if (t < n_surf) {
      vsurf[t] = make_double2(vx, vz);
    } else {
      const int i = head + t - n_surf;
      if constexpr (sizeof(R) == 4) remove_self(tx[0], tz[0], pass_a_source(src[i], rc), vx, vz);
      vel[i] = Vec2<R>{R(vx), R(vz)};
    }
  }
  __syncthreads();  // the tile buffer is staged again by the next round
}

// Persistent: each workgroup keeps its rollout's wake in workspace slot
// blockIdx.x (a.cap sources and velocities) and walks rollouts b, b + G, ...
// or, with a queue, claims them in planned order.
template <typename R, int TMAX, int NW, int TILE, bool EXT>
__global__ __launch_bounds__(64 * NW, 1) void rollout_stream_kernel(KArgs a, Queue qu) {
  using Src = typename SrcOf<R>::type;
  constexpr int kThr = 64 * NW;
  extern __shared__ __align__(32) unsigned char lds[];
  __shared__ Shared<R> sh;
  auto *tile = reinterpret_cast<typename PassAOf<R>::type *>(lds);
  Scl32 *const scl = nullptr;  // pass A converts each staged tile
  double2 *vsurf = reinterpret_cast<double2 *>(lds + a.off_vsurf);
  double *kinv = reinterpret_cast<double *>(lds + a.off_kinv);
  Src *src = reinterpret_cast<Src *>(a.ws_src) + (size_t)blockIdx.x * a.cap;
  Vec2<R> *vel = reinterpret_cast<Vec2<R> *>(a.ws_vel) + (size_t)blockIdx.x * a.cap;

  const int tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar (every lane is active here), so loops bounded by
  // it are counted in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n_surf = 2 * a.nb + 3;
  stage_inverses(a, kinv, tid, kThr);

  int next_static = blockIdx.x;
  for (;;) {
    int k;
    if (qu.list) {
      k = claim(qu, sh, tid, next_static);
    } else {
      k = next_static < a.K ? next_static : -1;
      next_static += gridDim.x;
    }
    if (k < 0) break;
    __syncthreads();
    if (!setup(a, sh, src, scl, k, opaque_tid(tid), kThr, 0)) continue;
    __syncthreads();
    for (int n = 0; n < a.H; ++n) {
      if (n == 0) {
        if (tid == 0) prologue<R, EXT>(a, sh, src, scl, 0);
        __syncthreads();
      }
      const int head = sh.head, n_w = sh.n_w, n_shed = sh.n_shed;
      const int NT = n_surf + n_w;
      double u_m = 0.0, u_e = 0.0;  // this step's control, loaded before pass A
      if (tid == 0) {
        u_m = a.u_mean[n];
        u_e = a.u_eps[(size_t)k * a.H + n];
      }
      // pass A in rounds of 64 * NW * T targets (T shrinks for the tail)
      for (int c0 = 0; c0 < NT;) {
        const int rem = NT - c0;
        int T = TMAX;
        while (T > 1 && 64 * NW * T > rem) T >>= 1;
        const int W = (rem + 63) / 64;
        if (T == 1 && 2 * W <= NW) {
          // a ragged last round: spread over source parts
          stream_pass_a_spread<R, NW, TILE>(a, sh, src, tile, vel, vsurf, c0, NT, head, n_w, tid,
                                            lane, wave, W, NW / W);
          break;
        }
        switch (T) {
          case 1: stream_pass_a_round<R, 1, NW, TILE>(a, sh, src, tile, vel, vsurf, c0, NT, head, n_w, tid, lane, wave); break;
          case 2: if constexpr (TMAX >= 2) stream_pass_a_round<R, 2, NW, TILE>(a, sh, src, tile, vel, vsurf, c0, NT, head, n_w, tid, lane, wave); break;
          default: if constexpr (TMAX >= 4) stream_pass_a_round<R, 4, NW, TILE>(a, sh, src, tile, vel, vsurf, c0, NT, head, n_w, tid, lane, wave); break;
        }
        c0 += 64 * NW * T;
      }
      __syncthreads();
      if (wave == 0)
        solve_section(a, sh, src, vel, vsurf, kinv, k, n, head, n_w, lane,
                      EXT ? u_m + u_e + sh.u_fb : u_m + u_e);
      __syncthreads();
      pass_b(a, sh, src, scl, vel, k, n == a.H - 1, head, n_w + n_shed, n_w, tid, kThr,
             reinterpret_cast<double2 *>(lds + a.off_red));
      __syncthreads();
      if (tid == 0) epilogue<R, EXT>(a, sh, src, scl, k, n, n_w);
      __syncthreads();
    }
    finish(a, sh, src, k, opaque_tid(tid), kThr);
  }
}

// ------------------------------------------------------- batch planning

constexpr int kPlanThreads = 1024;
constexpr int kBuckets = 128;  // 4 per octave of capacity
constexpr int kClasses = 3;    // 0: streamed, 1: large LDS, 2: small LDS

// One workgroup orders an uneven batch: the class of rollout k follows its
// capacity n0 + 2H (streamed above cap_l, large LDS above cap_s, small LDS
// otherwise); within a class rollouts are ordered by decreasing capacity in
// quarter-octave buckets (longest processing time first). Writes the order
// into list, the per-class slices into range and resets the cursors.
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(
    int K, int H, int max_wake0, int n_fields, const int64_t *field_off,
    const int32_t *field_of, int cap_s, int cap_l, int32_t *list, int2 *range,
    int32_t *next) {
  __shared__ int hist[kClasses * kBuckets];
  __shared__ int cursor[kClasses * kBuckets];
  const int t = threadIdx.x;
  for (int i = t; i < kClasses * kBuckets; i += kPlanThreads) hist[i] = 0;
  __syncthreads();
  auto key_of = [&](int k) -> int {
    const int fo = field_of ? field_of[k] : k;
    int cap = 0;
    if (fo >= 0 && fo < n_fields) {
      const long long n0 = field_off[fo + 1] - field_off[fo];
      if (n0 >= 0 && n0 <= max_wake0) cap = static_cast<int>(n0) + 2 * H;
    }
    const int cls = cap > cap_l ? 0 : cap > cap_s ? 1 : 2;
    int b = cap > 0 ? static_cast<int>(4.0f * log2f(static_cast<float>(cap))) : 0;
    b = b < 0 ? 0 : b >= kBuckets ? kBuckets - 1 : b;
    return cls * kBuckets + (kBuckets - 1 - b);  // larger capacity first
  };
  for (int k = t; k < K; k += kPlanThreads) atomicAdd(&hist[key_of(k)], 1);
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int c = 0; c < kClasses; ++c) {
      const int begin = acc;
      for (int b = 0; b < kBuckets; ++b) {
        cursor[c * kBuckets + b] = acc;
        acc += hist[c * kBuckets + b];
      }
      range[c] = make_int2(begin, acc);
      next[c] = begin;
    }
  }
  __syncthreads();
  for (int k = t; k < K; k += kPlanThreads) list[atomicAdd(&cursor[key_of(k)], 1)] = k;
}

// ------------------------------------------------------------------ host

// Doubles of plate inverse staged in LDS: the system of the shedding mode,
// and with the separation gate also the trailing-edge-only system.
int inverse_entries(const vpm_params *p) {
  const int s = system_size(p->n_bound, p->shed_mode);
  const int s_te = system_size(p->n_bound, VPM_SHED_TE);
  return s * s + (p->gate ? s_te * s_te : 0);
}

// The per-wave partial sums of pass A (64 T Vec2 per wave), which pass B
// reuses as FP64 scratch (64 double2 per wave): the larger of the two.
template <typename R>
size_t red_bytes(int nw, int tmax) {
  const size_t pass_a = (size_t)nw * 64 * tmax * sizeof(Vec2<R>);
  const size_t pass_b = (size_t)nw * 64 * sizeof(double2);
  return pass_a > pass_b ? pass_a : pass_b;
}

// n_inv: doubles of the staged inverse(s)
template <typename R>
size_t lds_fixed_bytes(int nb, int n_inv, int nw, int tmax) {
  return (size_t)n_inv * sizeof(double) + (size_t)(2 * nb + 3) * sizeof(double2) +
         red_bytes<R>(nw, tmax) + 32 + sizeof(Shared<R>);
}
// Per vortex: the wake entry, its pass-A velocity and (FP32) its scaled copy.
template <typename R, int NW> constexpr size_t scaled_bytes() {
  return lds_scaled<R, NW>() ? sizeof(Scl32) : 0;
}
template <typename R, int NW> constexpr size_t lds_per_vortex() {
  return sizeof(typename SrcOf<R>::type) + sizeof(Vec2<R>) + scaled_bytes<R, NW>();
}

// The wake arrays (src, its scaled copy, vel) hold n_surf + cap entries: the
// wake from entry n_surf on, the step's surface points just below it.
template <typename R, int NW>
int lds_layout(int cap, int nb, int tmax, KArgs &a) {
  constexpr int nw = NW;
  const size_t ent = (size_t)cap + 2 * nb + 3;
  size_t off = 0;
  off += ent * sizeof(typename SrcOf<R>::type);
  a.off_scl = static_cast<int>(off);
  off += ent * scaled_bytes<R, NW>();
  off = (off + 15) & ~size_t(15);
  a.off_kinv = static_cast<int>(off);
  off += (size_t)a.n_inv * sizeof(double);
  off = (off + 15) & ~size_t(15);  // 16-byte records follow
  a.off_vsurf = static_cast<int>(off);
  off += (size_t)(2 * nb + 3) * sizeof(double2);
  a.off_red = static_cast<int>(off);
  off += red_bytes<R>(nw, tmax);
  a.off_vel = static_cast<int>(off);
  off += ent * sizeof(Vec2<R>);
  return static_cast<int>(off);
}

template <typename R>
int stream_layout(int nb, KArgs &a) {
  size_t off = (size_t)kStreamTile * sizeof(typename PassAOf<R>::type);
  a.off_scl = 0;
  a.off_kinv = static_cast<int>(off);
  off += (size_t)a.n_inv * sizeof(double);
  off = (off + 15) & ~size_t(15);  // 16-byte records follow
  a.off_vsurf = static_cast<int>(off);
  off += (size_t)(2 * nb + 3) * sizeof(double2);
  a.off_red = a.off_vel = 0;
  return static_cast<int>(off);
}

template <typename Kern>
int set_lds(Kern kern, int bytes) {
  if (bytes > 65536)
    VPM_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    bytes));
  return VPM_OK;
}

// Launch the LDS kernel for wakes up to `cap` vortices; grid = `grid`
// workgroups (one per rollout without a queue).
template <typename R, int TMAX, int MINW, int NW, int TILE>
int launch_lds(vpm_ctx *ctx, KArgs a, int cap, int grid, const Queue &qu,
               hipStream_t stream) {
  a.cap = cap;
  const int lds = lds_layout<R, NW>(cap, a.nb, TMAX, a);
  if (lds + static_cast<int>(sizeof(Shared<R>)) > ctx->max_lds)
    return fail(VPM_ECAPACITY, "wake capacity " + std::to_string(cap) +
                                   " does not fit the LDS-resident kernel");
  auto kern = a.gate || a.fb_gain ? rollout_lds_kernel<R, TMAX, MINW, NW, TILE, true>
                                 : rollout_lds_kernel<R, TMAX, MINW, NW, TILE, false>;
  int rc = set_lds(kern, lds);
  if (rc != VPM_OK) return rc;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, stream, a, qu);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}


template <typename R, int TMAX, int NW, int TILE>
int launch_stream(vpm_ctx *ctx, KArgs a, int grid, const Queue &qu,
                  hipStream_t stream, bool capturing, void *fixed_ws) {
  const int lds = stream_layout<R>(a.nb, a);
  if (lds + static_cast<int>(sizeof(Shared<R>)) > ctx->max_lds)
    return fail(VPM_ECAPACITY, "streaming kernel LDS exceeds the device limit");
  auto kern = a.gate || a.fb_gain ? rollout_stream_kernel<R, TMAX, NW, TILE, true>
                                 : rollout_stream_kernel<R, TMAX, NW, TILE, false>;
  int rc = set_lds(kern, lds);
  if (rc != VPM_OK) return rc;
  void *ws = fixed_ws;  // the caller sized it for `grid` slots
  if (!ws) {
    const size_t slot = (size_t)a.cap * (sizeof(typename SrcOf<R>::type) + sizeof(Vec2<R>));
    rc = ensure_buffer(&ctx->ws, &ctx->ws_bytes, slot * grid, "streaming workspace", capturing);
    if (rc != VPM_OK) return rc;
    ws = ctx->ws;
  }
  a.ws_src = ws;
  a.ws_vel = static_cast<char *>(ws) + (size_t)grid * a.cap * sizeof(typename SrcOf<R>::type);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, stream, a, qu);
  VPM_HIP_TRY(hipGetLastError());
  return VPM_OK;
}

// Largest capacity a workgroup of the LDS kernel can hold within `bytes`.
template <typename R, int NW>
int lds_capacity(int nb, int n_inv, int tmax, size_t bytes) {
  // the surface-point entries below the wake take n_surf vortex records
  const size_t fixed = lds_fixed_bytes<R>(nb, n_inv, NW, tmax) +
                       (size_t)(2 * nb + 3) * lds_per_vortex<R, NW>();
  return bytes > fixed ? static_cast<int>((bytes - fixed) / lds_per_vortex<R, NW>()) : 0;
}

// Kernel instance for a class's tuning (targets per thread x compensation
// tile). FP32 compiles every pair of {1, 2, 4} x {64, 128, 256}; FP64 only
// its fixed shape (2 targets per thread, 64-source tiles).
template <typename R, int MINW, int NW>
int launch_lds_tuned(vpm_ctx *ctx, KArgs a, int cap, int grid, const Queue &qu,
                     hipStream_t stream, Tune t) {
  if constexpr (sizeof(R) == 8) {
    return launch_lds<R, 2, MINW, NW, 64>(ctx, a, cap, grid, qu, stream);
  } else {
    switch (t.tmax * 1000 + t.tile) {
      case 1064: return launch_lds<R, 1, MINW, NW, 64>(ctx, a, cap, grid, qu, stream);
      case 1128: return launch_lds<R, 1, MINW, NW, 128>(ctx, a, cap, grid, qu, stream);
      case 1256: return launch_lds<R, 1, MINW, NW, 256>(ctx, a, cap, grid, qu, stream);
      case 2064: return launch_lds<R, 2, MINW, NW, 64>(ctx, a, cap, grid, qu, stream);
      case 2128: return launch_lds<R, 2, MINW, NW, 128>(ctx, a, cap, grid, qu, stream);
      case 2256: return launch_lds<R, 2, MINW, NW, 256>(ctx, a, cap, grid, qu, stream);
      case 4064: return launch_lds<R, 4, MINW, NW, 64>(ctx, a, cap, grid, qu, stream);
      case 4128: return launch_lds<R, 4, MINW, NW, 128>(ctx, a, cap, grid, qu, stream);
      case 4256: return launch_lds<R, 4, MINW, NW, 256>(ctx, a, cap, grid, qu, stream);
      default: return fail(VPM_EINVAL, "unsupported kernel tuning");
    }
  }
}

template <typename R, int NW>
int launch_stream_tuned(vpm_ctx *ctx, KArgs a, int grid, const Queue &qu, hipStream_t stream,
                        bool capturing, Tune t, void *fixed_ws = nullptr) {
  if constexpr (sizeof(R) == 8) {
    return launch_stream<R, 2, NW, 64>(ctx, a, grid, qu, stream, capturing, fixed_ws);
  } else {
    switch (t.tmax * 1000 + t.tile) {
      case 1064: return launch_stream<R, 1, NW, 64>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 1128: return launch_stream<R, 1, NW, 128>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 1256: return launch_stream<R, 1, NW, 256>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 2064: return launch_stream<R, 2, NW, 64>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 2128: return launch_stream<R, 2, NW, 128>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 2256: return launch_stream<R, 2, NW, 256>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 4064: return launch_stream<R, 4, NW, 64>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 4128: return launch_stream<R, 4, NW, 128>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      case 4256: return launch_stream<R, 4, NW, 256>(ctx, a, grid, qu, stream, capturing, fixed_ws);
      default: return fail(VPM_EINVAL, "unsupported kernel tuning");
    }
  }
}

// The tuning a class runs with in precision R (FP64 shapes are fixed).
template <typename R> Tune class_tune(const vpm_ctx *ctx, int cls) {
  if constexpr (sizeof(R) == 8) return Tune{2, 64};
  return ctx->tune[cls];
}

// Bytes of one streaming-workspace slot (one resident workgroup's wake and
// velocities) for wakes of capacity `cap`.
template <typename R>
size_t stream_slot_bytes(int cap) {
  return (size_t)cap * (sizeof(typename SrcOf<R>::type) + sizeof(Vec2<R>));
}

// One batch of vpm_rollout_batch_noalloc: the kernels of run_batch with their
// scratch (the uneven-batch plan, then the streaming workspace) in the
// library's static device array [scratch, scratch + bytes), the streamed
// class on as many workgroups as whole slots fit there (at most one per CU),
// and the class kernels of an uneven batch one after another on the caller's
// stream. Allocates nothing and creates no stream or event.
template <typename R, int MINW_S, int NW_X>
int run_batch_noalloc(vpm_ctx *ctx, KArgs a, int path, hipStream_t stream, char *scratch,
                      size_t bytes) {
  constexpr int kNwSmall = 4, kNwLarge = sizeof(R) == 4 ? 16 : 8;
  std::lock_guard<std::mutex> lock(ctx->ws_mu);  // the tuning table
  const int cap = a.cap;
  const Tune t_s = class_tune<R>(ctx, VPM_CLASS_SMALL), t_l = class_tune<R>(ctx, VPM_CLASS_LARGE);
  const Tune t_x = class_tune<R>(ctx, VPM_CLASS_STREAM);
  const int cap_small = lds_capacity<R, kNwSmall>(a.nb, a.n_inv, t_s.tmax, ctx->max_lds / 4);
  const int cap_large = lds_capacity<R, kNwLarge>(a.nb, a.n_inv, t_l.tmax, ctx->max_lds);
  const Queue none{nullptr, nullptr, nullptr, 0};
  const bool stream_only = path == VPM_PATH_STREAM;
  const size_t slot = stream_slot_bytes<R>(cap);
  auto stream_grid = [&](size_t room) {
    size_t g = room / slot;
    g = g < (size_t)ctx->n_cu ? g : (size_t)ctx->n_cu;
    return (int)(g < (size_t)a.K ? g : (size_t)a.K);
  };
  if (a.n_fields == 1 || path == VPM_PATH_LDS || stream_only) {
    if (!stream_only && cap <= cap_small)
      return launch_lds_tuned<R, MINW_S, kNwSmall>(ctx, a, cap, a.K, none, stream, t_s);
    if (!stream_only && cap <= cap_large)
      return launch_lds_tuned<R, 1, kNwLarge>(ctx, a, cap, a.K, none, stream, t_l);
    if (path == VPM_PATH_LDS)
      return fail(VPM_ECAPACITY, "wake capacity " + std::to_string(cap) +
                                     " does not fit the LDS-resident kernel");
    const int grid = stream_grid(bytes);
    if (grid < 1)
      return fail(VPM_ECAPACITY, "one streaming slot of wake capacity " + std::to_string(cap) +
                                     " exceeds the static scratch of " +
                                     std::to_string(bytes) + " bytes");
    return launch_stream_tuned<R, NW_X>(ctx, a, grid, none, stream, false, t_x, scratch);
  }
  // uneven batch: the plan at the start of the scratch, 256-byte aligned
  const size_t plan_bytes = ((size_t)a.K * sizeof(int32_t) + 64 + 255) & ~size_t(255);
  if (plan_bytes > bytes)
    return fail(VPM_ECAPACITY, "the plan of " + std::to_string(a.K) +
                                   " rollouts exceeds the static scratch");
  int2 *range = reinterpret_cast<int2 *>(scratch);
  int32_t *next = reinterpret_cast<int32_t *>(scratch + 32);
  int32_t *list = reinterpret_cast<int32_t *>(scratch + 64);
  int grid_x = 0;
  if (cap > cap_large) {
    grid_x = stream_grid(bytes - plan_bytes);
    if (grid_x < 1)
      return fail(VPM_ECAPACITY, "one streaming slot of wake capacity " + std::to_string(cap) +
                                     " does not fit the static scratch beside the plan");
  }
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, a.K, a.H,
                     a.max_wake0, a.n_fields, a.field_off, a.field_of, cap_small,
                     cap_large, list, range, next);
  VPM_HIP_TRY(hipGetLastError());
  int rc = VPM_OK;
  if (cap > cap_large) {
    rc = launch_stream_tuned<R, NW_X>(ctx, a, grid_x, Queue{list, next, range, 0}, stream, false,
                                      t_x, scratch + plan_bytes);
    if (rc != VPM_OK) return rc;
  }
  if (cap > cap_small) {
    const int c1 = cap < cap_large ? cap : cap_large;
    const int grid = a.K < ctx->n_cu ? a.K : ctx->n_cu;
    rc = launch_lds_tuned<R, 1, kNwLarge>(ctx, a, c1, grid, Queue{list, next, range, 1}, stream,
                                          t_l);
    if (rc != VPM_OK) return rc;
  }
  const int c2 = cap < cap_small ? cap : cap_small;
  const int grid = a.K < 4 * ctx->n_cu ? a.K : 4 * ctx->n_cu;
  return launch_lds_tuned<R, MINW_S, kNwSmall>(ctx, a, c2, grid, Queue{list, next, range, 2},
                                               stream, t_s);
}

// One batch in a given precision. Uniform batches (one field) run one
// rollout per workgroup on the caller's stream. Uneven batches are planned
// on the device and run as up to three persistent class kernels on forked
// streams, joined back into the caller's stream. Calls that use the
// context's workspace are ordered by an event; while the caller's stream is
// being captured into a graph that ordering is the caller's (replays of a
// graph and other calls on the same context must not overlap).
template <typename R, int MINW_S, int NW_X>
int run_batch(vpm_ctx *ctx, KArgs a, int path, hipStream_t stream) {
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  VPM_HIP_TRY(hipStreamIsCapturing(stream, &cap_status));
  const bool capturing = cap_status != hipStreamCaptureStatusNone;
  // FP32 takes 16-wave large-class workgroups (128 VGPRs each), FP64 8
  constexpr int kNwSmall = 4, kNwLarge = sizeof(R) == 4 ? 16 : 8;
  const int cap = a.cap;  // max_wake0 + 2H
  const Tune t_s = class_tune<R>(ctx, VPM_CLASS_SMALL), t_l = class_tune<R>(ctx, VPM_CLASS_LARGE);
  const Tune t_x = class_tune<R>(ctx, VPM_CLASS_STREAM);
  const int cap_small = lds_capacity<R, kNwSmall>(a.nb, a.n_inv, t_s.tmax, ctx->max_lds / 4);
  const int cap_large = lds_capacity<R, kNwLarge>(a.nb, a.n_inv, t_l.tmax, ctx->max_lds);
  const Queue none{nullptr, nullptr, nullptr, 0};
  const bool stream_only = path == VPM_PATH_STREAM;
  if (a.n_fields == 1 || path == VPM_PATH_LDS || stream_only) {
    if (!stream_only && cap <= cap_small)
      return launch_lds_tuned<R, MINW_S, kNwSmall>(ctx, a, cap, a.K, none, stream, t_s);
    if (!stream_only && cap <= cap_large)
      return launch_lds_tuned<R, 1, kNwLarge>(ctx, a, cap, a.K, none, stream, t_l);
    if (path == VPM_PATH_LDS)
      return fail(VPM_ECAPACITY, "wake capacity " + std::to_string(cap) +
                                     " does not fit the LDS-resident kernel");
    std::lock_guard<std::mutex> lock(ctx->ws_mu);
    if (ctx->ws_event_valid && !capturing)
      VPM_HIP_TRY(hipStreamWaitEvent(stream, ctx->ws_event, 0));
    const int grid = a.K < ctx->n_cu ? a.K : ctx->n_cu;
    int rc = launch_stream_tuned<R, NW_X>(ctx, a, grid, none, stream, capturing, t_x);
    if (rc != VPM_OK) return rc;
    if (!capturing) {
      VPM_HIP_TRY(hipEventRecord(ctx->ws_event, stream));
      ctx->ws_event_valid = true;
    }
    return VPM_OK;
  }

  // uneven batch: plan, then the class kernels
  std::lock_guard<std::mutex> lock(ctx->ws_mu);
  int rc = ensure_side_streams(ctx, capturing);
  if (rc != VPM_OK) return rc;
  if (ctx->ws_event_valid && !capturing)
    VPM_HIP_TRY(hipStreamWaitEvent(stream, ctx->ws_event, 0));
  const size_t plan_bytes = (size_t)a.K * sizeof(int32_t) + 64;
  rc = ensure_buffer(&ctx->plan, &ctx->plan_bytes, plan_bytes, "batch plan", capturing);
  if (rc != VPM_OK) return rc;
  int2 *range = static_cast<int2 *>(ctx->plan);
  int32_t *next = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->plan) + 32);
  int32_t *list = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->plan) + 64);
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, a.K, a.H,
                     a.max_wake0, a.n_fields, a.field_off, a.field_of, cap_small,
                     cap_large, list, range, next);
  VPM_HIP_TRY(hipGetLastError());
  VPM_HIP_TRY(hipEventRecord(ctx->fork_event, stream));
  hipEvent_t joins[kClasses];
  int n_join = 0;
  // class 0: streamed (only when some rollout can exceed the large class)
  if (cap > cap_large) {
    hipStream_t s = ctx->side[0];
    VPM_HIP_TRY(hipStreamWaitEvent(s, ctx->fork_event, 0));
    const int grid = a.K < ctx->n_cu ? a.K : ctx->n_cu;
    rc = launch_stream_tuned<R, NW_X>(ctx, a, grid, Queue{list, next, range, 0}, s, capturing,
                                      t_x);
    if (rc != VPM_OK) return rc;
    VPM_HIP_TRY(hipEventRecord(ctx->join_event[0], s));
    joins[n_join++] = ctx->join_event[0];
  }
  // class 1: large rollouts, 16-wave LDS workgroups, one per CU
  if (cap > cap_small) {
    hipStream_t s = ctx->side[1];
    VPM_HIP_TRY(hipStreamWaitEvent(s, ctx->fork_event, 0));
    const int c1 = cap < cap_large ? cap : cap_large;
    const int grid = a.K < ctx->n_cu ? a.K : ctx->n_cu;
    rc = launch_lds_tuned<R, 1, kNwLarge>(ctx, a, c1, grid, Queue{list, next, range, 1}, s, t_l);
    if (rc != VPM_OK) return rc;
    VPM_HIP_TRY(hipEventRecord(ctx->join_event[1], s));
    joins[n_join++] = ctx->join_event[1];
  }
  // class 2: small rollouts, 4-wave LDS workgroups, four per CU
  {
    hipStream_t s = ctx->side[2];
    VPM_HIP_TRY(hipStreamWaitEvent(s, ctx->fork_event, 0));
    const int c2 = cap < cap_small ? cap : cap_small;
    const int grid = a.K < 4 * ctx->n_cu ? a.K : 4 * ctx->n_cu;
    rc = launch_lds_tuned<R, MINW_S, kNwSmall>(ctx, a, c2, grid, Queue{list, next, range, 2}, s,
                                               t_s);
    if (rc != VPM_OK) return rc;
    VPM_HIP_TRY(hipEventRecord(ctx->join_event[2], s));
    joins[n_join++] = ctx->join_event[2];
  }
  for (int i = 0; i < n_join; ++i) VPM_HIP_TRY(hipStreamWaitEvent(stream, joins[i], 0));
  if (!capturing) {
    VPM_HIP_TRY(hipEventRecord(ctx->ws_event, stream));
    ctx->ws_event_valid = true;
  }
  return VPM_OK;
}

}  // namespace

int ensure_side_streams(vpm_ctx *ctx, bool capturing) {
  if (ctx->side[2]) return VPM_OK;
  if (capturing)
    return fail(VPM_EINVAL, "an eager uneven batch must run on this context before graph "
                            "capture");
  for (int i = 0; i < 3; ++i) {
    if (!ctx->side[i]) VPM_HIP_TRY(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
    if (!ctx->join_event[i])
      VPM_HIP_TRY(hipEventCreateWithFlags(&ctx->join_event[i], hipEventDisableTiming));
  }
  return VPM_OK;
}

// Grow a context buffer to `bytes` (device-synchronises before freeing a
// smaller one). Under graph capture nothing may be allocated: the buffer must
// already have been grown by an eager call of the same shape.
int ensure_buffer(void **buf, size_t *have, size_t bytes, const char *what,
                  bool capturing) {
  if (*have >= bytes) return VPM_OK;
  if (capturing)
    return fail(VPM_EINVAL, std::string("the ") + what +
                                " must be sized by an eager call before graph capture");
  if (*buf) {
    VPM_HIP_TRY(hipDeviceSynchronize());
    VPM_HIP_TRY(hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  if (hipMalloc(buf, bytes) != hipSuccess) {
    *buf = nullptr;
    return fail(VPM_ENOMEM, std::string("hipMalloc of the ") + what + " failed");
  }
  *have = bytes;
  return VPM_OK;
}

// Grow the context buffers that a batch of these sizes would need (the same
// class decisions as run_batch), outside any stream capture.
template <typename R>
int reserve_batch(vpm_ctx *ctx, int nb, int n_inv, int K, int cap, int n_fields) {
  constexpr int kNwLarge = sizeof(R) == 4 ? 16 : 8;
  const int cap_large =
      lds_capacity<R, kNwLarge>(nb, n_inv, class_tune<R>(ctx, VPM_CLASS_LARGE).tmax, ctx->max_lds);
  const int path = ctx->path;
  std::lock_guard<std::mutex> lock(ctx->ws_mu);
  if (path == VPM_PATH_STREAM || (path == VPM_PATH_AUTO && cap > cap_large)) {
    const int grid = K < ctx->n_cu ? K : ctx->n_cu;
    const size_t slot = (size_t)cap * (sizeof(typename SrcOf<R>::type) + sizeof(Vec2<R>));
    const int rc = ensure_buffer(&ctx->ws, &ctx->ws_bytes, slot * grid, "streaming workspace",
                                 false);
    if (rc != VPM_OK) return rc;
  }
  if (path == VPM_PATH_AUTO && n_fields > 1) {
    const size_t plan_bytes = (size_t)K * sizeof(int32_t) + 64;
    int rc = ensure_buffer(&ctx->plan, &ctx->plan_bytes, plan_bytes, "batch plan", false);
    if (rc == VPM_OK) rc = ensure_side_streams(ctx, false);
    if (rc != VPM_OK) return rc;
  }
  return VPM_OK;
}

int reserve_rollout(vpm_ctx *ctx, const vpm_params *p, int K, int H, int max_wake0,
                    int n_fields) {
  const int cap = max_wake0 + 2 * H;
  const int n_inv = inverse_entries(p);
  if (p->precision == VPM_FP64)
    return reserve_batch<double>(ctx, p->n_bound, n_inv, K, cap, n_fields);
  return reserve_batch<float>(ctx, p->n_bound, n_inv, K, cap, n_fields);
}

int lds_resident_capacity(int nb, int precision) {
  const int n_inv = (nb + 2) * (nb + 2);
  return precision == VPM_FP64 ? lds_capacity<double, 8>(nb, n_inv, 2, 163840)
                               : lds_capacity<float, 16>(nb, n_inv, 2, 163840);
}

int launch_rollout(vpm_ctx *ctx, const vpm_params *p, const vpm_batch_in *in,
                   vpm_batch_out *out, const double *kinv_t, const double *kinv_te,
                   hipStream_t stream, bool noalloc) {
  KArgs a{};
  a.K = in->K;
  a.H = in->H;
  a.nb = p->n_bound;
  a.S = system_size(p->n_bound, p->shed_mode);
  a.mode = p->shed_mode;
  a.gate = p->gate;
  a.alpha_crit = p->alpha_crit;
  a.split_b = in->K <= ctx->n_cu;
  a.n_inv = inverse_entries(p);
  a.n_wake_max = p->n_wake_max;
  a.max_wake0 = in->max_wake0;
  a.n_pairs = in->n_pairs;
  a.n_fields = in->n_fields;
  a.cap = in->max_wake0 + 2 * in->H;
  a.dt = in->dt;
  a.chord = p->chord;
  a.shed_frac = p->shed_frac;
  a.r_core = p->r_core;
  a.decay = p->decay;
  a.rho = p->rho;
  a.span = p->span;
  a.grav = p->grav;
  a.mass = p->mass;
  a.inertia = p->inertia;
  a.inv_dt = 1.0 / in->dt;
  a.inv_lb = p->n_bound / p->chord;
  a.lb = p->chord / p->n_bound;
  a.inv_mass = 1.0 / p->mass;
  a.inv_inertia = 1.0 / p->inertia;
  a.l_body = p->l_body;
  a.l_wing = p->l_wing;
  a.l_elev = p->l_elev;
  a.s_elev = p->s_elev;
  for (int i = 0; i < 7; ++i) {
    a.x_goal[i] = in->x_goal[i];
    a.q_diag[i] = in->q_diag[i];
  }
  a.g0 = in->g0;
  a.gb0 = in->gb0;
  a.wx = in->wx;
  a.wz = in->wz;
  a.wg = in->wg;
  a.u_mean = in->u_mean;
  a.u_eps = in->u_eps;
  a.kinv_t = kinv_t;
  a.kinv_te = p->gate ? kinv_te : nullptr;
  a.field_off = in->field_off;
  a.field_of = in->field_of;
  a.pairs = in->n_pairs > 0 ? in->pairs : nullptr;
  a.g_final = out->g_final;
  a.cost = out->cost;
  a.traj = out->traj;
  a.gamma_s = out->gamma_s;
  a.status = out->status;
  a.pair_count = out->pair_count;
  const bool wake = out->wake_off && out->n_final;
  a.wake_off = wake ? out->wake_off : nullptr;
  a.n_final = out->n_final;
  a.wx_out = wake ? out->wx : nullptr;
  a.wz_out = wake ? out->wz : nullptr;
  a.wg_out = wake ? out->wg : nullptr;
  a.vel_last = wake ? out->vel_last : nullptr;
  a.n_vel_last = out->n_vel_last;
  a.gb_final = out->gb_final;
  a.fb_gain = in->fb_gain;
  a.fb_xref = in->fb_gain ? in->fb_xref : nullptr;
  if (noalloc) {
    char *sc = static_cast<char *>(ctx->scratch);
    if (!sc) return fail(VPM_EDEVICE, "the library's static scratch is not mapped");
    if (p->precision == VPM_FP64)
      return run_batch_noalloc<double, 2, 8>(ctx, a, ctx->path, stream, sc, kScratchBytes);
    return run_batch_noalloc<float, 4, 16>(ctx, a, ctx->path, stream, sc, kScratchBytes);
  }
  if (p->precision == VPM_FP64)
    return run_batch<double, 2, 8>(ctx, a, ctx->path, stream);
  return run_batch<float, 4, 16>(ctx, a, ctx->path, stream);
}

// The scratch of vpm_rollout_batch_noalloc: device memory of the library
// itself, one copy per GPU the library runs on, held until the process ends.
// In host code `scratch` names a host-side stand-in; the device address of
// each GPU's copy comes from hipGetSymbolAddress (static_scratch_address).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

int static_scratch_address(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices)
    return fail(VPM_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int cur = -1;
    VPM_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) return fail(VPM_EDEVICE, "the device must be current");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(VPM_EDEVICE, std::string("hipGetSymbolAddress of the static scratch: ") +
                                   hipGetErrorString(e));
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return VPM_OK;
}

}  // namespace vpm
