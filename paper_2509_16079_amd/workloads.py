"""Seeded synthetic workloads shaped like the paper's rollouts.

This module draws inputs only: glider initial states, wake fields,
disturbance pairs and the MPPI control perturbations. It holds none of the
method's arithmetic, so both the GPU path and the CPU oracle can consume the
same arrays. Every floating-point value is rounded to the nearest float32 so
that the FP32 and FP64 paths start from identical inputs.

Random numbers come from numpy's counter-based Philox generator, seeded per
workload; the MPPI perturbations are inputs to the rollout (they are never
drawn inside it).

Physical constants that the paper uses only as symbols (Sec. III-B) take the
fixed values in ``GLIDER``; the numerical settings of each workload follow
the paper where it gives them (delta_s = 2 % of chord, Sec. III-A; the cost
goal and weights of Sec. IV-A and Sec. V-A) and are stated per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# Glider constants (Sec. III-B names them; the values are this project's).
GLIDER = dict(rho=1.225, span=0.5, grav=9.81, mass=0.12, inertia=2.0e-3,
              l_body=0.35, l_wing=0.08, l_elev=0.03, s_elev=0.02)

# Perch goal of Sec. IV-A and the position/pitch weights of Sec. V-A.
X_GOAL = np.array([3.5, 0.0, math.pi / 4, 0.0, 0.5, -0.5, 0.0])
Q_POS_PITCH = np.array([10.0, 10.0, 1.0, 0.0, 0.0, 0.0, 0.0])

SHED_BOTH, SHED_TE, SHED_NONE = 0, 1, 2


def f32(a):
    """Round to the nearest float32, returned as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def make_params(n_bound, *, chord=0.3, r_core=0.01, decay=0.1, n_wake_max=0,
                shed_mode=SHED_BOTH, prescribed=0, gate=0, alpha_crit=0.0, **over):
    p = dict(n_bound=int(n_bound), n_wake_max=int(n_wake_max), shed_mode=int(shed_mode),
             prescribed=int(prescribed), chord=float(chord), shed_frac=0.02,
             r_core=float(r_core), decay=float(decay), gate=int(gate),
             alpha_crit=float(alpha_crit))
    p.update(GLIDER)
    p.update(over)
    for k, v in list(p.items()):
        if isinstance(v, float):
            p[k] = float(f32(v))
    return p


@dataclass
class Workload:
    """One batch of K rollouts of H steps (layout of the rollout entry point)."""
    name: str
    params: dict
    K: int
    H: int
    dt: float
    g0: np.ndarray          # [K, 7]  (x, z, theta, phi, xd, zd, thetad)
    gb0: np.ndarray         # [K, N_b] bound circulations carried in the state
    field_off: np.ndarray   # [F + 1]  int64 CSR offsets of the wake fields
    field_of: np.ndarray    # [K]      int32 field of each rollout
    wx: np.ndarray          # [N]      wake x, oldest first within a field
    wz: np.ndarray          # [N]
    wg: np.ndarray          # [N]      circulation
    pairs: np.ndarray       # [K, 2P]  int32 disturbance pair indices or -1
    u_mean: np.ndarray      # [H]      mean elevator-rate sequence
    u_eps: np.ndarray       # [K, H]   perturbations (MPPI samples)
    x_goal: np.ndarray = field(default_factory=lambda: X_GOAL.copy())
    q_diag: np.ndarray = field(default_factory=lambda: Q_POS_PITCH.copy())
    lam: float = 1.0
    precision: str = "fp32"
    meta: dict = field(default_factory=dict)

    @property
    def n0(self) -> np.ndarray:
        fo = self.field_of
        return (self.field_off[fo + 1] - self.field_off[fo]).astype(np.int64)

    @property
    def u(self) -> np.ndarray:
        return self.u_mean[None, :] + self.u_eps

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        return replace(self, K=int(idx.size), g0=self.g0[idx], gb0=self.gb0[idx],
                       field_of=self.field_of[idx],
                       pairs=self.pairs[idx], u_eps=self.u_eps[idx])


def _rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def _glider0(K, speed):
    g = np.zeros((K, 7))
    g[:, 4] = speed
    return f32(g)


def _pair(x, zc, gamma, sep=0.25):
    """Counter-rotating pair moving toward -x: top vortex clockwise (-gamma),
    bottom vortex counter-clockwise (+gamma)."""
    return (np.array([x, x]), np.array([zc + 0.5 * sep, zc - 0.5 * sep]),
            np.array([-gamma, gamma]))


def _eps(rng, K, H, sigma):
    return f32(rng.normal(0.0, sigma, size=(K, H)))


def _one_field(K, wx, wz, wg, pair_idx, H, n_pairs=1):
    field_off = np.array([0, len(wx)], dtype=np.int64)
    field_of = np.zeros(K, dtype=np.int32)
    pairs = np.full((K, 2 * n_pairs), -1, dtype=np.int32)
    for q, (a, b) in enumerate(pair_idx):
        pairs[:, 2 * q] = a
        pairs[:, 2 * q + 1] = b
    return field_off, field_of, pairs


def plain_single_plan(seed=0, K=32, H=100):
    """Plain FP64 single plan: K MPPI rollouts of H steps at dt = 5 ms, chord
    0.3 m with 16 bound vortices, 6 m/s level start, a +-0.4 m^2/s vortex pair
    0.25 m apart 2 m ahead, core radius 0.01 m, perturbations N(0, 0.15),
    merging above 200 wake vortices, lambda = 1."""
    rng = _rng(seed)
    p = make_params(16, n_wake_max=200)
    x, z, g = _pair(2.0, 0.0, 0.4)
    wx, wz, wg = f32(x), f32(z), f32(g)
    fo, fof, pairs = _one_field(K, wx, wz, wg, [(0, 1)], H)
    return Workload("plain_fp64_K32_H100", p, K, H, float(f32(0.005)), _glider0(K, 6.0),
                    np.zeros((K, 16)), fo, fof, wx, wz, wg, pairs,
                    np.zeros(H), _eps(rng, K, H, 0.15), precision="fp64")


def realtime(seed=1, K=1024, H=200):
    """FP32-vs-FP64 real-time size: K rollouts of H steps at dt = 2.5 ms,
    32 bound vortices, merging above 800, one disturbance pair with strength
    U(0.2, 0.8) at x ~ U(1.5, 2.5), centre z ~ U(-0.3, 0.3), shared by all
    rollouts."""
    rng = _rng(seed)
    p = make_params(32, n_wake_max=800)
    gam = rng.uniform(0.2, 0.8)
    xp = rng.uniform(1.5, 2.5)
    zc = rng.uniform(-0.3, 0.3)
    x, z, g = _pair(xp, zc, gam)
    wx, wz, wg = f32(x), f32(z), f32(g)
    fo, fof, pairs = _one_field(K, wx, wz, wg, [(0, 1)], H)
    return Workload("realtime_K%d_H%d" % (K, H), p, K, H, float(f32(0.0025)),
                    _glider0(K, 6.0), np.zeros((K, 32)), fo, fof, wx, wz, wg,
                    pairs, np.zeros(H), _eps(rng, K, H, 0.15),
                    meta=dict(pair_gamma=float(gam), pair_x=float(xp), pair_zc=float(zc)))


# Runtime-versus-batch table of the paper (Sec. III-C, Table I): 80 steps at
# dt = 10 ms, at most 60 wake particles before merging; batch sizes 1..1024.
TABLE1_BATCHES = (1, 128, 256, 512, 1024)
TABLE1_PAPER_MS = (8.0, 10.3, 12.2, 16.3, 27.2)   # RTX 5080, as printed


def table1(K, seed=7, n_bound=32):
    """The Table I configuration at batch K: H = 80, dt = 10 ms, merging
    above 60 wake vortices, 7 m/s level start (Sec. IV-A), one disturbance
    pair as in the realtime batch, perturbations N(0, 0.15^2). The paper does
    not state N_b for this run; 32 bound vortices are used."""
    rng = _rng(seed)
    H = 80
    p = make_params(n_bound, n_wake_max=60)
    gam = rng.uniform(0.2, 0.8)
    xp = rng.uniform(1.5, 2.5)
    zc = rng.uniform(-0.3, 0.3)
    x, z, g = _pair(xp, zc, gam)
    wx, wz, wg = f32(x), f32(z), f32(g)
    fo, fof, pairs = _one_field(K, wx, wz, wg, [(0, 1)], H)
    return Workload("table1_K%d" % K, p, K, H, float(f32(0.01)), _glider0(K, 7.0),
                    np.zeros((K, n_bound)), fo, fof, wx, wz, wg, pairs, np.zeros(H),
                    _eps(rng, K, H, 0.15))


# Perturbation scales of the policy rollouts (the paper tunes its
# covariances by sweeps and does not print them): positions 1 cm, angles
# 0.01 rad, velocities 0.05 m/s, pitch rate 0.05 rad/s; controls 0.15.
POLICY_SIGMA_X = np.array([0.01, 0.01, 0.01, 0.01, 0.05, 0.05, 0.05])
POLICY_SIGMA_U = 0.15


def policy_batch(seed=5, K=256, H=77, dt=0.01, n_bound=32):
    """Rollouts for the local feedback policy (Sec. IV-B) at the size of the
    paper's controller (MPPI batch 256, 77-step nominal, dt = 10 ms): rollout
    0 is the nominal (7 m/s level start, elevator-rate sequence u_mean, no
    perturbation); rollouts 1..K start from N(x_0, diag(POLICY_SIGMA_X)^2)
    with controls u_mean + N(0, POLICY_SIGMA_U^2); one disturbance pair as in
    the realtime batch. Returns a Workload of K + 1 rollouts."""
    rng = _rng(seed)
    p = make_params(n_bound, n_wake_max=800)
    gam = rng.uniform(0.2, 0.8)
    xp = rng.uniform(1.5, 2.5)
    zc = rng.uniform(-0.3, 0.3)
    x, z, g = _pair(xp, zc, gam)
    wx, wz, wg = f32(x), f32(z), f32(g)
    fo, fof, pairs = _one_field(K + 1, wx, wz, wg, [(0, 1)], H)
    g0 = np.zeros((K + 1, 7))
    g0[:, 4] = 7.0
    g0[1:] += rng.normal(size=(K, 7)) * POLICY_SIGMA_X
    eps = np.zeros((K + 1, H))
    eps[1:] = rng.normal(0.0, POLICY_SIGMA_U, size=(K, H))
    # elevator-rate sequence that pitches the glider up to about 40 degrees
    # while it slows from 7 to about 4 m/s, a perch-like manoeuvre
    u_mean = f32(-1.5 * np.sin(np.linspace(0.0, np.pi, H)))
    return Workload("policy_K%d_H%d" % (K, H), p, K + 1, H, float(f32(dt)), f32(g0),
                    np.zeros((K + 1, n_bound)), fo, fof, wx, wz, wg, pairs, u_mean, f32(eps),
                    precision="fp64",
                    meta=dict(pair_gamma=float(gam), pair_x=float(xp), pair_zc=float(zc)))


# Weights of the paper's controller experiments (Sec. V-A): the NMPC cost
# and the TVLQR weights.
Q_NMPC = np.array([10.0, 10.0, 1.0, 0.0, 0.2, 0.2, 0.2])
TVLQR_Q_F = np.array([400.0, 400.0, 10.0, 1.0, 1.0, 1.0, 1.0])
TVLQR_Q_C = np.array([0.1, 0.1, 5.0, 0.1, 0.1, 0.1, 5.0])
TVLQR_R_C = 0.01


def replan_case(seed=6, K=256, H=77, P=10, iterations=3, Kp=256, n_bound=32, dt=0.01):
    """Inputs of one replanning cycle at the paper's controller size (MPPI
    batch 256, 3 iterations, 77-step plan, dt = 10 ms, replanning every
    100 ms = 10 steps): the resident state is the 7 m/s level start with one
    disturbance pair ahead (as in the realtime batch) and no shed wake yet,
    the plan in force is the pitch-up of policy_batch (open loop), MPPI
    perturbations N(0, 0.15^2), policy perturbations as in policy_batch.
    Returns a dict of numpy arrays (rounded to binary32 like every input)."""
    rng = _rng(seed)
    p = make_params(n_bound, n_wake_max=0)
    gam = rng.uniform(0.2, 0.8)
    xp = rng.uniform(1.5, 2.5)
    zc = rng.uniform(-0.3, 0.3)
    x, z, g = _pair(xp, zc, gam)
    g0 = np.zeros(7)
    g0[4] = 7.0
    return dict(
        params=p, dt=float(f32(dt)), H=H, P=P, K=K, iterations=iterations, Kp=Kp,
        g=f32(g0), gb=np.zeros(n_bound), wx=f32(x), wz=f32(z), wg=f32(g),
        pairs=np.array([0, 1], dtype=np.int32),
        u_plan=f32(-1.5 * np.sin(np.linspace(0.0, np.pi, H))),
        u_eps=f32(rng.normal(0.0, 0.15, size=(iterations, K, H))),
        x_eps=f32(rng.normal(size=(Kp, 7)) * POLICY_SIGMA_X),
        du=f32(rng.normal(0.0, POLICY_SIGMA_U, size=(Kp, H))),
        lam=1.0, x_goal=X_GOAL.copy(), q_diag=Q_NMPC.copy(), q_f=TVLQR_Q_F.copy(),
        q_c=TVLQR_Q_C.copy(), r_c=TVLQR_R_C)


def random_field(rng, n, box=(0.0, 3.0, -0.5, 0.5), sigma_gamma=0.05):
    """n vortices uniform in the box with N(0, sigma^2) strengths, shifted to
    zero total circulation (the paper's flow starts at zero circulation)."""
    x = rng.uniform(box[0], box[1], size=n)
    z = rng.uniform(box[2], box[3], size=n)
    g = rng.normal(0.0, sigma_gamma, size=n)
    g = g - g.mean()
    return f32(x), f32(z), f32(g)


def uneven_batch(seed=2, K=4096, H=100, n_min=50, n_max=4000):
    """Uneven batch: each rollout has its own initial wake with a log-uniform
    count in [n_min, n_max], positions in a 3 m x 1 m box, strengths
    N(0, 0.05^2); H steps at dt = 5 ms, 32 bound vortices, no merging."""
    rng = _rng(seed)
    p = make_params(32, n_wake_max=0)
    n0 = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=K))).astype(np.int64)
    xs, zs, gs = [], [], []
    for k in range(K):
        x, z, g = random_field(rng, int(n0[k]))
        xs.append(x)
        zs.append(z)
        gs.append(g)
    off = np.zeros(K + 1, dtype=np.int64)
    off[1:] = np.cumsum(n0)
    return Workload("uneven_K%d_H%d" % (K, H), p, K, H, float(f32(0.005)), _glider0(K, 6.0),
                    np.zeros((K, 32)), off, np.arange(K, dtype=np.int32),
                    np.concatenate(xs), np.concatenate(zs), np.concatenate(gs),
                    np.full((K, 2), -1, dtype=np.int32), np.zeros(H), _eps(rng, K, H, 0.15))


def lamb_oseen_sheet(rng, per_blob=1023, r_lo=0.05, gamma0=0.3, n_pairs=4):
    """Two rows of 8 Lamb-Oseen vortices (z = +-0.15 m, x = 1.0 ... 2.75 m
    every 0.25 m, -gamma0 on the top row, +gamma0 below), each sampled as
    per_blob particles from its Gaussian vorticity (sigma = r_lo / sqrt 2 per
    axis) carrying gamma0 / per_blob each; plus n_pairs disturbance pairs of
    strength U(0.2, 0.8) at x ~ U(1.0, 3.0), centre z ~ U(-0.3, 0.3). The
    pairs come first in the field; returns (x, z, g, pair index list)."""
    sig = r_lo / math.sqrt(2.0)
    xs, zs, gs, pidx = [], [], [], []
    for q in range(n_pairs):
        x, z, g = _pair(rng.uniform(1.0, 3.0), rng.uniform(-0.3, 0.3), rng.uniform(0.2, 0.8))
        xs.append(x)
        zs.append(z)
        gs.append(g)
        pidx.append((2 * q, 2 * q + 1))
    for row, (zc, sgn) in enumerate(((0.15, -1.0), (-0.15, 1.0))):
        for i in range(8):
            xc = 1.0 + 0.25 * i
            xs.append(xc + rng.normal(0.0, sig, size=per_blob))
            zs.append(zc + rng.normal(0.0, sig, size=per_blob))
            gs.append(np.full(per_blob, sgn * gamma0 / per_blob))
    return (f32(np.concatenate(xs)), f32(np.concatenate(zs)), f32(np.concatenate(gs)), pidx)


def large_stress(seed=4, K=8192, H=150, per_blob=1023):
    """Large stress: K rollouts of H steps at dt = 5 ms, 64 bound vortices,
    merging above 16384, all starting from one Lamb-Oseen wake field of
    16 * per_blob particles plus 4 disturbance pairs."""
    rng = _rng(seed)
    p = make_params(64, n_wake_max=16384)
    wx, wz, wg, pidx = lamb_oseen_sheet(rng, per_blob=per_blob)
    fo, fof, pairs = _one_field(K, wx, wz, wg, pidx, H, n_pairs=len(pidx))
    return Workload("stress_K%d_H%d" % (K, H), p, K, H, float(f32(0.005)), _glider0(K, 6.0),
                    np.zeros((K, 64)), fo, fof, wx, wz, wg, pairs, np.zeros(H),
                    _eps(rng, K, H, 0.15))


@dataclass
class Request:
    """One replanning request of the serving trace."""
    t_arrive: float      # seconds from trace start
    state: int           # index of the resident state it plans from
    K: int
    H: int
    seed: int


def serving_trace(seed=3, n_requests=300, rate=100.0, n_states=16, k_range=(256, 2048),
                  h_range=(50, 200), n_range=(500, 6000)):
    """Replanning trace: Poisson arrivals at `rate` req/s; each request picks
    one of n_states resident fluid states (counts U{n_range}, generated like
    the uneven batch) and draws K ~ U{k_range}, H ~ U{h_range}. Returns
    (params, states, requests) with states a list of (wx, wz, wg)."""
    rng = _rng(seed)
    p = make_params(32, n_wake_max=0)
    states = []
    for _ in range(n_states):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        states.append(random_field(rng, n))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = []
    for i in range(n_requests):
        reqs.append(Request(float(t[i]), int(rng.integers(0, n_states)),
                            int(rng.integers(k_range[0], k_range[1] + 1)),
                            int(rng.integers(h_range[0], h_range[1] + 1)),
                            int(rng.integers(0, 2**31 - 1))))
    return p, states, reqs


def request_eps(req: Request, sigma=0.15):
    """The perturbations [K, H] of one request, from its own seed."""
    return _eps(_rng(req.seed), req.K, req.H, sigma)


def workload_from_state(name, params, state, K, H, eps, dt=0.005, speed=6.0):
    """A batch of K rollouts that all start from one resident wake state."""
    wx, wz, wg = state
    nb = params["n_bound"]
    fo = np.array([0, len(wx)], dtype=np.int64)
    return Workload(name, params, K, H, float(f32(dt)), _glider0(K, speed), np.zeros((K, nb)), fo, np.zeros(K, dtype=np.int32), wx, wz, wg,
                    np.full((K, 2), -1, dtype=np.int32), np.zeros(H), eps)


def pair_count(n0, H, n_bound, shed=2, n_wake_max=0):
    """Exact pair-interaction count of one rollout from its wake-count schedule
    (the method's own work, not what an implementation happens to evaluate):
    per step, N_w (2 N_b + 1) regularised pairs at the surface points,
    N_w' (N_w' - 1) regularised wake-wake pairs (N_w' = N_w + shed) and
    N_w' N_b singular wake-bound pairs. Returns (regularised, singular)."""
    reg = 0
    sing = 0
    n = int(n0)
    for _ in range(H):
        reg += n * (2 * n_bound + 1)
        m = n + shed
        reg += m * (m - 1)
        sing += m * n_bound
        n = m
        if n_wake_max > 0:
            while n > n_wake_max:
                n -= 1
    return reg, sing
