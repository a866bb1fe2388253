"""ctypes wrapper of the plain FP64 CPU oracle (``vpm_oracle.c``).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.

The oracle follows Gupta et al., arXiv 2509.16079: Sec. III-A (vortex
particle model, Eqs. 4-17), Sec. III-B (glider dynamics), Sec. IV-A (cost and
MPPI, Eqs. 24-25) and Sec. V (disturbance termination).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vpm_oracle.c")
LIB = os.path.join(HERE, "libvpm_oracle.so")
LIB_F32 = os.path.join(HERE, "libvpm_oracle_f32state.so")

SHED_BOTH, SHED_TE, SHED_NONE = 0, 1, 2
OK, NONFINITE, CAPACITY, SINGULAR = 0, 1, 2, 4


class Params(C.Structure):
    _fields_ = [
        ("n_bound", C.c_int32),
        ("n_wake_max", C.c_int32),
        ("shed_mode", C.c_int32),
        ("prescribed", C.c_int32),
        ("chord", C.c_double),
        ("shed_frac", C.c_double),
        ("r_core", C.c_double),
        ("decay", C.c_double),
        ("rho", C.c_double),
        ("span", C.c_double),
        ("grav", C.c_double),
        ("mass", C.c_double),
        ("inertia", C.c_double),
        ("l_body", C.c_double),
        ("l_wing", C.c_double),
        ("l_elev", C.c_double),
        ("s_elev", C.c_double),
        ("alpha_crit", C.c_double),
        ("gate", C.c_int32),
        ("lev_literal", C.c_int32),
    ]


def _stale(path):
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no fast-math, no contraction),
    and its binary32-state variant."""
    for path, extra in ((LIB, []), (LIB_F32, ["-DORC_F32_STATE"])):
        if force or _stale(path):
            cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                   "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"] + extra + \
                  [SRC, "-o", path + ".tmp", "-lm"]
            subprocess.check_call(cmd)
            os.replace(path + ".tmp", path)
    return LIB


_libs = {}


def lib(f32_state: bool = False):
    path = LIB_F32 if f32_state else LIB
    if path not in _libs:
        if _stale(path):
            build(force=True)
        L = C.CDLL(path)
        d, i32, P = C.c_double, C.c_int32, C.c_void_p
        L.orc_kernel_sing.argtypes = [d, d, P, P]
        L.orc_kernel_reg.argtypes = [d, d, d, P, P]
        L.orc_wake_velocities.argtypes = [i32, P, P, P, i32, P, P, P, d, i32, P, P]
        L.orc_advect.argtypes = [i32, P, P, P, P, P, d, d]
        L.orc_plate_geometry.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.orc_system_size.argtypes = [i32, i32]
        L.orc_system_size.restype = i32
        L.orc_surface_matrix.argtypes = [P, P, i32, P]
        L.orc_solve.argtypes = [i32, P, P, P]
        L.orc_solve.restype = i32
        L.orc_plate_solve_pose.argtypes = [P, P, P, d, i32, P]
        L.orc_plate_solve_pose.restype = i32
        L.orc_elevator.argtypes = [P, P, d, P, P]
        L.orc_elevator.restype = d
        L.orc_segment_hits_plate.argtypes = [P, P, P, P]
        L.orc_segment_hits_plate.restype = i32
        L.orc_rollout_batch.argtypes = ([P, i32, i32, d] + [P] * 8 + [i32] + [P] * 3 + [i32, i32]
                                        + [P] * 16)
        L.orc_rollout_batch.restype = i32
        L.orc_cost.argtypes = [P, P, P]
        L.orc_cost.restype = d
        L.orc_mppi.argtypes = [i32, i32, P, d, P, P, P, P, P, P]
        L.orc_wing_aoa.argtypes = [P, P]
        L.orc_wing_aoa.restype = d
        _libs[path] = L
    return _libs[path]


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        optional = name in ("gate", "alpha_crit", "lev_literal")
        setattr(p, name, d.get(name, 0) if optional else d[name])
    return p


def kernel_sing(dx, dz):
    kx, kz = np.zeros(1), np.zeros(1)
    lib().orc_kernel_sing(dx, dz, _p(kx), _p(kz))
    return kx[0], kz[0]


def kernel_reg(dx, dz, r_core):
    kx, kz = np.zeros(1), np.zeros(1)
    lib().orc_kernel_reg(dx, dz, r_core, _p(kx), _p(kz))
    return kx[0], kz[0]


def wake_velocities(wx, wz, wg, bx=None, bz=None, bg=None, r_core=0.01, reverse=False):
    wx, wz, wg = _f64(wx), _f64(wz), _f64(wg)
    n = wx.size
    if bx is None:
        bx = bz = bg = np.zeros(0)
    bx, bz, bg = _f64(bx), _f64(bz), _f64(bg)
    vx, vz = np.zeros(n), np.zeros(n)
    lib().orc_wake_velocities(n, _p(wx), _p(wz), _p(wg), bx.size, _p(bx), _p(bz), _p(bg),
                              r_core, int(reverse), _p(vx), _p(vz))
    return vx, vz


def advect(wx, wz, wg, vx, vz, dt, decay):
    """In-place Euler advection and decay; returns the arrays."""
    wx, wz, wg = _f64(wx).copy(), _f64(wz).copy(), _f64(wg).copy()
    vx, vz = _f64(vx), _f64(vz)
    lib().orc_advect(wx.size, _p(wx), _p(wz), _p(wg), _p(vx), _p(vz), dt, decay)
    return wx, wz, wg


def plate_geometry(params: dict, g):
    p = make_params(params)
    nb = params["n_bound"]
    g = _f64(g)
    out = dict(x_w=np.zeros(2), xw_dot=np.zeros(2), rc=np.zeros((nb + 1, 2)),
               rb=np.zeros((nb, 2)), r_lev=np.zeros(2), r_tev=np.zeros(2),
               n_hat=np.zeros(2), t_hat=np.zeros(2))
    lib().orc_plate_geometry(C.byref(p), _p(g), *[_p(out[k]) for k in
                             ("x_w", "xw_dot", "rc", "rb", "r_lev", "r_tev", "n_hat", "t_hat")])
    return out


def wing_aoa(params: dict, g) -> np.ndarray:
    """Sec. III-A: the wing's angle of attack (pitch minus the direction of
    the wing point's velocity) in each state of g [..., 7]."""
    p = make_params(params)
    g = _f64(g)
    flat = g.reshape(-1, 7)
    out = np.array([lib().orc_wing_aoa(C.byref(p), _p(np.ascontiguousarray(r))) for r in flat])
    return out.reshape(g.shape[:-1])


def system_size(n_bound, shed_mode=SHED_BOTH):
    return lib().orc_system_size(n_bound, shed_mode)


def surface_matrix(params: dict, g, shed_mode=SHED_BOTH):
    p = make_params(params)
    S = system_size(params["n_bound"], shed_mode)
    a = np.zeros((S, S))
    lib().orc_surface_matrix(C.byref(p), _p(_f64(g)), shed_mode, _p(a))
    return a


def solve(a, b):
    a = _f64(a).copy()
    b = _f64(b).copy()
    x = np.zeros(b.size)
    rc = lib().orc_solve(b.size, _p(a), _p(b), _p(x))
    if rc != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return x


def plate_solve_pose(params: dict, pose6, vw_c, sum_gw, shed_mode=SHED_BOTH):
    p = make_params(params)
    S = system_size(params["n_bound"], shed_mode)
    gs = np.zeros(S)
    rc = lib().orc_plate_solve_pose(C.byref(p), _p(_f64(pose6)), _p(_f64(vw_c)),
                                    float(sum_gw), shed_mode, _p(gs))
    return gs, rc


def elevator(params: dict, g, u):
    p = make_params(params)
    xe, fe = np.zeros(2), np.zeros(2)
    alpha = lib().orc_elevator(C.byref(p), _p(_f64(g)), float(u), _p(xe), _p(fe))
    return alpha, xe, fe


def segment_hits_plate(params: dict, g, a, b):
    p = make_params(params)
    return bool(lib().orc_segment_hits_plate(C.byref(p), _p(_f64(g)), _p(_f64(a)), _p(_f64(b))))


def cost(g_final, x_goal, q_diag):
    return lib().orc_cost(_p(_f64(g_final)), _p(_f64(x_goal)), _p(_f64(q_diag)))


def mppi(cost_arr, lam, mu, xi):
    cost_arr = _f64(cost_arr)
    xi = _f64(xi)
    mu = _f64(mu)
    K, H = xi.shape
    w, xs = np.zeros(K), np.zeros(H)
    am = np.zeros(1, dtype=np.int32)
    jm = np.zeros(1)
    lib().orc_mppi(K, H, _p(cost_arr), float(lam), _p(mu), _p(xi), _p(w), _p(xs), _p(am), _p(jm))
    return dict(w=w, xi_star=xs, argmin=int(am[0]), j_min=float(jm[0]))


def rollout_batch(params: dict, K, H, dt, g0, gb0, field_off, field_of, wx, wz, wg,
                  pairs, u, x_goal, q_diag, *, traj=False, gamma_s=False, force=False,
                  final_wake=False, vel_last=False, reverse=False, n_threads=0,
                  rollouts=None, f32_state=False, fb_gain=None, fb_xref=None,
                  gb_final=False):
    """Run the oracle on rollouts ``rollouts`` (default: all K) of a batch.

    Inputs follow the layout of ``orc_rollout_batch``; ``u`` is the full
    control (mean + perturbation), shape [K, H]. Returns a dict of numpy
    arrays indexed by position in ``rollouts``. ``f32_state`` runs the
    binary32-storage variant. ``fb_gain`` [H, 7] and ``fb_xref`` [H, 7]
    close the loop with the policy of Sec. IV-B: the control of step n is
    u[k, n] - fb_gain[n] . (x_n - fb_xref[n]).
    """
    p = make_params(params)
    nb = params["n_bound"]
    S = system_size(nb, params["shed_mode"])
    idx = np.arange(K) if rollouts is None else np.asarray(rollouts, dtype=np.int64)
    k = idx.size
    g0 = _f64(np.asarray(g0)[idx])
    gb0 = _f64(np.asarray(gb0)[idx])
    field_off = np.ascontiguousarray(field_off, dtype=np.int64)
    fo = np.arange(K, dtype=np.int32) if field_of is None else np.asarray(field_of, dtype=np.int32)
    fo = np.ascontiguousarray(fo[idx], dtype=np.int32)
    n_pairs = 0 if pairs is None else np.asarray(pairs).shape[1] // 2
    pr = None if pairs is None else np.ascontiguousarray(np.asarray(pairs)[idx], dtype=np.int32)
    u = _f64(np.asarray(u)[idx])
    wx, wz, wg = _f64(wx), _f64(wz), _f64(wg)
    out = dict(g_final=np.zeros((k, 7)), cost=np.zeros(k), status=np.zeros(k, dtype=np.int32))
    if gb_final:
        out["gb_final"] = np.zeros((k, nb))
    fbg = None if fb_gain is None else _f64(fb_gain)
    fbx = None if fb_gain is None else _f64(fb_xref)
    if traj:
        out["traj"] = np.zeros((k, H + 1, 7))
    if gamma_s:
        out["gamma_s"] = np.zeros((k, H, S))
    if force:
        out["force"] = np.zeros((k, H, 3))
    shed = {SHED_BOTH: 2, SHED_TE: 1, SHED_NONE: 0}[params["shed_mode"]]
    n0 = (field_off[fo + 1] - field_off[fo]).astype(np.int64)
    out_off = np.zeros(k + 1, dtype=np.int64)
    out_off[1:] = np.cumsum(n0 + shed * H)
    want_w = final_wake or vel_last
    if want_w:
        tot = int(out_off[-1])
        if final_wake:
            out["wx"], out["wz"], out["wg"] = np.zeros(tot), np.zeros(tot), np.zeros(tot)
        out["n_final"] = np.zeros(k, dtype=np.int32)
        if vel_last:
            out["vel_last"] = np.zeros((tot, 2))
            out["n_vel_last"] = np.zeros(k, dtype=np.int32)
        out["out_off"] = out_off
    lib(f32_state).orc_rollout_batch(
        C.byref(p), k, H, float(dt), _p(g0), _p(gb0), _p(field_off), _p(fo),
        _p(wx), _p(wz), _p(wg), _p(pr), n_pairs, _p(u), _p(_f64(x_goal)), _p(_f64(q_diag)),
        int(reverse), int(n_threads), _p(out["g_final"]), _p(out["cost"]), _p(out["status"]),
        _p(out.get("traj")), _p(out.get("gamma_s")), _p(out.get("force")),
        _p(out_off) if want_w else None, _p(out.get("wx")), _p(out.get("wz")), _p(out.get("wg")),
        _p(out.get("n_final")), _p(out.get("vel_last")), _p(out.get("n_vel_last")),
        _p(fbg), _p(fbx), _p(out.get("gb_final")))
    return out
