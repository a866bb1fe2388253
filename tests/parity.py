"""Helpers shared by the GPU parity tests: run one workload through the HIP
library and through the CPU oracle on the same seeded inputs and compare."""
from dataclasses import replace

import numpy as np

from oracle import oracle as O
from paper_2509_16079_amd import vpm as V

TOL = {V.FP32C: 1e-4, V.FP64: 1e-10}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def run_oracle(wl, rollouts=None, **want):
    return O.rollout_batch(wl.params, wl.K, wl.H, wl.dt, wl.g0, wl.gb0, wl.field_off,
                           wl.field_of, wl.wx, wl.wz, wl.wg, wl.pairs, wl.u, wl.x_goal,
                           wl.q_diag, rollouts=rollouts, **want)


def wake_segments(out, k):
    o = out["out_off"][k]
    n = out["n_final"][k]
    return out["wx"][o:o + n], out["wz"][o:o + n], out["wg"][o:o + n]


def vel_segment(out, k):
    o = out["out_off"][k]
    n = out["n_vel_last"][k]
    return out["vel_last"][o:o + n]


def describe(tag, **errs):
    return tag + " " + " ".join("%s=%.3e" % kv for kv in errs.items())


def with_params(wl, **over):
    """The workload with some plate/glider parameters replaced."""
    p = dict(wl.params)
    p.update(over)
    return replace(wl, params=p, name=wl.name + "+" + ",".join(sorted(over)))


def gated_at_median(wl):
    """The workload with the separation gate on and the critical angle half
    way between the two middle wing angles of attack of the ungated oracle
    run, so that about half of the steps shed from the leading edge."""
    o = run_oracle(wl, traj=True)
    a = np.sort(O.wing_aoa(wl.params, o["traj"][:, :-1]).ravel())
    i = a.size // 2
    return with_params(wl, gate=1, alpha_crit=float(0.5 * (a[i - 1] + a[i])))


def gate_margin(wl, traj):
    """Smallest distance of a step's wing angle of attack from the critical
    angle along the trajectories traj [K, H + 1, 7]."""
    return float(np.min(np.abs(O.wing_aoa(wl.params, traj[:, :-1]) - wl.params["alpha_crit"])))
