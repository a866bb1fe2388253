"""Helpers shared by the GPU parity tests: run one workload through the HIP
library and through the CPU oracle on the same seeded inputs and compare."""
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
