"""Self-sensitivity of the rollout map, measured on the FP64 oracle alone.

The oracle is run twice on the same inputs, once summing every interaction
list front to back and once back to front. The two differ by rounding only
(~1e-16 relative per step); D(n), the relative L2 gap of the glider states
after n steps, shows how much the dynamics amplify rounding. A horizon is
usable for an FP64 parity bar `tol` when D(n) stays well below `tol`, and for
FP32 when D(n) times 2**29 (the FP32/FP64 rounding ratio) does.

For the large stress field (16376 vortices, too slow to rerun in the CPU
suite) the script also records S(n), the relative L2 gap between the FP64
oracle and its binary32-storage variant (state rounded to float after every
step), which bounds the FP32 error any FP32-state implementation can reach.

Usage: python tests/golden/conditioning.py [--stress-only]
  -> writes conditioning.txt (and conditioning_stress.txt) here.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2509_16079_amd import workloads as W  # noqa: E402


def _traj(wl, H, **kw):
    return O.rollout_batch(wl.params, wl.K, H, wl.dt, wl.g0, wl.gb0, wl.field_off,
                           wl.field_of, wl.wx, wl.wz, wl.wg, wl.pairs, wl.u[:, :H],
                           wl.x_goal, wl.q_diag, traj=True, **kw)["traj"]


def _gap(a, b):
    return np.array([float(np.linalg.norm(a[:, n] - b[:, n]) / np.linalg.norm(a[:, n]))
                     for n in range(a.shape[1])])


def divergence_curve(wl, H=None):
    H = wl.H if H is None else H
    return _gap(_traj(wl, H), _traj(wl, H, reverse=True))


def stress_curves(H=150, rollouts=(0, 2730, 5460, 8190)):
    """D(n) and S(n) on rollouts of the large stress batch."""
    wl = W.large_stress(K=8192, H=H).subset(np.asarray(rollouts))
    a = _traj(wl, H)
    return _gap(a, _traj(wl, H, reverse=True)), _gap(a, _traj(wl, H, f32_state=True))


def read_stress(path=None):
    """{"D": array, "S": array, "step": int} from conditioning_stress.txt."""
    path = path or os.path.join(HERE, "conditioning_stress.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        key, _, vals = line.partition(":")
        name, step = key.split()[0], int(key.split("step")[1])
        out[name] = np.array([float(v) for v in vals.split()])
        out["step"] = step
    return out


CASES = {
    "plain_fp64_K32_H100": lambda: W.plain_single_plan(K=8),
    "realtime_K1024_H200": lambda: W.realtime(K=8, H=200),
    "uneven_K4096_H100": lambda: W.uneven_batch(K=4096, H=100).subset(np.arange(0, 4096, 512)),
}


def main_stress():
    d, s32 = stress_curves()
    lines = ["# Large stress batch (K=8192, H=150, N_b=64, 16376-vortex field), rollouts",
             "# 0, 2730, 5460, 8190. D: oracle forward vs reverse summation (FP64);",
             "# S: oracle vs its binary32-storage variant. Relative L2 of glider states,",
             "# n = 0..150. Written by tests/golden/conditioning.py.",
             "D step 5: " + " ".join("%.2e" % v for v in d[::5]),
             "S step 5: " + " ".join("%.2e" % v for v in s32[::5])]
    print("\n".join(lines), flush=True)
    with open(os.path.join(HERE, "conditioning_stress.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    lines = ["# D(n): relative L2 gap of glider states, oracle forward vs reverse summation",
             "# (8 rollouts of each workload). Written by tests/golden/conditioning.py."]
    for name, make in CASES.items():
        wl = make()
        d = divergence_curve(wl)
        lines.append("%s n=0..%d step 10: %s" % (
            name, wl.H, " ".join("%.2e" % v for v in d[::10])))
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "conditioning.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if "--stress-only" not in sys.argv:
        main()
    main_stress()
