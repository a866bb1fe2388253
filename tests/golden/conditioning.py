"""Self-sensitivity of the rollout map, measured on the FP64 oracle alone.

The oracle is run twice on the same inputs, once summing every interaction
list front to back and once back to front. The two differ by rounding only
(~1e-16 relative per step); D(n), the relative L2 gap of the glider states
after n steps, shows how much the dynamics amplify rounding. A horizon is
usable for an FP64 parity bar `tol` when D(n) stays well below `tol`, and for
FP32 when D(n) times 2**29 (the FP32/FP64 rounding ratio) does.

Usage: python tests/golden/conditioning.py  -> writes conditioning.txt here.
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


def divergence_curve(wl, H=None):
    H = wl.H if H is None else H
    runs = []
    for rev in (False, True):
        runs.append(O.rollout_batch(wl.params, wl.K, H, wl.dt, wl.g0, wl.gb0, wl.field_off,
                                    wl.field_of, wl.wx, wl.wz, wl.wg, wl.pairs, wl.u[:, :H],
                                    wl.x_goal, wl.q_diag, reverse=rev, traj=True)["traj"])
    a, b = runs
    d = []
    for n in range(H + 1):
        den = np.linalg.norm(a[:, n])
        d.append(float(np.linalg.norm(a[:, n] - b[:, n]) / den))
    return np.array(d)


CASES = {
    "plain_fp64_K32_H100": lambda: W.plain_single_plan(K=8),
    "realtime_K1024_H200": lambda: W.realtime(K=8, H=200),
    "uneven_K4096_H100": lambda: W.uneven_batch(K=4096, H=100).subset(np.arange(0, 4096, 512)),
}


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
    main()
