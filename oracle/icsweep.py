"""Plain FP64 oracle of the initial-condition sweep of the local feedback
policies (Sec. IV-B, Fig. 3): the replanning cycle's oracle gives the nominal
plan and its least-squares policy, the finite-difference oracle the second
policy, and closed-loop oracle rollouts from offset forward speeds compare
open loop, least-squares and finite-difference feedback.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.
"""
from __future__ import annotations

import numpy as np

from oracle import fd as F
from oracle import oracle as O
from oracle import policy as P
from oracle import replan as OR


def run(c, offsets, h_x, h_u):
    rp = OR.replan(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"], c["pairs"],
                   c["u_plan"], None, None, 0, c["u_eps"], c["x_eps"], c["du"], c["lam"],
                   c["x_goal"], c["q_diag"], c["q_f"], c["q_c"], c["r_c"])
    A, B, _ = F.fd_jacobians(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"],
                             c["pairs"], rp["u_new"], h_x, h_u)
    _, fd_gain = P.tvlqr(A, B, c["q_f"], c["q_c"], c["r_c"])
    offsets = np.asarray(offsets, dtype=np.float64)
    K, H = len(offsets), len(rp["u_new"])
    g0 = np.repeat(np.asarray(c["g"], dtype=np.float64)[None], K, 0)
    g0[:, 4] += offsets
    pr = None if c["pairs"] is None else np.repeat(np.asarray(c["pairs"])[None], K, 0)
    out = dict(u_nom=rp["u_new"], x_nom=rp["x_new"], ls_gain=rp["gain"], fd_gain=fd_gain)
    for name, gain in (("open", None), ("ls", rp["gain"]), ("fd", fd_gain)):
        fb = {} if gain is None else dict(fb_gain=gain, fb_xref=rp["x_new"][:-1])
        o = O.rollout_batch(c["params"], K, H, c["dt"], g0, np.repeat(c["gb"][None], K, 0),
                            np.array([0, len(c["wx"])], dtype=np.int64), np.zeros(K, dtype=np.int32),
                            c["wx"], c["wz"], c["wg"], pr, np.repeat(rp["u_new"][None], K, 0),
                            c["x_goal"], c["q_diag"], **fb)
        err = np.hypot(o["g_final"][:, 0] - rp["x_new"][-1, 0],
                       o["g_final"][:, 1] - rp["x_new"][-1, 1])
        out[name] = dict(g_final=o["g_final"], pos_err=err, cost=o["cost"])
    return out
