"""Plain FP64 oracle of the closed-loop simulation of the nonlinear MPC
(Sec. IV-C, with the disturbance scenarios of Sec. V): a truth instance of
the model follows the policy in force while the planner (the replanning
cycle's oracle) replans from the truth's state every P steps over a horizon
that shrinks to the manoeuvre's end; the planner's copy of the state lacks
the disturbance pair in the uncompensated scenario.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from oracle import replan as OR


def _truth(c, state, plan, steps):
    g, gb, wx, wz, wg, pairs = state
    u, x_ref, gain = plan
    fb = {} if gain is None else dict(fb_gain=np.asarray(gain)[:steps],
                                      fb_xref=np.asarray(x_ref)[:steps])
    o = O.rollout_batch(c["params"], 1, steps, c["dt"], np.asarray(g)[None], np.asarray(gb)[None],
                        np.array([0, len(wx)], dtype=np.int64), np.zeros(1, dtype=np.int32),
                        wx, wz, wg, None if pairs is None else np.asarray(pairs)[None],
                        np.asarray(u, dtype=np.float64)[None, :steps], c["x_goal"], c["q_diag"],
                        traj=True, final_wake=True, gb_final=True, **fb)
    n = int(o["n_final"][0])
    new = (o["g_final"][0], o["gb_final"][0], o["wx"][:n], o["wz"][:n], o["wg"][:n], pairs)
    return new, o["traj"][0]


def simulate(c, scenario):
    H, P = c["H"], c["P"]
    with_pair = scenario != "no_disturbance"
    state = (np.asarray(c["g"], dtype=np.float64), np.asarray(c["gb"], dtype=np.float64),
             np.asarray(c["wx"] if with_pair else np.zeros(0), dtype=np.float64),
             np.asarray(c["wz"] if with_pair else np.zeros(0), dtype=np.float64),
             np.asarray(c["wg"] if with_pair else np.zeros(0), dtype=np.float64),
             c["pairs"] if with_pair else None)
    plan = (np.asarray(c["u_plan"], dtype=np.float64), None, None)
    traj = [state[0]]
    jmin = []
    t = 0
    while H - t - P >= P:   # the projection needs P controls of the plan
        Hn = H - t - P
        g, gb, wx, wz, wg, pairs = state
        if scenario == "uncompensated" and pairs is not None:
            wx, wz, wg, pairs = wx[2:], wz[2:], wg[2:], None
        out = OR.replan(c["params"], c["dt"], g, gb, wx, wz, wg, pairs, plan[0][:Hn],
                        None if plan[1] is None else plan[1][:Hn],
                        None if plan[2] is None else plan[2][:Hn], P,
                        c["u_eps"][:, :, :Hn], c["x_eps"], c["du"][:, :Hn], c["lam"],
                        c["x_goal"], c["q_diag"], c["q_f"], c["q_c"], c["r_c"])
        jmin.append(float(out["jmin"][-1]))
        state, seg = _truth(c, state, plan, P)
        traj.extend(seg[1:])
        t += P
        plan = (out["u_new"], out["x_new"][:-1], out["gain"])
    if t < H:
        state, seg = _truth(c, state, plan, H - t)
        traj.extend(seg[1:])
    return dict(traj=np.array(traj), jmin=np.array(jmin))
