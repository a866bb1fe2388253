"""Closed-loop simulation of the nonlinear MPC (Sec. IV-C) on the GPU: a
"truth" instance of the model is stepped under the policy in force while the
planner replans from the truth's state every P steps, with a horizon that
shrinks to the fixed end of the manoeuvre. As in the paper's experiments
(Sec. V), the truth's wake may hold a disturbance pair that the planner's
copy of the state either includes (compensated) or lacks (uncompensated).
Every step runs in the library (vpm_replan for the cycle, vpm_rollout_batch
with feedback for the truth); this module only sequences the calls.

Timing of a cycle at step t: the planner takes the truth's state s_t,
projects it P steps under the policy in force (which the truth follows over
the same P steps), and plans the remaining horizon from t + P; the new plan
is in force from t + P. Once fewer than 2P steps remain, the last plan flies
the manoeuvre to its end.
"""
from __future__ import annotations

import numpy as np

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

SCENARIOS = ("no_disturbance", "compensated", "uncompensated")


def _dev(a):
    import torch
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    return torch.tensor(a, device="cuda",
                        dtype=torch.int32 if a.dtype == np.int32 else torch.float64)


def truth_segment(ctx, c, state, plan, steps, precision, stream=None):
    """`steps` steps of the truth from `state` = (g, gb, wx, wz, wg, pairs)
    under `plan` = (u [>= steps], x_ref or None, gain or None); returns the
    new state and the segment's trajectory [steps + 1, 7]."""
    import torch
    g, gb, wx, wz, wg, pairs = state
    u, x_ref, gain = plan
    wl = W.Workload("truth", c["params"], 1, steps, c["dt"], np.asarray(g)[None],
                    np.asarray(gb)[None], np.array([0, len(wx)], dtype=np.int64),
                    np.zeros(1, dtype=np.int32), wx, wz, wg,
                    None if pairs is None else np.asarray(pairs, dtype=np.int32)[None],
                    np.asarray(u[:steps], dtype=np.float64), np.zeros((1, steps)),
                    x_goal=c["x_goal"], q_diag=c["q_diag"])
    db = V.DeviceBatch(wl)
    if gain is not None:
        db.set_feedback(_dev(np.asarray(gain)[:steps]), _dev(np.asarray(x_ref)[:steps]))
    out = V.DeviceOutputs(db, traj=True, final_wake=True, gb_final=True)
    ctx.rollout(wl.params, db, out, precision, stream)
    torch.cuda.synchronize()
    o = out.to_numpy()
    n = int(o["n_final"][0])
    off = int(o["out_off"][0])
    new = (o["g_final"][0], o["gb_final"][0], o["wx"][off:off + n], o["wz"][off:off + n],
           o["wg"][off:off + n], pairs)
    return new, o["traj"][0]


def planner_view(state, scenario, n_pair_vortices=2):
    """The planner's copy of the truth's state: without the disturbance pair
    (the first vortices of the wake) when uncompensated."""
    g, gb, wx, wz, wg, pairs = state
    if scenario != "uncompensated" or pairs is None:
        return state
    k = n_pair_vortices
    return (g, gb, wx[k:], wz[k:], wg[k:], None)


def simulate(ctx, c, scenario, precision=V.FP32C, stream=None):
    """Returns the truth trajectory [H + 1, 7], the replanning latencies
    (ms) and the plans' best costs."""
    import time

    import torch
    H, P = c["H"], c["P"]
    with_pair = scenario != "no_disturbance"
    state = (np.asarray(c["g"], dtype=np.float64), np.asarray(c["gb"], dtype=np.float64),
             c["wx"] if with_pair else np.zeros(0), c["wz"] if with_pair else np.zeros(0),
             c["wg"] if with_pair else np.zeros(0), c["pairs"] if with_pair else None)
    plan = (np.asarray(c["u_plan"], dtype=np.float64), None, None)   # open loop at first
    traj = [state[0]]
    lat, jmin = [], []
    t = 0
    while H - t - P >= P:   # the projection needs P controls of the plan
        Hn = H - t - P                      # remaining horizon after the projection
        u_in = plan[0][:Hn]
        x_in = None if plan[1] is None else plan[1][:Hn]
        k_in = None if plan[2] is None else plan[2][:Hn]
        view = planner_view(state, scenario)
        t0 = time.perf_counter()
        out = V.replan(ctx, c["params"], precision, c["dt"], tuple(_dev(a) for a in view),
                       (_dev(u_in), _dev(x_in), _dev(k_in)),
                       _dev(c["u_eps"][:, :, :Hn]), _dev(c["x_eps"]), _dev(c["du"][:, :Hn]),
                       c["lam"], c["x_goal"], c["q_diag"], c["q_f"], c["q_c"], c["r_c"], P,
                       stream=stream)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t0))
        jmin.append(float(out["jmin"][-1].item()))
        # meanwhile the truth follows the policy in force for P steps
        state, seg = truth_segment(ctx, c, state, plan, P, precision, stream)
        traj.extend(seg[1:])
        t += P
        plan = (out["u_new"].cpu().numpy(), out["x_new"][:-1].cpu().numpy(),
                out["gain"].cpu().numpy())
    if t < H:   # the last steps under the last plan
        state, seg = truth_segment(ctx, c, state, plan, H - t, precision, stream)
        traj.extend(seg[1:])
    return dict(traj=np.array(traj), replan_ms=np.array(lat), jmin=np.array(jmin))


def open_loop(ctx, c, precision=V.FP32C, stream=None):
    """The initial plan flown without replanning, disturbance present."""
    state = (np.asarray(c["g"], dtype=np.float64), np.asarray(c["gb"], dtype=np.float64),
             c["wx"], c["wz"], c["wg"], c["pairs"])
    _, seg = truth_segment(ctx, c, state, (np.asarray(c["u_plan"]), None, None), c["H"],
                           precision, stream)
    return dict(traj=seg)


def final_error(c, traj):
    """Distance of the final position from the goal's, and the cost of
    Eq. 24 with the planner's weights."""
    g = traj[-1]
    d = g - c["x_goal"]
    return float(np.hypot(d[0], d[1])), float(np.sum(c["q_diag"] * d * d))
