"""Plain FP64 oracle of one replanning cycle of the nonlinear MPC (Sec. IV-C
of Gupta et al., arXiv 2509.16079), composed of the rollout, MPPI and policy
oracles in the cycle's order.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.

Readings: the plan in force is stepped P steps (the replanning time) from the
resident state under its own policy, u_n = u_plan[n] - gain[n] . (x_n -
x_plan[n]) (open loop without gains); the MPPI iterations start from the
plan in force shifted by P with its last control held; the policy is
synthesised from the nominal rollout under the final mean and Kp rollouts
from perturbed projected states under perturbed controls. (Everything here is
FP64.)
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from oracle import policy as P


def shift(u_plan, P_steps):
    """The plan in force from step P on, its last control held."""
    u_plan = np.asarray(u_plan, dtype=np.float64)
    H = u_plan.size
    return u_plan[np.minimum(np.arange(H) + P_steps, H - 1)]


def replan(params, dt, g, gb, wx, wz, wg, pairs, u_plan, x_plan, gain_plan, P_steps,
           u_eps, x_eps, du, lam, x_goal, q_diag, q_f, q_c, r_c):
    """One cycle. u_eps [I, K, H], x_eps [Kp, 7], du [Kp, H]; pairs [2P] or
    None. Returns g_proj, gb_proj, the projected wake, u_new [H], x_new
    [H + 1, 7], the policy (gain, A, B, S, status), and per MPPI iteration
    argmin and jmin."""
    g = np.asarray(g, dtype=np.float64)
    gb = np.asarray(gb, dtype=np.float64)
    wx, wz, wg = (np.asarray(a, dtype=np.float64) for a in (wx, wz, wg))
    n_pairs = 0 if pairs is None else len(pairs) // 2
    H = len(u_plan)
    pr1 = None if pairs is None else np.asarray(pairs, dtype=np.int32)[None]
    # 1. projection under the policy in force
    if P_steps > 0:
        fb = {} if gain_plan is None else dict(fb_gain=np.asarray(gain_plan)[:P_steps],
                                               fb_xref=np.asarray(x_plan)[:P_steps])
        pj = O.rollout_batch(params, 1, P_steps, dt, g[None], gb[None],
                             np.array([0, wx.size], dtype=np.int64), None, wx, wz, wg, pr1,
                             np.asarray(u_plan, dtype=np.float64)[None, :P_steps], x_goal, q_diag,
                             final_wake=True, gb_final=True, **fb)
        n = int(pj["n_final"][0])
        g_p, gb_p = pj["g_final"][0], pj["gb_final"][0]
        wx_p, wz_p, wg_p = pj["wx"][:n], pj["wz"][:n], pj["wg"][:n]
    else:
        g_p, gb_p, wx_p, wz_p, wg_p = g, gb, wx, wz, wg
    field_off = np.array([0, wx_p.size], dtype=np.int64)
    # 2. MPPI iterations (Eqs. 24-25)
    u_eps = np.asarray(u_eps, dtype=np.float64)
    iters, K, _ = u_eps.shape
    mu = shift(u_plan, P_steps)
    argmin, jmin = [], []
    for it in range(iters):
        out = O.rollout_batch(params, K, H, dt, np.repeat(g_p[None], K, 0),
                              np.repeat(gb_p[None], K, 0), field_off, np.zeros(K, dtype=np.int32),
                              wx_p, wz_p, wg_p,
                              None if pr1 is None else np.repeat(pr1, K, 0),
                              mu[None] + u_eps[it], x_goal, q_diag)
        m = O.mppi(out["cost"], lam, mu, mu[None] + u_eps[it])   # samples xi_i
        argmin.append(m["argmin"])
        jmin.append(m["j_min"])
        mu = m["xi_star"]
    # 3. nominal and perturbed rollouts, then the policy (Sec. IV-B)
    x_eps = np.asarray(x_eps, dtype=np.float64)
    du = np.asarray(du, dtype=np.float64)
    Kp = x_eps.shape[0]
    g0 = np.concatenate([g_p[None], g_p[None] + x_eps])
    uu = mu[None] + np.concatenate([np.zeros((1, H)), du])
    pol_roll = O.rollout_batch(params, Kp + 1, H, dt, g0, np.repeat(gb_p[None], Kp + 1, 0),
                               field_off, np.zeros(Kp + 1, dtype=np.int32), wx_p, wz_p, wg_p,
                               None if pr1 is None else np.repeat(pr1, Kp + 1, 0), uu, x_goal,
                               q_diag, traj=True)
    tr = pol_roll["traj"]
    pol = P.policy(tr[0], tr[1:], du, dt, q_f, q_c, r_c)
    return dict(g_proj=g_p, gb_proj=gb_p, wake=(wx_p, wz_p, wg_p), u_new=mu, x_new=tr[0],
                gain=pol["gain"], A=pol["A"], B=pol["B"], S=pol["S"], status=pol["status"],
                argmin=np.array(argmin), jmin=np.array(jmin), n_pairs=n_pairs)
