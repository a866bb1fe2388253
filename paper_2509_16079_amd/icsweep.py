"""Initial-condition sweep of the local feedback policies (Sec. IV-B, the
comparison of its Fig. 3) on the GPU: one replanning cycle gives the nominal
plan and its least-squares TVLQR policy; finite-difference Jacobians through
the model along the same nominal give the second policy; closed-loop
rollouts from initial states whose forward speed is offset by each sweep
value compare open loop, least-squares and finite-difference feedback by
the final position error against the nominal's. Every step runs in the
library (vpm_replan, vpm_fd_jacobians, vpm_tvlqr, vpm_rollout_batch); this
module only sequences the calls.
"""
from __future__ import annotations

import numpy as np

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

FD_H_X = (1e-4, 1e-4, 1e-4, 1e-4, 1e-4)   # theta, phi, x_dot, z_dot, theta_dot
FD_H_U = 1e-4
ROA_POS_ERR = 0.05                          # 5 cm final position error (Sec. IV-B)


def _dev(a):
    import torch
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    return torch.tensor(a, device="cuda",
                        dtype=torch.int32 if a.dtype == np.int32 else torch.float64)


def region_of_attraction(offsets, err, limit=ROA_POS_ERR):
    """Widest interval [lo, hi] of consecutive offsets around 0 whose final
    position errors stay below `limit` (None if the nominal itself fails)."""
    offsets = np.asarray(offsets)
    ok = np.asarray(err) < limit
    i0 = int(np.argmin(np.abs(offsets)))
    if not ok[i0]:
        return None
    lo = hi = i0
    while lo > 0 and ok[lo - 1]:
        lo -= 1
    while hi < len(ok) - 1 and ok[hi + 1]:
        hi += 1
    return float(offsets[lo]), float(offsets[hi])


def sweep_batch(c, offsets, u_nom, gain=None, x_ref=None):
    """The closed-loop (or open-loop) sweep rollouts as a Workload."""
    K, H = len(offsets), c["H"]
    g0 = np.repeat(np.asarray(c["g"])[None], K, 0)
    g0[:, 4] += offsets
    fo = np.array([0, len(c["wx"])], dtype=np.int64)
    pairs = np.repeat(np.asarray(c["pairs"])[None], K, 0) if c["pairs"] is not None else None
    return W.Workload("icsweep", c["params"], K, H, c["dt"], g0, np.repeat(c["gb"][None], K, 0), fo,
                      np.zeros(K, dtype=np.int32), c["wx"], c["wz"], c["wg"], pairs,
                      np.asarray(u_nom, dtype=np.float64), np.zeros((K, H)),
                      x_goal=c["x_goal"], q_diag=c["q_diag"])


def run(ctx, c, offsets, precision=V.FP64, stream=None):
    """Returns the nominal plan, both policies and, per policy, the final
    states, position errors and region of attraction."""
    import torch
    state = tuple(_dev(c[k]) for k in ("g", "gb", "wx", "wz", "wg", "pairs"))
    rp = V.replan(ctx, c["params"], precision, c["dt"], state, (_dev(c["u_plan"]), None, None),
                  _dev(c["u_eps"]), _dev(c["x_eps"]), _dev(c["du"]), c["lam"], c["x_goal"],
                  c["q_diag"], c["q_f"], c["q_c"], c["r_c"], 0, stream=stream)
    fd = V.fd_jacobians(ctx, c["params"], c["dt"], state, rp["u_new"], FD_H_X, FD_H_U,
                        stream=stream)
    fd_gain, _ = V.tvlqr(ctx, fd["a"], fd["b"], c["q_f"], c["q_c"], c["r_c"], want_s=False,
                         stream=stream)
    u_nom = rp["u_new"].cpu().numpy()
    x_nom = rp["x_new"].cpu().numpy()
    x_ref = rp["x_new"][:-1].contiguous()
    out = dict(u_nom=u_nom, x_nom=x_nom, ls_gain=rp["gain"].cpu().numpy(),
               fd_gain=fd_gain.cpu().numpy(), offsets=np.asarray(offsets, dtype=np.float64))
    wl = sweep_batch(c, offsets, u_nom)
    for name, gain in (("open", None), ("ls", rp["gain"]), ("fd", fd_gain)):
        db = V.DeviceBatch(wl)
        if gain is not None:
            db.set_feedback(gain.contiguous(), x_ref)
        o = V.DeviceOutputs(db)
        ctx.rollout(wl.params, db, o, precision, stream)
        torch.cuda.synchronize()
        gf = o.g_final.cpu().numpy()
        err = np.hypot(gf[:, 0] - x_nom[-1, 0], gf[:, 1] - x_nom[-1, 1])
        out[name] = dict(g_final=gf, pos_err=err, cost=o.cost.cpu().numpy(),
                         roa=region_of_attraction(offsets, err))
    return out
