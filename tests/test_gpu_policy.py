"""GPU parity of the local feedback policy (vpm_policy: least-squares
Jacobians and TVLQR, Sec. IV-B) against the FP64 policy oracle on the same
trajectories: synthetic linear data with known Jacobians, rank-deficient
steps, and oracle VPM rollouts at the paper's controller size (K = 256
perturbed rollouts, 77 steps). Both sides are FP64; the synthesis differs
only in rounding (normal equations with column scaling against an SVD-based
least squares; condition numbers of the scaled regressors stay below 1e3
on these inputs), so the bar is 1e-9 relative on A, B, S and the gains."""
import numpy as np
import pytest

from oracle import policy as P
from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import rel_l2, run_oracle
from tests.policy_data import euler_linear_data

pytestmark = pytest.mark.gpu
TOL = 1e-9


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = V.Context(0)
    yield c
    c.close()


def _gpu_policy(ctx, nom, traj, du, dt):
    import torch
    dev = dict(dtype=torch.float64, device="cuda")
    out = V.policy(ctx, torch.tensor(nom, **dev), torch.tensor(traj, **dev),
                   torch.tensor(du, **dev), dt, P.Q_F, P.Q_C, P.R_C)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _compare(g, o, tag):
    assert np.array_equal(g["status"], o["status"]), tag
    for key in ("A", "B", "S", "gain"):
        e = rel_l2(g[key.lower()] if key in ("A", "B", "S") else g[key], o[key])
        assert e <= TOL, "%s %s rel_l2=%.3e" % (tag, key, e)


@pytest.mark.parametrize("K,H", [(64, 12), (6, 5), (1000, 3)])
def test_linear_data_matches_oracle(ctx, K, H):
    rng = np.random.default_rng(10 + K)
    nom, traj, du = euler_linear_data(rng, K, H, 0.01, rng.normal(size=(H, 3, 5)),
                                      rng.normal(size=(H, 3)))
    g = _gpu_policy(ctx, nom, traj, du, 0.01)
    o = P.policy(nom, traj, du, 0.01, P.Q_F, P.Q_C, P.R_C)
    _compare(g, o, "linear K=%d H=%d" % (K, H))


def test_rank_deficient_steps_match_oracle(ctx):
    rng = np.random.default_rng(11)
    K, H = 32, 4
    nom, traj, du = euler_linear_data(rng, K, H, 0.01, rng.normal(size=(H, 3, 5)),
                                      rng.normal(size=(H, 3)))
    du[:, 1] = 0.0
    g = _gpu_policy(ctx, nom, traj, du, 0.01)
    o = P.policy(nom, traj, du, 0.01, P.Q_F, P.Q_C, P.R_C)
    assert list(g["status"]) == [0, 1, 0, 0]
    _compare(g, o, "rank-deficient")
    few = _gpu_policy(ctx, nom, traj[:5], du[:5], 0.01)
    assert np.all(few["status"] == 1)
    eye = np.eye(7)
    eye[0, 4] = eye[1, 5] = eye[2, 6] = 0.01
    assert np.array_equal(few["a"][0], eye)     # kinematic rows only


def test_vpm_rollouts_at_controller_size(ctx):
    wl = W.policy_batch(K=256, H=77)
    o_roll = run_oracle(wl, traj=True)
    tr = o_roll["traj"]
    args = (tr[0], tr[1:], wl.u_eps[1:], wl.dt)
    g = _gpu_policy(ctx, *args)
    o = P.policy(*args, P.Q_F, P.Q_C, P.R_C)
    assert np.all(o["status"] == 0)
    _compare(g, o, "vpm K=256 H=77")


def test_end_to_end_fp64_rollouts_then_policy(ctx):
    # GPU rollouts (FP64) feed the GPU policy; the oracle runs both steps on
    # its own. Over 20 steps the FP64 trajectories agree to ~1e-13, which the
    # regression divides by the perturbation size (~1e-2) and multiplies by
    # the regressor conditioning (< 1e2): 1e-7 bounds the gains' difference.
    import torch
    wl = W.policy_batch(K=256, H=20)
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, traj=True)
    ctx.rollout(wl.params, db, out, V.FP64)
    traj = out.traj
    pol = V.policy(ctx, traj[0], traj[1:], db.u_eps[1:], wl.dt, P.Q_F, P.Q_C, P.R_C)
    torch.cuda.synchronize()
    o_roll = run_oracle(wl, traj=True)
    tr = o_roll["traj"]
    o = P.policy(tr[0], tr[1:], wl.u_eps[1:], wl.dt, P.Q_F, P.Q_C, P.R_C)
    assert rel_l2(traj.cpu().numpy(), tr) <= 1e-10
    assert np.array_equal(pol["status"].cpu().numpy(), o["status"])
    for key, ref in (("gain", o["gain"]), ("a", o["A"]), ("b", o["B"])):
        e = rel_l2(pol[key].cpu().numpy(), ref)
        assert e <= 1e-7, "end-to-end %s rel_l2=%.3e" % (key, e)
