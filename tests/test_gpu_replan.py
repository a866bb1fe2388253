"""GPU parity of one replanning cycle of the nonlinear MPC (vpm_replan,
Sec. IV-C) against the cycle's oracle composed of the rollout, MPPI and
policy oracles: projection of the resident state (open loop, then under the
policy of a previous cycle), MPPI iterations from the projected state, the
nominal and perturbed rollouts and the policy. FP64; the MPPI argmin of
every iteration is identical, the plan within 1e-10, the gains within 1e-7
(the regression divides trajectory gaps of ~1e-13 by 1e-2 perturbations)."""
import numpy as np
import pytest

from oracle import replan as OR
from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import describe, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = V.Context(0)
    yield c
    c.close()


def _dev(a, dtype=None):
    import torch
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    return torch.tensor(a, dtype=dtype or (torch.int32 if a.dtype == np.int32 else torch.float64),
                        device="cuda")


def _gpu_cycle(ctx, c, state, plan):
    import torch
    out = V.replan(ctx, c["params"], V.FP64, c["dt"],
                   tuple(_dev(a) for a in state), tuple(_dev(a) for a in plan),
                   _dev(c["u_eps"]), _dev(c["x_eps"]), _dev(c["du"]), c["lam"], c["x_goal"],
                   c["q_diag"], c["q_f"], c["q_c"], c["r_c"], c["P"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _oracle_cycle(c, state, plan):
    g, gb, wx, wz, wg, pairs = state
    u_plan, x_plan, gain_plan = plan
    return OR.replan(c["params"], c["dt"], g, gb, wx, wz, wg, pairs, u_plan, x_plan, gain_plan,
                     c["P"], c["u_eps"], c["x_eps"], c["du"], c["lam"], c["x_goal"], c["q_diag"],
                     c["q_f"], c["q_c"], c["r_c"])


def _compare(g, o, tag):
    assert np.array_equal(g["argmin"], o["argmin"]), tag
    assert np.array_equal(g["status"], o["status"]), tag
    for key, tol in (("g_proj", 1e-10), ("jmin", 1e-10), ("u_new", 1e-10), ("x_new", 1e-10),
                     ("gain", 1e-7)):
        e = rel_l2(g[key], o[key])
        assert e <= tol, describe("%s %s" % (tag, key), err=e)


def test_two_chained_cycles_match_oracle(ctx):
    c = W.replan_case(K=48, H=24, P=4, iterations=3, Kp=24)
    state = (c["g"], c["gb"], c["wx"], c["wz"], c["wg"], c["pairs"])
    plan = (c["u_plan"], None, None)
    g1 = _gpu_cycle(ctx, c, state, plan)
    o1 = _oracle_cycle(c, state, plan)
    _compare(g1, o1, "cycle 1 (open-loop projection)")
    # cycle 2: each side continues from its own cycle-1 plan and policy, the
    # projection now closed by that policy
    g2 = _gpu_cycle(ctx, c, state, (g1["u_new"], g1["x_new"][:-1], g1["gain"]))
    o2 = _oracle_cycle(c, state, (o1["u_new"], o1["x_new"][:-1], o1["gain"]))
    _compare(g2, o2, "cycle 2 (closed-loop projection)")


def test_no_projection_and_empty_wake(ctx):
    c = W.replan_case(K=16, H=12, P=0, iterations=2, Kp=8)
    state = (c["g"], c["gb"], np.zeros(0), np.zeros(0), np.zeros(0), None)
    plan = (c["u_plan"], None, None)
    _compare(_gpu_cycle(ctx, c, state, plan), _oracle_cycle(c, state, plan), "P=0, no wake")
