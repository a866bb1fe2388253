"""GPU parity of the closed-loop simulation of the nonlinear MPC (a truth
model following the policy in force while the planner replans from its
state every P steps, horizon shrinking to the manoeuvre's end) against its
FP64 oracle, in the three disturbance scenarios of the paper's experiments,
at a reduced size. Every cycle's best cost agrees to 1e-8 and the truth
trajectory to 1e-7 (the gains of each cycle carry the regression's ~1e-7)."""
import numpy as np
import pytest

from oracle import nmpc as ON
from paper_2509_16079_amd import nmpc as N
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


@pytest.mark.parametrize("scenario", N.SCENARIOS)
def test_closed_loop_simulation_matches_oracle(ctx, scenario):
    c = W.replan_case(K=48, H=24, P=4, iterations=2, Kp=24)
    g = N.simulate(ctx, c, scenario, V.FP64)
    o = ON.simulate(c, scenario)
    assert g["traj"].shape == o["traj"].shape == (25, 7)
    e = rel_l2(g["jmin"], o["jmin"])
    assert e <= 1e-8, describe(scenario + " jmin", err=e)
    e = rel_l2(g["traj"], o["traj"])
    assert e <= 1e-7, describe(scenario + " truth trajectory", err=e)
