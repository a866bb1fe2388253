"""GPU parity of the initial-condition sweep of the local feedback policies
(Sec. IV-B, Fig. 3) against its FP64 oracle at a reduced size: the nominal
plan, both policies (least-squares and finite-difference TVLQR) and the
final states of the open- and closed-loop sweep rollouts. The closed-loop
bars follow from the gains' (1e-7, set by the regression and the central
differences)."""
import numpy as np
import pytest

from oracle import icsweep as OI
from paper_2509_16079_amd import icsweep as S
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


def test_sweep_matches_oracle(ctx):
    c = W.replan_case(K=48, H=24, P=0, iterations=2, Kp=24)
    offsets = np.linspace(-0.5, 0.5, 9)
    g = S.run(ctx, c, offsets, V.FP64)
    o = OI.run(c, offsets, S.FD_H_X, S.FD_H_U)
    assert rel_l2(g["u_nom"], o["u_nom"]) <= 1e-10
    for key in ("ls_gain", "fd_gain"):
        e = rel_l2(g[key], o[key])
        assert e <= 1e-7, describe(key, err=e)
    for name, tol in (("open", 1e-10), ("ls", 1e-7), ("fd", 1e-7)):
        e = rel_l2(g[name]["g_final"], o[name]["g_final"])
        assert e <= tol, describe(name + " g_final", err=e)
        assert S.region_of_attraction(offsets, g[name]["pos_err"]) == \
            S.region_of_attraction(offsets, o[name]["pos_err"])
