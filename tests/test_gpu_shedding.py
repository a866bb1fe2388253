"""GPU parity of the shedding modes and the separation gate (Sec. III-A)
against the FP64 oracle: trailing-edge-only shedding (N_b + 1 unknowns),
no shedding (N_b unknowns), and the gate that sheds from the leading edge
only on steps where the wing's angle of attack exceeds the critical angle.
Tolerances as for the both-edge path; where the gate decides, the oracle's
angles keep a margin from the critical angle far above the FP32 state
error, so both sides take every decision the same way."""
import numpy as np
import pytest

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import (TOL, describe, gate_margin, gated_at_median, rel_l2, run_oracle,
                          vel_segment, wake_segments, with_params)

pytestmark = pytest.mark.gpu

SHED_PER_STEP = {W.SHED_BOTH: 2, W.SHED_TE: 1, W.SHED_NONE: 0}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = V.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("mode", [W.SHED_TE, W.SHED_NONE])
@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_one_step_uneven_fields(ctx, mode, prec):
    # ragged counts over several tiles; every kernel class of the planned batch
    wl = with_params(W.uneven_batch(K=12, H=1, n_min=1, n_max=1500), shed_mode=mode)
    g = V.run_workload(ctx, wl, prec, final_wake=True, vel_last=True, gamma_s=True)
    o = run_oracle(wl, final_wake=True, vel_last=True, gamma_s=True)
    tol = TOL[prec]
    assert np.array_equal(g["n_final"], wl.n0 + SHED_PER_STEP[mode])
    assert np.array_equal(g["n_final"], o["n_final"])
    for k in range(wl.K):
        vg, vo = vel_segment(g, k), vel_segment(o, k)
        assert vg.shape == vo.shape
        e = rel_l2(vg, vo)
        assert e <= tol, describe(wl.name + " velocity k=%d" % k, err=e)
    for key in ("gamma_s", "g_final"):
        e = rel_l2(g[key], o[key])
        assert e <= tol, describe(wl.name + " " + key, err=e)


def _horizon(ctx, wl, prec):
    g = V.run_workload(ctx, wl, prec, final_wake=True, gamma_s=True, traj=True)
    o = run_oracle(wl, final_wake=True, gamma_s=True, traj=True)
    tol = TOL[prec]
    assert np.all(g["status"] == 0) and np.array_equal(g["n_final"], o["n_final"])
    for key in ("g_final", "traj", "gamma_s"):
        e = rel_l2(g[key], o[key])
        assert e <= tol, describe(wl.name + " " + key, err=e)
    e = np.max(np.abs(g["cost"] - o["cost"]) / np.abs(o["cost"]))
    assert e <= tol, describe(wl.name + " cost", err=e)
    for k in range(wl.K):
        for a, b in zip(wake_segments(g, k), wake_segments(o, k)):
            assert rel_l2(a, b) <= 10 * tol
    return g, o


@pytest.mark.parametrize("mode,prec,H", [
    (W.SHED_TE, V.FP64, 40), (W.SHED_TE, V.FP32C, 15),
    (W.SHED_NONE, V.FP64, 40), (W.SHED_NONE, V.FP32C, 15)])
def test_horizon_parity_realtime(ctx, mode, prec, H):
    wl = with_params(W.realtime(K=16, H=H), shed_mode=mode)
    g, _ = _horizon(ctx, wl, prec)
    n0, nb = int(wl.n0[0]), wl.params["n_bound"]
    reg, sing = W.pair_count(n0, H, nb, shed=SHED_PER_STEP[mode],
                             n_wake_max=wl.params["n_wake_max"])
    assert np.all(g["pair_count"] == reg + sing)


@pytest.mark.parametrize("prec,H", [(V.FP64, 40), (V.FP32C, 20)])
def test_gated_realtime_switches_modes_like_the_oracle(ctx, prec, H):
    wl = gated_at_median(W.realtime(K=16, H=H))
    g, o = _horizon(ctx, wl, prec)
    # far above each precision's state error over this horizon
    assert gate_margin(wl, o["traj"]) > (1e-4 if prec == V.FP32C else 1e-8)
    n0 = int(wl.n0[0])
    both = o["n_final"] - n0 - H          # steps that shed from the leading edge
    assert np.all(both > 0) and np.all(both < H)


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_gated_uneven_batch(ctx, prec):
    # planned classes with the two staged inverses in every kernel's LDS
    wl = gated_at_median(W.uneven_batch(K=8, H=10, n_min=50, n_max=1500))
    _, o = _horizon(ctx, wl, prec)
    assert gate_margin(wl, o["traj"]) > 1e-5


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_gated_streaming_kernel(ctx, prec):
    wl = gated_at_median(W.realtime(K=4, H=10))
    ctx.set_path(V.PATH_STREAM)
    try:
        _, o = _horizon(ctx, wl, prec)
    finally:
        ctx.set_path(V.PATH_AUTO)
    assert gate_margin(wl, o["traj"]) > 1e-5
