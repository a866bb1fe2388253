"""GPU: uneven batches run as a device-planned set of persistent class
kernels (small and large LDS-resident workgroups, streamed beyond LDS)."""
import numpy as np
import pytest

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import TOL, describe, rel_l2, run_oracle, vel_segment, wake_segments

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = V.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_all_classes_match_oracle(ctx, prec):
    # counts from 10 to 7000 reach the small, large and streamed classes
    wl = W.uneven_batch(K=24, H=3, n_min=10, n_max=7000)
    g = V.run_workload(ctx, wl, prec, vel_last=True, gamma_s=True, final_wake=True)
    o = run_oracle(wl, vel_last=True, gamma_s=True, final_wake=True)
    assert np.all(g["status"] == 0)
    for k in range(wl.K):
        e = rel_l2(vel_segment(g, k), vel_segment(o, k))
        assert e <= TOL[prec], describe("class velocity k=%d n0=%d" % (k, wl.n0[k]), err=e)
        for a, b in zip(wake_segments(g, k), wake_segments(o, k)):
            assert rel_l2(a, b) <= TOL[prec]
    assert rel_l2(g["g_final"], o["g_final"]) <= TOL[prec]
    assert np.array_equal(g["pair_count"],
                          [V.pair_count(n, wl.H, 32, 0) for n in wl.n0])


def test_planned_batch_is_deterministic_and_matches_alone(ctx):
    wl = W.uneven_batch(K=40, H=6, n_min=20, n_max=6500)
    a = V.run_workload(ctx, wl, V.FP32C, final_wake=True)
    b = V.run_workload(ctx, wl, V.FP32C, final_wake=True)
    for key in ("g_final", "cost", "wx", "wz", "wg"):
        assert np.array_equal(a[key], b[key]), key
    # a rollout run alone takes the same kernel class and gives the same bits
    for k in (0, 7, int(np.argmax(wl.n0)), int(np.argmin(wl.n0))):
        s = slice(wl.field_off[k], wl.field_off[k + 1])
        alone = W.workload_from_state("alone", wl.params, (wl.wx[s], wl.wz[s], wl.wg[s]),
                                      K=1, H=wl.H, eps=wl.u_eps[k:k + 1], dt=wl.dt)
        r = V.run_workload(ctx, alone, V.FP32C, final_wake=True)
        assert np.array_equal(r["g_final"][0], a["g_final"][k]), k
        for x, y in zip(wake_segments(r, 0), wake_segments(a, k)):
            assert np.array_equal(x, y), k


def test_uneven_full_size_horizon(ctx):
    """All 4096 uneven rollouts (N_0 in [50, 4000]) over 15 steps in FP32 in
    one planned launch; 12 rollouts stratified by N_0 checked by the oracle."""
    wl = W.uneven_batch(K=4096, H=15)
    g = V.run_workload(ctx, wl, V.FP32C, traj=True)
    order = np.argsort(wl.n0)
    idx = order[np.linspace(0, 4095, 12).astype(int)]
    o = run_oracle(wl, rollouts=idx, traj=True)
    e = rel_l2(g["traj"][idx], o["traj"])
    assert e <= 1e-4, describe("uneven 4096 H15 traj", err=e)
    assert np.all(g["status"] == 0)


@pytest.mark.parametrize("shape", [(1, 64), (1, 256), (2, 128), (4, 64), (4, 256)])
def test_every_kernel_shape_matches_oracle(ctx, shape):
    """The autotuner's shapes (targets per thread x compensated tile), set
    for all three classes, on a batch that reaches all three."""
    wl = W.uneven_batch(K=24, H=2, n_min=10, n_max=7000)
    try:
        for cls in (V.CLASS_SMALL, V.CLASS_LARGE, V.CLASS_STREAM):
            ctx.set_tuning(cls, *shape)
        g = V.run_workload(ctx, wl, V.FP32C, vel_last=True)
    finally:
        ctx.set_tuning(V.CLASS_SMALL, 4, 64)
        ctx.set_tuning(V.CLASS_LARGE, 2, 64)
        ctx.set_tuning(V.CLASS_STREAM, 4, 64)
    o = run_oracle(wl, vel_last=True)
    assert np.all(g["status"] == 0)
    for k in range(wl.K):
        e = rel_l2(vel_segment(g, k), vel_segment(o, k))
        assert e <= TOL[V.FP32C], describe("shape %s k=%d" % (shape, k), err=e)
    assert rel_l2(g["g_final"], o["g_final"]) <= TOL[V.FP32C]
