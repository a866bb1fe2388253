"""GPU parity of the streaming rollout kernel (wake in a device workspace,
source tiles staged through LDS) against the FP64 oracle, including the
full-size stress shape: 16 Lamb-Oseen blobs of 1023 particles plus 4
disturbance pairs (16376 vortices), 64 bound vortices, merging above 16384."""
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


@pytest.fixture
def stream_ctx(ctx):
    ctx.set_path(V.PATH_STREAM)
    yield ctx
    ctx.set_path(V.PATH_AUTO)


def test_set_path_rejects_unknown(ctx):
    with pytest.raises(V.VpmError):
        ctx.set_path(7)


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_stream_one_step_uneven(stream_ctx, prec):
    # ragged counts around the 1024-source stage and 64-source tiles
    wl = W.uneven_batch(K=10, H=1, n_min=1, n_max=2600)
    g = V.run_workload(stream_ctx, wl, prec, vel_last=True, gamma_s=True, final_wake=True)
    o = run_oracle(wl, vel_last=True, gamma_s=True, final_wake=True)
    for k in range(wl.K):
        e = rel_l2(vel_segment(g, k), vel_segment(o, k))
        assert e <= TOL[prec], describe("stream velocity k=%d n0=%d" % (k, wl.n0[k]), err=e)
    assert rel_l2(g["gamma_s"], o["gamma_s"]) <= TOL[prec]
    assert rel_l2(g["g_final"], o["g_final"]) <= TOL[prec]


@pytest.mark.parametrize("prec,H", [(V.FP32C, 20), (V.FP64, 50)])
def test_stream_horizon_parity_realtime(stream_ctx, prec, H):
    wl = W.realtime(K=16, H=H)
    g = V.run_workload(stream_ctx, wl, prec, traj=True, gamma_s=True, final_wake=True)
    o = run_oracle(wl, traj=True, gamma_s=True, final_wake=True)
    for key in ("g_final", "traj", "gamma_s"):
        e = rel_l2(g[key], o[key])
        assert e <= TOL[prec], describe("stream realtime " + key, err=e)
    assert np.array_equal(g["n_final"], o["n_final"])


def test_stream_and_lds_paths_agree(ctx):
    wl = W.realtime(K=8, H=30)
    a = V.run_workload(ctx, wl, V.FP64, traj=True)
    ctx.set_path(V.PATH_STREAM)
    try:
        b = V.run_workload(ctx, wl, V.FP64, traj=True)
    finally:
        ctx.set_path(V.PATH_AUTO)
    assert rel_l2(a["traj"], b["traj"]) <= 1e-11


def test_stress_full_size_one_step():
    """K=8192 rollouts of the 16376-vortex field in the persistent launch the
    stress benchmark uses (auto path: the wake exceeds LDS); two rollouts
    checked by the oracle, all velocities identical across rollouts."""
    c = V.Context(0)
    try:
        wl = W.large_stress(K=8192, H=1)
        g = V.run_workload(c, wl, V.FP32C, vel_last=True, gamma_s=True)
        o = run_oracle(wl, rollouts=[0, 4097], vel_last=True, gamma_s=True)
        ref = vel_segment(o, 0)
        for k in (0, 1, 4097, 8191):
            e = rel_l2(vel_segment(g, k), ref)
            assert e <= 1e-4, describe("stress velocity k=%d" % k, err=e)
        assert rel_l2(g["gamma_s"][[0, 4097]], o["gamma_s"]) <= 1e-4
        assert rel_l2(g["g_final"][[0, 4097]], o["g_final"]) <= 1e-4
        assert np.all(g["status"] == 0)
        assert np.all(g["pair_count"] == V.pair_count(16376, 1, 64, 16384))
    finally:
        c.close()


def test_stress_shape_through_merging():
    """Five steps from the stress field: the wake crosses N_w,max = 16384 and
    the two oldest are merged each step from the fourth on."""
    c = V.Context(0)
    try:
        wl = W.large_stress(K=4, H=5)
        g = V.run_workload(c, wl, V.FP64, final_wake=True, traj=True)
        o = run_oracle(wl, rollouts=[0, 3], final_wake=True, traj=True)
        assert np.array_equal(g["n_final"][[0, 3]], o["n_final"]) and o["n_final"][0] == 16384
        assert rel_l2(g["traj"][[0, 3]], o["traj"]) <= 1e-10
        gw = [wake_segments(g, k) for k in (0, 3)]
        for j in range(2):
            for a, b in zip(gw[j], wake_segments(o, j)):
                assert rel_l2(a, b) <= 1e-10
    finally:
        c.close()
