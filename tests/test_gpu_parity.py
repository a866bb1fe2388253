"""GPU parity: the HIP rollout path against the FP64 CPU oracle on the same
seeded inputs. Tolerances: relative L2 <= 1e-4 in FP32 (compensated) mode and
<= 1e-10 in FP64 mode on velocities, surface circulations and final states;
MPPI argmin identical."""
import numpy as np
import pytest

from oracle import oracle as O
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


def _compare_one_step(ctx, wl, prec):
    g = V.run_workload(ctx, wl, prec, final_wake=True, vel_last=True, gamma_s=True)
    o = run_oracle(wl, final_wake=True, vel_last=True, gamma_s=True)
    tol = TOL[prec]
    for k in range(wl.K):
        vg, vo = vel_segment(g, k), vel_segment(o, k)
        assert vg.shape == vo.shape
        e = rel_l2(vg, vo)
        assert e <= tol, describe(wl.name + " velocity k=%d" % k, err=e)
    e = rel_l2(g["gamma_s"], o["gamma_s"])
    assert e <= tol, describe(wl.name + " gamma_s", err=e)
    e = rel_l2(g["g_final"], o["g_final"])
    assert e <= tol, describe(wl.name + " g_final", err=e)
    assert np.array_equal(g["n_final"], o["n_final"])


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_one_step_velocities_uneven_random_fields(ctx, prec):
    # ragged initial counts spanning several 64-source tiles and all chunk sizes
    wl = W.uneven_batch(K=12, H=1, n_min=1, n_max=1500)
    _compare_one_step(ctx, wl, prec)


def test_fp64_one_step_at_binary64_accuracy(ctx):
    # the FP64 pair's 1/sqrt and 1/r^2 are hardware estimates refined by
    # Newton-Raphson steps: one step of every target stays within a few
    # hundred ulp of the oracle over sums of up to 1500 terms (the bar
    # elsewhere is 1e-10)
    wl = W.uneven_batch(K=12, H=1, n_min=1, n_max=1500)
    g = V.run_workload(ctx, wl, V.FP64, final_wake=True, vel_last=True, gamma_s=True)
    o = run_oracle(wl, final_wake=True, vel_last=True, gamma_s=True)
    for k in range(wl.K):
        e = rel_l2(vel_segment(g, k), vel_segment(o, k))
        assert e <= 1e-13, describe("FP64 one-step velocity k=%d" % k, err=e)
    e = rel_l2(g["gamma_s"], o["gamma_s"])
    assert e <= 1e-13, describe("FP64 one-step gamma_s", err=e)


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_one_step_velocities_realtime_pair(ctx, prec):
    _compare_one_step(ctx, W.realtime(K=4, H=1), prec)


# Wake counts whose step target count NT = n + 2 N_b + 3 leaves a last pass-A
# chunk (NT mod 256) of every kind: 1..5 targets (too few lanes per part for
# the pads below the wake at N_b = 1: the tail path), 41 and 63 (one target
# per lane over several source parts), 64, 65, 128 and 191 (2..4 targets per
# lane), 255, and none (NT a multiple of 256); three steps move NT by the two
# vortices shed per step, so the spread plan changes between steps. On the
# streamed path (forced) the same counts give last rounds of one to eight
# waves of targets over 16 .. 2 source parts, and none beyond 512 targets.
@pytest.mark.parametrize("path", [V.PATH_AUTO, V.PATH_STREAM])
@pytest.mark.parametrize("nb", [1, 32])
@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_spread_last_chunk_every_remainder(ctx, path, nb, prec):
    n_surf = 2 * nb + 3
    rng = np.random.default_rng(17)
    for r in (1, 2, 3, 5, 41, 63, 64, 65, 128, 191, 255, 256):
        n = 256 + r - n_surf if r + 256 - n_surf < 512 else r - n_surf
        wl = W.workload_from_state("spread nb=%d r=%d" % (nb, r), W.make_params(nb),
                                   W.random_field(rng, n), K=2, H=3,
                                   eps=W.f32(np.full((2, 3), 0.05)))
        ctx.set_path(path)
        try:
            g = V.run_workload(ctx, wl, prec, final_wake=True, vel_last=True, gamma_s=True)
        finally:
            ctx.set_path(V.PATH_AUTO)
        o = run_oracle(wl, final_wake=True, vel_last=True, gamma_s=True)
        tol = TOL[prec]
        for k in range(wl.K):
            e = rel_l2(vel_segment(g, k), vel_segment(o, k))
            assert e <= tol, describe(wl.name + " velocity k=%d" % k, err=e)
        e = rel_l2(g["gamma_s"], o["gamma_s"])
        assert e <= tol, describe(wl.name + " gamma_s", err=e)
        assert np.array_equal(g["n_final"], o["n_final"])
        # both rollouts start from the same field: the same bits
        assert np.array_equal(vel_segment(g, 0), vel_segment(g, 1))


def test_empty_initial_wake(ctx):
    wl = W.workload_from_state("empty", W.make_params(16), (np.zeros(0), np.zeros(0), np.zeros(0)),
                               K=3, H=5, eps=W.f32(np.full((3, 5), 0.1)))
    for prec in (V.FP32C, V.FP64):
        g = V.run_workload(ctx, wl, prec, final_wake=True, traj=True)
        o = run_oracle(wl, final_wake=True, traj=True)
        assert rel_l2(g["traj"], o["traj"]) <= TOL[prec]
        assert np.array_equal(g["n_final"], o["n_final"]) and g["n_final"][0] == 10


def _horizon_parity(ctx, wl, prec):
    g = V.run_workload(ctx, wl, prec, final_wake=True, gamma_s=True, traj=True)
    o = run_oracle(wl, final_wake=True, gamma_s=True, traj=True)
    tol = TOL[prec]
    assert np.all(g["status"] == 0) and np.array_equal(g["n_final"], o["n_final"])
    for name in ("g_final", "traj", "gamma_s"):
        e = rel_l2(g[name], o[name])
        assert e <= tol, describe(wl.name + " " + name, err=e)
    e = np.max(np.abs(g["cost"] - o["cost"]) / np.abs(o["cost"]))
    assert e <= tol, describe(wl.name + " cost", err=e)
    for k in range(wl.K):
        for a, b in zip(wake_segments(g, k), wake_segments(o, k)):
            assert rel_l2(a, b) <= 10 * tol
    return g, o


def _case(case, H):
    if case == "plain":
        return W.plain_single_plan(H=H)                 # K = 32, N_b = 16
    if case == "realtime":
        return W.realtime(K=16, H=H)                    # N_b = 32
    return W.uneven_batch(K=8, H=H, n_min=50, n_max=1500)


# Horizons where rounding sensitivity permits each bar: FP64 by the oracle's
# own summation-order gap, FP32 by the oracle's binary32-storage variant
# (both enforced on the CPU by tests/test_conditioning.py).
@pytest.mark.parametrize("case,prec,H", [
    ("plain", V.FP64, 40), ("plain", V.FP32C, 15),
    ("realtime", V.FP64, 50), ("realtime", V.FP32C, 20),
    ("uneven", V.FP64, 20), ("uneven", V.FP32C, 15)])
def test_horizon_parity(ctx, case, prec, H):
    _horizon_parity(ctx, _case(case, H), prec)


@pytest.mark.parametrize("case,H", [("plain", 30), ("realtime", 40), ("uneven", 25)])
def test_fp32_error_at_the_binary32_storage_floor(ctx, case, H):
    """Beyond those horizons the FP32 path stays within a small factor of the
    error that storing the state in binary32 alone causes."""
    wl = _case(case, H)
    g = V.run_workload(ctx, wl, V.FP32C, traj=True)
    o = run_oracle(wl, traj=True)
    f = run_oracle(wl, traj=True, f32_state=True)
    for key in ("g_final", "traj"):
        floor = rel_l2(f[key], o[key])
        e = rel_l2(g[key], o[key])
        assert e <= 4 * floor + 1e-6, describe(wl.name + " " + key, err=e, floor=floor)


def test_plain_fp64_full_horizon_within_rounding_envelope(ctx):
    """K=32, H=100, merging above 200: at the full horizon the GPU stays
    within a small multiple of the gap between two FP64 summation orders of
    the oracle itself."""
    from tests.golden.conditioning import divergence_curve
    wl = W.plain_single_plan()
    g = V.run_workload(ctx, wl, V.FP64, final_wake=True)
    o = run_oracle(wl, final_wake=True)
    envelope = divergence_curve(wl)[-1]
    e = rel_l2(g["g_final"], o["g_final"])
    assert e <= 5 * envelope + 1e-12, describe("plain H100", err=e, envelope=envelope)
    assert np.all(g["n_final"] == 200) and np.array_equal(g["n_final"], o["n_final"])
    assert int(np.argmin(g["cost"])) == int(np.argmin(o["cost"]))
    assert np.all(g["pair_count"] == V.pair_count(2, wl.H, 16, 200))


def _restart_workload(wl, o, idx, K):
    """A one-step batch of K rollouts that start from oracle states after
    wl.H steps of rollouts idx (rounded to float32 like every input);
    rollout k uses state k % len(idx) and the perturbation of step wl.H of
    rollout k."""
    m = len(idx)
    xs, zs, gs, off = [], [], [], [0]
    for j in range(m):
        x, z, gm = wake_segments(o, j)
        xs.append(x)
        zs.append(z)
        gs.append(gm)
        off.append(off[-1] + len(x))
    nb = wl.params["n_bound"]
    full = W.realtime(K=K, H=wl.H + 1)
    sel = np.arange(K) % m
    return W.Workload("restart", wl.params, K, 1, wl.dt, W.f32(o["g_final"][sel]),
                      o["gamma_s"][sel, -1, :nb], np.array(off, dtype=np.int64),
                      sel.astype(np.int32), W.f32(np.concatenate(xs)), W.f32(np.concatenate(zs)),
                      W.f32(np.concatenate(gs)), np.full((K, 2), -1, dtype=np.int32),
                      np.zeros(1), full.u_eps[:, wl.H:wl.H + 1])


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_full_size_realtime_one_step_from_late_states(ctx, prec):
    """The full K=1024 batch in the benchmark's launch configuration, one step
    from 16 oracle states at step 199 of the 200-step horizon (N_w = 400)."""
    wl = W.realtime(K=1024, H=199)
    idx = np.arange(0, 1024, 64)
    o = run_oracle(wl, rollouts=idx, final_wake=True, gamma_s=True)
    rs = _restart_workload(wl, o, idx, 1024)
    g = V.run_workload(ctx, rs, prec, final_wake=True, vel_last=True, gamma_s=True)
    ref = run_oracle(rs, rollouts=np.arange(len(idx)), final_wake=True, vel_last=True,
                     gamma_s=True)
    tol = TOL[prec]
    m = len(idx)
    assert np.all(g["n_vel_last"] == 402)
    for k in range(rs.K):
        e = rel_l2(vel_segment(g, k), vel_segment(ref, k % m))
        assert e <= tol, describe("restart velocity k=%d" % k, err=e)
        e = rel_l2(g["gamma_s"][k], ref["gamma_s"][k % m])
        assert e <= tol, describe("restart gamma_s k=%d" % k, err=e)
    e = rel_l2(g["g_final"][:m], ref["g_final"])
    assert e <= tol, describe("restart g_final", err=e)


def test_full_size_uneven_one_step(ctx):
    """All 4096 uneven rollouts (N_0 log-uniform in [50, 4000]) for one step
    in FP32; the oracle checks 24 rollouts stratified by N_0."""
    wl = W.uneven_batch(K=4096, H=1)
    g = V.run_workload(ctx, wl, V.FP32C, vel_last=True, gamma_s=True)
    order = np.argsort(wl.n0)
    idx = order[np.linspace(0, 4095, 24).astype(int)]
    o = run_oracle(wl, rollouts=idx, vel_last=True, gamma_s=True)
    for j, k in enumerate(idx):
        e = rel_l2(vel_segment(g, k), vel_segment(o, j))
        assert e <= 1e-4, describe("uneven velocity k=%d n0=%d" % (k, wl.n0[k]), err=e)
        assert rel_l2(g["gamma_s"][k], o["gamma_s"][j]) <= 1e-4
    assert np.all(g["status"] == 0)


def test_merging_and_termination(ctx):
    # a small cap forces two merges per step; a disturbance pair starts
    # straddling the chord so the termination test fires on the first step
    p = W.make_params(8, n_wake_max=30, decay=0.2)
    geo = O.plate_geometry(p, [0, 0, 0, 0, 6.0, 0, 0])
    mid = 0.5 * (geo["rc"][0] + geo["rc"][-1])
    wx = W.f32(np.array([mid[0], mid[0], 0.9, 1.1, 1.4]))
    wz = W.f32(np.array([0.1, -0.1, 0.2, -0.3, 0.05]))
    wg = W.f32(np.array([-0.2, 0.2, 0.05, -0.05, 0.01]))
    wl = W.workload_from_state("merge_term", p, (wx, wz, wg), K=3, H=40,
                               eps=W.f32(np.random.default_rng(0).normal(0, 0.15, (3, 40))))
    wl.pairs = np.tile(np.array([[0, 1]], dtype=np.int32), (3, 1))
    for prec in (V.FP32C, V.FP64):
        g = V.run_workload(ctx, wl, prec, final_wake=True)
        o = run_oracle(wl, final_wake=True)
        assert np.all(g["n_final"] == 30) and np.array_equal(g["n_final"], o["n_final"])
        assert rel_l2(g["g_final"], o["g_final"]) <= TOL[prec]
        for k in range(3):
            for a, b in zip(wake_segments(g, k), wake_segments(o, k)):
                assert rel_l2(a, b) <= TOL[prec] * 10


def test_capacity_status_for_oversized_field(ctx):
    import torch
    wl = W.uneven_batch(K=3, H=2, n_min=10, n_max=20)
    db = V.DeviceBatch(wl)
    db.max_wake0 = int(np.min(np.diff(wl.field_off)))   # the others exceed it
    out = V.DeviceOutputs(db)
    ctx.rollout(wl.params, db, out, V.FP32C)
    torch.cuda.synchronize()
    r = out.to_numpy()
    big = np.diff(wl.field_off) > db.max_wake0
    assert np.all((r["status"][big] & V.ROLLOUT_CAPACITY) != 0)
    assert np.all(np.isinf(r["cost"][big])) and np.all(r["status"][~big] == 0)


def test_deterministic(ctx):
    wl = W.realtime(K=8, H=20)
    a = V.run_workload(ctx, wl, V.FP32C, final_wake=True)
    b = V.run_workload(ctx, wl, V.FP32C, final_wake=True)
    for key in ("g_final", "cost", "wx", "wz", "wg"):
        assert np.array_equal(a[key], b[key])


def test_plate_solve_all_modes(ctx):
    import torch
    rng = np.random.default_rng(7)
    for nb in (1, 16, 32, 64):
        p = W.make_params(nb)
        B = 37
        pose = np.column_stack([rng.normal(size=2 * B).reshape(B, 2), rng.uniform(-1, 1, B),
                                rng.normal(size=(B, 2)) + [6, 0], rng.normal(size=B)])
        vw = rng.normal(size=(B, nb + 1, 2)) * 0.3
        sg = rng.normal(size=B) * 0.1
        for mode in (V.SHED_BOTH, V.SHED_TE, V.SHED_NONE):
            if mode == V.SHED_NONE and nb < 2:
                continue
            t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
            gs = ctx.plate_solve(p, t(pose), t(vw), t(sg), mode).cpu().numpy()
            for b in range(B):
                ref, rc = O.plate_solve_pose(p, pose[b], vw[b], sg[b], mode)
                assert rc == 0
                assert rel_l2(gs[b], ref) <= 1e-10, (nb, mode, b)


def test_mppi_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(3)
    for K, H in ((1, 1), (3, 5), (1024, 200), (5000, 77)):
        cost = rng.uniform(10, 40, K)
        if K > 3:
            cost[rng.integers(0, K, 3)] = np.inf
            cost[5] = cost[7] = cost.min() - 1.0    # a tie at the minimum
        mu = rng.normal(size=H) * 0.1
        eps = rng.normal(size=(K, H)) * 0.15
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
        w, un, am, jm = ctx.mppi(t(cost), 1.0, t(mu), t(eps))
        ref = O.mppi(cost, 1.0, mu, mu[None, :] + eps)
        assert int(am.item()) == ref["argmin"]
        assert jm.item() == ref["j_min"]
        assert np.max(np.abs(w.cpu().numpy() - ref["w"])) <= 1e-14
        assert rel_l2(un.cpu().numpy(), ref["xi_star"]) <= 1e-12
    cost = np.array([np.inf, np.nan])
    mu = np.array([0.5, -0.5])
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    w, un, am, jm = ctx.mppi(t(cost), 1.0, t(mu), t(np.ones((2, 2))))
    assert int(am.item()) == -1 and np.all(w.cpu().numpy() == 0)
    assert np.array_equal(un.cpu().numpy(), mu)


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_table1_configuration_full_horizon(ctx, prec):
    """The paper's runtime-table configuration (80 steps, dt = 10 ms, merging
    above 60 vortices) at its full horizon: well conditioned (the oracle's
    reverse-order gap is 5e-15, binary32 storage drifts 1e-6), so both bars
    hold over all 80 steps."""
    wl = W.table1(16)
    _horizon_parity(ctx, wl, prec)


@pytest.mark.parametrize("prec,H", [(V.FP32C, 15), (V.FP64, 30)])
def test_inputs_that_binary32_cannot_hold(ctx, prec, H):
    """The generator rounds every value to binary32 so that both precisions
    start from the same numbers; here the wake, the glider state, the
    controls and the plate parameters carry FP64 digits beyond binary32 (a
    relative offset of ~1e-9), so the FP32C path's own conversion of its
    inputs is exercised: FP32C stays within its bar, FP64 within its own."""
    from dataclasses import replace
    wl = W.realtime(K=8, H=H)
    rng = np.random.default_rng(77)
    jig = lambda a: np.asarray(a, dtype=np.float64) * (1.0 + 1e-9 * rng.uniform(0.5, 1.5,
                                                                                np.shape(a)))
    p = dict(wl.params)
    for key in ("chord", "r_core", "rho", "mass", "inertia", "l_wing", "l_elev"):
        p[key] = float(jig(p[key]))
    wl = replace(wl, params=p, wx=jig(wl.wx), wz=jig(wl.wz), wg=jig(wl.wg), g0=jig(wl.g0),
                 u_eps=jig(wl.u_eps) + 1e-12, u_mean=wl.u_mean + 3e-11, name="unrounded")
    assert not np.array_equal(wl.wx, wl.wx.astype(np.float32).astype(np.float64))
    g = V.run_workload(ctx, wl, prec, traj=True, gamma_s=True)
    o = run_oracle(wl, traj=True, gamma_s=True)
    for key in ("traj", "gamma_s", "g_final"):
        e = rel_l2(g[key], o[key])
        assert e <= TOL[prec], describe("unrounded inputs " + key, err=e)
