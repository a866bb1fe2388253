"""GPU: the replanning service. Results of served requests equal the same
computation issued directly (bitwise, alone or in any mix); admission
respects the HBM budget; errors surface as status codes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import sampling as S
from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu


def _states(n_states=3, seed=11):
    rng = np.random.default_rng(seed)
    return [W.random_field(np.random.Generator(np.random.Philox(seed + i)),
                           int(rng.integers(300, 1500))) for i in range(n_states)]


def _requests(n, n_states, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        K, H = int(rng.integers(32, 257)), int(rng.integers(8, 31))
        out.append(dict(state=int(rng.integers(0, n_states)), K=K, H=H,
                        eps=W.f32(rng.normal(0, 0.15, (K, H))), mu=W.f32(rng.normal(0, 0.05, H))))
    return out


def _direct(ctx, params, state, req, prec=V.FP32C):
    wl = W.workload_from_state("direct", params, state, K=req["K"], H=req["H"], eps=req["eps"])
    wl.u_mean = req["mu"]
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db)
    ctx.rollout(params, db, out, prec)
    w, un, am, jm = ctx.mppi(out.cost, 1.0, db.u_mean, db.u_eps)
    torch.cuda.synchronize()
    return dict(cost=out.cost.cpu().numpy(), w=w.cpu().numpy(), u_new=un.cpu().numpy(),
                argmin=int(am.item()), g_final=out.g_final.cpu().numpy())


def _serve(planner, sids, params, reqs):
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    dt = float(W.f32(0.005))      # the step the direct calls use
    tickets = [planner.submit(sids[r["state"]], params, r["mu"], r["eps"], dt) for r in reqs]
    return [planner.poll(t, timeout_us=-1) for t in tickets]


def test_served_results_equal_direct_calls_alone_and_in_the_mix():
    params = W.make_params(32)
    states = _states()
    reqs = _requests(10, len(states))
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    mix = V.Planner(max_slots=4)
    alone = V.Planner(max_slots=1)
    try:
        sids = [mix.put_state(*s, g0, np.zeros(32)) for s in states]
        sids1 = [alone.put_state(*s, g0, np.zeros(32)) for s in states]
        served = _serve(mix, sids, params, reqs)
        serial = _serve(alone, sids1, params, reqs)
        ctx = V.Context(0)
        for r, a, b in zip(reqs, served, serial):
            d = _direct(ctx, params, states[r["state"]], r)
            assert a["status"] == 0 and b["status"] == 0
            for key in ("cost", "w", "u_new", "g_final"):
                assert np.array_equal(a[key], d[key]), key
                assert np.array_equal(b[key], d[key]), key
            assert a["argmin"] == d["argmin"] == b["argmin"]
            assert a["pairs"] == r["K"] * V.pair_count(len(states[r["state"]][0]), r["H"], 32, 0)
            assert a["t_arrive_us"] <= a["t_admit_us"] <= a["t_done_us"]
        ctx.close()
        # with four slots, some requests ran concurrently
        iv = sorted((s["t_admit_us"], s["t_done_us"]) for s in served)
        assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))
    finally:
        mix.close()
        alone.close()


def test_budget_admits_one_request_at_a_time():
    params = W.make_params(32)
    states = _states(1)
    reqs = _requests(6, 1, seed=9)
    for r in reqs:                                 # equal footprints: 1.5 of one fits one
        r["eps"], r["mu"] = r["eps"][:32, :8], r["mu"][:8]
    fp = V.planner_footprint(params, 32, 8, len(states[0][0]))
    p = V.Planner(max_slots=4, budget_bytes=fp + fp // 2)
    try:
        g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
        sids = [p.put_state(*s, g0, np.zeros(32)) for s in states]
        res = _serve(p, sids, params, reqs)
        iv = sorted((s["t_admit_us"], s["t_done_us"]) for s in res)
        assert all(iv[i + 1][0] >= iv[i][1] for i in range(len(iv) - 1))
        with pytest.raises(V.VpmError) as e:
            p.submit(sids[0], params, np.zeros(400), np.zeros((4096, 400)), 0.005)
        assert e.value.code == V.EBUDGET
    finally:
        p.close()


def test_errors_and_oracle_check():
    params = W.make_params(16, n_wake_max=200)
    wl = W.plain_single_plan(K=16, H=12)
    p = V.Planner(max_slots=2)
    try:
        sid = p.put_state(wl.wx, wl.wz, wl.wg, wl.g0[0], np.zeros(16))
        with pytest.raises(V.VpmError) as e:
            p.submit(sid + 99, params, wl.u_mean, wl.u_eps, wl.dt)
        assert e.value.code == V.ENOTFOUND
        with pytest.raises(V.VpmError) as e:
            p.submit(sid, W.make_params(32), wl.u_mean, wl.u_eps, wl.dt)
        assert e.value.code == V.EINVAL
        t = p.submit(sid, params, wl.u_mean, wl.u_eps, wl.dt)
        r = p.poll(t)
        assert r["status"] == 0
        wl.pairs = np.full((wl.K, 2), -1, dtype=np.int32)    # the state carries no pair tags
        o = O.rollout_batch(wl.params, wl.K, wl.H, wl.dt, wl.g0, wl.gb0, wl.field_off,
                            wl.field_of, wl.wx, wl.wz, wl.wg, wl.pairs, wl.u, wl.x_goal,
                            wl.q_diag)
        assert rel_l2(r["g_final"], o["g_final"]) <= 1e-4
        ref = O.mppi(o["cost"], 1.0, wl.u_mean, wl.u)
        assert r["argmin"] == ref["argmin"]
        assert np.max(np.abs(r["u_new"] - ref["xi_star"])) <= 1e-6
        with pytest.raises(V.VpmError) as e:
            p.poll(t)                                         # the ticket was released
        assert e.value.code == V.ENOTFOUND
        p.drop_state(sid)
    finally:
        p.close()


def test_multi_iteration_request_equals_chained_direct_calls():
    """A request of three MPPI iterations (the paper's planner runs three per
    replan) equals three direct rollout batches from the same initial state,
    each around the previous iteration's update, bitwise."""
    params = W.make_params(32)
    state = _states(1)[0]
    rng = np.random.default_rng(8)
    K, H, iters = 96, 12, 3
    eps = W.f32(rng.normal(0, 0.15, (iters, K, H)))
    mu = W.f32(rng.normal(0, 0.05, H))
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    planner = V.Planner(max_slots=2)
    try:
        sid = planner.put_state(*state, g0, np.zeros(32))
        res = planner.poll(planner.submit(sid, params, mu, eps, float(W.f32(0.005))), -1)
    finally:
        planner.close()
    assert res["status"] == 0
    ctx = V.Context(0)
    try:
        mean = mu.astype(np.float64)
        for i in range(iters):
            d = _direct(ctx, params, state, dict(K=K, H=H, eps=eps[i], mu=mean))
            mean = d["u_new"]
    finally:
        ctx.close()
    for key in ("cost", "w", "u_new", "g_final"):
        assert np.array_equal(res[key], d[key]), key
    assert res["argmin"] == d["argmin"]
    assert res["pairs"] == iters * K * V.pair_count(len(state[0]), H, 32, 0)


def test_seeded_request_equals_explicit_perturbations_bitwise():
    """A request whose perturbations the library draws from a seed (Sec. IV-A
    sampling) equals the same request with the oracle's independently drawn
    perturbations passed in, and both equal direct calls, bitwise."""
    params = W.make_params(32)
    state = _states(1, seed=21)[0]
    K, H, iters, seed, sigma = 80, 14, 2, 2**40 + 3, 0.15
    eps = np.array([S.eps(seed, i, K, H, sigma) for i in range(iters)])
    mu = W.f32(np.linspace(-0.05, 0.05, H))
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    dt = float(W.f32(0.005))
    p = V.Planner(max_slots=2)
    try:
        sid = p.put_state(*state, g0, np.zeros(32))
        a = p.poll(p.submit(sid, params, mu, None, dt, seed=seed, sigma=sigma, K=K,
                            iterations=iters))
        b = p.poll(p.submit(sid, params, mu, eps, dt))
    finally:
        p.close()
    assert a["status"] == 0 and b["status"] == 0
    for key in ("cost", "w", "u_new", "g_final"):
        assert np.array_equal(a[key], b[key]), key
    assert a["argmin"] == b["argmin"]
    ctx = V.Context(0)
    try:
        mean = mu.astype(np.float64)
        for i in range(iters):
            d = _direct(ctx, params, state, dict(K=K, H=H, eps=eps[i], mu=mean))
            mean = d["u_new"]
    finally:
        ctx.close()
    for key in ("cost", "w", "u_new", "g_final"):
        assert np.array_equal(a[key], d[key]), key


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
def test_advanced_state_equals_a_direct_rollout_and_the_oracle(prec):
    """advance = P carries the resident state P steps under the updated
    controls and keeps it resident (the receding-horizon step of Sec. IV-C):
    the new state equals a direct one-rollout batch under u_new (bitwise) and
    the oracle's (to the parity bar); a request from it runs."""
    params = W.make_params(32)
    state = _states(1, seed=31)[0]
    K, H, P = 64, 16, 5
    rng = np.random.default_rng(4)
    eps = W.f32(rng.normal(0, 0.15, (K, H)))
    mu = np.zeros(H)
    g0 = np.array([0, 0, 0.02, 0, 6.0, 0.1, 0])
    gb0 = np.linspace(-0.01, 0.01, 32)
    dt = float(W.f32(0.005))
    p = V.Planner(max_slots=2)
    try:
        sid = p.put_state(*state, g0, gb0)
        r = p.poll(p.submit(sid, params, mu, eps, dt, precision=prec, advance=P))
        assert r["status"] == 0 and r["new_state_id"] > 0 and r["new_state_status"] == 0
        wx, wz, wg, g7, gb = p.get_state(r["new_state_id"], 32)
        # a request from the advanced state
        r2 = p.poll(p.submit(r["new_state_id"], params, np.zeros(H), eps, dt, precision=prec))
        assert r2["status"] == 0
        with pytest.raises(V.VpmError):
            p.get_state(r["new_state_id"] + 100, 32)
        p.drop_state(r["new_state_id"])
    finally:
        p.close()
    assert len(wx) == len(state[0]) + 2 * P
    # direct: one rollout of P steps from the state under u_new[:P]
    wl = W.workload_from_state("adv", params, state, K=1, H=P, eps=np.zeros((1, P)))
    wl.u_mean = r["u_new"][:P]
    wl.g0 = g0[None, :]
    wl.gb0 = gb0[None, :]
    ctx = V.Context(0)
    try:
        db = V.DeviceBatch(wl)
        out = V.DeviceOutputs(db, final_wake=True, gb_final=True)
        ctx.rollout(params, db, out, prec)
        torch.cuda.synchronize()
        d = out.to_numpy()
    finally:
        ctx.close()
    n = int(d["n_final"][0])
    assert n == len(wx)
    assert np.array_equal(d["wx"][:n], wx) and np.array_equal(d["wz"][:n], wz)
    assert np.array_equal(d["wg"][:n], wg)
    assert np.array_equal(d["g_final"][0], g7) and np.array_equal(d["gb_final"][0], gb)
    o = O.rollout_batch(wl.params, 1, P, wl.dt, wl.g0, wl.gb0, wl.field_off, wl.field_of,
                        wl.wx, wl.wz, wl.wg, None, wl.u, wl.x_goal, wl.q_diag,
                        final_wake=True, gb_final=True)
    tol = 1e-4 if prec == V.FP32C else 1e-10
    assert rel_l2(g7, o["g_final"][0]) <= tol
    assert rel_l2(np.concatenate([wx, wz]), np.concatenate([o["wx"][:n], o["wz"][:n]])) <= tol
    assert rel_l2(gb, o["gb_final"][0]) <= tol


def test_reserve_and_tuning_keep_results_equal_to_direct_calls():
    """planner_reserve sizes every slot up front and planner_set_tuning sets
    the kernel shape of every slot; served results equal direct calls with
    the same shape, bitwise. Reserve needs an idle planner."""
    params = W.make_params(32)
    states = _states(2, seed=41)
    reqs = _requests(6, len(states), seed=13)
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    p = V.Planner(max_slots=3)
    try:
        sids = [p.put_state(*s, g0, np.zeros(32)) for s in states]
        p.reserve(params, K=256, H=30, n0=max(len(s[0]) for s in states))
        for cls in (V.CLASS_SMALL, V.CLASS_LARGE):
            p.set_tuning(cls, 2, 128)
        # a long request first, so that the service is surely busy below
        long_t = p.submit(sids[0], params, np.zeros(120), None, float(W.f32(0.005)), seed=1,
                          sigma=0.15, K=1024)
        tickets = [p.submit(sids[r["state"]], params, r["mu"], r["eps"], float(W.f32(0.005)))
                   for r in reqs]
        with pytest.raises(V.VpmError) as e:
            p.reserve(params, K=8, H=8, n0=10)
        assert e.value.code == V.EINVAL
        served = [p.poll(t) for t in tickets]
        assert p.poll(long_t)["status"] == 0
        p.reserve(params, K=8, H=8, n0=10)          # idle again
    finally:
        p.close()
    ctx = V.Context(0)
    try:
        for cls in (V.CLASS_SMALL, V.CLASS_LARGE):
            ctx.set_tuning(cls, 2, 128)
        for r, a in zip(reqs, served):
            d = _direct(ctx, params, states[r["state"]], r)
            for key in ("cost", "w", "u_new", "g_final"):
                assert np.array_equal(a[key], d[key]), key
    finally:
        ctx.close()
