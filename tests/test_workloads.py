"""Seeded input generators: reproducible, float32-exact, shaped as stated."""
import numpy as np

from paper_2509_16079_amd import workloads as W


def _f32_exact(a):
    return np.array_equal(a, a.astype(np.float32).astype(np.float64))


def test_seeded_and_reproducible():
    a, b = W.realtime(K=8, H=10), W.realtime(K=8, H=10)
    for f in ("wx", "wz", "wg", "u_eps", "g0"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = W.realtime(seed=7, K=8, H=10)
    assert not np.array_equal(a.u_eps, c.u_eps)


def test_inputs_are_float32_exact():
    for wl in (W.plain_single_plan(K=4, H=5), W.realtime(K=4, H=5),
               W.uneven_batch(K=6, H=5), W.large_stress(K=2, H=3, per_blob=31)):
        for f in ("wx", "wz", "wg", "u_eps", "g0"):
            assert _f32_exact(getattr(wl, f)), (wl.name, f)
        assert float(np.float32(wl.dt)) == wl.dt


def test_shapes_and_structure():
    wl = W.plain_single_plan()
    assert (wl.K, wl.H, wl.params["n_bound"], wl.params["n_wake_max"]) == (32, 100, 16, 200)
    assert wl.wg[0] == -wl.wg[1] and abs(wl.wg[0]) == np.float32(0.4)
    assert wl.wz[0] - wl.wz[1] == np.float32(0.125) - np.float32(-0.125)
    assert wl.u_eps.shape == (32, 100) and abs(wl.u_eps.std() - 0.15) < 0.02
    rt = W.realtime(K=16, H=20)
    assert 0.2 <= rt.meta["pair_gamma"] <= 0.8 and 1.5 <= rt.meta["pair_x"] <= 2.5
    ub = W.uneven_batch(K=64, H=5)
    n0 = ub.n0
    assert n0.min() >= 50 and n0.max() <= 4000 and len(ub.field_off) == 65
    for k in range(64):
        s = slice(ub.field_off[k], ub.field_off[k + 1])
        assert abs(ub.wg[s].sum()) < 1e-6          # zero total circulation
        assert ub.wx[s].min() >= 0 and ub.wx[s].max() <= 3.0
    st = W.large_stress(K=2, H=2)
    assert st.n0[0] == 16 * 1023 + 8 and st.pairs.shape == (2, 8)
    assert abs(st.wg.sum()) < 1e-5


def test_pair_count_matches_schedule():
    # two steps from 2 vortices, N_b = 1, both edges, no cap
    reg, sing = W.pair_count(2, 2, 1)
    # step 0: surface 2*3, wake 4*3, bound 4*1; step 1: surface 4*3, wake 6*5, bound 6
    assert reg == 2 * 3 + 4 * 3 + 4 * 3 + 6 * 5 and sing == 4 + 6
    reg, sing = W.pair_count(0, 3, 2, n_wake_max=3)
    # counts 0 -> 2 -> (4 -> 3) -> (5 -> 3)
    assert sing == 2 * 2 + 4 * 2 + 5 * 2


def test_serving_trace():
    p, states, reqs = W.serving_trace(n_requests=50)
    assert len(states) == 16 and len(reqs) == 50
    t = np.array([r.t_arrive for r in reqs])
    assert np.all(np.diff(t) > 0) and 0.2 < t[-1] < 1.0
    assert all(256 <= r.K <= 2048 and 50 <= r.H <= 200 for r in reqs)
    assert all(500 <= len(s[0]) <= 6000 for s in states)
    e1, e2 = W.request_eps(reqs[0]), W.request_eps(reqs[0])
    assert np.array_equal(e1, e2) and e1.shape == (reqs[0].K, reqs[0].H)
