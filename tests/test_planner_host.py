"""Host-side planner contract (no GPU needed): the footprint arithmetic and
argument checks that run before any device call."""
import ctypes as C

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

P32 = W.make_params(32)


def test_footprint_counts_inputs_outputs_and_streaming_workspace():
    small = V.planner_footprint(P32, 256, 50, 500)
    assert small >= 8 * 256 * 50                       # the perturbations alone
    assert V.planner_footprint(P32, 512, 50, 500) > small
    # a wake beyond the LDS-resident kernel adds 256 workgroup slots of 24 B
    big = V.planner_footprint(P32, 256, 50, 8000)
    assert big - V.planner_footprint(P32, 256, 50, 100) >= 256 * 8100 * 24


def test_footprint_follows_the_precision():
    # FP64 wakes take twice the LDS per vortex, so they stream from smaller
    # sizes and their workspace slots are 48 B per vortex
    n = 3500
    f32 = V.planner_footprint(P32, 256, 50, n, precision=V.FP32C)
    f64 = V.planner_footprint(P32, 256, 50, n, precision=V.FP64)
    assert f64 - f32 >= 256 * (n + 100) * 48
    big32 = V.planner_footprint(P32, 256, 50, 9000, precision=V.FP32C)
    big64 = V.planner_footprint(P32, 256, 50, 9000, precision=V.FP64)
    assert big64 - big32 == 256 * 9100 * 24


def test_footprint_counts_the_advanced_state():
    base = V.planner_footprint(P32, 256, 50, 500)
    adv = V.planner_footprint(P32, 256, 50, 500, advance=10)
    assert adv - base == 8 * (3 * (500 + 20) + 9 + 32)


def test_create_rejects_bad_options():
    L = V._planner_lib()
    h = C.c_void_p()
    for slots, budget in ((0, 1 << 30), (17, 1 << 30), (2, 0)):
        o = V.PlannerOpts(0, slots, budget)
        assert L.planner_create(C.byref(h), C.byref(o)) == V.EINVAL
    assert L.planner_submit(None, None, None) == V.EINVAL
    assert L.planner_poll(None, 1, None, 0) == V.EINVAL
    assert L.planner_reserve(None, None, 1, 1, 0, 1) == V.EINVAL
    assert L.planner_footprint(None, 1, 1, 0, 1, 0) == 0


def test_footprint_counts_the_perturbations_of_every_iteration():
    one = V.planner_footprint(P32, 256, 50, 500)
    three = V.planner_footprint(P32, 256, 50, 500, iterations=3)
    assert three - one == 2 * 8 * 256 * 50
