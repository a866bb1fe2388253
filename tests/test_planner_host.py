"""Host-side planner contract (no GPU needed)."""
import ctypes as C

from paper_2509_16079_amd import vpm as V


def test_footprint_counts_inputs_outputs_and_streaming_workspace():
    small = V.planner_footprint(256, 50, 500, 32)
    assert small >= 8 * 256 * 50                       # the perturbations alone
    assert V.planner_footprint(512, 50, 500, 32) > small
    # a wake beyond the LDS-resident kernel adds 256 workgroup slots of 24 B
    big = V.planner_footprint(256, 50, 8000, 32)
    assert big - V.planner_footprint(256, 50, 100, 32) >= 256 * 8100 * 24


def test_create_rejects_bad_options():
    L = V._planner_lib()
    h = C.c_void_p()
    for slots, budget in ((0, 1 << 30), (17, 1 << 30), (2, 0)):
        o = V.PlannerOpts(0, slots, budget)
        assert L.planner_create(C.byref(h), C.byref(o)) == V.EINVAL
    assert L.planner_submit(None, None, None) == V.EINVAL
    assert L.planner_poll(None, 1, None, 0) == V.EINVAL


def test_footprint_counts_the_perturbations_of_every_iteration():
    one = V.planner_footprint(256, 50, 500, 32)
    three = V.planner_footprint(256, 50, 500, 32, iterations=3)
    assert three - one == 2 * 8 * 256 * 50
