"""The horizons used by the GPU horizon-parity tests are justified by the
oracle alone. FP64 bars: the oracle's forward- and reverse-order runs (pure
rounding perturbations) stay far below the bar. FP32 bars: the oracle's
binary32-storage variant (state rounded to float after every step) stays far
below the bar -- storing the state in FP32 is the dominant FP32 error."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_16079_amd import workloads as W
from tests.golden.conditioning import divergence_curve, read_stress
from tests.parity import rel_l2, run_oracle

# (case, horizon, bar) -- the same horizons test_gpu_parity uses
FP64_HORIZONS = [("plain", 40, 1e-10), ("realtime", 50, 1e-10), ("uneven", 20, 1e-10)]
FP32_HORIZONS = [("plain", 15, 1e-4), ("realtime", 20, 1e-4), ("uneven", 15, 1e-4)]


def make(case, H):
    if case == "plain":
        return W.plain_single_plan(K=4, H=H)
    if case == "realtime":
        return W.realtime(K=4, H=H)
    return W.uneven_batch(K=8, H=H, n_min=50, n_max=1500)


@pytest.mark.parametrize("case,H,bar", FP64_HORIZONS)
def test_fp64_horizon_is_well_conditioned(case, H, bar):
    d = divergence_curve(make(case, H))
    assert d[-1] <= 0.1 * bar, (case, H, d[-1])


@pytest.mark.parametrize("case,H,bar", FP32_HORIZONS)
def test_fp32_storage_error_is_below_the_bar(case, H, bar):
    wl = make(case, H)
    a = run_oracle(wl, traj=True, gamma_s=True)
    b = run_oracle(wl, traj=True, gamma_s=True, f32_state=True)
    for key in ("g_final", "traj", "gamma_s"):
        assert rel_l2(b[key], a[key]) <= 0.3 * bar, (case, H, key)


def test_f32_state_variant_stores_binary32():
    wl = W.realtime(K=2, H=7)
    b = run_oracle(wl, final_wake=True, f32_state=True)
    for key in ("g_final", "wx", "wz", "wg"):
        v = b[key][np.isfinite(b[key])]
        assert np.array_equal(v, v.astype(np.float32).astype(np.float64)), key
    a = run_oracle(wl)
    assert 0 < rel_l2(b["g_final"], a["g_final"]) < 1e-6


def test_full_horizons_are_not():
    # the full realtime horizon amplifies FP64 rounding beyond 1e-6 on its own
    d = divergence_curve(W.realtime(K=2, H=120))
    assert d[-1] > 1e-7


# The stress field (16376 vortices) is too slow for the CPU suite: its curves
# come from tests/golden/conditioning_stress.txt, written by the committed
# script from the oracle alone. The GPU stress horizon tests use H = 20.
STRESS_H = 20


def test_stress_horizon_is_well_conditioned():
    g = read_stress()
    i = STRESS_H // g["step"]
    assert g["D"][i] <= 0.1 * 1e-10, g["D"][i]          # FP64 bar
    assert g["S"][i] <= 0.3 * 1e-4, g["S"][i]           # FP32 bar
    # and the full 150-step horizon is not: rounding alone grows past both bars
    assert g["D"][-1] > 1e-10 and g["S"][-1] > 1e-4
