"""GPU: vpm_rollout_batch_noalloc, the rollout entry point for callers that
cannot allocate device memory, against vpm_rollout_batch through the C ABI:
identical outputs (bitwise: the same kernels on the same inputs) on two
calls in a row, the second with a smaller input, for uniform streamed
batches and uneven batches that use the plan and all three kernel classes;
and its error paths."""
import numpy as np
import pytest
import torch

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("g_final", "cost", "status", "traj", "gamma_s", "pair_count", "n_final", "wx", "wz",
        "wg", "gb_final")


def _run(ctx, wl, prec, noalloc):
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, traj=True, gamma_s=True, final_wake=True, gb_final=True)
    ctx.rollout(wl.params, db, out, prec, noalloc=noalloc)
    torch.cuda.synchronize()
    return out.to_numpy()


def _same(a, b):
    for k in KEYS:
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def _streamed(K, n0, H, seed):
    """K rollouts from one shared wake of n0 vortices (a uniform batch)."""
    rng = np.random.Generator(np.random.Philox(seed))
    state = W.random_field(rng, n0)
    eps = W.f32(rng.normal(0, 0.15, (K, H)))
    return W.workload_from_state("streamed", W.make_params(32), state, K=K, H=H, eps=eps)


@pytest.mark.parametrize("prec", [V.FP32C, V.FP64])
@pytest.mark.parametrize("kind", ["uniform", "uneven"])
def test_noalloc_equals_rollout_batch_on_two_calls(prec, kind):
    if kind == "uniform":   # wakes beyond the LDS classes: the streamed kernel
        big, small = _streamed(300, 9000, 4, 1), _streamed(40, 7000, 3, 2)
    else:                   # plan + streamed + large + small class kernels
        big = W.uneven_batch(seed=3, K=96, H=4, n_min=50, n_max=9000)
        small = W.uneven_batch(seed=5, K=16, H=3, n_min=20, n_max=7000)
    ctx = V.Context(0)
    try:
        # plate inverse built (and context buffers sized) by the set-up call
        ctx.reserve(big.params, big.K, big.H, int(np.max(big.n0)), len(big.field_off) - 1,
                    precision=prec)
        refs = [_run(ctx, wl, prec, False) for wl in (big, small)]
        gots = [_run(ctx, wl, prec, True) for wl in (big, small)]   # two calls in a row
        for got, ref in zip(gots, refs):
            _same(got, ref)
            assert np.all(ref["status"] == 0)
    finally:
        ctx.close()


def test_noalloc_error_paths():
    ctx = V.Context(0)
    try:
        wl = _streamed(4, 100, 2, 3)
        with pytest.raises(V.VpmError) as e:           # no plate inverse cached yet
            _run(ctx, wl, V.FP32C, True)
        assert e.value.code == V.EINVAL
        # one FP64 streaming slot of 1.5M vortices (72 MB) exceeds the 64 MiB
        # array: refused on the host before any launch
        huge = _streamed(1, 1_500_000, 1, 4)
        ctx.reserve(huge.params, 1, 1, 10, 1, precision=V.FP64)   # the inverse only
        with pytest.raises(V.VpmError) as e:
            _run(ctx, huge, V.FP64, True)
        assert e.value.code == V.ECAPACITY
        # the context still works afterwards
        ctx.reserve(wl.params, wl.K, wl.H, 100, 1)
        _same(_run(ctx, wl, V.FP32C, True), _run(ctx, wl, V.FP32C, False))
    finally:
        ctx.close()
