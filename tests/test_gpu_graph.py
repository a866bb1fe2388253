"""GPU: one MPPI step (rollout batch + weights) captured into a HIP graph and
replayed several times, with eager work in between, gives the eager bits
every time -- for a uniform LDS-resident batch and for a planned uneven
batch whose class kernels run on forked streams (including the streamed
class)."""
import numpy as np
import pytest
import torch

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["uniform", "uneven"])
def test_graph_replay_matches_eager(case):
    wl = W.realtime(K=64, H=20) if case == "uniform" else \
        W.uneven_batch(K=24, H=3, n_min=10, n_max=7000)
    ctx = V.Context(0)
    try:
        db = V.DeviceBatch(wl)
        out = V.DeviceOutputs(db)
        ctx.rollout(wl.params, db, out, V.FP32C)           # eager: sizes every buffer
        w, un, am, jm = ctx.mppi(out.cost, 1.0, db.u_mean, db.u_eps)
        torch.cuda.synchronize()
        ref = dict(g=out.g_final.clone(), c=out.cost.clone(), w=w.clone(), u=un.clone())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.rollout(wl.params, db, out, V.FP32C)
            gw, gun, gam, gjm = ctx.mppi(out.cost, 1.0, db.u_mean, db.u_eps)
        for rep in range(3):
            out.g_final.fill_(float("nan"))
            out.cost.fill_(float("nan"))
            gw.fill_(float("nan"))
            x = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out.g_final, ref["g"]), rep
            assert torch.equal(out.cost, ref["c"]), rep
            assert torch.equal(gw, ref["w"]) and torch.equal(gun, ref["u"]), rep
            assert int(gam.item()) == int(am.item())
        del g
    finally:
        ctx.close()


def test_capture_refuses_to_allocate():
    """A first call (plate inverse and buffers not yet built) inside a capture
    is refused with VPM_EINVAL instead of allocating on the captured stream."""
    wl = W.uneven_batch(K=8, H=2, n_min=10, n_max=300)
    ctx = V.Context(0)
    try:
        db = V.DeviceBatch(wl)
        out = V.DeviceOutputs(db)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        raised = None
        try:
            with torch.cuda.graph(g):
                try:
                    ctx.rollout(wl.params, db, out, V.FP32C)
                except V.VpmError as e:
                    raised = e
        except RuntimeError:
            pass      # ending a capture that recorded nothing may be reported
        assert raised is not None and raised.code == V.EINVAL
        del g
        torch.cuda.synchronize()
        ctx.rollout(wl.params, db, out, V.FP32C)    # eager use still works
        torch.cuda.synchronize()
        assert torch.all(out.status == 0)
    finally:
        ctx.close()


def test_reserve_allows_capturing_a_first_call():
    """After vpm_reserve, a batch that was never run eagerly can be captured
    (nothing to allocate) and its replays equal an eager run."""
    wl = W.uneven_batch(K=24, H=3, n_min=10, n_max=7000)
    ctx = V.Context(0)
    try:
        db = V.DeviceBatch(wl)
        out = V.DeviceOutputs(db)
        ctx.reserve(wl.params, wl.K, wl.H, db.max_wake0, db.n_fields, V.FP32C)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.rollout(wl.params, db, out, V.FP32C)
        g.replay()
        torch.cuda.synchronize()
        got = out.g_final.clone()
        ref_out = V.DeviceOutputs(db)
        ctx.rollout(wl.params, db, ref_out, V.FP32C)
        torch.cuda.synchronize()
        assert torch.equal(got, ref_out.g_final)
        del g
    finally:
        ctx.close()
