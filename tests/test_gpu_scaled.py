"""GPU parity of the FP32 kernels' pre-scaled sources (q = 1/g, Sec. III
kernel of Eq. 5 in rearranged form) at the edges of that form, on the
hardware's v_rcp_f32 and v_rsq_f32: exactly zero strengths, a strength below
the 1e-30 cut, strengths whose scaled terms overflow to a zero term, and a
strong pair 30 m downstream, whose self terms (the rounding of q x) would add
~6e-3 m/s to a 0.6 m/s mutual velocity were they not removed. Each FP32
class is run: small (scaled copy of the wake), large (sources scaled per
chunk) and streamed (scaled tiles)."""
import numpy as np
import pytest

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W
from tests.parity import TOL, describe, rel_l2, run_oracle, vel_segment

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = V.Context(0)
    yield c
    c.close()


def _edge_field(n_extra):
    x, z, g = W.random_field(np.random.default_rng(11), 60)
    xe = ze = ge = np.zeros(0)
    if n_extra:
        xe, ze, ge = W.random_field(np.random.default_rng(12), n_extra, sigma_gamma=0.005)
    x = np.concatenate([x, xe, [30.0, 30.0, 1.2, 1.5, 2.0, 2.4, 0.8]])
    z = np.concatenate([z, ze, [0.25, -0.25, 0.1, -0.2, 0.3, -0.1, 0.05]])
    g = np.concatenate([g, ge, [-2.0, 2.0, 0.0, 0.0, 1e-33, 1e-20, -1e-12]])
    return W.f32(x), W.f32(z), W.f32(g)


# N_b = 16: the small class holds up to 689 vortices at its default shape,
# so 67 + 6 runs there and 867 + 6 in the large class
@pytest.mark.parametrize("name,n_extra,path", [("small", 0, V.PATH_AUTO),
                                               ("large", 800, V.PATH_AUTO),
                                               ("streamed", 0, V.PATH_STREAM)])
def test_scaled_source_edges_match_oracle(ctx, name, n_extra, path):
    wl = W.workload_from_state("scaled_edges_" + name, W.make_params(16), _edge_field(n_extra),
                               K=2, H=3, eps=W.f32(np.full((2, 3), 0.05)))
    o = run_oracle(wl, final_wake=True, vel_last=True, gamma_s=True)
    ctx.set_path(path)
    try:
        g = V.run_workload(ctx, wl, V.FP32C, final_wake=True, vel_last=True, gamma_s=True)
    finally:
        ctx.set_path(V.PATH_AUTO)
    tol = TOL[V.FP32C]
    assert np.all(g["status"] == 0), g["status"]
    assert np.array_equal(g["n_final"], o["n_final"])
    for k in range(wl.K):
        e = rel_l2(vel_segment(g, k), vel_segment(o, k))
        assert e <= tol, describe(wl.name + " velocity k=%d" % k, err=e)
    for key in ("gamma_s", "g_final"):
        e = rel_l2(g[key], o[key])
        assert e <= tol, describe(wl.name + " " + key, err=e)
