"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and validates arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_16079_amd import vpm as V
from paper_2509_16079_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"VPM_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt)
    return names


def test_library_exports_every_declared_symbol():
    lib = V.lib()
    names = declared_symbols()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


def _valid_args():
    wl = W.realtime(K=4, H=3)
    p = V.make_params(wl.params)
    b = V.BatchIn()
    b.K, b.H, b.dt, b.n_fields, b.max_wake0, b.n_pairs = 4, 3, wl.dt, 1, 2, 1
    fake = C.c_void_p(0x1000)   # never dereferenced: validation is host-only
    for f in ("g0", "gb0", "field_off", "field_of", "wx", "wz", "wg", "pairs", "u_mean", "u_eps"):
        setattr(b, f, fake)
    for i in range(7):
        b.x_goal[i] = wl.x_goal[i]
        b.q_diag[i] = wl.q_diag[i]
    o = V.BatchOut()
    o.g_final = o.cost = o.status = fake
    return p, b, o


def _validate(p, b, o):
    return V.lib().vpm_validate_batch(C.byref(p), C.byref(b), C.byref(o))


def test_validation_accepts_valid_arguments():
    assert _validate(*_valid_args()) == V.OK


@pytest.mark.parametrize("field,value,code", [
    ("K", 0, V.EINVAL), ("H", 0, V.EINVAL), ("dt", 0.0, V.EINVAL), ("dt", float("nan"), V.EINVAL),
    ("n_fields", 0, V.EINVAL), ("max_wake0", -1, V.EINVAL), ("n_pairs", 5, V.EINVAL),
    ("g0", None, V.EINVAL), ("u_eps", None, V.EINVAL), ("wx", None, V.EINVAL),
])
def test_validation_rejects_bad_batch(field, value, code):
    p, b, o = _valid_args()
    setattr(b, field, value)
    assert _validate(p, b, o) == code
    assert V.lib().vpm_last_error()


@pytest.mark.parametrize("field,value", [
    ("n_bound", 0), ("n_bound", 65), ("shed_mode", 3), ("shed_mode", -1), ("gate", 2),
    ("precision", 2), ("chord", 0.0),
    ("r_core", 0.0), ("mass", -1.0), ("inertia", 0.0), ("decay", -0.1), ("rho", float("inf")),
])
def test_validation_rejects_bad_params(field, value):
    p, b, o = _valid_args()
    setattr(p, field, value)
    assert _validate(p, b, o) == V.EINVAL


def test_shedding_modes_and_gate_rules():
    for mode in (V.SHED_BOTH, V.SHED_TE, V.SHED_NONE):
        p, b, o = _valid_args()
        p.shed_mode = mode
        assert _validate(p, b, o) == V.OK
    p, b, o = _valid_args()
    p.gate, p.alpha_crit = 1, 0.1
    assert _validate(p, b, o) == V.OK
    for mode, crit in ((V.SHED_TE, 0.1), (V.SHED_NONE, 0.1), (V.SHED_BOTH, float("nan"))):
        p, b, o = _valid_args()      # the gate switches between BOTH and TE only
        p.gate, p.shed_mode, p.alpha_crit = 1, mode, crit
        assert _validate(p, b, o) == V.EINVAL
    p, b, o = _valid_args()
    p.shed_mode, p.n_bound = V.SHED_NONE, 1  # no collocation row would remain
    assert _validate(p, b, o) == V.EINVAL


def test_validation_output_rules():
    p, b, o = _valid_args()
    o.cost = None
    assert _validate(p, b, o) == V.EINVAL
    p, b, o = _valid_args()
    o.wx = C.c_void_p(0x1000)     # a wake output without wake_off / n_final
    assert _validate(p, b, o) == V.EINVAL
    p, b, o = _valid_args()
    b.field_of = None             # one field cannot serve 4 rollouts by index
    assert _validate(p, b, o) == V.EINVAL


def test_null_context_is_rejected():
    p, b, o = _valid_args()
    assert V.lib().vpm_rollout_batch(None, C.byref(p), C.byref(b), C.byref(o), None) == V.EINVAL
    assert V.lib().mppi_weights(None, 1, 1, None, 1.0, None, None, None, None, None, None,
                                None) == V.EINVAL


def test_pair_count_agrees_with_schedule():
    for n0, H, nb, cap in ((2, 100, 16, 200), (2, 200, 32, 800), (900, 100, 32, 0), (0, 5, 3, 4)):
        reg, sing = W.pair_count(n0, H, nb, n_wake_max=cap)
        assert V.pair_count(n0, H, nb, cap) == reg + sing


def test_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2509_16079_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower() or f == "workloads.py", f
                assert "vpm_oracle" not in txt, f


def test_tuning_arguments_are_checked_without_a_gpu():
    L = V.lib()
    t, tile = C.c_int32(), C.c_int32()
    assert L.vpm_set_tuning(None, 0, 4, 64) == V.EINVAL
    assert L.vpm_get_tuning(None, 0, C.byref(t), C.byref(tile)) == V.EINVAL


def test_policy_arguments_are_checked_without_a_gpu():
    L = V.lib()
    fake = C.c_void_p(0x1000)     # never dereferenced: validation is host-only
    pin = V.PolicyIn(8, 5, 0.01, fake, fake, fake)
    for i in range(7):
        pin.q_f[i], pin.q_c[i] = 1.0, 0.1
    pin.r_c = 0.01
    pout = V.PolicyOut(fake, fake, fake, None, fake)
    assert L.vpm_policy(None, C.byref(pin), C.byref(pout), None) == V.EINVAL
    bad = [("K", 0), ("H", 0), ("dt", 0.0), ("r_c", 0.0), ("r_c", float("nan")), ("du", None)]
    for field, value in bad:
        b = V.PolicyIn.from_buffer_copy(pin)
        setattr(b, field, value)
        assert L.vpm_policy(fake, C.byref(b), C.byref(pout), None) == V.EINVAL, field
    b = V.PolicyIn.from_buffer_copy(pin)
    b.q_c[3] = -1.0
    assert L.vpm_policy(fake, C.byref(b), C.byref(pout), None) == V.EINVAL
    o = V.PolicyOut.from_buffer_copy(pout)
    o.gain = None
    assert L.vpm_policy(fake, C.byref(pin), C.byref(o), None) == V.EINVAL


def test_replan_arguments_are_checked_without_a_gpu():
    L = V.lib()
    fake = C.c_void_p(0x1000)     # never dereferenced: validation is host-only
    p = V.make_params(W.make_params(16), V.FP64)

    def good():
        r = V.ReplanIn(0.01, 10, 2, 8, 2, 8, 4, 0, 0, fake, fake, fake, fake, fake, None, fake,
                       None, None, fake, fake, fake, 1.0)
        r.r_c = 0.01
        return r
    o = V.ReplanOut(*([fake] * 7))
    assert L.vpm_replan(None, C.byref(p), C.byref(good()), C.byref(o), None) == V.EINVAL
    bad = [("H", 0), ("P", 11), ("P", -1), ("K", 0), ("iterations", 0), ("Kp", 0),
           ("n_wake", -1), ("n_pairs", 5), ("lam", 0.0), ("dt", float("nan")), ("u_eps", None),
           ("x_plan", fake)]   # x_plan without gain_plan
    for field, value in bad:
        r = good()
        setattr(r, field, value)
        assert L.vpm_replan(fake, C.byref(p), C.byref(r), C.byref(o), None) == V.EINVAL, field
    r = good()
    r.n_pairs, r.pairs = 1, fake                     # pairs with a wake that may merge
    p2 = V.make_params(W.make_params(16, n_wake_max=20), V.FP64)
    assert L.vpm_replan(fake, C.byref(p2), C.byref(r), C.byref(o), None) == V.EINVAL
    o2 = V.ReplanOut(*([fake] * 6 + [None]))
    assert L.vpm_replan(fake, C.byref(p), C.byref(good()), C.byref(o2), None) == V.EINVAL


def test_tvlqr_and_fd_arguments_are_checked_without_a_gpu():
    L = V.lib()
    fake = C.c_void_p(0x1000)     # never dereferenced: validation is host-only
    q = (C.c_double * 7)(*([1.0] * 7))
    assert L.vpm_tvlqr(None, 5, fake, fake, q, q, 0.01, fake, None, None) == V.EINVAL
    assert L.vpm_tvlqr(fake, 0, fake, fake, q, q, 0.01, fake, None, None) == V.EINVAL
    assert L.vpm_tvlqr(fake, 5, fake, fake, q, q, 0.0, fake, None, None) == V.EINVAL
    assert L.vpm_tvlqr(fake, 5, None, fake, q, q, 0.01, fake, None, None) == V.EINVAL
    p = V.make_params(W.make_params(16), V.FP64)

    def good():
        return V.FdIn(0.01, 10, 4, 0, 0, fake, fake, fake, fake, fake, None, fake,
                      (C.c_double * 5)(*([1e-4] * 5)), 1e-4)
    o = V.FdOut(fake, fake, None)
    for field, value in [("H", 0), ("n_wake", -1), ("n_pairs", 5), ("h_u", 0.0),
                         ("dt", 0.0), ("u_nom", None)]:
        r = good()
        setattr(r, field, value)
        assert L.vpm_fd_jacobians(fake, C.byref(p), C.byref(r), C.byref(o), None) == V.EINVAL
    r = good()
    r.h_x[2] = -1e-4
    assert L.vpm_fd_jacobians(fake, C.byref(p), C.byref(r), C.byref(o), None) == V.EINVAL
    assert L.vpm_fd_jacobians(fake, C.byref(p), C.byref(good()), C.byref(V.FdOut(fake, None, None)),
                              None) == V.EINVAL
