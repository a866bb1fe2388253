"""CPU: the rollout kernels' logic, compiled for the CPU against an emulation
of the HIP subset they use (tests/emu), against the FP64 oracle: indexing,
task partitioning, synchronisation (a deadlock fails the test by timeout)
and the results to the GPU parity tolerances, over horizons short enough
that the conditioning of the flow does not enter. It does not replace the
GPU tests (it does not see the compiler's code generation)."""
import json
import os
import subprocess
import sys

import pytest

from tests.parity import TOL

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def emu_lib():
    r = subprocess.run([sys.executable, os.path.join(EMU, "build.py")], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return r.stdout.strip()


@pytest.mark.parametrize("case", ["empty", "realtime", "nb64", "uneven", "large", "large_tuned",
                                  "shed_te", "shed_none", "gated", "feedback", "scaled_edges",
                                  "tail_t1"])
def test_emulated_kernels_match_oracle(emu_lib, case):
    try:
        r = subprocess.run([sys.executable, os.path.join(EMU, "run_cases.py"), case],
                           capture_output=True, text=True, timeout=300, cwd=ROOT)
    except subprocess.TimeoutExpired:
        pytest.fail("emulated kernels did not finish (deadlock?) on case " + case)
    assert r.returncode == 0, r.stderr[-3000:]
    rows = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")]
    assert len(rows) == 2
    for row in rows:
        tol = TOL[row["prec"]]
        assert all(s == 0 for s in row["status"]), row
        assert row["n_final_equal"], row
        if row["gate_margin"] is not None:  # the decisions are robust to rounding
            assert row["gate_margin"] > 1e-5, row
        for key in ("traj", "gamma_s", "g_final", "gb_final", "vel_last"):
            assert row[key] <= tol, (key, row)
        assert row["wake"] <= 10 * tol, row


@pytest.mark.parametrize("case,deficient", [("policy_linear", 1), ("policy_vpm", 0)])
def test_emulated_policy_kernels_match_oracle(emu_lib, case, deficient):
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_cases.py"), case],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    row = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")][0]
    assert row["status_equal"] and row["n_rank_deficient"] == deficient, row
    for key in ("A", "B", "S", "gain"):
        assert row[key] <= 1e-9, (key, row)


def test_emulated_replanning_cycle_matches_oracle(emu_lib):
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_cases.py"), "replan"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    row = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")][0]
    for cyc in ("cycle0", "cycle1"):
        c = row[cyc]
        assert c["argmin_equal"] and c["status_equal"], row
        for key in ("g_proj", "jmin", "u_new", "x_new"):
            assert c[key] <= 1e-10, (cyc, key, row)
        assert c["gain"] <= 1e-7, (cyc, row)


def test_emulated_fd_jacobians_match_oracle(emu_lib):
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_cases.py"), "fd"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    row = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")][0]
    assert row["x_nom"] <= 1e-13 and row["A"] <= 1e-10 and row["B"] <= 1e-10, row
    assert row["gain"] <= 1e-7, row
