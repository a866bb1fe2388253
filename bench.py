"""Benchmark of the rollout hot path on one MI355X.

One step = one MPPI iteration of the planner's hot path on one batch:
``vpm_rollout_batch`` (K rollouts x H steps of the VPM-glider model and the
terminal cost) followed by ``mppi_weights`` (softmin weights and the control
update). Inputs are resident in HBM before the timed region starts.

Workloads (``--workload``):
  realtime (default)  K=1024, H=200, dt=2.5 ms, 32 bound vortices, one
                      disturbance pair, FP32 with compensated sums
  plain               K=32, H=100, dt=5 ms, 16 bound vortices, merging above
                      200, FP64
  uneven              K=4096, H=100, initial wakes of 50..4000 vortices each
                      (log-uniform), FP32, planned persistent class kernels
  stress              K=8192, H=150, 16376-vortex Lamb-Oseen field, 64 bound
                      vortices, merging above 16384, FP32 (streamed wakes)
  policy              the local feedback policy (Sec. IV-B) at the paper's
                      controller size: least-squares Jacobians from K=256
                      perturbed FP64 rollouts of 77 steps (dt = 10 ms) and
                      the TVLQR recursion; one step = one vpm_policy call on
                      resident trajectories
  table1              the paper's runtime-versus-batch table (Table I): batches
                      of 1, 128, 256, 512 and 1024 rollouts of 80 steps at
                      dt = 10 ms with at most 60 wake vortices; one step = one
                      rollout batch + MPPI weights; the paper's RTX 5080
                      runtimes are printed beside ours as context
  icsweep             the comparison of Sec. IV-B's Fig. 3: open loop,
                      least-squares and finite-difference TVLQR feedback
                      from 41 initial forward speeds offset by -0.5..0.5 m/s
                      around the nominal of one replanning cycle; reports
                      each policy's region of attraction (5 cm final
                      position error) and the time of the whole pipeline
  nmpc                the nonlinear MPC closed in simulation: a truth model
                      flies the 77-step manoeuvre under the policy in force
                      while the planner replans every 10 steps (horizon
                      shrinking to the end), with the disturbance pair
                      absent, known to the planner or unknown to it, and
                      the open-loop plan for comparison
  replan              one replanning cycle of the nonlinear MPC (Sec. IV-C)
                      at the paper's controller size: projection by 10 steps
                      under the policy in force, 3 MPPI iterations of 256
                      rollouts x 77 steps, 257 policy rollouts and the
                      policy; one step = one vpm_replan call
The default run also replays the first requests of the serving trace through
the replanning service (8 slots) and through the plain one-at-a-time path,
reporting p50/p99 latency and rollouts/s for both, and times one whole MPPI
step of the large stress batch (all 8192 rollouts x 150 steps, as 8
launches of 1024 rollouts) under the ``stress`` key, with its error against
the FP64 oracle on a 64-rollout subsample. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
FLOP_REG, FLOP_SING = 13, 11  # algorithmic FLOP per regularised / singular pair
METRIC = "vortex pair-interactions/s, MPPI rollouts/s, p50/p99 replan latency vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["realtime", "plain", "uneven", "stress", "policy",
                                           "replan", "table1", "icsweep", "nmpc"],
                    default="realtime")
    ap.add_argument("--precision", choices=["fp32c", "fp64"], default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="also replay the serving requests at 0.25/0.5/0.8 of capacity")
    ap.add_argument("--tuning", default=None,
                    help="kernel-shape table written by paper_2509_16079_amd.autotune "
                         "(default: the packaged table if present; 'none': library defaults)")
    ap.add_argument("--graph", choices=["on", "off"], default=None,
                    help="capture one MPPI step (rollout batch + weights) in a HIP graph after "
                         "the warm-up and time its replays (default: on for the uneven batch)")
    ap.add_argument("--serving-slots", type=int, default=8,
                    help="concurrent slots of the served replay (default 8)")
    ap.add_argument("--serving-requests", type=int, default=None,
                    help="requests of the serving trace to replay (0: skip)")
    ap.add_argument("--slice", type=int, default=None,
                    help="launch the batch in slices of this many rollouts, reporting each "
                         "finished slice (default: whole batch; 1024 for stress)")
    ap.add_argument("--stress-record", choices=["on", "off"], default=None,
                    help="time one full MPPI step of the stress batch after the realtime "
                         "line (default: on for the realtime workload)")
    ap.add_argument("--max-k", type=int, default=None,
                    help="run only the first K rollouts of the workload (profiling runs of "
                         "one launch)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def make_workload(name):
    from paper_2509_16079_amd import workloads as W
    if name == "realtime":
        wl = W.realtime()
        desc = ("realtime FP32-vs-FP64 batch: K=1024 rollouts, H=200 steps, dt=2.5 ms, "
                "N_b=32, N_w<=402, one disturbance pair")
        return wl, desc, "fp32c", (10, 3)
    if name == "plain":
        wl = W.plain_single_plan()
        desc = ("plain single plan: K=32 rollouts, H=100 steps, dt=5 ms, N_b=16, "
                "N_w,max=200, one disturbance pair")
        return wl, desc, "fp64", (20, 3)
    if name == "uneven":
        wl = W.uneven_batch()
        desc = ("uneven batch: K=4096 rollouts, H=100 steps, dt=5 ms, N_b=32, initial wakes "
                "log-uniform in [50, 4000] vortices, one planned persistent launch")
        return wl, desc, "fp32c", (3, 1)
    wl = W.large_stress()
    desc = ("large stress: K=8192 rollouts, H=150 steps, dt=5 ms, N_b=64, 16376-vortex "
            "Lamb-Oseen field + 4 pairs, N_w,max=16384")
    return wl, desc, "fp32c", (1, 0)


def work_counts(wl):
    from paper_2509_16079_amd import workloads as W
    cache = {}
    n_reg = n_sing = 0
    for n in wl.n0:
        n = int(n)
        if n not in cache:
            cache[n] = W.pair_count(n, wl.H, wl.params["n_bound"],
                                    n_wake_max=wl.params["n_wake_max"])
        r, s = cache[n]
        n_reg += r
        n_sing += s
    return n_reg, n_sing


# Committed rocprofv3 summary holding the measured HBM traffic of the
# dominant kernel per workload (FETCH_SIZE and WRITE_SIZE passes, scaled by a
# copy-kernel calibration); it is reported only while the kernel source still
# has the hash recorded beside it.
TRAFFIC_PROFILE = {"realtime": "profiles/rollout_lds_kernel_realtime_K1024_H200.md",
                   "stress": "profiles/rollout_stream_kernel_stress_K8192_H150.md"}


def measured_traffic(workload):
    import hashlib
    path = TRAFFIC_PROFILE.get(workload)
    if path is None:
        return None
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(here, path)).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        key, _, val = line.strip().partition(":")
        if key in ("traffic_bytes_per_launch", "source_sha256"):
            fields[key] = val.strip()
    src = os.path.join(here, "paper_2509_16079_amd", "csrc", "rollout.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if fields.get("source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(name, wl):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload, all host cores (OpenMP over rollouts). Returns the baseline
    record, the sampled workload and the oracle's outputs on it."""
    from oracle import oracle as O
    from paper_2509_16079_amd import workloads as W
    O.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    H = wl.H
    if name == "realtime":
        idx = np.linspace(0, wl.K - 1, 256).astype(np.int64)
        what = "256 of the 1024 rollouts (evenly spaced), full horizon H=200"
    elif name == "plain":
        idx = np.arange(wl.K)
        what = "all 32 rollouts, full horizon H=100"
    elif name == "uneven":
        order = np.argsort(wl.n0)
        idx = order[np.linspace(0, wl.K - 1, 64).astype(np.int64)]
        what = "64 rollouts stratified by initial wake size, full horizon H=100"
    else:
        idx = np.linspace(0, wl.K - 1, 64).astype(np.int64)
        H = STRESS_ORACLE_STEPS
        what = ("64 rollouts (evenly spaced), first %d of 150 steps, per-pair rate"
                % STRESS_ORACLE_STEPS)
    sub = wl.subset(idx)
    if H != wl.H:
        from dataclasses import replace
        sub = replace(sub, H=H, u_mean=sub.u_mean[:H], u_eps=sub.u_eps[:, :H])
    t0 = time.perf_counter()
    o = O.rollout_batch(sub.params, sub.K, sub.H, sub.dt, sub.g0, sub.gb0, sub.field_off,
                        sub.field_of, sub.wx, sub.wz, sub.wg, sub.pairs, sub.u, sub.x_goal,
                        sub.q_diag, final_wake=True, n_threads=threads,
                        vel_last=name == "stress", gamma_s=name == "stress",
                        traj=name == "stress")
    dt = time.perf_counter() - t0
    pairs = sum(sum(W.pair_count(int(n), H, sub.params["n_bound"],
                                 n_wake_max=sub.params["n_wake_max"])) for n in sub.n0)
    out = {"value": pairs / dt, "unit": "pair-interactions/s", "cores": threads,
           "kind": "oracle", "seconds": dt, "sample": what + "; OpenMP over rollouts",
           "cpu_model": cpu_model()}
    if name in ("plain", "realtime"):
        # one thread, on the first 32 rollouts of the sample
        one = sub.subset(np.arange(min(32, sub.K)))
        t1 = time.perf_counter()
        O.rollout_batch(one.params, one.K, one.H, one.dt, one.g0, one.gb0, one.field_off,
                        one.field_of, one.wx, one.wz, one.wg, one.pairs, one.u, one.x_goal,
                        one.q_diag, n_threads=1)
        d1 = time.perf_counter() - t1
        p1 = sum(sum(W.pair_count(int(n), H, one.params["n_bound"],
                                  n_wake_max=one.params["n_wake_max"])) for n in one.n0)
        out["single_thread"] = {"value": p1 / d1, "rollouts_per_s": one.K / d1,
                                "seconds": d1, "sample": "%d rollouts, full horizon" % one.K}
    if H == wl.H:
        out["rollouts_per_s"] = len(idx) / dt
    o["mppi"] = O.mppi(o["cost"], sub.lam, sub.u_mean, sub.u_eps)
    if name in ("realtime", "plain", "uneven"):
        # the oracle against itself with every velocity sum in reverse order:
        # the amplification of rounding differences by the flow over this
        # horizon, i.e. the floor no other summation order can beat
        r = O.rollout_batch(sub.params, sub.K, sub.H, sub.dt, sub.g0, sub.gb0, sub.field_off,
                            sub.field_of, sub.wx, sub.wz, sub.wg, sub.pairs, sub.u, sub.x_goal,
                            sub.q_diag, reverse=True, n_threads=threads)
        o["self_divergence"] = {
            "final_state_rel_l2": _rel_l2(r["g_final"], o["g_final"]),
            "mppi_argmin_equal": O.mppi(r["cost"], sub.lam, sub.u_mean, sub.u_eps)["argmin"]
                                 == o["mppi"]["argmin"]}
    return out, sub, o


def apply_tuning(ctx, path):
    """Load the autotuner's table into the context; returns what runs."""
    from paper_2509_16079_amd import autotune as A
    from paper_2509_16079_amd import vpm as V
    if path is None:
        path = A.DEFAULT_TABLE if os.path.exists(A.DEFAULT_TABLE) else "none"
    if path != "none":
        A.apply(ctx, A.load(path))
    shapes = {V.CLASS_NAMES[c]: "%d targets/thread, %d-source tiles" % ctx.get_tuning(c)
              for c in (V.CLASS_SMALL, V.CLASS_LARGE, V.CLASS_STREAM)}
    return {"table": os.path.relpath(path, os.path.dirname(os.path.abspath(__file__)))
            if path != "none" else None, "fp32_shapes": shapes}


def gpu_clock():
    """Current shader and memory clock levels from the driver's sysfs tables
    (the entry marked '*'), read after the timed region; None if absent.
    A file read, not a tool: nothing is spawned inside the GPU process."""
    import glob
    out = {}
    for card in sorted(glob.glob("/sys/class/drm/card*/device")):
        for name in ("pp_dpm_sclk", "pp_dpm_mclk"):
            try:
                for line in open(os.path.join(card, name)):
                    if line.rstrip().endswith("*"):
                        out[name[7:]] = line.split(":", 1)[1].strip(" *\n")
            except OSError:
                continue
        if out:
            out["card"] = os.path.basename(os.path.dirname(card))
            return out
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def error_vs_oracle(V, ctx, sub, o, prec, horizon_note):
    """The GPU path on the oracle's sample (same inputs, same horizon), in an
    extra launch outside the timed region, against the oracle's outputs."""
    import torch
    db = V.DeviceBatch(sub)
    out = V.DeviceOutputs(db, final_wake=True)
    ctx.rollout(sub.params, db, out, prec)
    w, _, am, _ = ctx.mppi(out.cost, sub.lam, db.u_mean, db.u_eps)
    torch.cuda.synchronize()
    g = out.to_numpy()
    seg_g, seg_o, circ = [], [], []
    for k in range(sub.K):
        n = int(g["n_final"][k])
        a0, b0 = int(g["out_off"][k]), int(o["out_off"][k])
        gx = np.concatenate([g["wx"][a0:a0 + n], g["wz"][a0:a0 + n]])
        ox = np.concatenate([o["wx"][b0:b0 + n], o["wz"][b0:b0 + n]])
        seg_g.append(gx)
        seg_o.append(ox)
        og = o["wg"][b0:b0 + n]
        circ.append(abs(g["wg"][a0:a0 + n].sum() - og.sum()) / max(np.abs(og).sum(), 1e-300))
    finite = np.isfinite(o["cost"])
    return {
        "horizon": horizon_note,
        "final_state_rel_l2": _rel_l2(g["g_final"], o["g_final"]),
        "cost_max_rel": float(np.max(np.abs(g["cost"][finite] - o["cost"][finite])
                                     / np.abs(o["cost"][finite]))) if finite.any() else None,
        "final_wake_positions_rel_l2": _rel_l2(np.concatenate(seg_g), np.concatenate(seg_o)),
        "circulation_drift_max": float(max(circ)) if circ else 0.0,
        "wake_counts_equal": bool(np.array_equal(g["n_final"], o["n_final"])),
        "mppi_weights_max_abs": float(np.max(np.abs(w.cpu().numpy() - o["mppi"]["w"]))),
        "mppi_argmin_equal": int(am.item()) == o["mppi"]["argmin"],
    }


def serving(n_requests, sweep=False, slots=8, tuning=None):
    """Replay the first requests of the serving trace (Poisson arrivals at
    100 req/s, K~U{256..2048}, H~U{50..200}, 16 resident states of
    500..6000 vortices, perturbations drawn by the library from each
    request's seed) through the service with `slots` concurrent slots and
    through the plain path (the same service with one slot: one request at a
    time, same kernels). Both are sized up front for the trace's largest
    request (planner_reserve) and run the tuned kernel shapes. With `sweep`,
    also replay them at offered loads of 0.25, 0.5 and 0.8 of the capacity
    measured in the saturated replay (arrival gaps stretched)."""
    from paper_2509_16079_amd import autotune as A
    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    params, states, reqs = W.serving_trace()
    reqs = reqs[:n_requests]
    dt = float(W.f32(0.005))
    g0 = np.array([0, 0, 0, 0, 6.0, 0, 0])
    if tuning is None:
        tuning = A.DEFAULT_TABLE if os.path.exists(A.DEFAULT_TABLE) else "none"
    table = A.load(tuning) if tuning != "none" else None
    k_max, h_max = max(r.K for r in reqs), max(r.H for r in reqs)
    n_max = max(len(st[0]) for st in states)

    def replay(n_slots, stretch=1.0):
        p = V.Planner(max_slots=n_slots, budget_bytes=64 << 30)
        try:
            sids = [p.put_state(*st, g0, np.zeros(32)) for st in states]
            if table is not None:
                A.apply(p, table)
            p.reserve(params, K=k_max, H=h_max, n0=n_max)
            # warm-up (not timed): one small request per resident state
            for sid in sids:
                p.poll(p.submit(sid, params, np.zeros(4), np.zeros((64, 4)), dt))
            t_start = time.perf_counter()
            tickets = []
            for r in reqs:
                delay = (t_start + stretch * (r.t_arrive - reqs[0].t_arrive)
                         - time.perf_counter())
                if delay > 0:
                    time.sleep(delay)
                tickets.append(p.submit(sids[r.state], params, np.zeros(r.H), None, dt,
                                        seed=r.seed, sigma=0.15, K=r.K))
            res = [p.poll(t) for t in tickets]
        finally:
            p.close()
        assert all(x["status"] == 0 for x in res)
        lat = np.array([x["t_done_us"] - x["t_arrive_us"] for x in res]) * 1e-3
        span = (max(x["t_done_us"] for x in res) - min(x["t_arrive_us"] for x in res)) * 1e-6
        rollouts = sum(r.K for r in reqs)
        pairs = sum(x["pairs"] for x in res)
        print("serving replay with %d slot(s) done" % n_slots, file=sys.stderr, flush=True)
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "rollouts_per_s": rollouts / span, "pair_interactions_per_s": pairs / span,
                "makespan_s": span}

    served = replay(slots)
    plain = replay(1)
    out = {"requests": len(reqs), "trace": "first %d requests of the seeded 100 req/s "
           "trace (K~U{256..2048}, H~U{50..200}, resident states of 500..6000 vortices)"
           % len(reqs),
           "latency_sample": "%d requests (p99 interpolated between the two slowest)"
           % len(reqs),
           "tuning": os.path.relpath(tuning, ROOT) if tuning != "none" else None,
           "served_slots": slots,
           "served": served, "plain_one_at_a_time": plain,
           "p99_speedup": plain["p99_ms"] / served["p99_ms"],
           "rollouts_speedup": served["rollouts_per_s"] / plain["rollouts_per_s"]}
    if sweep:
        # capacity in requests/s from the saturated replay; the trace offers
        # len(reqs) requests over its arrival span
        cap = len(reqs) / max(served["makespan_s"], plain["makespan_s"])
        offered = (len(reqs) - 1) / max(reqs[-1].t_arrive - reqs[0].t_arrive, 1e-9)
        out["capacity_req_per_s"] = cap
        out["sweep"] = []
        for f in (0.25, 0.5, 0.8):
            stretch = offered / (f * cap)
            s8, s1 = replay(slots, stretch), replay(1, stretch)
            out["sweep"].append({"load": f, "served": s8, "plain_one_at_a_time": s1,
                                 "p99_speedup": s1["p99_ms"] / s8["p99_ms"]})
            print("serving sweep load %.2f done" % f, file=sys.stderr, flush=True)
    return out


STRESS_DESC = ("large stress: K=8192 rollouts, H=150 steps, dt=5 ms, N_b=64, 16376-vortex "
               "Lamb-Oseen field + 4 pairs, N_w,max=16384")


def stress_record(args, with_oracle=True):
    """One whole MPPI step of the large stress batch, timed once after a
    256-rollout warm-up launch: 8 launches of 1024 rollouts (HIP events
    around each, on the launch stream) and the weights over all 8192. Then
    the GPU path on a 64-rollout subsample (evenly spaced) for the first
    STRESS_ORACLE_STEPS steps in FP32C and FP64 against the FP64 oracle on
    the machine's host cores, which also gives the oracle's CPU rate."""
    import torch

    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    wl = W.large_stress()
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, pair_count=True)
    stream = torch.cuda.current_stream()
    n_reg, n_sing = work_counts(wl)
    slice_k = 1024
    n_launch = wl.K // slice_k
    ctx.rollout(wl.params, db, out, V.FP32C, stream, 0, 256)
    torch.cuda.synchronize()
    print("stress warm-up done", file=sys.stderr, flush=True)
    evs = []
    t0 = time.perf_counter()
    for k0 in range(0, wl.K, slice_k):
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(stream)
        ctx.rollout(wl.params, db, out, V.FP32C, stream, k0, k0 + slice_k)
        ev[1].record(stream)
        ev[1].synchronize()
        evs.append(ev)
        print("stress launch %d..%d done" % (k0, k0 + slice_k), file=sys.stderr, flush=True)
    ctx.mppi(out.cost, wl.lam, db.u_mean, db.u_eps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = n_reg + n_sing
    assert int(out.pair_count.sum().item()) == pairs
    kern = [a.elapsed_time(b) for a, b in evs]
    kern_ms = float(np.mean(kern))
    flop_launch = (FLOP_REG * n_reg + FLOP_SING * n_sing) / n_launch
    achieved = flop_launch / (kern_ms * 1e-3) / 1e12
    status = out.status.cpu().numpy()
    rec = {"workload": STRESS_DESC, "K": wl.K, "H": wl.H, "n_bound": wl.params["n_bound"],
           "precision": "fp32c", "steps": 1, "warmup": "one 256-rollout launch",
           "seconds_per_mppi_step": wall, "pair_interactions_per_s": pairs / wall,
           "rollouts_per_s": wl.K / wall, "pairs_per_step": pairs, "launches": n_launch,
           "rollout_kernel_ms_per_launch": kern_ms,
           "rollout_kernel_ms_min_max": [float(min(kern)), float(max(kern))],
           "kernel_timing": "HIP events around each 1024-rollout launch on its stream",
           "nonfinite_rollouts": int(np.sum(status != 0)), "tuning": tuning,
           "gpu_clock_after_timed_region": gpu_clock(),
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                        "traffic": measured_traffic("stress")}}
    del db, out
    ctx.close()
    if with_oracle:
        base, sub, o = cpu_baseline("stress", wl)
        rec["cpu_baseline"] = base
        ctx = V.Context(0)
        rec["error_vs_oracle"] = {
            name: stress_errors(V, ctx, sub, o, prec)
            for name, prec in (("fp32c", V.FP32C), ("fp64", V.FP64))}
        ctx.close()
    return rec


STRESS_ORACLE_STEPS = 4


def stress_errors(V, ctx, sub, o, prec):
    """GPU against the oracle on the stress subsample: the C4 error figures,
    with the circulation drift max over steps of |sum Gamma_W (GPU) - sum
    Gamma_W (oracle)|, where the wake's total after each solve is minus the
    surface total (Kelvin row of the solve)."""
    import torch
    db = V.DeviceBatch(sub)
    out = V.DeviceOutputs(db, final_wake=True, vel_last=True, gamma_s=True, traj=True)
    ctx.rollout(sub.params, db, out, prec)
    w, _, am, _ = ctx.mppi(out.cost, sub.lam, db.u_mean, db.u_eps)
    torch.cuda.synchronize()
    g = out.to_numpy()
    vel = max(_rel_l2(g["vel_last"][g["out_off"][k]:g["out_off"][k] + g["n_vel_last"][k]],
                      o["vel_last"][o["out_off"][k]:o["out_off"][k] + o["n_vel_last"][k]])
              for k in range(sub.K))
    seg_g, seg_o = [], []
    for k in range(sub.K):
        n = int(g["n_final"][k])
        a0, b0 = int(g["out_off"][k]), int(o["out_off"][k])
        seg_g.append(np.concatenate([g["wx"][a0:a0 + n], g["wz"][a0:a0 + n]]))
        seg_o.append(np.concatenate([o["wx"][b0:b0 + n], o["wz"][b0:b0 + n]]))
    drift = np.abs(g["gamma_s"].sum(axis=2) - o["gamma_s"].sum(axis=2))
    return {"horizon": "%d steps, 64 rollouts (evenly spaced)" % sub.H,
            "velocities_last_step_rel_l2_max": vel,
            "gamma_s_rel_l2": _rel_l2(g["gamma_s"], o["gamma_s"]),
            "traj_rel_l2": _rel_l2(g["traj"], o["traj"]),
            "final_state_rel_l2": _rel_l2(g["g_final"], o["g_final"]),
            "final_wake_positions_rel_l2": _rel_l2(np.concatenate(seg_g), np.concatenate(seg_o)),
            "circulation_drift_max": float(drift.max()),
            "wake_counts_equal": bool(np.array_equal(g["n_final"], o["n_final"])),
            "mppi_weights_max_abs": float(np.max(np.abs(w.cpu().numpy() - o["mppi"]["w"]))),
            "mppi_argmin_equal": int(am.item()) == o["mppi"]["argmin"]}


def policy_bytes(K, H):
    """Algorithmic bytes of one vpm_policy call: trajectories, control
    deviations and the nominal read once; A, B, gains, S and status written
    once."""
    return 8 * (K * (H + 1) * 7 + K * H + (H + 1) * 7) + 8 * H * (49 + 7 + 7) \
        + 8 * (H + 1) * 49 + 4 * H


def policy_main(args):
    import torch

    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    K, H = 256, 77
    steps = 50 if args.steps is None else args.steps
    warmup = 5 if args.warmup is None else args.warmup
    wl = W.policy_batch(K=K, H=H)
    ctx = V.Context(0)
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, traj=True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.rollout(wl.params, db, out, V.FP64, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    rollout_ms = e0.elapsed_time(e1)
    traj, du = out.traj, db.u_eps[1:]
    q_f = [400.0, 400.0, 10.0, 1.0, 1.0, 1.0, 1.0]   # TVLQR weights of Sec. V-A
    q_c = [0.1, 0.1, 5.0, 0.1, 0.1, 0.1, 5.0]
    r_c = 0.01
    for _ in range(warmup):
        pol = V.policy(ctx, traj[0], traj[1:], du, wl.dt, q_f, q_c, r_c, stream=stream)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(stream)
        pol = V.policy(ctx, traj[0], traj[1:], du, wl.dt, q_f, q_c, r_c, stream=stream)
        ev[1].record(stream)
        evs.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    each = [a.elapsed_time(b) for a, b in evs]
    kern = float(np.mean(each))
    ms = 1e3 * wall / steps
    nbytes = policy_bytes(K, H)
    achieved = nbytes / (kern * 1e-3) / 1e9
    line = {
        "metric": "local feedback policy construction time (LS Jacobians + TVLQR)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "policy: K=256 perturbed FP64 rollouts + nominal, H=77, "
                               "dt=10 ms, N_b=32, one disturbance pair", "K": K, "H": H},
        "policy_kernels_ms": kern,
        "policy_kernels_ms_median": float(np.median(each)),
        "rollout_batch_ms_fp64": rollout_ms,
        "rank_deficient_steps": int(pol["status"].sum().item()),
        "kernel_timing": "HIP events around each vpm_policy call (synthesis + Riccati) on its "
                         "stream",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "traffic": None},
        "gpu_clock_after_timed_region": gpu_clock(),
    }
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import policy as P
        tr = traj.cpu().numpy()
        dun = du.cpu().numpy()
        reps = 0
        with threadpool_limits(1):          # the oracle on one core
            t0 = time.perf_counter()
            while reps < 20 or time.perf_counter() - t0 < 2.0:
                o = P.policy(tr[0], tr[1:], dun, wl.dt, q_f, q_c, r_c)
                reps += 1
            cpu_ms = 1e3 * (time.perf_counter() - t0) / reps
        line["cpu_baseline"] = {"value": cpu_ms, "unit": "ms", "cores": 1, "kind": "oracle",
                                "sample": "the whole workload (same trajectories), %d calls"
                                          % reps}
        g = {k: v.cpu().numpy() for k, v in pol.items() if v is not None}
        line["error_vs_oracle"] = {
            "gain_rel_l2": _rel_l2(g["gain"], o["gain"]),
            "A_rel_l2": _rel_l2(g["a"], o["A"]), "S_rel_l2": _rel_l2(g["s"], o["S"]),
            "status_equal": bool(np.array_equal(g["status"], o["status"]))}
    ctx.close()
    print(json.dumps(line), flush=True)


def replan_main(args):
    import torch

    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    steps = 30 if args.steps is None else args.steps
    warmup = 3 if args.warmup is None else args.warmup
    prec_name = args.precision or "fp32c"
    prec = V.FP32C if prec_name == "fp32c" else V.FP64
    c = W.replan_case()
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    dev = lambda a: None if a is None else torch.tensor(
        np.ascontiguousarray(a), device="cuda",
        dtype=torch.int32 if np.asarray(a).dtype == np.int32 else torch.float64)
    state = tuple(dev(c[k]) for k in ("g", "gb", "wx", "wz", "wg", "pairs"))
    args_d = (dev(c["u_eps"]), dev(c["x_eps"]), dev(c["du"]))
    stream = torch.cuda.current_stream()

    def cycle(plan):
        return V.replan(ctx, c["params"], prec, c["dt"], state, plan, *args_d, c["lam"],
                        c["x_goal"], c["q_diag"], c["q_f"], c["q_c"], c["r_c"], c["P"],
                        stream=stream)
    # the first cycle projects open loop; later cycles project under the
    # policy the previous cycle produced (same resident state each time)
    out = cycle((dev(c["u_plan"]), None, None))
    for _ in range(warmup):
        out = cycle((out["u_new"].clone(), out["x_new"][:-1].contiguous(), out["gain"].clone()))
    torch.cuda.synchronize()
    plan = (out["u_new"].clone(), out["x_new"][:-1].contiguous(), out["gain"].clone())
    evs, walls = [], []
    for _ in range(steps):
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        t0 = time.perf_counter()
        ev[0].record(stream)
        out = cycle(plan)
        ev[1].record(stream)
        ev[1].synchronize()
        walls.append(1e3 * (time.perf_counter() - t0))
        evs.append(ev)
    each = [a.elapsed_time(b) for a, b in evs]
    H, K, I, Kp, P = c["H"], c["K"], c["iterations"], c["Kp"], c["P"]
    ms = float(np.mean(walls))
    line = {
        "metric": "replanning-cycle latency (projection + MPPI iterations + LS-TVLQR policy)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == V.FP32C else "f64", "data": "synthetic",
        "config": {"workload": "replan: project %d steps, %d MPPI iterations of K=%d x H=%d, "
                               "%d policy rollouts, dt=10 ms, N_b=32, one disturbance pair"
                               % (P, I, K, H, Kp + 1), "K": K, "H": H, "P": P,
                   "iterations": I, "Kp": Kp, "precision": prec_name},
        "latency_ms_p50": float(np.percentile(walls, 50)),
        "latency_ms_p99": float(np.percentile(walls, 99)),
        "gpu_ms_mean": float(np.mean(each)),
        "replan_budget_ms": 100.0,
        "rollouts_per_cycle": 1 + I * K + Kp + 1,
        "argmin_last": out["argmin"].cpu().tolist(),
        "tuning": tuning,
        "kernel_timing": "HIP events around each vpm_replan call on its stream; wall time "
                         "from the call to its completion",
        "gpu_clock_after_timed_region": gpu_clock(),
    }
    if not args.no_cpu_baseline:
        from oracle import replan as OR
        u_plan, x_plan, gain_plan = (t.cpu().numpy() for t in plan)
        t0 = time.perf_counter()
        o = OR.replan(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"],
                      c["pairs"], u_plan, x_plan, gain_plan, P, c["u_eps"], c["x_eps"], c["du"],
                      c["lam"], c["x_goal"], c["q_diag"], c["q_f"], c["q_c"], c["r_c"])
        cpu_ms = 1e3 * (time.perf_counter() - t0)
        line["cpu_baseline"] = {"value": cpu_ms, "unit": "ms",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle",
                                "sample": "one whole cycle (FP64, OpenMP over rollouts)"}
        g = {k: v.cpu().numpy() for k, v in out.items()}
        line["error_vs_oracle"] = {
            "precision": prec_name,
            "argmin_equal": bool(np.array_equal(g["argmin"], o["argmin"])),
            "u_new_rel_l2": _rel_l2(g["u_new"], o["u_new"]),
            "x_new_rel_l2": _rel_l2(g["x_new"], o["x_new"]),
            "gain_rel_l2": _rel_l2(g["gain"], o["gain"])}
    ctx.close()
    print(json.dumps(line), flush=True)


def table1_main(args):
    import torch

    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    steps = 20 if args.steps is None else args.steps
    warmup = 3 if args.warmup is None else args.warmup
    prec_name = args.precision or "fp32c"
    prec = V.FP32C if prec_name == "fp32c" else V.FP64
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    stream = torch.cuda.current_stream()
    rows = []
    for K, paper_ms in zip(W.TABLE1_BATCHES, W.TABLE1_PAPER_MS):
        wl = W.table1(K)
        db = V.DeviceBatch(wl)
        out = V.DeviceOutputs(db)

        def step():
            ctx.rollout(wl.params, db, out, prec, stream)
            ctx.mppi(out.cost, wl.lam, db.u_mean, db.u_eps, stream)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record(stream)
            step()
            ev[1].record(stream)
            evs.append(ev)
        torch.cuda.synchronize()
        wall = 1e3 * (time.perf_counter() - t0) / steps
        gpu = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        pairs = int(out.pair_count.sum().item())
        rows.append({"K": K, "ms_per_step": wall, "gpu_ms": gpu, "rollouts_per_s": K / (wall * 1e-3),
                     "pairs_per_s": pairs / (wall * 1e-3),
                     "nonfinite_rollouts": int((out.status != 0).sum().item()),
                     "paper_rtx5080_ms": paper_ms})
    top = rows[-1]
    line = {
        "metric": "MPPI rollouts/s (the paper's runtime-versus-batch table)",
        "value": top["rollouts_per_s"], "unit": "rollouts/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": top["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == V.FP32C else "f64", "data": "synthetic",
        "config": {"workload": "table1: 80 steps, dt=10 ms, merging above 60 wake vortices, "
                               "N_b=32, one disturbance pair; batch 1024 is the value",
                   "H": 80, "n_bound": 32, "precision": prec_name},
        "batches": rows,
        "paper_context": "RTX 5080 runtimes of the paper's table (precision, N_b and what the "
                         "timing includes are not stated): 8.0 / 10.3 / 12.2 / 16.3 / 27.2 ms",
        "tuning": tuning,
        "kernel_timing": "HIP events around each step (rollout batch + MPPI weights); "
                         "ms_per_step is wall time per step with launches enqueued back to back",
        "gpu_clock_after_timed_region": gpu_clock(),
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def icsweep_main(args):
    import torch

    from paper_2509_16079_amd import icsweep as S
    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    steps = 3 if args.steps is None else args.steps
    prec_name = args.precision or "fp64"
    prec = V.FP32C if prec_name == "fp32c" else V.FP64
    c = W.replan_case(P=0)
    offsets = np.linspace(-0.5, 0.5, 41)
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    g = S.run(ctx, c, offsets, prec)        # warm-up (builds inverses, workspaces)
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = S.run(ctx, c, offsets, prec)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    roa = {k: g[k]["roa"] for k in ("open", "ls", "fd")}
    width = {k: (v[1] - v[0]) if v else 0.0 for k, v in roa.items()}
    line = {
        "metric": "initial-condition sweep: region of attraction per policy (5 cm final "
                  "position error) and pipeline time",
        "value": float(np.median(times)), "unit": "ms", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": float(np.median(times)), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == V.FP64 else "f32", "data": "synthetic",
        "config": {"workload": "icsweep: replanning cycle (3 x 256 MPPI rollouts, 77 steps, "
                               "257 policy rollouts), FD Jacobians along its nominal, 3 x 41 "
                               "sweep rollouts over x_dot offsets -0.5..0.5 m/s",
                   "precision": prec_name},
        "region_of_attraction_m_per_s": roa,
        "roa_width_m_per_s": width,
        "final_pos_err_m": {k: [round(float(x), 4) for x in g[k]["pos_err"]]
                            for k in ("open", "ls", "fd")},
        "offsets_m_per_s": [round(float(x), 4) for x in offsets],
        "tuning": tuning,
        "kernel_timing": "wall time of the whole pipeline (every stage synchronised)",
    }
    if not args.no_cpu_baseline:
        from oracle import icsweep as OI
        t0 = time.perf_counter()
        o = OI.run(c, offsets, S.FD_H_X, S.FD_H_U)
        line["cpu_baseline"] = {"value": 1e3 * (time.perf_counter() - t0), "unit": "ms",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle", "sample": "the whole sweep (FP64)"}
        line["error_vs_oracle"] = {
            k: {"g_final_rel_l2": _rel_l2(g[k]["g_final"], o[k]["g_final"]),
                "roa_equal": S.region_of_attraction(offsets, o[k]["pos_err"]) == g[k]["roa"]}
            for k in ("open", "ls", "fd")}
    ctx.close()
    print(json.dumps(line), flush=True)


def nmpc_main(args):
    import torch

    from paper_2509_16079_amd import nmpc as N
    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W
    prec_name = args.precision or "fp32c"
    prec = V.FP32C if prec_name == "fp32c" else V.FP64
    c = W.replan_case()
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    N.simulate(ctx, c, "compensated", prec)          # warm-up (inverses, workspaces)
    res, lat = {}, []
    t0 = time.perf_counter()
    for sc in N.SCENARIOS:
        r = N.simulate(ctx, c, sc, prec)
        err, cost = N.final_error(c, r["traj"])
        res[sc] = {"final_pos_err_m": err, "final_cost": cost,
                   "replan_ms": [round(float(x), 3) for x in r["replan_ms"]]}
        lat.extend(r["replan_ms"])
    wall = 1e3 * (time.perf_counter() - t0)
    ol = N.open_loop(ctx, c, prec)
    err, cost = N.final_error(c, ol["traj"])
    res["open_loop_with_disturbance"] = {"final_pos_err_m": err, "final_cost": cost}
    torch.cuda.synchronize()
    line = {
        "metric": "closed-loop NMPC in simulation: final perch error per scenario and "
                  "replanning latency",
        "value": float(np.percentile(lat, 50)), "unit": "ms (replanning cycle, p50)",
        "n_gpus": 1, "steps": len(lat), "warmup": 1, "ms_per_step": float(np.mean(lat)),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == V.FP32C else "f64", "data": "synthetic",
        "config": {"workload": "nmpc: 77-step manoeuvre at dt=10 ms, replanning every 10 "
                               "steps (3 x 256 MPPI rollouts, 257 policy rollouts), goal x_d of "
                               "Sec. IV-A, one disturbance pair", "precision": prec_name},
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "replan_budget_ms": 100.0,
        "scenarios": res,
        "simulation_wall_ms": wall,
        "tuning": tuning,
        "kernel_timing": "wall time of each vpm_replan call to its completion",
    }
    if not args.no_cpu_baseline:
        from oracle import nmpc as ON
        t0 = time.perf_counter()
        o = ON.simulate(c, "compensated")
        line["cpu_baseline"] = {"value": 1e3 * (time.perf_counter() - t0), "unit": "ms",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle",
                                "sample": "the compensated scenario's whole simulation (FP64)"}
        g64 = N.simulate(ctx, c, "compensated", V.FP64)
        line["error_vs_oracle"] = {"fp64_truth_traj_rel_l2": _rel_l2(g64["traj"], o["traj"]),
                                   "fp64_jmin_rel_l2": _rel_l2(g64["jmin"], o["jmin"])}
    ctx.close()
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the rollouts of one batch are independent and "
              "this build measures one GPU's share; see the sharding notes in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "policy":
        return policy_main(args)
    if args.workload == "replan":
        return replan_main(args)
    if args.workload == "table1":
        return table1_main(args)
    if args.workload == "icsweep":
        return icsweep_main(args)
    if args.workload == "nmpc":
        return nmpc_main(args)
    import torch

    from paper_2509_16079_amd import vpm as V

    wl, desc, prec_name, (steps_d, warm_d) = make_workload(args.workload)
    if args.max_k is not None and args.max_k < wl.K:
        wl = wl.subset(np.arange(args.max_k))
        desc += "; first %d rollouts only" % args.max_k
    steps = steps_d if args.steps is None else args.steps
    warmup = warm_d if args.warmup is None else args.warmup
    prec_name = args.precision or prec_name
    prec = V.FP32C if prec_name == "fp32c" else V.FP64
    ctx = V.Context(0)
    tuning = apply_tuning(ctx, args.tuning)
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, pair_count=True)
    stream = torch.cuda.current_stream()
    n_reg, n_sing = work_counts(wl)
    pairs_per_step = n_reg + n_sing
    flop_per_launch = FLOP_REG * n_reg + FLOP_SING * n_sing

    slice_k = args.slice if args.slice is not None else (1024 if args.workload == "stress" else 0)
    kernel_ms = []

    def step(timed=False):
        if slice_k <= 0 or slice_k >= wl.K:
            if timed:
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                ev[0].record(stream)
            ctx.rollout(wl.params, db, out, prec, stream)
            if timed:
                ev[1].record(stream)
                kernel_ms.append(ev)
        else:
            for k0 in range(0, wl.K, slice_k):
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                ev[0].record(stream)
                ctx.rollout(wl.params, db, out, prec, stream, k0, min(wl.K, k0 + slice_k))
                ev[1].record(stream)
                ev[1].synchronize()
                if timed:
                    kernel_ms.append(ev)
                print("slice %d..%d done" % (k0, min(wl.K, k0 + slice_k)), file=sys.stderr,
                      flush=True)
        ctx.mppi(out.cost, wl.lam, db.u_mean, db.u_eps, stream)

    if args.calibrate_copy_mb > 0:
        src = torch.empty(args.calibrate_copy_mb << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    use_graph = (args.graph == "on") or (args.graph is None and args.workload == "uneven")
    if use_graph and 0 < slice_k < wl.K:
        sys.exit("--graph needs the whole batch in one launch (use --slice 0)")
    for _ in range(max(warmup, 1 if use_graph else 0)):
        step()
    torch.cuda.synchronize()
    graph = None
    if use_graph:
        # the eager warm-up sized every buffer; the capture allocates nothing
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            cs = torch.cuda.current_stream()
            ctx.rollout(wl.params, db, out, prec, cs)
            ctx.mppi(out.cost, wl.lam, db.u_mean, db.u_eps, cs)
        graph.replay()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if graph is None:
            step(timed=True)
        else:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record(stream)
            graph.replay()
            ev[1].record(stream)
            kernel_ms.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(out.pair_count.sum().item()) == pairs_per_step
    kern_each = [a.elapsed_time(b) for a, b in kernel_ms]
    kern_avg = float(sum(kern_each) / steps)
    ms = 1e3 * wall / steps
    status = out.status.cpu().numpy()
    achieved = flop_per_launch / (kern_avg * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": pairs_per_step / (ms * 1e-3),
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == V.FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "K": wl.K, "H": wl.H, "n_bound": wl.params["n_bound"],
                   "precision": prec_name},
        "rollouts_per_s": wl.K / (ms * 1e-3),
        "pairs_per_step": pairs_per_step,
        "rollout_kernel_ms": kern_avg,
        "rollout_kernel_ms_median": float(np.median(kern_each)) if kern_each else None,
        "gpu_clock_after_timed_region": gpu_clock(),
        "launch_slices": 1 if slice_k <= 0 or slice_k >= wl.K else -(-wl.K // slice_k),
        "hip_graph": graph is not None,
        "tuning": tuning,
        "kernel_timing": ("HIP events around each replay of the captured graph (rollout batch "
                          "+ MPPI weights)") if graph is not None else
                         "HIP events around each rollout launch on its stream",
        "nonfinite_rollouts": int(np.sum(status != 0)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(args.workload)},
    }
    ctx.close()
    n_serve = args.serving_requests
    if n_serve is None:
        n_serve = 64 if args.workload == "realtime" and args.max_k is None else 0
    if n_serve > 0:
        line["serving"] = serving(n_serve, sweep=args.serving_sweep, slots=args.serving_slots,
                                  tuning=args.tuning)
    if args.stress_record == "on" or (args.stress_record is None and
                                      args.workload == "realtime" and args.max_k is None):
        line["stress"] = stress_record(args, with_oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        base, sub, o = cpu_baseline(args.workload, wl)
        line["cpu_baseline"] = base
        ctx = V.Context(0)
        note = "%d steps on the oracle's sample (%s)" % (sub.H, base["sample"])
        line["error_vs_oracle"] = {prec_name: error_vs_oracle(V, ctx, sub, o, prec, note)}
        if prec == V.FP32C:
            line["error_vs_oracle"]["fp64"] = error_vs_oracle(V, ctx, sub, o, V.FP64, note)
        if "self_divergence" in o:
            line["error_vs_oracle"]["oracle_reverse_order"] = o["self_divergence"]
        ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
