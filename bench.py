"""Benchmark of the rollout hot path on one MI355X.

One step = one MPPI iteration of the planner's hot path on one batch:
``vpm_rollout_batch`` (K rollouts x H steps of the VPM-glider model, terminal
cost) followed by ``mppi_weights`` (softmin weights and the control update).
Inputs are resident in HBM before the timed region starts.

Default workload: K = 1024 rollouts, H = 200 steps at dt = 2.5 ms, 32 bound
vortices, one disturbance pair, FP32 with compensated sums (FP64 surface
solve). Prints one JSON line.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp32c", "fp64"], default="fp32c")
    ap.add_argument("--K", type=int, default=1024)
    ap.add_argument("--H", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256, help="rollouts timed on the oracle")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def cpu_baseline(wl, n_sample):
    """The FP64 oracle on a bounded sample of the same workload, all host cores."""
    from oracle import oracle as O
    O.build(force=False)
    idx = np.linspace(0, wl.K - 1, n_sample).astype(np.int64)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    O.rollout_batch(wl.params, wl.K, wl.H, wl.dt, wl.g0, wl.gb0, wl.field_off, wl.field_of,
                    wl.wx, wl.wz, wl.wg, wl.pairs, wl.u, wl.x_goal, wl.q_diag,
                    rollouts=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    from paper_2509_16079_amd import workloads as W
    pairs = sum(sum(W.pair_count(wl.n0[k], wl.H, wl.params["n_bound"],
                                 n_wake_max=wl.params["n_wake_max"])) for k in idx)
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle", "rollouts_per_s": n_sample / dt, "seconds": dt,
            "sample": "%d of the %d rollouts (evenly spaced indices), full horizon H=%d, "
                      "OpenMP over rollouts" % (n_sample, wl.K, wl.H)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the rollouts of one batch are independent and "
              "this build measures one GPU's share; see the sharding notes in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2509_16079_amd import vpm as V
    from paper_2509_16079_amd import workloads as W

    prec = V.FP32C if args.precision == "fp32c" else V.FP64
    wl = W.realtime(K=args.K, H=args.H)
    ctx = V.Context(0)
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db, pair_count=True)
    stream = torch.cuda.current_stream()
    reg_sing = [W.pair_count(n, wl.H, wl.params["n_bound"], n_wake_max=wl.params["n_wake_max"])
                for n in wl.n0]
    n_reg = sum(r for r, _ in reg_sing)
    n_sing = sum(s for _, s in reg_sing)
    pairs_per_step = n_reg + n_sing
    flop_per_launch = FLOP_REG * n_reg + FLOP_SING * n_sing

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.rollout(wl.params, db, out, prec, stream)
        if ev is not None:
            ev[1].record(stream)
        ctx.mppi(out.cost, wl.lam, db.u_mean, db.u_eps, stream)

    if args.calibrate_copy_mb > 0:
        src = torch.empty(args.calibrate_copy_mb << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert int(out.pair_count.sum().item()) == pairs_per_step
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    kern_avg = float(np.mean(kern_ms))
    ms = 1e3 * wall / args.steps
    status = out.status.cpu().numpy()
    achieved = flop_per_launch / (kern_avg * 1e-3) / 1e12
    line = {
        "metric": "vortex pair-interactions/s, MPPI rollouts/s, p50/p99 replan latency vs plain",
        "value": pairs_per_step / (ms * 1e-3),
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == V.FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": "realtime FP32-vs-FP64 batch: K=%d rollouts, H=%d steps, "
                               "dt=2.5 ms, N_b=32, N_w<=%d, one disturbance pair"
                               % (wl.K, wl.H, 2 + 2 * wl.H),
                   "K": wl.K, "H": wl.H, "n_bound": 32, "precision": args.precision},
        "rollouts_per_s": wl.K / (ms * 1e-3),
        "pairs_per_step": pairs_per_step,
        "rollout_kernel_ms": kern_avg,
        "nonfinite_rollouts": int(np.sum(status != 0)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
