"""Autotuner for the FP32 rollout kernels.

For a workload, it times every kernel shape of each class that the workload
runs: targets per thread in {1, 2, 4} and sources per compensated tile in
{64, 128, 256}. The timing uses HIP events around `vpm_rollout_batch` on the
current stream, and the median of a few launches is taken. The classes are
tuned one at a time, the others held at their best shape so far, because an
uneven batch runs its classes concurrently. The result is a JSON table keyed
by GPU architecture and kernel class, which `apply` loads into a context
through `vpm_set_tuning`.

    python -m paper_2509_16079_amd.autotune --workload realtime --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import vpm as V
from . import workloads as W

SHAPES = [(t, tile) for t in (1, 2, 4) for tile in (64, 128, 256)]
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def classes_used(ctx_caps, wl):
    """Kernel classes a batch runs, from its wake capacities (N_0 + 2H) and
    the class capacities (cap_small, cap_large) for its plate."""
    cap_small, cap_large = ctx_caps
    caps = np.asarray(wl.n0) + 2 * wl.H
    out = set()
    for c in np.unique(caps):
        out.add(V.CLASS_SMALL if c <= cap_small else V.CLASS_LARGE if c <= cap_large
                else V.CLASS_STREAM)
    return sorted(out)


def time_batch(ctx, wl, db, out, reps=3, precision=V.FP32C):
    import torch
    ctx.rollout(wl.params, db, out, precision)          # warm-up (and buffer sizing)
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.rollout(wl.params, db, out, precision)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def sweep(ctx, wl, classes, reps=3, log=print):
    """Coordinate search over the classes; returns {class: (t, tile, ms, {shape: ms})}."""
    db = V.DeviceBatch(wl)
    out = V.DeviceOutputs(db)
    best = {}
    for cls in classes:
        results = {}
        for t, tile in SHAPES:
            ctx.set_tuning(cls, t, tile)
            ms = time_batch(ctx, wl, db, out, reps)
            results["%d/%d" % (t, tile)] = ms
            log("  %s T=%d tile=%d: %.3f ms" % (V.CLASS_NAMES[cls], t, tile, ms))
        key = min(results, key=results.get)
        t, tile = (int(x) for x in key.split("/"))
        ctx.set_tuning(cls, t, tile)
        best[cls] = (t, tile, results[key], results)
    return best


def class_capacities(wl):
    """cap_small / cap_large of the library's class rule for this plate, at
    the default shapes (4-wave workgroups within a quarter of the 160 KB LDS,
    16-wave within all of it): fixed bytes per rollout plus 24 B per vortex
    (the small class 40 B: it also holds the scaled pass-A copy)."""
    nb = wl.params["n_bound"]
    S = nb + 2

    def cap(nw, tmax, budget, per_vortex):
        fixed = S * S * 8 + (2 * nb + 3) * 16 + nw * 64 * tmax * 8 + 32 + 2600
        return (budget - fixed) // per_vortex
    return cap(4, 4, 163840 // 4, 40), cap(16, 2, 163840, 24)


def table_entry(wl_name, wl, best):
    return {V.CLASS_NAMES[c]: {"targets_per_thread": t, "tile": tile, "ms": ms,
                               "workload": wl_name, "n_bound": wl.params["n_bound"],
                               "candidates_ms": res}
            for c, (t, tile, ms, res) in best.items()}


def apply(ctx, table):
    """Load a table written by `main` into a context."""
    for name, e in table.get("classes", {}).items():
        cls = {v: k for k, v in V.CLASS_NAMES.items()}[name]
        ctx.set_tuning(cls, int(e["targets_per_thread"]), int(e["tile"]))


def load(path=DEFAULT_TABLE):
    with open(path) as f:
        return json.load(f)


def _short(wl, H):
    from dataclasses import replace
    return replace(wl, H=H, u_mean=wl.u_mean[:H], u_eps=wl.u_eps[:, :H])


WORKLOADS = {
    "realtime": lambda: W.realtime(),
    "uneven": lambda: W.uneven_batch(),
    "uneven_small": lambda: W.uneven_batch(K=1024, H=30),
    "stress_slice": lambda: _short(W.large_stress().subset(np.arange(256)), 10),
}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", action="append", choices=sorted(WORKLOADS),
                    help="workloads whose classes to tune, in order (repeatable)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args(argv)
    names = args.workload or ["realtime", "uneven_small", "stress_slice"]
    import torch
    ctx = V.Context(0)
    table = {"arch": "gfx950", "method": "median of %d HIP-event-timed launches per shape; "
             "classes tuned in turn, others at their best" % args.reps, "classes": {}}
    done = set()
    try:
        for name in names:
            wl = WORKLOADS[name]()
            classes = [c for c in classes_used(class_capacities(wl), wl) if c not in done]
            if not classes:
                continue
            print("%s: tuning %s" % (name, [V.CLASS_NAMES[c] for c in classes]), flush=True)
            best = sweep(ctx, wl, classes, args.reps,
                         log=lambda m: print(m, flush=True))
            table["classes"].update(table_entry(name, wl, best))
            done.update(classes)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
