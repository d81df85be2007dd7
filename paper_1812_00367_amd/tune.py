"""Launch-shape tuner for nb_evaluate.

For each active-set size it times every compiled shape (bodies per lane, waves per
workgroup, LDS tile) at several j-split targets, on the device it runs on, and
keeps the fastest. The result is a table for Simulation.eval_table() /
nb_eval_table(): rows (n_act_max, ipl, waves, tile, target_waves), where a row
covers active sets up to the geometric midpoint to the next tuned size.

    python -m paper_1812_00367_amd.tune [--n 65536] [--precision fp64|split]

prints the table as JSON (and as a C initializer).
"""
from __future__ import annotations

import argparse
import json
import math

SHAPES = [(1, 1, 64), (1, 1, 128), (1, 2, 128), (1, 1, 256), (1, 2, 256), (1, 4, 256),
          (2, 1, 64), (2, 1, 128), (2, 2, 128), (2, 1, 256), (2, 2, 256), (2, 4, 256)]
TARGETS = [1024, 2048, 4096, 8192, 16384, 32768]
DEFAULT_SIZES = [1, 4, 16, 64, 256, 1024, 4096, 16384, 65536]


def time_eval(sim, idx, out, reps, warm):
    import torch
    stream = sim.stream
    for _ in range(warm):
        sim.evaluate_into(idx, out)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        sim.evaluate_into(idx, out)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return ms[len(ms) // 2]


def tune(sim, sizes=None, seed=20, shapes=SHAPES, targets=TARGETS, log=None):
    """Returns (rows, results); results[n_act] = (best_ms, shape, target, plan)."""
    import torch

    import nbody_inputs as ni
    n = sim.n
    sizes = [s for s in (sizes or DEFAULT_SIZES) if s <= n]
    out = torch.empty((10, n), dtype=torch.float64, device=sim.device)
    results = {}
    for k, na in enumerate(sizes):
        idx = torch.as_tensor(ni.active_subset(n, na, seed + k), device=sim.device)
        work = na * n
        reps = 3 if work > 1e9 else 7
        best = None
        seen = set()
        for shape in shapes:
            for tw in targets:
                sim.eval_table([(1 << 30, *shape, tw)])
                plan = sim.eval_config(None, na)
                key = (plan["ipl"], plan["waves"], plan["tile"], plan["splits"])
                if key in seen:
                    continue
                seen.add(key)
                ms = time_eval(sim, idx, out, reps, 2)
                if best is None or ms < best[0]:
                    best = (ms, shape, tw, plan)
        results[na] = best
        if log:
            log(f"n_act={na}: {best[0]:.4f} ms shape={best[1]} target={best[2]} plan={best[3]} "
                f"({na * n / (best[0] / 1e3):.3e} interactions/s)")
    sim.eval_table(None)
    rows = []
    for k, na in enumerate(sizes):
        upper = (1 << 30) if k + 1 == len(sizes) else int(math.sqrt(na * sizes[k + 1]))
        ms, shape, tw, _ = results[na]
        rows.append((upper, *shape, tw))
    # merge neighbouring rows with the same choice
    merged = []
    for r in rows:
        if merged and merged[-1][1:] == r[1:]:
            merged[-1] = r
        else:
            merged.append(r)
    return merged, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--precision", choices=("fp64", "split"), default="fp64")
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args()
    import nbody_inputs as ni
    import paper_1812_00367_amd as nb
    ic = ni.plummer(args.n, args.seed)
    sim = nb.Simulation(args.n, eps=1e-4,
                        precision=nb.NB_SPLIT if args.precision == "split" else nb.NB_FP64)
    sim.set_state(ic.m, ic.x, ic.v, a=ni.plummer_mean_field_acc(ic.x))
    sim.predict(0)
    rows, results = tune(sim, log=lambda s: print(s, flush=True))
    print(json.dumps({"n": args.n, "precision": args.precision, "rows": rows,
                      "best_ms": {str(k): v[0] for k, v in results.items()}}), flush=True)
    print("C: " + ", ".join("{%d, %d, %d, %d, %d}" % tuple(r) for r in rows), flush=True)


if __name__ == "__main__":
    main()
