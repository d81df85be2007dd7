"""Launch-shape tuner for nb_evaluate.

For each active-set size it times every compiled shape (bodies per lane, waves per
workgroup, LDS tile) at several j-split targets, on the device it runs on, and
keeps the fastest. The result is a table for Simulation.eval_table() /
nb_eval_table(): rows (n_act_max, ipl, waves, tile, target_waves), where a row
covers active sets up to the geometric midpoint to the next tuned size.

    python -m paper_1812_00367_amd.tune [--n 65536] [--precision fp64|split]

prints the table as JSON (and as a C initializer).

    python -m paper_1812_00367_amd.tune --time-shapes '1024=default,-128/8/256/32'

times the given shapes (interleaved rounds) instead, one JSON line per shape.

    python -m paper_1812_00367_amd.tune --batch 128 [--sweep split|factors] [--precision fp64|split]

tunes the batch path instead: it times an ensemble of clusters for each pair of
(j-records per lane, work items per job), or for each setting of the chunk-length
factors of the three item classes, and prints the fastest, to be passed to
Batch(jchunk=..., items_per_job=..., chunk_tile=..., chunk_wide=..., chunk_direct=...)
/ nb_batch_params.
"""
from __future__ import annotations

import argparse
import json
import math

SHAPES = [(1, 1, 64), (1, 1, 128), (1, 2, 128), (1, 1, 256), (1, 2, 256), (1, 4, 256),
          (2, 1, 64), (2, 1, 128), (2, 2, 128), (2, 1, 256), (2, 2, 256), (2, 4, 256)]
# the small-set kernel (FP64): at most P active bodies per wave on 64 / P lanes each,
# records from LDS tiles (tile 64) or straight from memory (tile 0); timed only for
# active sets up to SMALL_MAX
SMALL_SHAPES = [(-p, 1, t) for t in (0, 64) for p in (1, 2, 4, 8, 16, 32, 64)]
SMALL_MAX = 1024
# the group kernel (FP64): every wave of a workgroup on one group of at most P active
# bodies, the waves sharing the split's records from LDS tiles of 256 (all sizes) or
# read straight from memory (tile 0; timed only up to GROUP_DIRECT_MAX active bodies)
GROUP_SHAPES = [(-p, w, 256) for w in (4, 8) for p in (2, 4, 8, 16, 32, 64, 128)]
GROUP_DIRECT = [(-p, w, 0) for w in (4, 8) for p in (1, 2, 4, 8, 16)]
GROUP_DIRECT_MAX = 64
TARGETS = [128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768]
# active-set sizes up to n / 2: a full set (n_act = n) takes the pairwise-symmetric
# kernel, which the table does not choose
DEFAULT_SIZES = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768]


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


def tune(sim, sizes=None, seed=20, shapes=SHAPES, targets=TARGETS, log=None, small=True):
    """Returns (rows, results); results[n_act] = (best_ms, shape, target, plan).
    small: also time the small-set and group kernels' shapes (FP64 contexts only)."""
    import torch

    import nbody_inputs as ni
    n = sim.n
    sizes = [s for s in (sizes or DEFAULT_SIZES) if s < n]
    out = torch.empty((10, n), dtype=torch.float64, device=sim.device)
    results = {}
    for k, na in enumerate(sizes):
        idx = torch.as_tensor(ni.active_subset(n, na, seed + k), device=sim.device)
        work = na * n
        reps = 3 if work > 1e9 else 7
        best = None
        seen = set()
        cands = list(shapes)
        if small:
            cands += (SMALL_SHAPES if na <= SMALL_MAX else []) + GROUP_SHAPES
            cands += GROUP_DIRECT if na <= GROUP_DIRECT_MAX else []
        for shape in cands:
            for tw in targets:
                sim.eval_table([(1 << 30, *shape, tw)])
                plan = sim.eval_config(None, na)
                key = (plan["ipl"], plan["waves"], plan["tile"], plan["splits"], plan["fused"])
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


BATCH_JCHUNKS = [64, 128, 192, 256]
BATCH_TARGETS = [512, 2048, 8192]
# chunk-length factors of the tile, wide and direct item classes
BATCH_FACTORS = [(1, 4, 1), (2, 4, 1), (4, 4, 1), (2, 2, 1), (2, 8, 1), (2, 4, 2)]


def batch_configs(sweep):
    """Batch keyword arguments to time: sweep "split" covers (jchunk, items_per_job),
    "factors" the class factors (chunk_tile, chunk_wide, chunk_direct) at the default
    jchunk and items_per_job."""
    if sweep == "split":
        return [dict(jchunk=jc, items_per_job=tg) for jc in BATCH_JCHUNKS for tg in BATCH_TARGETS]
    if sweep == "factors":
        return [dict(chunk_tile=t, chunk_wide=w, chunk_direct=d) for t, w, d in BATCH_FACTORS]
    raise ValueError(f"unknown sweep {sweep!r}")


def tune_batch(clusters, tick_end, precision, configs, steps_per_call=32, log=None):
    """Time the batch path on an ensemble once for every configuration (a dict of
    Batch keyword arguments) and return (best configuration, [interactions/s per
    configuration]). `clusters` is a list of objects with m, x, v (one job each), all
    integrated to tick_end."""
    import time

    import torch

    from .batch import Batch
    cap = sum(len(ic.m) for ic in clusters)
    rates = []
    for cfg in configs:
        b = Batch(cap, len(clusters), precision=precision, **cfg)
        for ic in clusters:
            if b.add(ic.m, ic.x, ic.v, tick_end) is None:
                raise RuntimeError("ensemble does not fit")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inter = 0
        while True:
            _, _, _, it, taken = b.run_steps(steps_per_call)
            inter += it
            if taken < steps_per_call:
                break
        dt = time.perf_counter() - t0
        rates.append(inter / dt)
        if log:
            log(f"{cfg}: {inter / dt:.3e} interactions/s ({dt:.2f} s)")
        b.close()
    best = max(range(len(configs)), key=lambda k: rates[k])
    return configs[best], rates


def parse_shapes(spec):
    """'1024=default,-128/8/256/32;8192=default' -> {1024: [None, (-128, 8, 256, 32)], ...}"""
    out = {}
    for part in filter(None, spec.split(";")):
        na, cfgs = part.split("=")
        out[int(na)] = [None if c == "default" else tuple(int(v) for v in c.split("/"))
                        for c in cfgs.split(",")]
    return out


def time_shapes(sim, cases, rounds=5, reps=3, seed=20, log=print):
    """Interleaved timing of forced launch shapes (None: the built-in table): for each
    active-set size, `rounds` passes over its shapes, each timing `reps` calls after one
    warm-up call; returns and logs the median per shape. Also logs the event time of a
    one-element add, the floor under any single-launch figure."""
    import torch

    import nbody_inputs as ni
    x = torch.zeros(1, dtype=torch.float64, device=sim.device)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(50)]
    for a, b in ev:
        a.record()
        x.add_(1.0)
        b.record()
    torch.cuda.synchronize()
    tiny = sorted(a.elapsed_time(b) for a, b in ev)[25]
    log(json.dumps({"one_tiny_kernel_event_us": round(tiny * 1e3, 2)}))
    out = torch.empty((10, sim.n), dtype=torch.float64, device=sim.device)
    res = []
    for na, cfgs in cases.items():
        idx = torch.as_tensor(ni.active_subset(sim.n, na, seed + na), device=sim.device)
        times = {k: [] for k in range(len(cfgs))}
        for _ in range(rounds):
            for k, cfg in enumerate(cfgs):
                sim.eval_config(cfg, na)
                times[k].append(time_eval(sim, idx, out, reps, 1))
        for k, cfg in enumerate(cfgs):
            shape = sim.eval_config(cfg, na)
            ms = sorted(times[k])[len(times[k]) // 2]
            r = {"n_act": na, "cfg": cfg, "us": round(ms * 1e3, 2),
                 "frac_fp64": round(79.0 * na * sim.n / (ms * 1e-3) / 78.6e12, 4), "shape": shape}
            res.append(r)
            log(json.dumps(r))
    sim.eval_config(None)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--precision", choices=("fp64", "split"), default="fp64")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--sizes", default="", help="comma-separated active-set sizes to tune "
                    "(default: powers of two up to n / 2)")
    ap.add_argument("--batch", type=int, default=0,
                    help="tune the batch path instead, on an ensemble of this many Plummer "
                         "clusters (N log-uniform in [256, 16384], Kroupa masses) to t = 0.125")
    ap.add_argument("--sweep", choices=("split", "factors"), default="split",
                    help="batch: sweep (jchunk, items_per_job) or the item-class chunk factors")
    ap.add_argument("--time-shapes", default="",
                    help="time given shapes instead of tuning, e.g. "
                         "'1024=default,-128/8/256/32;8192=default' (ipl/waves/tile/S)")
    ap.add_argument("--rounds", type=int, default=5, help="--time-shapes: interleaved passes")
    args = ap.parse_args()
    if args.batch:
        import nbody_inputs as ni
        import paper_1812_00367_amd as nb
        g = ni.rng(args.seed)
        clusters = []
        for _ in range(args.batch):
            n = ni.log_uniform_n(g, 256, 16384)
            s = int(g.integers(0, 2**31 - 1))
            clusters.append(ni.plummer(n, s, masses=ni.kroupa_masses(n, s + 1)))
        prec = nb.NB_SPLIT if args.precision == "split" else nb.NB_FP64
        configs = batch_configs(args.sweep)
        best, rates = tune_batch(clusters, 1 << 37, prec, configs, log=lambda m: print(m, flush=True))
        print(json.dumps({"clusters": args.batch, "precision": args.precision, "sweep": args.sweep,
                          "best": best, "rates": [dict(c, rate=r) for c, r in zip(configs, rates)]}),
              flush=True)
        return
    import nbody_inputs as ni
    import paper_1812_00367_amd as nb
    ic = ni.plummer(args.n, args.seed)
    sim = nb.Simulation(args.n, eps=1e-4,
                        precision=nb.NB_SPLIT if args.precision == "split" else nb.NB_FP64)
    sim.set_state(ic.m, ic.x, ic.v, a=ni.plummer_mean_field_acc(ic.x))
    sim.predict(0)
    if args.time_shapes:
        time_shapes(sim, parse_shapes(args.time_shapes), rounds=args.rounds,
                    log=lambda m: print(m, flush=True))
        return
    sizes = [int(v) for v in args.sizes.split(",")] if args.sizes else None
    rows, results = tune(sim, sizes=sizes, log=lambda s: print(s, flush=True),
                         small=args.precision == "fp64")
    print(json.dumps({"n": args.n, "precision": args.precision, "rows": rows,
                      "best_ms": {str(k): v[0] for k, v in results.items()}}), flush=True)
    print("C: " + ", ".join("{%d, %d, %d, %d, %d}" % tuple(r) for r in rows), flush=True)


if __name__ == "__main__":
    main()
