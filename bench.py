"""Throughput of the Hermite-6 block-step path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--precision fp64|split]

Workload: a Plummer sphere of N = 65536 bodies (seed 2, equal masses, eps = 1e-4,
Henon units), after the Hermite start-up on the GPU. A step is one whole block
step over the full active set (all N bodies due): active-set selection, prediction
of every body, pairwise evaluation of acceleration/jerk/snap/potential (N x N
interactions), j-split reduction, corrector and new step levels. The timed region
ends with one energy diagnostic (O(N^2), at the output time). Inputs are resident
in HBM before timing starts.

Before each step every body's time and level are reset so that all N bodies are
due together (at the smallest level any body needed at start-up); positions and
derivatives carry on from the previous step, so each step is a genuine
shared-level Hermite step of the whole system with identical work.

Prints one JSON line: value = interactions per second over the timed region
(K * N^2 interactions / elapsed), the roofline of the evaluation kernel (stated 79
flop per interaction against the FP64 vector peak), the nb_evaluate sweep over
active-set sizes (median and p99 latency), and the CPU oracle timed on a bounded
sample of the same evaluation.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_INTERACTION = 79          # stated count (see the design notes)
PEAK_FP64_TFLOPS = 78.6            # 256 CU x 2.4 GHz x 128 FP64 flop/clk (vector)
N_BODIES = 65536
EPS = 1e-4
DT_MAX, DT_MIN = -3, -40
SWEEP = (1, 64, 1024, 8192, 65536)
METRIC = "pairwise interactions/s (acc+jerk+snap) and % of FP64/FP32 vector peak; p99"
PEAK_FP32_TFLOPS = 157.3           # the chip's FP32 vector peak (packed instructions)
# sources of the full-N evaluation kernel (k_eval_sym and the k_sym_reduce pass); the
# traffic figure below is valid only for them
KERNEL_SRCS = [os.path.join(ROOT, "paper_1812_00367_amd", "csrc", f)
               for f in ("nbody_sym.hip", "nb_math.h", "nb_internal.h")]
# HBM bytes per full-N FP64 evaluation launch of k_eval_sym (FETCH_SIZE x 2.00 +
# WRITE_SIZE x 1.00, both calibrated on a 512 MiB device copy) from
# profiles/eval_sym_plummer65536.md, keyed by the sha256 prefix of the sources above;
# any edit of them turns the figure to null until the counters are taken again.
TRAFFIC = {"35b8a367b0d3ebaa": {"fp64": 2.00 * 164221 * 1024 + 1.00 * 693827 * 1024}}
# FP64 flops per interaction the kernel executes (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes /
# N^2, same profile), keyed the same way.
EXECUTED_FLOPS = {"35b8a367b0d3ebaa": {"fp64": 54.9}}


def kernel_name(shape, fp64):
    """The evaluation kernel a launch shape (nb_eval_config's report) selects."""
    if not fp64:
        return "k_eval_split"
    if shape["ipl"] == 0:
        return "k_eval_sym"   # every body active: each pair once, added to both bodies
    return "k_eval_lanes_f64" if shape["ipl"] < 0 else "k_eval_f64"


def kernel_sources_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=("fp64", "split"), default="fp64")
    ap.add_argument("--n", type=int, default=N_BODIES)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eval-only", type=int, default=0,
                    help="time only K nb_evaluate calls of the full active set (for profiling)")
    ap.add_argument("--config", choices=("c2", "c3", "c4", "c5"), default="c2",
                    help="c2: N=65536 block steps (the headline line); c3: N=2^20 Kroupa-mass "
                         "sphere, one full evaluation + 16 block steps on both precisions; "
                         "c4: ensemble of 512 clusters integrated together to t=0.25; "
                         "c5: continuous-batching server under Poisson arrivals (rate sweep)")
    ap.add_argument("--rates", default="0.5,1,2,3", help="c5: arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=24, help="c5: requests per rate")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="c5: HBM budget of the pool")
    ap.add_argument("--slots", type=int, default=64, help="c5: job-table size")
    ap.add_argument("--serve-t-end", type=float, default=1.0, help="c5: end time of every job")
    ap.add_argument("--clusters", type=int, default=512, help="c4: number of clusters")
    ap.add_argument("--t-end", type=float, default=0.25, help="c4: end time (multiple of 2^-3)")
    ap.add_argument("--jchunk", type=int, default=0, help="c4: j-chunk per work item (0 = default)")
    ap.add_argument("--precisions", default="fp64,split", help="c4: precisions to run")
    ap.add_argument("--steps-per-call", type=int, default=32,
                    help="c4: batch steps enqueued per call without a host wait")
    ap.add_argument("--energy-seconds", type=float, default=3.0,
                    help="length of the untimed run of the same step under the GPU energy "
                         "counter (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the split-precision, ensemble and serving objects of the "
                         "default line")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size "
                         "kernel against which HBM byte counters are scaled)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path "
              "(the design notes describe how the evaluation would shard).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import nbody_inputs as ni
    import paper_1812_00367_amd as nb

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.config == "c3":
        print(json.dumps(large_workload()), flush=True)
        return
    if args.config == "c5":
        print(json.dumps(serving_workload([float(r) for r in args.rates.split(",")], args.requests,
                                          args.budget_gib, args.slots, args.serve_t_end,
                                          args.precision, args.steps_per_call)), flush=True)
        return
    if args.config == "c4":
        print(json.dumps(ensemble_workload(args.clusters, args.t_end, args.jchunk,
                                           args.precisions.split(","), args.steps_per_call)),
              flush=True)
        return
    n = args.n
    prec = nb.NB_SPLIT if args.precision == "split" else nb.NB_FP64
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    ic = ni.plummer(n, 2)
    sim = nb.Simulation(n, eps=EPS, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, precision=prec,
                        device=dev)
    sim.set_state(ic.m, ic.x, ic.v)
    sim.start()
    st = sim.get_state()
    L = DT_MAX - DT_MIN
    kmax = int(st["level"].max().item())
    # every body due at the same block time 2^(L - kmax): the smallest step any body needs
    snap = {}
    snap["tick"] = torch.zeros(n, dtype=torch.int64, device=dev)
    snap["level"] = torch.full((n,), kmax, dtype=torch.int32, device=dev)
    idx_buf = torch.empty(n, dtype=torch.int32, device=dev)

    def restore():
        # every body due at the same block time again; the physical state carries on,
        # so each step is a shared-level step of the whole system
        sim.set_times(snap["tick"], snap["level"])

    def one_step(timed_eval=None):
        idx, tn = sim.active(idx_buf)
        sim.predict(tn)
        if timed_eval is not None:
            timed_eval[0].record(stream)
        sim.evaluate_into(idx, out_buf)
        if timed_eval is not None:
            timed_eval[1].record(stream)
        sim.correct(idx, tn)
        sim.timesteps(idx)
        return idx.shape[0]

    out_buf = torch.empty((10, n), dtype=torch.float64, device=dev)

    if args.calib_copy_mib:
        a = torch.ones(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.eval_only:
        restore()
        idx, tn = sim.active(idx_buf)
        sim.predict(tn)
        for _ in range(args.warmup):
            sim.evaluate_into(idx, out_buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.eval_only):
            sim.evaluate_into(idx, out_buf)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.eval_only
        print(json.dumps({"eval_only_ms": dt * 1e3, "interactions_per_s": n * n / dt}), flush=True)
        return

    for _ in range(args.warmup):
        restore()
        one_step()
    torch.cuda.synchronize()
    pairs = []
    inter = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        na = one_step((e0, e1))
        pairs.append((e0, e1))
        inter += na * n
    torch.cuda.synchronize()
    te = time.perf_counter()
    ek, ep = sim.energy(1 << (L - kmax))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    t_energy = t1 - te
    elapsed = t1 - t0
    eval_ms = [a.elapsed_time(b) for a, b in pairs]
    eval_avg_s = sum(eval_ms) / len(eval_ms) / 1e3
    shape = sim.eval_config(None, n)
    achieved = FLOP_PER_INTERACTION * n * n / eval_avg_s / 1e12
    peak = PEAK_FP64_TFLOPS if prec == nb.NB_FP64 else PEAK_FP32_TFLOPS
    value = inter / elapsed
    src_hash = kernel_sources_hash()
    traffic = TRAFFIC.get(src_hash, {}).get(args.precision) if n == N_BODIES else None
    executed = EXECUTED_FLOPS.get(src_hash, {}).get(args.precision)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == nb.NB_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plummer-65536 full block step (Hermite-6, all bodies due)",
                   "n": n, "n_act": n, "eps": EPS, "seed": 2, "precision": args.precision,
                   "eta": 0.45, "level": kmax, "eval_shape": shape},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": kernel_name(shape, prec == nb.NB_FP64),
                     "flop_per_interaction": FLOP_PER_INTERACTION,
                     "algorithmic_bytes": 80 * n + 152 * n,
                     "eval_ms_avg": eval_avg_s * 1e3, "kernel_src": src_hash,
                     "executed_flop_per_interaction": executed,
                     "executed_tflops": None if executed is None else executed * n * n / eval_avg_s / 1e12},
        "energy": {"ekin": ek, "epot": ep, "ms": t_energy * 1e3},
    }

    # the sweep and the crackle leg evaluate the state predicted by the energy call
    # above; the energy leg then runs further steps
    if not args.no_sweep:
        result["sweep"] = sweep(sim, ic, n, stream, dev, peak)
        result["crackle"] = crackle_leg(sim, n, stream)
    if args.energy_seconds > 0:
        result["energy_per_interaction"] = energy_leg(restore, one_step, n, args.energy_seconds)
    if not args.no_extras and prec == nb.NB_FP64:
        del sim
        torch.cuda.empty_cache()
        result["split"] = split_leg(ic, n)
        result["ensemble"] = ensemble_workload(512, 0.25, 0, ("fp64",), 32)
        result["serving"] = serving_workload([3.0], count=12, steps_per_call=32)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(ic, n, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def split_leg(ic, n, reps=10):
    """The full N x N evaluation of the sphere's initial state (predicted accelerations:
    the smooth Plummer field) on the split-precision path and on the FP64 path, each
    timed over `reps` calls: interactions/s, the ratio of the two, the stated rate as a
    share of the FP64 and of the FP32 vector peak, and the split path's relative error
    of a, j, s and phi against the FP64 path on every body (the FP64 path matches the
    oracle within 1e-13, so this is the split path's error to that accuracy)."""
    import numpy as np
    import torch

    import nbody_inputs as ni
    import paper_1812_00367_amd as nb
    dev = torch.device("cuda", 0)
    ap = ni.plummer_mean_field_acc(ic.x)
    idx = torch.arange(n, dtype=torch.int32, device=dev)
    res, outs = {}, {}
    for name, prec in (("fp64", nb.NB_FP64), ("split", nb.NB_SPLIT)):
        sim = nb.Simulation(n, eps=EPS, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, precision=prec,
                            device=dev)
        sim.set_state(ic.m, ic.x, ic.v, a=ap)
        sim.predict(0)
        out = torch.empty((10, n), dtype=torch.float64, device=dev)
        sim.evaluate_into(idx, out)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(sim.stream)
            sim.evaluate_into(idx, out)
            b.record(sim.stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        res[name] = ms
        outs[name] = out.cpu().numpy()
        sim.close()
        del sim
    rate = n * n / (res["split"] / 1e3)
    err = {}
    for lab, c0, c1 in (("a", 0, 3), ("j", 3, 6), ("s", 6, 9), ("phi", 9, 10)):
        ref = outs["fp64"][c0:c1]
        e = np.linalg.norm(outs["split"][c0:c1] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        err[lab] = {"p50": float(np.median(e)), "p99": float(np.percentile(e, 99)),
                    "max": float(e.max())}
    return {"workload": f"plummer-{n} initial state, all {n} bodies active",
            "median_ms": res["split"], "fp64_median_ms": res["fp64"],
            "interactions_per_s": rate, "speedup_vs_fp64": res["fp64"] / res["split"],
            "frac_fp64_peak": rate * FLOP_PER_INTERACTION / (PEAK_FP64_TFLOPS * 1e12),
            "frac_fp32_peak": rate * FLOP_PER_INTERACTION / (PEAK_FP32_TFLOPS * 1e12),
            "rel_error_vs_fp64_path": err,
            "integrates": False,
            "note": "evaluation only: the 6th-order step criterion cannot be driven by it "
                    "(FP32 force noise amplified by the interpolated higher derivatives)"}


FLOP_PER_INTERACTION_CRACKLE = 127   # the 79 above plus 48 for the crackle term


def crackle_leg(sim, n, stream, reps=5):
    """nb_evaluate_crackle over the full active set of the predicted state (FP64)."""
    import torch
    idx = torch.arange(n, dtype=torch.int32, device=sim.device)
    out = torch.empty((13, n), dtype=torch.float64, device=sim.device)
    sim.evaluate_crackle(idx, out)              # warm-up
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        sim.evaluate_crackle(idx, out)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
    rate = n * n / (ms / 1e3)
    return {"n_act": n, "median_ms": ms, "interactions_per_s": rate,
            "flop_per_interaction": FLOP_PER_INTERACTION_CRACKLE,
            "tflops": rate * FLOP_PER_INTERACTION_CRACKLE / 1e12,
            "peak_frac": rate * FLOP_PER_INTERACTION_CRACKLE / (PEAK_FP64_TFLOPS * 1e12)}


def energy_leg(restore, one_step, n, seconds):
    """GPU energy per interaction: the headline step repeated for about `seconds`
    under the device's accumulated-energy counter (sampled socket power beside it).
    Separate from the timed region; reported as nJ per interaction."""
    import torch

    from paper_1812_00367_amd.power import EnergyMeter
    meter = EnergyMeter(0)
    if not meter.available:
        return {"nJ": None, "reason": meter.reason}
    # size the run from one timed step
    torch.cuda.synchronize()
    t = time.perf_counter()
    restore()
    one_step()
    torch.cuda.synchronize()
    per = time.perf_counter() - t
    steps = max(1, int(seconds / max(per, 1e-4)))
    meter.start()
    inter = 0
    for _ in range(steps):
        restore()
        inter += one_step() * n
    torch.cuda.synchronize()
    rec = meter.stop()
    meter.close()
    rec.update({"steps": steps, "interactions": inter,
                "nJ": rec["joules"] / inter * 1e9 if rec.get("joules") else None,
                "interactions_per_joule": inter / rec["joules"] if rec.get("joules") else None})
    return rec


def sweep(sim, ic, n, stream, dev, peak):
    """Single nb_evaluate calls over active-set sizes: median / p99 latency."""
    import numpy as np
    import torch

    import nbody_inputs as ni
    res = []
    out = torch.empty((10, n), dtype=torch.float64, device=dev)
    for k, na in enumerate(SWEEP):
        if na > n:
            continue
        idx = torch.as_tensor(ni.active_subset(n, na, 20 + k), device=dev)
        reps = 200 if na <= 1024 else 50
        for _ in range(20):
            sim.evaluate_into(idx, out)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            sim.evaluate_into(idx, out)
            b.record(stream)
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        med = float(np.median(ms))
        res.append({"n_act": na, "median_ms": med, "p99_ms": float(np.percentile(ms, 99)),
                    "interactions_per_s": na * n / (med / 1e3),
                    "peak_frac": FLOP_PER_INTERACTION * na * n / (med / 1e3) / 1e12 / peak,
                    "shape": sim.eval_config(None, na)})
    return res


def large_workload(n=1 << 20, steps=16):
    """Plummer sphere of 2^20 bodies with Kroupa masses (seed 3, eps = 1e-4): Hermite
    start-up, one timed full evaluation and 16 timed block steps on each precision,
    with the relative energy drift of each run and the split-vs-FP64 difference of
    a, j, s on the 4096-body subsample (seed 33)."""
    import numpy as np
    import torch

    import nbody_inputs as ni
    import paper_1812_00367_amd as nb
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    ic = ni.plummer(n, 3, masses=ni.kroupa_masses(n, 3))
    sub = torch.as_tensor(ni.active_subset(n, 4096, 33), device=dev)
    allidx = torch.arange(n, dtype=torch.int32, device=dev)
    res = {"workload": "plummer-2^20 kroupa, full evaluation + 16 block steps", "n": n}
    subs = {}
    for name, prec in (("fp64", nb.NB_FP64), ("split", nb.NB_SPLIT)):
        sim = nb.Simulation(n, eps=EPS, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, precision=prec,
                            device=dev)
        sim.set_state(ic.m, ic.x, ic.v)
        e0 = sum(sim.energy(0))
        sim.set_state(ic.m, ic.x, ic.v)
        sim.start()
        out = torch.empty((10, n), dtype=torch.float64, device=dev)
        sim.predict(0)
        sim.evaluate_into(allidx, out)           # warm-up of the full-N shape
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.evaluate_into(allidx, out)
        b.record(stream)
        torch.cuda.synchronize()
        full_ms = a.elapsed_time(b)
        subs[name] = sim.evaluate(sub).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inter, tick, done, status, nacts, levels = 0, 0, 0, "ok", [], []
        for _ in range(steps):
            try:
                na, tick = sim.step()
            except nb.NBodyError as e:
                status = f"stopped after {done} block steps: {e}"
                break
            inter += na * n
            nacts.append(na)
            done += 1
            print(f"[c3 {name}] block step {done}: n_act={na} t={tick * 2.0 ** DT_MIN:.6e}",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the level trajectory, replayed from the same start outside the timed loop: after
        # each block step the deepest level (smallest step 2^-level) and its body count
        sim.set_state(ic.m, ic.x, ic.v)
        sim.start()
        for _ in range(done):
            try:
                sim.step()
                lvl = sim.get_state()["level"]
            except nb.NBodyError:
                break
            top = int(lvl.max().item())
            levels.append({"max_level": top, "bodies_at_max": int((lvl == top).sum().item())})
        try:
            lv = sim.get_state()["level"]
            ek, ep = sim.energy(tick) if done else (float("nan"), float("nan"))
        except nb.NBodyError:
            # the failed step is reported by the next wait; the deepest level reached
            # before it is in the trajectory
            lv = torch.tensor([levels[-1]["max_level"] if levels else -1])
            ek, ep = float("nan"), float("nan")
        res[name] = {"full_eval_ms": full_ms,
                     "full_eval_interactions_per_s": n * n / (full_ms / 1e3),
                     "block_steps": done, "status": status, "n_act": nacts,
                     "block_step_interactions": inter,
                     "block_steps_interactions_per_s": inter / dt if dt > 0 else None,
                     "time_reached": tick * 2.0 ** DT_MIN,
                     "max_level": int(lv.max().item()),
                     "level_trajectory": levels,
                     "energy_drift": (ek + ep - e0) / abs(e0)}
        del sim
    d = {}
    for c, lab in ((0, "a"), (3, "j"), (6, "s")):
        ref = subs["fp64"][c:c + 3]
        rel = np.linalg.norm(subs["split"][c:c + 3] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        d[lab] = {"p50": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
                  "max": float(rel.max())}
    res["split_vs_fp64_rel_diff"] = d
    return res


def ensemble_clusters(count, seed=4, lo=256, hi=16384):
    """Plummer clusters with N log-uniform in [lo, hi] and Kroupa masses, each from its
    own seed derived from `seed`."""
    import nbody_inputs as ni
    g = ni.rng(seed)
    out = []
    for k in range(count):
        n = ni.log_uniform_n(g, lo, hi)
        s = int(g.integers(0, 2**31 - 1))
        out.append(ni.plummer(n, s, masses=ni.kroupa_masses(n, s + 1)))
    return out


def ensemble_workload(count=512, t_end=0.25, jchunk=0, precisions=("fp64", "split"), chunk=32):
    """Many independent clusters advanced together by the batch entry points, each
    with its own block steps, to t_end. Reports whole-run interactions/s (start-up
    excluded, every batch step and its host bookkeeping included), the share of the
    stated FP64 / FP32 vector peak, and the relative energy drift of every cluster."""
    import numpy as np
    import torch

    import paper_1812_00367_amd as nb
    dev = torch.device("cuda", 0)
    L = DT_MAX - DT_MIN
    tick_end = int(round(t_end * 2.0 ** -DT_MIN))
    if tick_end % (1 << L):
        raise SystemExit("t_end must be a multiple of 2^-3")
    ics = ensemble_clusters(count)
    ns = np.array([ic.m.size for ic in ics], dtype=np.int64)
    res = {"workload": f"ensemble of {count} plummer clusters, N log-uniform [256, 16384], "
                       f"kroupa masses, eps=1e-4, to t={t_end}",
           "clusters": count, "sum_n": int(ns.sum()), "sum_n2": float((ns * ns).sum())}
    for name in precisions:
        prec = nb.NB_SPLIT if name == "split" else nb.NB_FP64
        b = nb.Batch(int(ns.sum()), count, eps=EPS, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN,
                     precision=prec, jchunk=jchunk, device=dev)
        t0 = time.perf_counter()
        jobs = []
        for ic in ics:
            j = b.add(ic.m, ic.x, ic.v, tick_end)
            if j is None:
                raise SystemExit("ensemble does not fit the batch")
            jobs.append(j)
        torch.cuda.synchronize()
        t_start = time.perf_counter() - t0
        e0 = np.array([sum(b.energy(j, 0)) for j in jobs])
        print(f"[c4 {name}] {count} clusters admitted, start-up {t_start:.2f} s", file=sys.stderr,
              flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = inter = 0
        errs = {}
        last = t0
        while True:
            # `chunk` batch steps per call with no host wait in between; a call whose
            # steps advance no job means every cluster has reached t_end (or failed)
            nact, tnext, err, it, taken = b.run_steps(chunk)
            steps += taken
            inter += it
            for j in jobs:
                if err[j]:
                    errs[j] = err[j]
            if taken < chunk:
                break
            now = time.perf_counter()
            if now - last > 20:
                last = now
                live = sum(1 for j in jobs if nact[j])
                print(f"[c4 {name}] batch step {steps}: {live} clusters stepping, "
                      f"{inter:.3e} interactions, {now - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # energy drift over the clusters that reached t_end: a cluster stopped by an
        # error word would be extrapolated to t_end by the predictor, which is no
        # energy error of the integration
        done = [k for k, j in enumerate(jobs) if j not in errs]
        e1 = np.array([sum(b.energy(jobs[k], tick_end)) for k in done])
        de = np.abs((e1 - e0[done]) / np.abs(e0[done]))
        rate = inter / wall
        peak = PEAK_FP32_TFLOPS if name == "split" else PEAK_FP64_TFLOPS
        res[name] = {"status": "completed" if not errs else
                               f"not completed: {len(errs)} of {count} clusters stopped with an error word",
                     "wall_s": wall, "startup_s": t_start, "batch_steps": steps, "steps_per_call": chunk,
                     "interactions": inter, "interactions_per_s": rate,
                     "tflops_at_79": rate * FLOP_PER_INTERACTION / 1e12,
                     "peak_frac": rate * FLOP_PER_INTERACTION / (peak * 1e12),
                     "failed_clusters": len(errs), "completed_clusters": len(done),
                     "energy_drift_completed": None if not done else
                         {"p50": float(np.median(de)), "p99": float(np.percentile(de, 99)),
                          "max": float(de.max())}}
        print(f"[c4 {name}] {steps} batch steps, {inter:.3e} interactions in {wall:.1f} s "
              f"= {rate:.3e}/s", file=sys.stderr, flush=True)
        b.close()
        del b
        torch.cuda.empty_cache()
    return res


# Work items per job of the serving batch: four times the library default, which gives
# the large, sparse serving jobs more parallel items for a larger partial-sum buffer
# inside the same HBM budget (at 3 requests/s, interleaved: p50 1.94 s against 1.99 s
# with 4096 items and 2.19 s with 2048; 16384 items, 2.00-2.02 s, leave less pool).
SERVE_ITEMS_PER_JOB = 8192


def serving_workload(rates, count=24, budget_gib=32.0, slots=64, t_end=1.0, precision="fp64",
                     steps_per_call=8, seed=5):
    """Continuous-batching serving: for each arrival rate, `count` seeded requests
    (90 % Plummer clusters with N log-uniform in [1024, 65536], 10 % parabolic pairs
    of two N/2 spheres 10 apart), each integrated to t_end, arrive as a Poisson
    stream; the server keeps admitted jobs resident in a pool sized from an HBM
    budget and advances them together. Reports p50/p99 latency (arrival to result,
    queueing and start-up included) and aggregate interactions/s."""
    import torch

    import nbody_inputs as ni
    import paper_1812_00367_amd as nb
    from paper_1812_00367_amd.serve import Request, Server, capacity_for_budget
    dev = torch.device("cuda", 0)
    prec = nb.NB_SPLIT if precision == "split" else nb.NB_FP64
    tick_end = int(round(t_end * 2.0 ** -DT_MIN))
    cap = capacity_for_budget(int(budget_gib * (1 << 30)), slots, prec, items_per_job=SERVE_ITEMS_PER_JOB)
    res = {"workload": f"serving: Poisson arrivals, 90% plummer N log-uniform [1024, 65536], "
                       f"10% parabolic pairs, to t={t_end}",
           "budget_gib": budget_gib, "pool_bodies": cap, "slots": slots, "precision": precision,
           "items_per_job": SERVE_ITEMS_PER_JOB,
           "steps_per_call": steps_per_call, "rates": []}
    for k, rate in enumerate(rates):
        stream = ni.serving_requests(count, rate, seed + k)
        reqs = [Request(rid=i, arrival=q["arrival"], m=q["ic"].m, x=q["ic"].x, v=q["ic"].v,
                        tick_end=tick_end, kind=q["kind"]) for i, q in enumerate(stream)]
        b = nb.Batch(cap, slots, eps=EPS, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, precision=prec,
                     items_per_job=SERVE_ITEMS_PER_JOB, device=dev)
        t0 = time.perf_counter()
        summ = Server(b, steps_per_call=steps_per_call).run(
            reqs, log=lambda msg: print(f"[c5 rate {rate}] {msg}", file=sys.stderr, flush=True))
        summ["rate_per_s"] = rate
        summ["mean_n"] = sum(r.n for r in reqs) / len(reqs)
        summ["wall_s"] = time.perf_counter() - t0
        res["rates"].append(summ)
        print(f"[c5] rate {rate}/s: p50 {summ['latency_p50_s']:.2f} s, p99 {summ['latency_p99_s']:.2f} s, "
              f"{summ['interactions_per_s']:.3e} interactions/s", file=sys.stderr, flush=True)
        b.close()
        del b
        torch.cuda.empty_cache()
    return res


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's string."""
    import platform
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(ic, n, seconds):
    """The oracle's evaluation on a bounded sample of the active set, on every host
    core (the reported value), then on one core over a sample a fifth as long."""
    import numpy as np

    import nbody_inputs as ni
    import oracle
    threads = oracle.default_threads()
    ap = ni.plummer_mean_field_acc(ic.x)

    def timed(k, nthreads):
        idx = ni.active_subset(n, k, 99)
        t0 = time.perf_counter()
        oracle.evaluate(ic.m, ic.x, ic.v, ap, EPS, idx=idx, nthreads=nthreads)
        return time.perf_counter() - t0

    probe = min(n, 64)
    k = int(min(n, max(probe, probe * seconds / max(timed(probe, threads), 1e-6))))
    k = min(n, max(threads, k // threads * threads))
    dt = timed(k, threads)
    per_body_one_core = dt * threads / k   # seconds, if the threads scaled perfectly
    k1 = int(min(n, max(1, 0.2 * seconds / per_body_one_core)))
    dt1 = timed(k1, 1)
    return {"value": k * n / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} active bodies x {n} bodies (plummer-{n}), "
                      f"{k * n:.3e} interactions in {dt:.1f} s",
            "cpu": cpu_model(), "one_core_value": k1 * n / dt1,
            "one_core_sample": f"{k1} active bodies x {n} bodies in {dt1:.1f} s"}


if __name__ == "__main__":
    main()
