"""Continuous-batching serving loop over the batch entry points (nb_batch_*).

Integration requests (a cluster and an end time) arrive over time. The server keeps
every admitted job's state resident in one batch pool on the GPU and advances all
resident jobs together, a few batch steps per call (each job takes its own block
steps). Between calls it retires finished jobs, freeing their bodies, and admits
waiting requests in arrival order while the pool (sized from an HBM budget) and the
job table have room. A request that arrives while others run therefore overlaps
with them on the device, and, because a job's arithmetic does not depend on the
other jobs, its result is the same as if it had run alone.

All arithmetic runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

from ._abi import NB_FP64


@dataclass
class Request:
    """One integration job: bodies (m[n], x[3][n], v[3][n]) integrated from t = 0 to
    `tick_end` (ticks of 2^dt_min_log2); `arrival` in seconds from the start."""
    rid: int
    arrival: float
    m: object
    x: object
    v: object
    tick_end: int
    kind: str = "cluster"
    # filled in by the server
    admitted: float | None = None
    finished: float | None = None
    error: int = 0
    result: dict | None = field(default=None, repr=False)
    # (tick_next, n_act) of every block step the job took, when the server traces
    trace: list | None = field(default=None, repr=False)

    @property
    def n(self):
        return len(self.m)

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def capacity_for_budget(budget_bytes, max_jobs, precision=NB_FP64, **kw):
    """Largest pool (bodies) whose batch workspace fits `budget_bytes` of HBM."""
    from .batch import batch_workspace_bytes
    lo, hi = 1, 1 << 30
    if batch_workspace_bytes(lo, max_jobs, precision, **kw) > budget_bytes:
        raise ValueError("the budget does not hold even a one-body pool")
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if batch_workspace_bytes(mid, max_jobs, precision, **kw) <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    return lo


def _percentile(values, q):
    v = sorted(values)
    if not v:
        return None
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class Server:
    """Drives an executor with the Batch interface (add / remove / run_steps / get).

    steps_per_call: batch steps enqueued between two scheduling decisions (one host
    wait each). keep_state: copy each finished job's final state to the host.
    trace: record every job's block steps, (tick_next, n_act) each, in its request
    (needs steps_per_call = 1, since a multi-step call reports only its last step).
    clock / sleep: time source (seconds) and wait, replaceable for tests."""

    def __init__(self, executor, steps_per_call=8, keep_state=False, clock=time.perf_counter,
                 sleep=time.sleep, trace=False):
        self.ex = executor
        self.steps_per_call = int(steps_per_call)
        if trace and self.steps_per_call != 1:
            raise ValueError("tracing every block step needs steps_per_call = 1")
        self.keep_state = keep_state
        self.trace = bool(trace)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests, log=None):
        """Serve `requests` to completion; returns a summary dict (latency p50/p99,
        interactions/s) and fills each request's admitted/finished/error/result."""
        ex = self.ex
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        resident = {}
        t0 = self.clock()
        inter = 0
        busy = 0.0
        calls = 0
        peak_resident = 0
        while queue or waiting or resident:
            now = self.clock() - t0
            while queue and queue[0].arrival <= now:
                waiting.append(queue.popleft())
            # admission in arrival order while the pool and the job table have room
            while waiting:
                r = waiting[0]
                job = ex.add(r.m, r.x, r.v, r.tick_end)
                if job is None:
                    break
                waiting.popleft()
                r.admitted = self.clock() - t0
                if self.trace:
                    r.trace = []
                resident[job] = r
            if not resident:
                if waiting:
                    raise RuntimeError(f"request {waiting[0].rid} ({waiting[0].n} bodies) can "
                                       "never be admitted: it exceeds the pool or job table")
                if queue:
                    self.sleep(max(0.0, queue[0].arrival - (self.clock() - t0)))
                continue
            peak_resident = max(peak_resident, len(resident))
            c0 = self.clock()
            nact, tnext, err, it, _ = ex.run_steps(self.steps_per_call)
            t = self.clock() - t0
            busy += self.clock() - c0
            calls += 1
            inter += it
            if self.trace:
                for job, r in resident.items():
                    if nact[job] > 0:
                        r.trace.append((tnext[job], nact[job]))
            for job in list(resident):
                if nact[job] == 0 or err[job]:
                    r = resident.pop(job)
                    r.finished = t
                    r.error = err[job]
                    if self.keep_state:
                        r.result = {k: v.detach().cpu().numpy() for k, v in ex.get(job).items()}
                    ex.remove(job)
                    if log:
                        log(f"request {r.rid} ({r.kind}, n={r.n}) done at {t:.3f} s, "
                            f"latency {r.latency:.3f} s, error {r.error}")
        makespan = self.clock() - t0
        # latency percentiles over the requests that completed without an error (a
        # failed job's latency is its time to failure); failures are counted apart
        ok = [r for r in requests if not r.error]
        lat = [r.latency for r in ok]
        wait = [r.admitted - r.arrival for r in requests]
        return {
            "requests": len(requests),
            "completed": len(ok),
            "failed": len(requests) - len(ok),
            "latency_p50_s": _percentile(lat, 50),
            # with fewer than 100 completed requests p99 is interpolated between the
            # two largest latencies; the maximum is reported beside it
            "latency_p99_s": _percentile(lat, 99),
            "latency_max_s": max(lat) if lat else None,
            "queue_wait_p50_s": _percentile(wait, 50),
            "queue_wait_p99_s": _percentile(wait, 99),
            "makespan_s": makespan,
            "interactions": inter,
            "interactions_per_s": inter / makespan if makespan > 0 else None,
            "interactions_per_busy_s": inter / busy if busy > 0 else None,
            "calls": calls,
            "peak_resident": peak_resident,
        }
