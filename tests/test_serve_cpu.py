"""The serving loop's scheduling, driven on the CPU by a stand-in executor with the
Batch interface: first-fit pool admission, a job table, and jobs that finish after
a number of steps growing with their size. Time is simulated (each call of
run_steps advances the clock), so the checks are deterministic."""
import numpy as np
import pytest

from paper_1812_00367_amd.serve import Request, Server, _percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeBatch:
    """Pool of `capacity` bodies, `max_jobs` slots; a job of n bodies needs
    ceil(n / 100) steps; each run_steps call costs 1 ms of clock per resident job."""

    def __init__(self, capacity, max_jobs, clock):
        self.capacity, self.max_jobs, self.clock = capacity, max_jobs, clock
        self.ranges = [(0, capacity)]
        self.jobs = {}      # job -> [off, n, steps_left]
        self.log = []       # (event, job, n, resident bodies)

    def add(self, m, x, v, tick_end):
        n = len(m)
        free = [k for k in range(self.max_jobs) if k not in self.jobs]
        if not free:
            return None
        for i, (o, ln) in enumerate(self.ranges):
            if ln >= n:
                self.ranges[i] = (o + n, ln - n)
                job = free[0]
                self.jobs[job] = [o, n, -(-n // 100)]
                self.log.append(("add", job, n, sum(j[1] for j in self.jobs.values())))
                return job
        return None

    def remove(self, job):
        o, n, _ = self.jobs.pop(job)
        self.ranges.append((o, n))
        self.ranges.sort()
        merged = []
        for o2, l2 in self.ranges:
            if merged and merged[-1][0] + merged[-1][1] == o2:
                merged[-1] = (merged[-1][0], merged[-1][1] + l2)
            else:
                merged.append((o2, l2))
        self.ranges = [r for r in merged if r[1] > 0] or [(0, 0)]
        self.log.append(("remove", job, n, sum(j[1] for j in self.jobs.values())))

    def run_steps(self, k):
        nact = [0] * self.max_jobs
        tnext = [0] * self.max_jobs
        err = [0] * self.max_jobs
        inter = 0
        for job, st in self.jobs.items():
            if st[1] == 13:       # a job of 13 bodies fails in its first step
                err[job] = 2
                continue
            done = min(k, st[2])
            st[2] -= done
            inter += done * st[1] * st[1]
            nact[job] = st[1] if st[2] > 0 else 0
            tnext[job] = -(-st[1] // 100) - st[2]   # block steps taken so far
        self.clock.t += 1e-3 * len(self.jobs)
        return nact, tnext, err, inter, k

    def get(self, job):
        raise AssertionError("not used")


def requests(sizes, gaps):
    t, out = 0.0, []
    for k, (n, g) in enumerate(zip(sizes, gaps)):
        t += g
        out.append(Request(rid=k, arrival=t, m=np.ones(n), x=None, v=None, tick_end=1))
    return out


def test_all_requests_finish_in_arrival_order_of_admission():
    clock = FakeClock()
    ex = FakeBatch(1000, 4, clock)
    reqs = requests([300, 500, 200, 700, 100, 900, 50], [0, 0.001, 0.001, 0.002, 0, 0.01, 0.003])
    summ = Server(ex, steps_per_call=2, clock=clock, sleep=clock.sleep).run(reqs)
    assert summ["requests"] == 7 and summ["failed"] == 0
    for r in reqs:
        assert r.admitted >= r.arrival and r.finished >= r.admitted
    # first-in first-admitted
    adm = [r.admitted for r in sorted(reqs, key=lambda r: r.arrival)]
    assert adm == sorted(adm)
    # the pool and the job table were never over-committed
    assert all(ev[3] <= 1000 for ev in ex.log)
    assert max(sum(1 for e in ex.log[:k + 1] if e[0] == "add") -
               sum(1 for e in ex.log[:k + 1] if e[0] == "remove") for k in range(len(ex.log))) <= 4
    # every job took exactly its step count: interactions = sum of steps * n^2
    assert summ["interactions"] == sum(-(-r.n // 100) * r.n * r.n for r in reqs)
    assert summ["latency_p99_s"] >= summ["latency_p50_s"] > 0


def test_overlap_when_requests_arrive_while_others_run():
    clock = FakeClock()
    ex = FakeBatch(10000, 8, clock)
    reqs = requests([2000] * 4, [0, 0.0005, 0.0005, 0.0005])
    summ = Server(ex, steps_per_call=1, clock=clock, sleep=clock.sleep).run(reqs)
    assert summ["peak_resident"] >= 3


def test_idle_server_waits_for_the_next_arrival():
    clock = FakeClock()
    ex = FakeBatch(1000, 2, clock)
    reqs = requests([100, 100], [0, 5.0])
    Server(ex, steps_per_call=4, clock=clock, sleep=clock.sleep).run(reqs)
    assert reqs[1].admitted >= 5.0 and reqs[0].finished < 1.0


def test_a_request_that_can_never_fit_is_reported():
    clock = FakeClock()
    ex = FakeBatch(1000, 2, clock)
    with pytest.raises(RuntimeError):
        Server(ex, clock=clock, sleep=clock.sleep).run(requests([1001], [0]))


def test_failed_requests_are_counted_apart_from_the_latencies():
    """A failing job leaves at its time to failure; the latency percentiles cover
    only the completed requests."""
    clock = FakeClock()
    ex = FakeBatch(1000, 4, clock)
    reqs = requests([13, 400, 300], [0, 0, 0])
    summ = Server(ex, steps_per_call=1, clock=clock, sleep=clock.sleep).run(reqs)
    assert summ["failed"] == 1 and summ["completed"] == 2
    assert reqs[0].error == 2
    ok = sorted(r.latency for r in reqs[1:])
    assert summ["latency_p50_s"] == pytest.approx(0.5 * (ok[0] + ok[1]))
    assert summ["latency_max_s"] == ok[1]
    assert reqs[0].latency < ok[0]


def test_trace_records_every_block_step():
    """With steps_per_call = 1 the server records each job's (block time, n_act) per
    step; a multi-step call cannot be traced."""
    clock = FakeClock()
    ex = FakeBatch(1000, 4, clock)
    reqs = requests([250, 120], [0, 0.0015])
    Server(ex, steps_per_call=1, clock=clock, sleep=clock.sleep, trace=True).run(reqs)
    for r in reqs:
        steps = -(-r.n // 100)
        # the last step reports n_act 0 (the job is done), the others n bodies
        assert [t for t, _ in r.trace] == list(range(1, steps))
        assert all(k == r.n for _, k in r.trace)
    with pytest.raises(ValueError):
        Server(ex, steps_per_call=2, trace=True)


def test_percentile_interpolates():
    assert _percentile([1, 2, 3, 4], 50) == 2.5
    assert _percentile([5], 99) == 5
    assert _percentile([1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11], 100) == 11


def test_energy_counter_arithmetic():
    from paper_1812_00367_amd.power import joules_from_counter, mean_power
    assert joules_from_counter(100, 1100, 15.3) == pytest.approx(1000 * 15.3e-6)
    # wrap-around of a 64-bit accumulator
    assert joules_from_counter((1 << 64) - 10, 5, 1.0) == pytest.approx(15e-6)
    # trapezoid mean of a ramp 100 W -> 300 W over 2 s with an extra sample is 200 W
    assert mean_power([(0.0, 100.0), (1.0, 200.0), (2.0, 300.0)]) == pytest.approx(200.0)
    assert mean_power([(0.0, 100.0), (2.0, 300.0), (0.5, 150.0)]) == pytest.approx(200.0)
    assert mean_power([]) is None
