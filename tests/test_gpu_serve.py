"""GPU check of the continuous-batching server: requests arriving while others run
are admitted into the resident batch, and every job's final state is bitwise the
state of the same job run alone."""
import sys

import numpy as np
import pytest

import nbody_inputs as ni
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DT_MIN, DT_MAX = -40, -3
L = DT_MAX - DT_MIN


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_00367_amd as nb
    return nb


def test_served_jobs_equal_their_solo_runs(nb):
    from paper_1812_00367_amd.serve import Request, Server
    reqs = []
    g = ni.rng(77)
    t = 0.0
    for k in range(7):
        pair = k in (2, 5)
        n = ni.log_uniform_n(g, 128, 1500, even=pair)
        s = int(g.integers(0, 2**31 - 1))
        ic = ni.parabolic_pair(n, s) if pair else ni.plummer(n, s, masses=ni.kroupa_masses(n, s + 1))
        # the first three arrive together (resident at once), the rest while they run
        reqs.append(Request(rid=k, arrival=t, m=ic.m, x=ic.x, v=ic.v, tick_end=1 << L,
                            kind="pair" if pair else "cluster"))
        t += 0.0 if k < 2 else 0.002
    # a pool for about three of them at a time: later requests wait for room
    cap = 3000
    b = nb.Batch(cap, 4, eps=1e-4, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN)
    summ = Server(b, steps_per_call=4, keep_state=True).run(
        reqs, log=lambda s: print(s, flush=True))
    print(summ, flush=True)
    assert summ["failed"] == 0 and summ["latency_p99_s"] >= summ["latency_p50_s"] > 0
    assert summ["peak_resident"] >= 2
    for r in reqs:
        solo = nb.Batch(r.n, 1, eps=1e-4, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN)
        j = solo.add(r.m, r.x, r.v, r.tick_end)
        solo.run()
        st = {k: v.detach().cpu().numpy() for k, v in solo.get(j).items()}
        for key in st:
            assert np.array_equal(st[key], r.result[key]), (r.rid, key)
        solo.close()
        sys.stdout.flush()


def test_served_jobs_match_oracle(nb):
    """Jobs of the serving mix served together, each against the oracle's integration
    of the same initial state: a Plummer cluster of 4096 bodies, a parabolic pair of
    two 2048-body spheres and a cluster of 9000 bodies (above 8192, where a job's
    next block time comes from the previous step's minima instead of a scan), all to
    t = 0.125. The third arrives while the first two run. Every job takes exactly the
    oracle's block steps (the same block times and active counts in the same order),
    ends with the oracle's levels, and its positions and velocities agree within
    1e-9."""
    from paper_1812_00367_amd.serve import Request, Server
    t_end = 1 << L
    # each job takes a few tens of milliseconds: the third arrives 2 ms in
    specs = [("cluster", 4096, 0.0), ("pair", 4096, 0.0), ("cluster", 9000, 0.002)]
    reqs = []
    for k, (kind, n, arrival) in enumerate(specs):
        ic = ni.parabolic_pair(n, 810 + k) if kind == "pair" else ni.plummer(n, 810 + k)
        reqs.append(Request(rid=k, arrival=arrival, m=ic.m, x=ic.x, v=ic.v, tick_end=t_end,
                            kind=kind))
    b = nb.Batch(sum(n for _, n, _ in specs) + 100, 4, eps=1e-4, dt_max_log2=DT_MAX,
                 dt_min_log2=DT_MIN, items_per_job=8192)
    summ = Server(b, steps_per_call=1, keep_state=True, trace=True).run(
        reqs, log=lambda s: print(s, flush=True))
    print(summ, flush=True)
    assert summ["failed"] == 0
    # the third was admitted while the first two were still resident
    assert 0.0 < reqs[2].admitted < min(reqs[0].finished, reqs[1].finished)
    assert summ["peak_resident"] == 3
    for r in reqs:
        ost = oracle.State(m=r.m, x=r.x, v=r.v)
        osteps, ostt, osna, _ = oracle.integrate(ost, 1e-4, 0.45, 0.01, DT_MAX, DT_MIN, t_end)
        gt = np.array([t for t, _ in r.trace])
        gn = np.array([k for _, k in r.trace])
        dx = np.abs(r.result["x"] - ost.x).max()
        dv = np.abs(r.result["v"] - ost.v).max()
        print(f"request {r.rid} ({r.kind}, n={r.n}): block steps served {len(gt)}, oracle {osteps}; "
              f"max |dx| {dx:.2e}, max |dv| {dv:.2e}", flush=True)
        assert len(gt) == osteps, r.rid
        assert np.array_equal(gt, ostt) and np.array_equal(gn, osna), r.rid
        assert np.all(r.result["tick"] == t_end), r.rid
        assert np.array_equal(r.result["level"], ost.level), r.rid
        assert dx < 1e-9 and dv < 1e-9, (r.rid, dx, dv)
    b.close()
