"""GPU check of the continuous-batching server: requests arriving while others run
are admitted into the resident batch, and every job's final state is bitwise the
state of the same job run alone."""
import sys

import numpy as np
import pytest

import nbody_inputs as ni

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
