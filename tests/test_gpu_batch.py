"""GPU checks of the batch entry points (nb_batch_*): many independent clusters of
uneven size advanced together, each with its own block steps.

  * every job takes exactly the oracle's block steps (same block times, same active
    counts, same final levels) and reaches the oracle's positions within 1e-9 and
    its energy change within 1e-9 of |E| (the criterion of the single-system
    end-to-end test);
  * a job's results are bitwise the same alone and in any mix of jobs, at any pool
    offset, in both precisions;
  * admission (NB_ERR_SPACE when the pool or the job table has no room), removal
    and reuse of freed ranges;
  * resume from a checkpoint taken with nb_batch_get is bitwise exact;
  * a failing job is flagged in its own error word and the others are unaffected.
"""
import sys

import numpy as np
import pytest

import nbody_inputs as ni
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DT_MIN = -40
DT_MAX = -3
L = DT_MAX - DT_MIN


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_00367_amd as nb
    return nb


def host(t):
    return t.detach().cpu().numpy()


def make_batch(nb, capacity, max_jobs, **kw):
    kw.setdefault("eps", 1e-4)
    return nb.Batch(capacity, max_jobs, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, **kw)


def cluster(n, seed, kroupa=True):
    m = ni.kroupa_masses(n, seed + 7) if kroupa else None
    return ni.plummer(n, seed, masses=m)


def run_to_end(b):
    steps, inter, logs = b.run()
    return steps, inter, logs


def states(b, jobs):
    return {j: {k: host(t) for k, t in b.get(j).items()} for j in jobs}


# --------------------------------------------------------------- oracle parity --
def test_batch_large_job_matches_oracle(nb):
    """A 9000-body job (above 8192 bodies: after its first step the next block time
    comes from the previous step's minima instead of a scan) beside two small ones,
    run to its end with steps capped at 2^-6: the same block times, active counts
    and final levels as the oracle's integration, positions and velocities within
    1e-9."""
    dt_max = -6
    t_end = 1 << (dt_max - DT_MIN)
    ics = [cluster(9000, 1200), cluster(300, 1201), cluster(2500, 1202)]
    b = nb.Batch(12000, 3, eps=1e-4, dt_max_log2=dt_max, dt_min_log2=DT_MIN)
    jobs = [b.add(ic.m, ic.x, ic.v, t_end) for ic in ics]
    steps, inter, logs = run_to_end(b)
    st = states(b, jobs)
    for j, ic in zip(jobs, ics):
        ost = oracle.State(m=ic.m, x=ic.x, v=ic.v)
        osteps, ostt, osna, _ = oracle.integrate(ost, 1e-4, 0.45, 0.01, dt_max, DT_MIN, t_end)
        gt = np.array([t for t, _ in logs[j]])
        gn = np.array([k for _, k in logs[j]])
        dx = np.abs(st[j]["x"] - ost.x).max()
        dv = np.abs(st[j]["v"] - ost.v).max()
        say("large-job batch: job", j, "n", ic.m.size, "steps gpu/oracle", len(gt), osteps,
            "max |dx|", dx, "max |dv|", dv)
        assert len(gt) == osteps
        assert np.array_equal(gt, ostt) and np.array_equal(gn, osna)
        assert np.all(st[j]["tick"] == t_end)
        assert np.array_equal(st[j]["level"], ost.level)
        assert dx < 1e-9 and dv < 1e-9, (j, dx, dv)
    b.close()



# default chunk factors of the item classes, and another setting of all three
@pytest.mark.parametrize("factors", [None, (1, 8, 2)])
def test_batch_jobs_match_oracle(nb, factors):
    sizes = [70, 200, 333, 1024, 64, 1]
    # end times are whole multiples of dt_max, where every body of a job is synchronised
    ends = [1 << L, 2 << L, 3 << L, 1 << L, 2 << L, 1 << L]
    ics = [cluster(n, 100 + k) for k, n in enumerate(sizes)]
    kw = {} if factors is None else dict(chunk_tile=factors[0], chunk_wide=factors[1],
                                         chunk_direct=factors[2])
    b = make_batch(nb, sum(sizes) + 500, 8, **kw)
    jobs = []
    for ic, te in zip(ics, ends):
        jobs.append(b.add(ic.m, ic.x, ic.v, te))
    e0 = {j: sum(b.energy(j, 0)) if ic.m.size > 1 else 0.0 for j, ic in zip(jobs, ics)}
    steps, inter, logs = run_to_end(b)
    say("batch steps", steps, "interactions", inter)
    st = states(b, jobs)
    total_inter = 0
    for j, ic, te in zip(jobs, ics, ends):
        ost = oracle.State(m=ic.m, x=ic.x, v=ic.v)
        osteps, ostt, osna, ointer = oracle.integrate(ost, 1e-4, 0.45, 0.01, DT_MAX, DT_MIN, te)
        gt = np.array([t for t, _ in logs[j]])
        gn = np.array([k for _, k in logs[j]])
        say("job", j, "n", ic.m.size, "steps gpu/oracle", len(gt), osteps)
        assert len(gt) == osteps
        assert np.array_equal(gt, ostt) and np.array_equal(gn, osna)
        assert np.all(st[j]["tick"] == te)
        assert np.array_equal(st[j]["level"], ost.level)
        dx = np.abs(st[j]["x"] - ost.x).max()
        assert dx < 1e-9, (j, dx)
        if ic.m.size > 1:
            e1 = sum(b.energy(j, te))
            ro = sum(oracle.energy(ic.m, ic.x, ic.v, 1e-4))
            r1 = sum(oracle.energy(ost.m, ost.x, ost.v, 1e-4))
            assert abs((e1 - e0[j]) - (r1 - ro)) < 1e-9 * abs(ro), j
        total_inter += int(ointer) - 2 * ic.m.size ** 2  # the oracle counts its start-up too
    assert inter == total_inter
    # nothing is left to do
    nact, _, err, it = b.step()
    assert it == 0 and not any(nact) and not any(err)


# ------------------------------------------------------- alone vs mix, bitwise --
@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_batch_alone_and_mixed_are_bitwise_equal(nb, precision):
    """Three target jobs, 777, 9000 and 17001 bodies (above 8192 bodies, after its first
    step a job's next block time comes from the previous step's minima instead of a
    scan; above 16384 its bodies are kept in level order), each run alone and then in
    a mix where they sit at other pool offsets, another job ends earlier, one is
    removed mid-run and two are admitted later: every field of every target's final
    state is bitwise the same."""
    prec = nb.NB_FP64 if precision == "fp64" else nb.NB_SPLIT
    t_end = 1 << (L - 2)
    targets = [cluster(777, 5), cluster(9000, 6), cluster(17001, 7)]
    others = [cluster(n, 200 + n) for n in (300, 1500, 64, 129)]
    kw = dict(precision=prec, jchunk=256)
    alone, b1s = [], []
    for ic in targets:
        b1 = make_batch(nb, ic.m.size, 1, **kw)
        j1 = b1.add(ic.m, ic.x, ic.v, t_end)
        run_to_end(b1)
        alone.append(states(b1, [j1])[j1])
        b1s.append((b1, j1))
    b2 = make_batch(nb, 32768, 8, **kw)
    oj = [b2.add(ic.m, ic.x, ic.v, t_end if k != 1 else t_end // 2) for k, ic in enumerate(others[:2])]
    j2 = [b2.add(ic.m, ic.x, ic.v, t_end) for ic in targets]
    for (b1, j1), j in zip(b1s, j2):
        assert b2.info(j)[0] != b1.info(j1)[0]
    for k in range(5):
        b2.step()
    b2.remove(oj[0])
    b2.add(others[2].m, others[2].x, others[2].v, t_end)
    b2.add(others[3].m, others[3].x, others[3].v, t_end)
    run_to_end(b2)
    for a, j, (b1, j1) in zip(alone, j2, b1s):
        mixed = states(b2, [j])[j]
        for k in a:
            assert np.array_equal(a[k], mixed[k]), (j, k)
        assert sum(b1.energy(j1, t_end)) == sum(b2.energy(j, t_end))


def test_batch_job_at_a_high_pool_offset(nb):
    """A job placed after 2^25 + 123 parked bodies (its records start 2.7 GB into the
    record array, so byte offsets pass 2^31) takes the same block steps, bitwise, as
    in a pool of its own. The parked job is given as a state already at its end
    time, so it never steps and needs no start-up."""
    t_end = 1 << (L - 2)
    target = cluster(1000, 77)
    b1 = make_batch(nb, 1000, 1)
    j1 = b1.add(target.m, target.x, target.v, t_end)
    run_to_end(b1)
    alone = states(b1, [j1])[j1]
    b1.close()
    big = (1 << 25) + 123
    say("parked bodies", big)
    b2 = make_batch(nb, big + 1000, 2)
    g = ni.rng(78)
    park = b2.add(np.full(big, 1.0 / big), g.normal(0, 1, (3, big)), np.zeros((3, big)), 0,
                  tick=np.zeros(big, np.int64), level=np.zeros(big, np.int32))
    j2 = b2.add(target.m, target.x, target.v, t_end)
    assert b2.info(j2)[0] == big
    steps, _, _ = run_to_end(b2)
    assert steps > 10
    high = states(b2, [j2])[j2]
    for k in alone:
        assert np.array_equal(alone[k], high[k]), k
    assert b2.info(park) == (0, big)
    b2.close()


def test_batch_coincident_bodies_without_softening(nb):
    """A job with two bodies at one place and eps = 0 has a non-finite start-up: its
    error word says so (1) and it never steps; a good job beside it is unaffected."""
    m = np.array([0.4, 0.35, 0.25])
    x = np.array([[0.1, 0.1, -0.6], [0.2, 0.2, 0.3], [0.0, 0.0, 0.1]])
    v = np.array([[0.0, 0.3, 0.1], [0.1, 0.0, -0.2], [0.0, 0.0, 0.05]])
    good = cluster(200, 31)
    t_end = 1 << (L - 3)
    b = make_batch(nb, 203, 2, eps=0.0)
    jb = b.add(m, x, v, t_end)
    jg = b.add(good.m, good.x, good.v, t_end)
    nact, tnext, err, _ = b.step()
    assert err[jb] == 1 and nact[jb] == 0
    assert err[jg] == 0 and nact[jg] > 0
    b.close()


# ------------------------------------------------------------- admission ------
def test_batch_admission_remove_and_reuse(nb):
    b = make_batch(nb, 1000, 3)
    ics = {n: cluster(n, n) for n in (400, 300, 200, 500, 700, 1001)}
    t_end = 1 << (L - 6)
    a = b.add(ics[400].m, ics[400].x, ics[400].v, t_end)
    c = b.add(ics[300].m, ics[300].x, ics[300].v, t_end)
    assert b.add(ics[500].m, ics[500].x, ics[500].v, t_end) is None      # 300 bodies free
    assert b.add(ics[1001].m, ics[1001].x, ics[1001].v, t_end) is None   # above capacity
    d = b.add(ics[200].m, ics[200].x, ics[200].v, t_end)
    assert b.add(ics[200].m[:50], ics[200].x[:, :50], ics[200].v[:, :50], t_end) is None  # table full
    assert (b.info(a), b.info(c), b.info(d)) == ((0, 400), (400, 300), (700, 200))
    b.step()
    b.remove(c)
    with pytest.raises(nb.NBodyError):
        b.remove(c)
    assert b.add(ics[500].m, ics[500].x, ics[500].v, t_end) is None      # 300 + 100 not adjacent
    b.remove(a)                                                          # 0..700 merged
    e = b.add(ics[700].m, ics[700].x, ics[700].v, t_end)
    assert b.info(e) == (0, 700)
    steps, inter, logs = run_to_end(b)
    assert steps > 0
    st = b.get(e)
    tick, level = host(st["tick"]), host(st["level"]).astype(np.int64)
    # t_end is not a multiple of every step: each body stopped at its last time
    # not beyond t_end, and its next time is beyond it
    assert np.all(tick <= t_end) and np.all(tick + (np.int64(1) << (L - level)) > t_end)
    # a partial-sum buffer below the bound every step fits is raised to it: any job
    # that fits the pool is admitted
    small = make_batch(nb, 4096, 2, jchunk=64, partial_slots=1000)
    big = cluster(1024, 3)
    assert small.add(big.m, big.x, big.v, t_end) == 0
    with pytest.raises(nb.NBodyError):
        small.get(1)


# ------------------------------------------------------------ checkpointing ------
def test_batch_checkpoint_resume_bitwise(nb):
    """Run to t_mid, checkpoint with nb_batch_get, resume the checkpoints (full state)
    in a fresh batch to t_end: bitwise the uninterrupted run to t_end."""
    t_mid, t_end = 1 << (L - 2), 1 << (L - 1)
    ics = [cluster(n, 40 + n) for n in (256, 640)]
    b = make_batch(nb, 2048, 4)
    jobs = [b.add(ic.m, ic.x, ic.v, t_mid) for ic in ics]
    run_to_end(b)
    ck = states(b, jobs)
    b_res = make_batch(nb, 2048, 4)
    jr = [b_res.add(s["m"], s["x"], s["v"], t_end, a=s["a"], j=s["j"], s=s["s"], c=s["c"],
                    a4n=s["a4n"], a5n=s["a5n"], tick=s["tick"], level=s["level"])
          for s in (ck[j] for j in jobs)]
    run_to_end(b_res)
    resumed = states(b_res, jr)
    b_ref = make_batch(nb, 2048, 4)
    jref = [b_ref.add(ic.m, ic.x, ic.v, t_end) for ic in ics]
    run_to_end(b_ref)
    ref = states(b_ref, jref)
    for a_, r_ in zip(jr, jref):
        for k in ("x", "v", "a", "j", "s", "c", "a4n", "a5n", "tick", "level"):
            assert np.array_equal(resumed[a_][k], ref[r_][k]), k


# ------------------------------------------------------------ error isolation ----
def test_batch_failing_job_is_isolated(nb):
    t_end = 1 << (L - 3)
    good = [cluster(n, 60 + n) for n in (128, 500)]
    # a job with a non-finite velocity: its corrector produces non-finite values
    bad = cluster(100, 9)
    bad_v = bad.v.copy()
    bad_v[1, 17] = np.nan
    # a tight pair of very heavy bodies: its initial step, eta_init sqrt(|a| / |s|)
    # ~ 0.01 sqrt(r^3 / M) ~ 3e-13, is below dt_min = 2^-40 ~ 9.1e-13
    heavy_x = np.array([[-5e-4, 5e-4], [0.0, 0.0], [0.0, 0.0]])
    heavy_v = np.array([[0.0, 0.0], [0.5, -0.5], [0.0, 0.0]])
    heavy_m = np.array([1e12, 1e12])
    b = make_batch(nb, 2048, 6)
    jg = [b.add(ic.m, ic.x, ic.v, t_end) for ic in good]
    # the non-finite jerk and snap give the largest step (a non-finite step estimate
    # counts as no limit), so this job first steps, and fails, at t = dt_max
    jb = b.add(bad.m, bad.x, bad_v, 1 << L)
    jh = b.add(heavy_m, heavy_x, heavy_v, 1 << L)
    errs = {}
    for _ in range(100000):
        nact, tnext, err, it = b.step()
        for j in (jb, jh):
            if err[j]:
                errs.setdefault(j, err[j])
        if not any(nact):
            break
    say("error words", errs)
    assert errs.get(jb, 0) == 1 and errs.get(jh, 0) == 2
    # the good jobs are bitwise what they are alone
    mixed = states(b, jg)
    for ic, j in zip(good, jg):
        b1 = make_batch(nb, 1024, 1)
        k = b1.add(ic.m, ic.x, ic.v, t_end)
        run_to_end(b1)
        alone = states(b1, [k])[k]
        for key in alone:
            assert np.array_equal(alone[key], mixed[j][key]), key


# ------------------------------------------------------ multi-step calls ------
def test_run_steps_on_the_null_stream(nb):
    """The null stream cannot be captured, so there nb_batch_run launches every step
    directly; the states are bitwise those of the captured graphs on a stream of the
    batch's own."""
    ics = [cluster(n, 40 + n) for n in (700, 90)]
    t_end = 1 << L
    out = []
    for stream in (None, torch.cuda.default_stream()):
        b = make_batch(nb, 790, 2, stream=stream)
        jobs = [b.add(ic.m, ic.x, ic.v, t_end) for ic in ics]
        steps = 0
        while True:
            *_, taken = b.run_steps(16)
            steps += taken
            if taken < 16:
                break
        out.append((steps, states(b, jobs)))
        b.close()
    assert out[0][0] == out[1][0] > 16
    for j in out[0][1]:
        for k in out[0][1][j]:
            assert np.array_equal(out[0][1][j][k], out[1][1][j][k]), (j, k)


def test_run_steps_equals_single_steps(nb):
    """nb_batch_run (many steps, one wait) gives bitwise the states of the same number
    of nb_batch_step calls, and counts the same interactions."""
    # 9000 bodies: above 8192, the next block time comes from the previous step's
    # minima; 17001: above 16384, the bodies are kept in level order
    ics = [cluster(n, 300 + n) for n in (90, 700, 1300, 9000, 17001)]
    t_end = 1 << L
    b1 = make_batch(nb, 30000, 5)
    b2 = make_batch(nb, 30000, 5)
    j1 = [b1.add(ic.m, ic.x, ic.v, t_end) for ic in ics]
    j2 = [b2.add(ic.m, ic.x, ic.v, t_end) for ic in ics]
    inter1 = 0
    for _ in range(40):
        inter1 += b1.step()[3]
    # 13 = one replay of the eight-step graph and five of the one-step graph, 27 = three
    # and three
    _, _, _, inter2a, taken_a = b2.run_steps(13)
    nact, tnext, err, inter2b, taken_b = b2.run_steps(27)
    assert inter2a + inter2b == inter1 and taken_a + taken_b == 40
    s1, s2 = states(b1, j1), states(b2, j2)
    for a, c in zip(j1, j2):
        for k in s1[a]:
            assert np.array_equal(s1[a][k], s2[c][k]), k
    # finishing with big calls: the last call reports fewer steps than asked
    total = 40
    while True:
        *_, it, taken = b2.run_steps(64)
        total += taken
        if taken < 64:
            break
    steps_alone, _, _ = run_to_end(b1)
    assert total == 40 + steps_alone


# ------------------------------------------------ many small jobs, eps = 0 ------
def test_many_small_jobs_and_unsoftened(nb):
    """1500 jobs of 2..40 bodies: the work split and its prefix sums run over more
    than one 1024-job pass, and the item / body searches leave the 1024-entry LDS
    cache for global memory. eps = 0 exercises the self-pair mask. Every job must
    take the oracle's block steps; a sample is compared in full."""
    g = ni.rng(91)
    sizes = [int(v) for v in g.integers(2, 41, 1500)]
    t_end = 1 << L
    b = make_batch(nb, sum(sizes), 1500, eps=0.0)
    ics = []
    jobs = []
    for k, n in enumerate(sizes):
        ic = ni.plummer(n, 5000 + k)
        ics.append(ic)
        jobs.append(b.add(ic.m, ic.x, ic.v, t_end))
    assert all(j is not None for j in jobs)
    steps, inter, logs = run_to_end(b)
    say("many small jobs: batch steps", steps, "interactions", inter)
    for k in list(range(0, 1500, 97)) + [1499]:
        j, ic = jobs[k], ics[k]
        ost = oracle.State(m=ic.m, x=ic.x, v=ic.v)
        osteps, ostt, osna, _ = oracle.integrate(ost, 0.0, 0.45, 0.01, DT_MAX, DT_MIN, t_end)
        gt = np.array([t for t, _ in logs[j]])
        gn = np.array([x for _, x in logs[j]])
        assert len(gt) == osteps and np.array_equal(gt, ostt) and np.array_equal(gn, osna), k
        st = {key: host(v) for key, v in b.get(j).items()}
        assert np.array_equal(st["level"], ost.level), k
        assert np.abs(st["x"] - ost.x).max() < 1e-9, k


# --------------------------------------------- split precision against the oracle --
def test_batch_split_startup_within_rounding_bound(nb):
    """The batch path's split-precision evaluation (tile and direct classes) at the
    Hermite start-up of jobs of 5..1500 bodies, against the FP64 oracle evaluated on
    the same inputs (positions, velocities, and the start-up accelerations read
    back), within the FP32 rounding bound of the split-precision tests."""
    from test_gpu_split import check_split, envelope
    sizes = [5, 70, 300, 1500]
    b = make_batch(nb, sum(sizes), 4, precision=nb.NB_SPLIT)
    for k, n in enumerate(sizes):
        ic = cluster(n, 700 + k)
        j = b.add(ic.m, ic.x, ic.v, 1 << L)
        st = {key: host(v) for key, v in b.get(j).items()}
        got = np.concatenate([st["a"], st["j"], st["s"], st["phi"][None, :]])
        ref = oracle.evaluate(ic.m, ic.x, ic.v, st["a"], 1e-4)
        env = envelope(ic.m, ic.x, ic.v, st["a"], 1e-4, np.arange(n))
        check_split(got, ref, env, f"batch split n={n}")


# ------------------------------------------ active sets of jobs over 8192 bodies --
def test_batch_active_sets_of_large_jobs(nb):
    """Jobs of 9000 and 17001 bodies (the active-set scan takes 8192 bodies per round:
    two and three rounds, the last ragged; after their first step both take the next
    block time from the previous step's minima instead of a scan) beside a small one:
    after every batch step the bodies that advanced are exactly the oracle's active
    set computed from the job's times and levels before the step, and the reported
    count and block time match it."""
    sizes = [9000, 300, 17001]
    b = make_batch(nb, sum(sizes), 3)
    jobs = []
    for k, n in enumerate(sizes):
        ic = cluster(n, 900 + k)
        jobs.append(b.add(ic.m, ic.x, ic.v, 1 << L))
    checked = {j: 0 for j in jobs}
    for step in range(24):
        before = {j: {k: host(t) for k, t in b.get(j).items() if k in ("tick", "level")} for j in jobs}
        nact, tnext, err, _ = b.step()
        for j in jobs:
            assert err[j] == 0, (step, j, err[j])
            idx, tn = oracle.active(before[j]["tick"], before[j]["level"], L)
            after = host(b.get(j)["tick"])
            if nact[j] == 0:
                assert tn > (1 << L) or len(idx) == 0, (step, j)
                assert np.array_equal(after, before[j]["tick"]), (step, j)
                continue
            assert tnext[j] == tn and nact[j] == len(idx), (step, j, tnext[j], tn, nact[j], len(idx))
            moved = np.flatnonzero(after != before[j]["tick"]).astype(np.int32)
            assert np.array_equal(moved, idx), (step, j)
            assert np.all(after[idx] == tn), (step, j)
            checked[j] += 1
    say("large-job active sets checked per job:", checked)
    assert all(v > 0 for v in checked.values())


# ------------------------------------- the full ensemble of the batched benchmark --
def test_c4_full_ensemble_sampled(nb):
    """The 512-cluster ensemble of `bench.py --config c4` (2.04 M bodies, the same
    batch parameters): the start-up a, j, s, phi of sampled bodies of nine sampled
    clusters (smallest, median, largest, and others) against the oracle on the same
    inputs, then ten batch steps replayed: one oracle block step from each sampled
    cluster's state before the step gives the same block time and active set (bit
    exact), the same new levels, and positions and velocities within 1e-12."""
    import bench
    from test_gpu_parity import TOL_EVAL, eval_errors
    ics = bench.ensemble_clusters(512)
    ns = np.array([ic.m.size for ic in ics])
    tick_end = int(round(0.25 * 2.0 ** -DT_MIN))
    b = nb.Batch(int(ns.sum()), 512, eps=bench.EPS, dt_max_log2=bench.DT_MAX, dt_min_log2=bench.DT_MIN)
    jobs = [b.add(ic.m, ic.x, ic.v, tick_end) for ic in ics]
    assert all(j is not None for j in jobs)
    order = np.argsort(ns, kind="stable")
    sample = [int(order[0]), int(order[1]), int(order[255]), int(order[256]), int(order[-2]),
              int(order[-1]), 17, 100, 333]
    say("c4 sampled clusters", [(k, int(ns[k])) for k in sample])
    for k in sample:
        st = {key: host(t) for key, t in b.get(jobs[k]).items()}
        n = int(ns[k])
        pick = np.unique(np.linspace(0, n - 1, min(n, 64)).astype(np.int32))
        ref = oracle.evaluate(ics[k].m, ics[k].x, ics[k].v, st["a"], bench.EPS, idx=pick)
        got = np.concatenate([st["a"], st["j"], st["s"], st["phi"][None, :]])[:, pick]
        errs = eval_errors(got, ref)
        assert max(errs) <= TOL_EVAL, (k, n, errs)
    for step in range(10):
        before = {k: {key: host(t) for key, t in b.get(jobs[k]).items()} for k in sample}
        nact, tnext, err, _ = b.step()
        for k in sample:
            j = jobs[k]
            assert err[j] == 0, (step, k, err[j])
            s0 = before[k]
            ost = oracle.State(m=s0["m"], x=s0["x"], v=s0["v"], a=s0["a"], j=s0["j"], s=s0["s"],
                               c=s0["c"], a4n=s0["a4n"], a5n=s0["a5n"], tick=s0["tick"],
                               level=s0["level"])
            idx, tn = oracle.active(ost.tick, ost.level, L)
            assert nact[j] == len(idx) and tnext[j] == tn, (step, k)
            xp, vp, ap = oracle.predict(ost.tick, tn, DT_MIN, ost.x, ost.v, ost.a, ost.j, ost.s, ost.c)
            anew = oracle.evaluate(ost.m, xp, vp, ap, bench.EPS, idx=idx)
            oracle.correct(ost, idx, tn, DT_MIN, anew)
            oracle.timesteps(ost, idx, 0, 0.45, 0.01, DT_MAX, DT_MIN)
            s1 = {key: host(t) for key, t in b.get(j).items()}
            assert np.array_equal(s1["tick"], ost.tick), (step, k)
            assert np.array_equal(s1["level"], ost.level), (step, k)
            assert np.abs(s1["x"] - ost.x).max() < 1e-12, (step, k)
            assert np.abs(s1["v"] - ost.v).max() < 1e-12, (step, k)
    b.close()


# ------------------------------------------------ level-ordered active sets ----
def test_large_job_resumes_bitwise_from_a_checkpoint(nb):
    """A job above 16384 bodies keeps its bodies in (level, index) order. Checkpoint it
    after some steps, admit the checkpoint in a fresh batch (its first active-set pass
    rebuilds the order from the levels and the latest body time) and step both: the
    states stay bitwise equal, so the order depends on the levels alone."""
    ic = cluster(17001, 1201)
    b = make_batch(nb, 17001, 1)
    j = b.add(ic.m, ic.x, ic.v, 1 << L)
    for _ in range(12):
        b.step()
    ck = {k: host(t) for k, t in b.get(j).items()}
    b2 = make_batch(nb, 17001, 1)
    j2 = b2.add(ck["m"], ck["x"], ck["v"], 1 << L, a=ck["a"], j=ck["j"], s=ck["s"], c=ck["c"],
                a4n=ck["a4n"], a5n=ck["a5n"], tick=ck["tick"], level=ck["level"])
    for step in range(20):
        na1, tn1, e1, _ = b.step()
        na2, tn2, e2, _ = b2.step()
        assert e1[j] == 0 and e2[j2] == 0, (step, e1, e2)
        assert na1[j] == na2[j2] and tn1[j] == tn2[j2], (step, na1[j], na2[j2], tn1[j], tn2[j2])
    s1 = {k: host(t) for k, t in b.get(j).items()}
    s2 = {k: host(t) for k, t in b2.get(j2).items()}
    for k in ("x", "v", "a", "j", "s", "c", "a4n", "a5n", "tick", "level"):
        assert np.array_equal(s1[k], s2[k]), k


def test_large_job_off_its_level_grid_is_scanned(nb):
    """A job above 16384 bodies loaded with times that are not multiples of their own
    steps (each body less than one step behind the latest, so that none is due before
    it) is off its level grid and cannot use the level counts; it falls back to the
    scans, and every step still advances exactly the oracle's active set at the
    oracle's block time."""
    n = 17001
    ic = cluster(n, 1301)
    b0 = make_batch(nb, n, 1)
    j0 = b0.add(ic.m, ic.x, ic.v, 1 << L)  # the Hermite start-up gives a, j, s and levels
    st0 = {k: host(t) for k, t in b0.get(j0).items()}
    level = st0["level"]
    dt = np.int64(1) << (L - level.astype(np.int64))
    t0 = np.int64(4) << (L - int(level.min()))
    back = (ni.rng(1302).random(n) * dt).astype(np.int64)  # in [0, dt)
    back[:: 7] = 0
    tick = t0 - back
    assert tick.max() < (tick + dt).min() and np.any(tick % dt != 0)
    # the start-up state is taken to hold at t0; a body behind is moved back along its
    # Taylor series, so that the forces the first steps see match its derivatives
    tau = (-back.astype(np.float64) * 2.0 ** DT_MIN)[None, :]
    x0, v0, a0, j0, s0 = (st0[k] for k in ("x", "v", "a", "j", "s"))
    x = x0 + tau * (v0 + tau / 2 * (a0 + tau / 3 * (j0 + tau / 4 * s0)))
    v = v0 + tau * (a0 + tau / 2 * (j0 + tau / 3 * s0))
    a = a0 + tau * (j0 + tau / 2 * s0)
    jj = j0 + tau * s0
    b = make_batch(nb, n, 1)
    j = b.add(ic.m, x, v, 1 << (L + 3), a=a, j=jj, s=s0, c=st0["c"],
              a4n=st0["a4n"], a5n=st0["a5n"], tick=tick, level=level)
    checked = 0
    for step in range(10):
        before = {k: host(t) for k, t in b.get(j).items() if k in ("tick", "level")}
        nact, tnext, err, _ = b.step()
        idx, tn = oracle.active(before["tick"], before["level"], L)
        if err[j] != 0:
            say("off-grid job: error word", err[j], "at step", step)
            break  # a start this far from a real orbit may fail; what was taken is checked
        assert tnext[j] == tn and nact[j] == len(idx), (step, tnext[j], tn, nact[j], len(idx))
        after = host(b.get(j)["tick"])
        moved = np.flatnonzero(after != before["tick"]).astype(np.int32)
        assert np.array_equal(moved, idx), step
        checked += 1
    say("off-grid job: steps checked", checked)
    assert checked >= 3
