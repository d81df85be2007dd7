"""GPU parity of every step of the block-step cycle against the CPU oracle, on the
same seeded inputs, through the C ABI.

Tolerances (written here, derived in the design notes):
  * evaluation, FP64 path: per-body relative error of the a, j and s 3-vectors
    (Euclidean norm) <= 1e-13; potential relative error <= 1e-13;
  * predictor / corrector: a few FP64 rounding units of the magnitude of the terms
    in each formula (they are short sums of products evaluated in another order);
  * step levels and the active set: bit-exact (integer results of IEEE-exact
    decisions taken in FP64 on both sides);
  * energy: relative 1e-12 (a sum of n^2 / 2 terms in a different order).
"""
import math
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
TOL_EVAL = 1e-13
U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_00367_amd as nb
    return nb


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def rel_vec_err(got, ref):
    """Per-body relative error of the 3-vectors rows [3][k]."""
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def error_stats(got, ref):
    """(p50, p99, max) of the per-body relative errors of a, j and s."""
    out = []
    for c in range(3):
        e = rel_vec_err(got[3 * c:3 * c + 3], ref[3 * c:3 * c + 3])
        out.append((float(np.median(e)), float(np.percentile(e, 99)), float(e.max())))
    return out


def condition_numbers(m, xp, vp, ap, eps, idx):
    """kappa_i = sum_j |q_ij| / |q_i| for q = a, j, s of the bodies idx (a report of
    how much the sums cancel, not a reference: the oracle is the reference)."""
    kap = np.zeros((3, len(idx)))
    for col, i in enumerate(idx):
        r = xp - xp[:, i:i + 1]
        v = vp - vp[:, i:i + 1]
        a = ap - ap[:, i:i + 1]
        R = (r * r).sum(0) + eps * eps
        mm = m.copy()
        mm[i] = 0.0
        R[i] = 1.0
        m3 = mm * R ** -1.5
        alpha = (r * v).sum(0) / R
        beta = ((v * v).sum(0) + (r * a).sum(0)) / R + alpha * alpha
        A = m3 * r
        J = m3 * v - 3 * alpha * A
        S = m3 * a - 6 * alpha * J - 3 * beta * A
        for c, q in enumerate((A, J, S)):
            kap[c, col] = np.linalg.norm(q, axis=0).sum() / np.linalg.norm(q.sum(1))
    return kap


# A body whose sum cancels (condition number kappa = sum_j |q_ij| / |q_i| large) can
# exceed TOL_EVAL: an uncompensated FP64 sum in any order is only as accurate as a
# few rounding units times kappa. Such a body is held to KAPPA_C * U * kappa instead.
KAPPA_C = 8


def assert_eval_within(got, ref, m, xp, vp, ap, eps, idx, label):
    """Every body within TOL_EVAL for a, j, s and phi, except bodies whose sums
    cancel: a, j or s of a body above TOL_EVAL must be within KAPPA_C * U * kappa of
    the oracle, and such bodies must be rare (at most 1 in 1000, or 4)."""
    phi = (np.abs(got[9] - ref[9]) / np.abs(ref[9])).max()
    assert phi <= TOL_EVAL, (label, "phi", phi)
    for c, q in enumerate("ajs"):
        e = rel_vec_err(got[3 * c:3 * c + 3], ref[3 * c:3 * c + 3])
        over = np.flatnonzero(e > TOL_EVAL)
        if over.size == 0:
            continue
        assert over.size <= max(4, e.size // 1000), (label, q, over.size)
        kap = condition_numbers(m, xp, vp, ap, eps, np.asarray(idx)[over])[c]
        say(f"{label}: {q} of {over.size} bodies above {TOL_EVAL:g}: errors {e[over]}, "
            f"kappa {kap}, error / (U kappa) {e[over] / (U * kap)}")
        assert np.all(e[over] <= KAPPA_C * U * kap), (label, q, e[over], kap)


def eval_errors(got, ref):
    return (rel_vec_err(got[0:3], ref[0:3]).max(), rel_vec_err(got[3:6], ref[3:6]).max(),
            rel_vec_err(got[6:9], ref[6:9]).max(),
            (np.abs(got[9] - ref[9]) / np.abs(ref[9])).max())


def system(n, seed, eps=1e-4):
    ic = ni.plummer(n, seed)
    ap = ni.plummer_mean_field_acc(ic.x) * (1.0 + 0.1 * ni.rng(seed + 1).normal(size=(3, n)))
    return ic, ap


def make_sim(nb, n, eps=1e-4, **kw):
    return nb.Simulation(n, eps=eps, dt_max_log2=DT_MAX, dt_min_log2=DT_MIN, **kw)


# ------------------------------------------------------------------ evaluation --
SHAPES = [(1, 1, 64, 1), (1, 1, 64, 3), (1, 1, 64, 47), (1, 4, 256, 1), (1, 4, 256, 5),
          (2, 4, 256, 1), (2, 4, 256, 2), (2, 4, 256, 12),
          # the small-set kernel: P bodies per wave on 64 / P lanes, direct or LDS tiles
          (-1, 1, 0, 1), (-1, 1, 0, 37), (-8, 1, 0, 5), (-2, 1, 64, 3), (-16, 1, 64, 16),
          (-64, 1, 64, 7), (-4, 1, 0, 24),
          # the group kernel: every wave of a workgroup on the same G bodies
          (-128, 8, 256, 1), (-128, 8, 256, 5), (-128, 8, 256, 12), (-128, 4, 256, 3),
          (-16, 8, 256, 7), (-64, 4, 256, 12), (-2, 8, 256, 6), (-1, 4, 0, 9),
          (-4, 8, 0, 30), (-32, 8, 256, 40)]


@pytest.mark.parametrize("eps", [1e-4, 0.0])
def test_eval_fp64_every_shape(nb, eps):
    n = 3001  # ragged against every tile size
    ic, ap = system(n, 101)
    sim = make_sim(nb, n, eps=eps)
    sim.set_state(ic.m, ic.x, ic.v, tick0=0, a=ap)
    sim.predict(0)  # h = 0: the predicted state is the state itself
    for n_act, seed in [(n, 0), (1, 1), (7, 2), (600, 3), (2999, 4)]:
        idx = ni.active_subset(n, n_act, 500 + seed)
        ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, eps, idx=idx)
        for cfg in SHAPES:
            say("eval fp64", eps, n_act, cfg)
            sim.eval_config(cfg, n_act)
            got = host(sim.evaluate(idx))
            errs = eval_errors(got, ref)
            assert max(errs) <= TOL_EVAL, (cfg, n_act, errs)
    sim.eval_config(None)


@pytest.mark.parametrize("n,eps", [(9001, 1e-4), (8192, 0.0), (13 * 768, 1e-4), (30000, 1e-4),
                                   (49000, 1e-4), (65536, 1e-4)])
def test_eval_symmetric_full_set(nb, n, eps):
    """Every body active (n_act = n >= 8192): the pairwise-symmetric kernel (each pair
    once, added to both bodies). Ragged n (the last block and its halves partly
    filled) and n a whole number of blocks; every body within the FP64 bound of the
    oracle (bodies whose sums cancel: within a few rounding units times their condition
    number); bitwise the same on a second call; within the bound of the one-sided
    kernel forced by a launch shape; Newton's third law to round-off. At 30000, 49000
    and 65536 bodies the last units are claimed in pieces (of 64, 128 and 128 records;
    at 65536 a unit is a whole block of 768 records)."""
    ic, ap = system(n, 131 + n)
    sim = make_sim(nb, n, eps=eps)
    sim.set_state(ic.m, ic.x, ic.v, tick0=0, a=ap)
    sim.predict(0)
    idx = np.arange(n, dtype=np.int32)
    shape = sim.eval_config(None, n)
    say("symmetric shape", n, shape)
    assert shape["ipl"] == 0  # the symmetric kernel
    got = host(sim.evaluate(idx))
    again = host(sim.evaluate(idx))
    assert np.array_equal(got, again)
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, eps, idx=idx)
    errs = eval_errors(got, ref)
    stats = error_stats(got, ref)
    say("symmetric", n, eps, "max errors a/j/s/phi", errs, "p50/p99/max", stats)
    assert_eval_within(got, ref, ic.m, ic.x, ic.v, ap, eps, idx, f"symmetric {n}")
    # Newton's third law: sum m a = sum m j = sum m s = 0 to round-off of the terms
    for c0 in (0, 3, 6):
        tot = (ic.m * got[c0:c0 + 3]).sum(axis=1)
        scale = (ic.m * np.abs(got[c0:c0 + 3])).sum(axis=1)
        assert np.all(np.abs(tot) <= 1e-12 * scale), (c0, tot, scale)
    sim.eval_config((2, 4, 256, 16), n)
    one = host(sim.evaluate(idx))
    sim.eval_config(None)
    say("one-sided", n, eps, "max errors a/j/s/phi", eval_errors(one, ref))
    assert_eval_within(one, ref, ic.m, ic.x, ic.v, ap, eps, idx, f"one-sided {n}")


GROUP_SHAPES = [(-128, 8, 256), (-128, 4, 256), (-64, 8, 256), (-16, 8, 256), (-4, 4, 256),
                (-1, 4, 0), (-2, 8, 0)]


@pytest.mark.parametrize("n_act", [1, 3, 64, 333, 1024, 4099])
def test_eval_group_kernel(nb, n_act):
    """The group kernel at several split counts, with the splits added by a separate
    pass or inside the launch (the last workgroup of each group): within the FP64 bound
    of the oracle, and bitwise the same on a repeated call (the group counters are back
    at zero after every launch)."""
    n = 20001
    ic, ap = system(n, 151)
    sim = make_sim(nb, n, eps=1e-4)
    sim.set_state(ic.m, ic.x, ic.v, tick0=0, a=ap)
    sim.predict(0)
    idx = ni.active_subset(n, n_act, 152 + n_act)
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=idx)
    seen = set()
    for pmax, waves, tile in GROUP_SHAPES:
        for S in (1, 2, 7, 16, 64):
            shape = sim.eval_config((pmax, waves, tile, S), n_act)
            say("group", n_act, (pmax, waves, tile, S), shape)
            got = host(sim.evaluate(idx))
            errs = eval_errors(got, ref)
            assert max(errs) <= TOL_EVAL, (shape, n_act, errs)
            again = host(sim.evaluate(idx))
            assert np.array_equal(got, again), shape
            seen.add((shape["splits"] > 1, shape["fused"]))
    sim.eval_config(None)
    # both ways of adding the splits ran (one split only for a single group)
    assert (True, 1) in seen and (False, 0) in seen, seen
    if n_act >= 64:
        assert (True, 0) in seen, seen


def test_eval_group_kernel_bad_index_and_xcd_grid(nb):
    """An index out of range in a group-kernel launch (in-launch reduction) is reported
    and the next call is correct again; split counts that are multiples of 8 take the
    XCD-aware 1-D grid."""
    n = 16284  # 64 tiles of 256, the last one partly filled
    ic, ap = system(n, 161)
    sim = make_sim(nb, n)
    sim.set_state(ic.m, ic.x, ic.v, tick0=0, a=ap)
    sim.predict(0)
    idx = ni.active_subset(n, 700, 162)
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=idx)
    for cfg in [(-128, 8, 256, 8), (-16, 8, 256, 16), (-64, 4, 256, 32)]:
        shape = sim.eval_config(cfg, len(idx))
        assert shape["splits"] == cfg[3], shape
        got = host(sim.evaluate(idx))
        assert max(eval_errors(got, ref)) <= TOL_EVAL, (cfg, shape)
    sim.eval_config((-16, 8, 256, 4), 40)
    assert sim.eval_config((-16, 8, 256, 4), 40)["fused"] == 1
    bad = np.array(list(range(0, 39)) + [n + 7], np.int32)
    sim.evaluate(bad)
    with pytest.raises(nb.NBodyError) as e:
        sim.energy(0)
    assert e.value.status == 1
    good = np.arange(100, 140, dtype=np.int32)
    got = host(sim.evaluate(good))
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=good)
    assert max(eval_errors(got, ref)) <= TOL_EVAL
    sim.eval_config(None)


def test_eval_symmetric_reports_a_bad_index(nb):
    n = 8192
    ic, ap = system(n, 141)
    sim = make_sim(nb, n)
    sim.set_state(ic.m, ic.x, ic.v, a=ap)
    sim.predict(0)
    idx = np.arange(n, dtype=np.int32)
    idx[100] = n + 5
    sim.evaluate(idx)
    with pytest.raises(nb.NBodyError) as e:
        sim.energy(0)
    assert e.value.status == 1


def test_eval_fp64_xcd_mapping(nb):
    """Split counts that are multiples of 8 use the XCD-aware 1-D grid."""
    n = 16401
    ic, ap = system(n, 111)
    sim = make_sim(nb, n)
    sim.set_state(ic.m, ic.x, ic.v, tick0=0, a=ap)
    sim.predict(0)
    idx = ni.active_subset(n, 700, 112)
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=idx)
    for cfg, want in [((2, 4, 256, 8), 8), ((1, 1, 64, 16), 16), ((1, 1, 64, 24), 24),
                      ((1, 4, 256, 8), 8)]:
        shape = sim.eval_config(cfg, len(idx))
        assert shape["splits"] == want, shape
        got = host(sim.evaluate(idx))
        errs = eval_errors(got, ref)
        say("xcd", cfg, errs)
        assert max(errs) <= TOL_EVAL, (cfg, errs)
    sim.eval_config(None)


def test_eval_tiny_systems(nb):
    # n = 1: no partner, everything zero; n = 2: closed form
    sim = make_sim(nb, 1)
    sim.set_state(np.array([1.0]), np.zeros((3, 1)), np.zeros((3, 1)))
    sim.predict(0)
    out = host(sim.evaluate(np.array([0], np.int32)))
    assert np.array_equal(out, np.zeros((10, 1)))
    m = np.array([0.7, 0.3])
    x = np.array([[0.0, 0.75], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [0.0, 0.4], [0.0, 0.0]])
    sim = make_sim(nb, 2, eps=0.1)
    sim.set_state(m, x, v)
    sim.predict(0)
    got = host(sim.evaluate(np.array([0, 1], np.int32)))
    ref = oracle.evaluate(m, x, v, np.zeros((3, 2)), 0.1)
    assert max(eval_errors(got, ref)[:1]) <= TOL_EVAL
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-300)


def test_coincident_bodies(nb):
    """Two bodies at the same place: with softening every term is finite and matches
    the oracle; without it their pair term is not finite, and the first block step
    reports NB_ERR_NUMERIC instead of carrying non-finite values on."""
    m = np.array([0.4, 0.35, 0.25])
    x = np.array([[0.1, 0.1, -0.6], [0.2, 0.2, 0.3], [0.0, 0.0, 0.1]])
    v = np.array([[0.0, 0.3, 0.1], [0.1, 0.0, -0.2], [0.0, 0.0, 0.05]])
    sim = make_sim(nb, 3, eps=1e-2)
    sim.set_state(m, x, v)
    sim.predict(0)
    got = host(sim.evaluate(np.arange(3, dtype=np.int32)))
    ref = oracle.evaluate(m, x, v, np.zeros((3, 3)), 1e-2)
    assert np.isfinite(got).all()
    assert max(eval_errors(got, ref)) <= TOL_EVAL
    sim0 = make_sim(nb, 3, eps=0.0)
    sim0.set_state(m, x, v)
    sim0.start()
    with pytest.raises(nb.NBodyError) as e:
        sim0.step()   # its first wait reports the start-up's non-finite values
    assert e.value.status == 5 and "non-finite" in str(e.value), str(e.value)


def test_eval_empty_active_set_is_noop(nb):
    n = 100
    ic, ap = system(n, 7)
    sim = make_sim(nb, n)
    sim.set_state(ic.m, ic.x, ic.v)
    sim.predict(0)
    out = sim.evaluate(np.zeros(0, np.int32))
    assert out.shape == (10, 0)


# ------------------------------------------------------------------- predictor --
def test_predict_parity(nb):
    n = 5003
    g = ni.rng(202)
    x, v, a, j, s, c = (g.normal(0, sc, (3, n)) for sc in (1.0, 1.0, 2.0, 10.0, 100.0, 1e3))
    tick, level = ni.block_state(n, 203, L, max_level=12)
    tick_next = int(tick.max()) + (1 << (L - 2))
    sim = make_sim(nb, n)
    sim.set_state(np.full(n, 1.0 / n), x, v, a=a, j=j, s=s, c=c, tick=tick, level=level)
    sim.predict(tick_next)
    xp, vp, ap = (host(t) for t in sim.get_predicted())
    rx, rv, ra = oracle.predict(tick, tick_next, DT_MIN, x, v, a, j, s, c)
    h = (tick_next - tick) * 2.0 ** DT_MIN
    sx = np.abs(x) + h * np.abs(v) + h**2 / 2 * np.abs(a) + h**3 / 6 * np.abs(j) \
        + h**4 / 24 * np.abs(s) + h**5 / 120 * np.abs(c)
    sv = np.abs(v) + h * np.abs(a) + h**2 / 2 * np.abs(j) + h**3 / 6 * np.abs(s) + h**4 / 24 * np.abs(c)
    sa = np.abs(a) + h * np.abs(j) + h**2 / 2 * np.abs(s) + h**3 / 6 * np.abs(c)
    assert np.all(np.abs(xp - rx) <= 8 * U * sx)
    assert np.all(np.abs(vp - rv) <= 8 * U * sv)
    assert np.all(np.abs(ap - ra) <= 8 * U * sa)


# ------------------------------------------------------------------- corrector --
def test_correct_parity(nb):
    n = 4001
    g = ni.rng(303)
    x, v, a, j, s = (g.normal(0, sc, (3, n)) for sc in (1.0, 1.0, 2.0, 10.0, 100.0))
    tick, level = ni.block_state(n, 304, L, max_level=14)
    # the active bodies are those due at the next block time of this state
    idx, tick_next = oracle.active(tick, level, L)
    na = idx.shape[0]
    assert na > 0
    h = (tick_next - tick[idx]) * 2.0 ** DT_MIN
    # new evaluation: old values plus a smooth change over the step
    anew = np.concatenate([a[:, idx] + h * j[:, idx] + g.normal(0, 1e-3, (3, na)),
                           j[:, idx] + h * s[:, idx] + g.normal(0, 1e-2, (3, na)),
                           s[:, idx] + g.normal(0, 1e-1, (3, na)),
                           g.normal(0, 1, (1, na))])
    sim = make_sim(nb, n)
    sim.set_state(np.full(n, 1.0 / n), x, v, a=a, j=j, s=s, tick=tick, level=level)
    sim.set_evaluation(idx, anew)
    sim.correct(idx, tick_next)
    st = {k: host(t) for k, t in sim.get_state().items()}
    ost = oracle.State(m=np.full(n, 1.0 / n), x=x, v=v, a=a, j=j, s=s, tick=tick, level=level)
    oracle.correct(ost, idx, tick_next, DT_MIN, anew)
    assert np.array_equal(st["tick"], ost.tick)
    for k in ("a", "j", "s"):
        assert np.array_equal(st[k], getattr(ost, k))
    A0, J0, S0, V0, X0 = (np.abs(q[:, idx]) for q in (a, j, s, v, x))
    A1, J1, S1 = np.abs(anew[0:3]), np.abs(anew[3:6]), np.abs(anew[6:9])
    scv = V0 + h / 2 * (A0 + A1) + h**2 / 10 * (J0 + J1) + h**3 / 120 * (S0 + S1)
    scx = X0 + h / 2 * (V0 + np.abs(st["v"][:, idx])) + h**2 / 10 * (A0 + A1) + h**3 / 120 * (J0 + J1)
    assert np.all(np.abs(st["v"][:, idx] - ost.v[:, idx]) <= 16 * U * scv)
    assert np.all(np.abs(st["x"][:, idx] - ost.x[:, idx]) <= 16 * U * (scx + scv * h))
    sc3 = (60 * (A0 + A1) + h * (36 * J1 + 24 * J0) + h**2 * (9 * S1 + 3 * S0)) / h**3
    assert np.all(np.abs(st["c"][:, idx] - ost.c[:, idx]) <= 32 * U * sc3)
    sc4 = (360 * (A0 + A1) + h * (192 * J1 + 168 * J0) + h**2 * (36 * S1 + 24 * S0)) / h**4
    sc5 = (720 * (A0 + A1) + 360 * h * (J1 + J0) + 60 * h**2 * (S1 + S0)) / h**5
    assert np.all(np.abs(st["a4n"][idx] - ost.a4n[idx]) <= 32 * U * np.linalg.norm(sc4, axis=0))
    assert np.all(np.abs(st["a5n"][idx] - ost.a5n[idx]) <= 32 * U * np.linalg.norm(sc5, axis=0))
    untouched = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(st["x"][:, untouched], x[:, untouched])


# ----------------------------------------------------------------- step levels --
@pytest.mark.parametrize("init", [0, 1])
def test_timesteps_parity_bit_exact(nb, init):
    n = 6007
    g = ni.rng(404 + init)
    # magnitudes spread over many decades so that every level and rule is exercised
    mags = lambda sc: g.normal(0, 1, (3, n)) * 10.0 ** g.uniform(-3, 3, n) * sc
    a, j, s, c = mags(1.0), mags(30.0), mags(1e3), mags(3e4)
    a4n = np.abs(g.normal(0, 1, n)) * 10.0 ** g.uniform(2, 8, n)
    a5n = np.abs(g.normal(0, 1, n)) * 10.0 ** g.uniform(3, 10, n)
    if init:
        tick = np.zeros(n, np.int64)
        level = np.zeros(n, np.int32)
    else:
        tick, level = ni.block_state(n, 405, L, max_level=20)
    idx = ni.active_subset(n, 4000, 406)
    sim = make_sim(nb, n)
    sim.set_state(np.full(n, 1.0 / n), np.zeros((3, n)), np.zeros((3, n)), a=a, j=j, s=s, c=c,
                  a4n=a4n, a5n=a5n, tick=tick, level=level)
    sim.timesteps(idx, init=bool(init))
    got = host(sim.get_state()["level"])
    ost = oracle.State(m=np.full(n, 1.0 / n), x=np.zeros((3, n)), v=np.zeros((3, n)), a=a, j=j,
                       s=s, c=c, a4n=a4n, a5n=a5n, tick=tick, level=level)
    rc = oracle.timesteps(ost, idx, init, 0.45, 0.01, DT_MAX, DT_MIN, check=False)
    assert rc in (0, 2)
    assert np.array_equal(got, ost.level)
    assert len(np.unique(ost.level[idx])) > 5


# ------------------------------------------------------------------ active set --
@pytest.mark.parametrize("n", [1, 5000, 3 * 2048 + 17])
def test_active_parity_bit_exact(nb, n):
    sim = make_sim(nb, n)
    for seed in range(3):
        tick, level = ni.block_state(n, 500 + seed, L, max_level=16)
        sim.set_state(np.full(n, 1.0 / n), np.zeros((3, n)), np.zeros((3, n)), tick=tick,
                      level=level)
        idx, tn = sim.active()
        ridx, rtn = oracle.active(tick, level, L)
        assert tn == rtn
        assert np.array_equal(host(idx), ridx)


# ---------------------------------------------------------------------- energy --
@pytest.mark.parametrize("n,eps", [(3001, 1e-4), (2, 0.0), (700, 0.05)])
def test_energy_parity(nb, n, eps):
    ic = ni.plummer(n, 606)
    sim = make_sim(nb, n, eps=eps)
    sim.set_state(ic.m, ic.x, ic.v)
    ek, ep = sim.energy(0)
    rk, rp = oracle.energy(ic.m, ic.x, ic.v, eps)
    assert abs(ek - rk) <= 1e-12 * abs(rk)
    assert abs(ep - rp) <= 1e-12 * abs(rp)


# ----------------------------------------------------------- whole integration --
def _c1(nb, n=1024, seed=1):
    ic = ni.plummer(n, seed)
    sim = make_sim(nb, n, eps=1e-4)
    sim.set_state(ic.m, ic.x, ic.v)
    return ic, sim


def test_c1_block_steps_match_oracle(nb):
    ic, sim = _c1(nb)
    t_end = 1 << L  # t = 0.125 = dt_max
    e0 = sum(sim.energy(0))
    sim.set_state(ic.m, ic.x, ic.v)
    sim.start()
    steps, log, inter = sim.integrate(t_end)
    e1 = sum(sim.energy(t_end))
    st = {k: host(t) for k, t in sim.get_state().items()}
    ost = oracle.State(m=ic.m, x=ic.x, v=ic.v)
    osteps, ostt, osna, ointer = oracle.integrate(ost, 1e-4, 0.45, 0.01, DT_MAX, DT_MIN, t_end)
    ro = oracle.energy(ic.m, ic.x, ic.v, 1e-4)
    r1 = oracle.energy(ost.m, ost.x, ost.v, 1e-4)
    say("c1 steps gpu/oracle", steps, osteps, "dE gpu", (e1 - e0) / abs(e0),
        "dE oracle", (sum(r1) - sum(ro)) / abs(sum(ro)))
    gt = np.array([t for t, _ in log])
    gn = np.array([k for _, k in log])
    # the two runs take the same block steps (level decisions are FP64 on both sides;
    # round-off differences could flip a level at a power-of-two boundary, which would
    # show up here first)
    assert steps == osteps
    assert np.array_equal(gt, ostt) and np.array_equal(gn, osna)
    assert np.all(st["tick"] == t_end)
    assert np.array_equal(st["level"], ost.level)
    dx = np.abs(st["x"] - ost.x).max()
    assert dx < 1e-9, dx
    assert abs((e1 - e0) - (sum(r1) - sum(ro))) < 1e-9 * abs(sum(ro))


def test_c1_per_step_replay_errors(nb):
    """W1 block steps on the GPU, replayed: at every block step the oracle evaluates
    the active bodies from the GPU's own predicted positions, velocities and
    accelerations (identical inputs), and every per-body relative error of a, j, s
    (and phi) stays within the FP64 bound. Prints the max and p99 over all steps
    and bodies."""
    ic, sim = _c1(nb)
    t_end = 1 << L
    sim.start()
    errs = {"a": [], "j": [], "s": [], "phi": []}
    steps = inter = 0
    while True:
        idx, tn = sim.active()
        if len(idx) == 0 or tn > t_end:
            break
        sim.predict(tn)
        got = host(sim.evaluate(idx))
        xp, vp, ap = (host(t) for t in sim.get_predicted())
        ref = oracle.evaluate(ic.m, xp, vp, ap, 1e-4, idx=host(idx))
        errs["a"].append(rel_vec_err(got[0:3], ref[0:3]))
        errs["j"].append(rel_vec_err(got[3:6], ref[3:6]))
        errs["s"].append(rel_vec_err(got[6:9], ref[6:9]))
        errs["phi"].append(np.abs(got[9] - ref[9]) / np.abs(ref[9]))
        sim.correct(idx, tn)
        sim.timesteps(idx)
        steps += 1
        inter += len(idx) * ic.m.size
    summary = {k: (float(np.concatenate(v).max()), float(np.percentile(np.concatenate(v), 99)))
               for k, v in errs.items()}
    say("c1 replay: steps", steps, "interactions", inter, "max / p99 relative error", summary)
    assert steps == 215
    for k, (mx, _) in summary.items():
        assert mx <= TOL_EVAL, (k, mx)


def test_determinism_and_checkpoint_resume(nb):
    ic, sim = _c1(nb, n=512, seed=11)
    sim.start()
    t_mid, t_end = 1 << (L - 1), 1 << L
    sim.integrate(t_mid)
    ck = sim.get_state()
    sim.integrate(t_end)
    a = {k: host(t) for k, t in sim.get_state().items()}
    # same run again from scratch: bitwise identical
    ic2, sim2 = _c1(nb, n=512, seed=11)
    sim2.start()
    sim2.integrate(t_end)
    b = {k: host(t) for k, t in sim2.get_state().items()}
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # resume from the checkpoint in a fresh context: bitwise identical
    sim3 = make_sim(nb, 512, eps=1e-4)
    sim3.set_state(ck["m"], ck["x"], ck["v"], a=ck["a"], j=ck["j"], s=ck["s"], c=ck["c"],
                   a4n=ck["a4n"], a5n=ck["a5n"], tick=ck["tick"], level=ck["level"])
    sim3.integrate(t_end)
    c = {k: host(t) for k, t in sim3.get_state().items()}
    for k in a:
        if k == "phi":
            continue  # phi of bodies not stepped after the restore is not part of the state
        assert np.array_equal(a[k], c[k]), k


# --------------------------------------------------------------- error paths --
def test_errors_are_reported(nb):
    n = 64
    ic, ap = system(n, 9)
    sim = make_sim(nb, n)
    sim.set_state(ic.m, ic.x, ic.v)
    with pytest.raises(nb.NBodyError) as e:
        sim.evaluate(np.arange(4, dtype=np.int32))  # no prediction yet
    assert e.value.status == 4
    sim.predict(0)
    bad = np.array([0, 5, n + 3], np.int32)   # out of range: clamped in-kernel, reported
    sim.evaluate(bad)
    with pytest.raises(nb.NBodyError) as e:
        sim.energy(0)
    assert e.value.status == 1
    sim.energy(0)  # the latched error was cleared
    with pytest.raises(nb.NBodyError) as e:
        sim.correct(np.arange(4, dtype=np.int32), 1 << 10)
    assert e.value.status == 4
    # a list that is not strictly ascending is refused by the corrector's check
    for dup in (np.array([3, 5, 5, 9], np.int32), np.array([7, 2, 11], np.int32)):
        sim2 = make_sim(nb, n)
        sim2.set_state(ic.m, ic.x, ic.v, a=ap)
        sim2.predict(1 << 10)
        sim2.evaluate(dup)
        sim2.correct(dup, 1 << 10)
        with pytest.raises(nb.NBodyError) as e:
            sim2.energy(1 << 10)
        assert e.value.status == 1 and "ascending" in str(e.value), str(e.value)


# ------------------------------------------------ a large system, sampled outputs --
def test_large_system_sampled(nb):
    """2^25 + 777 bodies (a 13 GB workspace, 2.7 GB of j-records, so byte offsets
    pass 2^31): the active set of a random block state bit-exact against the
    oracle, then the prediction of every body and the evaluation of 64 active
    bodies, eight of them sampled against the oracle."""
    n = (1 << 25) + 777
    say("large system", n)
    tick, level = ni.block_state(n, 505, L, max_level=16)
    ic = ni.plummer(n, 5)
    ap = ni.plummer_mean_field_acc(ic.x)
    sim = make_sim(nb, n, eps=1e-4, partial_slots=1 << 20)
    sim.set_state(ic.m, ic.x, ic.v, a=ap, tick=tick, level=level)
    idx, tn = sim.active()
    ridx, rtn = oracle.active(tick, level, L)
    assert tn == rtn
    assert np.array_equal(host(idx), ridx)
    sim.set_state(ic.m, ic.x, ic.v, a=ap)
    sim.predict(0)
    act = ni.active_subset(n, 64, 506)
    got = host(sim.evaluate(act))
    pick = np.arange(0, 64, 8)
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=act[pick])
    errs = eval_errors(got[:, pick], ref)
    say("large system errors", errs)
    assert max(errs) <= TOL_EVAL, errs
    del sim


# --------------------------------------------------- full-size, sampled outputs --
@pytest.fixture(scope="module")
def c2_inputs():
    """The N = 65536 Plummer sphere (seed 2) with its predicted accelerations taken
    from the oracle: the first pass of the Hermite start-up (a of every body from x
    and v), as the N = 65536 sweep workload specifies."""
    n = 65536
    ic = ni.plummer(n, 2)
    first = oracle.evaluate(ic.m, ic.x, ic.v, np.zeros((3, n)), 1e-4)
    return ic, np.ascontiguousarray(first[0:3])


@pytest.mark.parametrize("n_act", [1, 64, 1024, 8192, 65536])
def test_c2_full_size_sampled(nb, c2_inputs, n_act):
    n = 65536
    ic, ap = c2_inputs
    sim = make_sim(nb, n, eps=1e-4)
    sim.set_state(ic.m, ic.x, ic.v, a=ap)
    sim.predict(0)
    k = [1, 64, 1024, 8192, 65536].index(n_act)
    idx = ni.active_subset(n, n_act, 20 + k)
    say("c2 sampled", n_act, sim.eval_config(None, n_act))
    got = host(sim.evaluate(idx))
    pick = np.unique(np.linspace(0, n_act - 1, min(n_act, 256)).astype(np.int64))
    ref = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4, idx=idx[pick])
    errs = eval_errors(got[:, pick], ref)
    say("c2 errors", n_act, errs)
    stats = error_stats(got[:, pick], ref)
    kap = condition_numbers(ic.m, ic.x, ic.v, ap, 1e-4, idx[pick][:64])
    for c, q in enumerate("ajs"):
        say(f"c2 n_act {n_act} {q}: relative error p50 {stats[c][0]:.2e} p99 {stats[c][1]:.2e} "
            f"max {stats[c][2]:.2e}; kappa p50 {np.median(kap[c]):.1f} max {kap[c].max():.1f}")
    assert max(errs) <= TOL_EVAL, errs
