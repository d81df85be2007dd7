"""Pins of the oracle's predictor, corrector, block steps, active set, energy and
integration loop.

  * predictor: exact (to round-off) on polynomial motion of degree <= 5 whose
    derivatives are given at the start;
  * corrector: the velocity update is exact for accelerations of degree <= 5, the
    position update for degree <= 4, and its residual for a pure t^5 term is
    h^7/840 times that coefficient; the interpolated 3rd/4th/5th derivatives are
    exact for degree 5;
  * block rules: hand cases with outcomes fixed by the rules;
  * active set: brute force over the definition on random block states;
  * energy: closed-form two-body value;
  * integration: closed-form Kepler orbit (Kepler's equation), 6th-order
    convergence with fixed steps, energy conservation, block invariants;
  * step criterion and start rule: the circular-orbit closed form (eta / omega and
    eta_init / omega at any radius); the criterion itself is a reading of the
    literature, since the paper prints no formula.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import nbody_inputs as ni
import oracle

DT_MIN_LOG2 = -40


def _poly(coef, t, deriv=0):
    """Value of the deriv-th derivative of sum_k coef[k] t^k (coef[k] arrays)."""
    tot = np.zeros_like(coef[0])
    for k in range(deriv, len(coef)):
        f = math.factorial(k) / math.factorial(k - deriv)
        tot = tot + coef[k] * f * t ** (k - deriv)
    return tot


def test_predictor_exact_on_degree5_motion():
    n = 40
    g = ni.rng(21)
    coef = [g.normal(0, 1, (3, n)) for _ in range(6)]
    tick = g.integers(0, 1 << 20, n).astype(np.int64) * (1 << 10)
    tick_next = int(tick.max()) + (1 << 32)
    x, v, a, j, s, c = (_poly(coef, 0.0, d) for d in range(6))
    xp, vp, ap = oracle.predict(tick, tick_next, DT_MIN_LOG2, x, v, a, j, s, c)
    h = (tick_next - tick) * 2.0**DT_MIN_LOG2
    mp.mp.dps = 30
    for i in range(0, n, 7):
        for k in range(3):
            cs = [mp.mpf(coef[d][k, i]) for d in range(6)]
            H = mp.mpf(h[i])
            ex = [sum(cs[d] * mp.factorial(d) / mp.factorial(d - q) * H ** (d - q)
                      for d in range(q, 6)) for q in range(3)]
            scale = [sum(abs(cs[d]) * mp.factorial(d) / mp.factorial(d - q) * H ** (d - q)
                         for d in range(q, 6)) for q in range(3)]
            for got, e, sc in zip((xp[k, i], vp[k, i], ap[k, i]), ex, scale):
                assert abs(got - float(e)) <= 4 * 2.0**-53 * float(sc)


@pytest.mark.parametrize("deg,hlog2", [(3, -7), (4, -7), (5, -7), (5, -1)])
def test_corrector_polynomial_exactness(deg, hlog2):
    n = 24
    g = ni.rng(30 + deg)
    # acceleration a(t) = sum_{k<=deg} ca[k] t^k ; v, x its integrals with v(0), x(0)
    ca = [g.normal(0, 1, (3, n)) for _ in range(deg + 1)]
    v0 = g.normal(0, 1, (3, n))
    x0 = g.normal(0, 1, (3, n))
    level = np.zeros(n, dtype=np.int32)
    dt_ticks = 1 << (hlog2 - DT_MIN_LOG2)
    h = dt_ticks * 2.0**DT_MIN_LOG2

    def a_t(t, d=0):
        return _poly(ca, t, d)

    def v_t(t):
        return v0 + sum(ca[k] * t ** (k + 1) / (k + 1) for k in range(len(ca)))

    def x_t(t):
        return x0 + v0 * t + sum(ca[k] * t ** (k + 2) / ((k + 1) * (k + 2))
                                 for k in range(len(ca)))

    st = oracle.State(m=np.full(n, 1.0 / n), x=x0, v=v0, a=a_t(0.0), j=a_t(0.0, 1),
                      s=a_t(0.0, 2), c=np.zeros((3, n)), tick=np.zeros(n, np.int64),
                      level=level)
    anew = np.concatenate([a_t(h), a_t(h, 1), a_t(h, 2), np.zeros((1, n))])
    idx = np.arange(n, dtype=np.int32)
    oracle.correct(st, idx, dt_ticks, DT_MIN_LOG2, anew)
    assert np.all(st.tick == dt_ticks)
    tol = 1e-14
    assert np.abs(st.v - v_t(h)).max() < tol
    if deg <= 4:
        assert np.abs(st.x - x_t(h)).max() < tol
    else:
        # x-corrector residual for the t^5 term: formula - exact = c5 h^7 / 840
        resid = st.x - x_t(h)
        assert np.all(np.abs(resid - ca[5] * h**7 / 840.0) < tol)
        if hlog2 == -1:
            assert np.abs(ca[5] * h**7 / 840.0).max() > 1e3 * tol
    # interpolated derivatives at t1 are exact for degree <= 5
    # (round-off of the divided differences scales as u * |terms| / h^k)
    a3, a4, a5 = a_t(h, 3), a_t(h, 4), a_t(h, 5)
    A0, A1 = np.abs(a_t(0.0)), np.abs(a_t(h))
    J0, J1 = np.abs(a_t(0.0, 1)), np.abs(a_t(h, 1))
    S0, S1 = np.abs(a_t(0.0, 2)), np.abs(a_t(h, 2))
    u = 2.0**-53
    sc3 = (60 * (A0 + A1) + h * (36 * J1 + 24 * J0) + h * h * (9 * S1 + 3 * S0)) / h**3
    sc4 = (360 * (A0 + A1) + h * (192 * J1 + 168 * J0) + h * h * (36 * S1 + 24 * S0)) / h**4
    sc5 = (720 * (A0 + A1) + 360 * h * (J1 + J0) + 60 * h * h * (S1 + S0)) / h**5
    assert np.all(np.abs(st.c - a3) <= 8 * u * sc3)
    assert np.all(np.abs(st.a4n - np.linalg.norm(a4, axis=0)) <= 16 * u * np.linalg.norm(sc4, axis=0))
    assert np.all(np.abs(st.a5n - np.linalg.norm(a5, axis=0)) <= 16 * u * np.linalg.norm(sc5, axis=0))
    assert np.array_equal(st.a, anew[0:3]) and np.array_equal(st.s, anew[6:9])


def _ts_state(a, j, s, c, a4n, a5n, tick, level):
    n = 1
    st = oracle.State(m=np.ones(n), x=np.zeros((3, n)), v=np.zeros((3, n)),
                      a=np.array(a, float).reshape(3, 1), j=np.array(j, float).reshape(3, 1),
                      s=np.array(s, float).reshape(3, 1), c=np.array(c, float).reshape(3, 1),
                      a4n=np.array([a4n]), a5n=np.array([a5n]),
                      tick=np.array([tick]), level=np.array([level]))
    return st


ETA = 0.45
L = -3 - DT_MIN_LOG2


def _ticks(k):
    return 1 << (L - k)


def test_block_rule_shrink_is_free():
    # |a| = |s| = 1, j = 0 -> numerator 1 ; c = 0, |a4| = 1/ratio -> denominator 1/ratio
    # criterion: dt^3 <= eta^3 * ratio. Scale ratio to put Delta between 2^-12 and 2^-11.
    ratio = (1.5 * 2.0**-12) ** 3 / ETA**3
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / ratio, 0.0,
                   tick=7 * _ticks(3), level=3)
    oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 9      # dt = 2^(-3-9) = 2^-12


def test_block_rule_grow_one_level_only_at_even_time():
    big = 1e6  # criterion allows any step
    # time is an odd multiple of the current step: no growth
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / big, 0.0,
                   tick=3 * _ticks(5), level=5)
    oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 5
    # even multiple: grows by exactly one level
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / big, 0.0,
                   tick=6 * _ticks(5), level=5)
    oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 4
    # level 0 cannot grow beyond dt_max
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / big, 0.0,
                   tick=8 * _ticks(0), level=0)
    oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 0


def test_block_rule_no_growth_when_double_step_does_not_fit():
    ratio = (1.5 * 2.0**-10) ** 3 / ETA**3      # Delta in [2^-10, 2^-9)
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / ratio, 0.0,
                   tick=4 * _ticks(7), level=7)   # dt = 2^-10, 2 dt = 2^-9 does not fit
    oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 7


def test_block_rule_below_dt_min_is_an_error():
    ratio = (2.0**-45) ** 3 / ETA**3
    st = _ts_state([1, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0], 1 / ratio, 0.0,
                   tick=0, level=3)
    rc = oracle.timesteps(st, [0], 0, ETA, 0.01, -3, DT_MIN_LOG2, check=False)
    assert rc == 2 and st.level[0] == L


def test_initial_step_rule():
    # |a| = 2, |j| = 8, |s| = 2  -> min(|a|/|j|, sqrt(|a|/|s|)) = 0.25 ; eta_init 0.01
    # Delta0 = 2.5e-3 -> largest power of two below it is 2^-9 -> level 6
    st = _ts_state([2, 0, 0], [0, 8, 0], [0, 0, 2], [0, 0, 0], 0.0, 0.0, tick=0, level=0)
    oracle.timesteps(st, [0], 1, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 6
    # at a time that the candidate step does not divide, the level is lowered until it does
    st = _ts_state([2, 0, 0], [0, 8, 0], [0, 0, 2], [0, 0, 0], 0.0, 0.0,
                   tick=_ticks(8), level=0)
    oracle.timesteps(st, [0], 1, ETA, 0.01, -3, DT_MIN_LOG2)
    assert st.level[0] == 8


def _circular_derivatives(omega, radius, phase, rot):
    """a, a', ..., a^(5) of uniform circular motion at angular speed omega, radius
    radius and phase phase, in the plane turned by the rotation matrix rot: with
    r = radius (cos th, sin th, 0), a = -omega^2 r and the k-th derivative turns the
    vector by k quarter turns and scales it by omega^k."""
    out = []
    for k in range(6):
        th = phase + k * math.pi / 2
        out.append(rot @ (-(omega ** (k + 2)) * radius * np.array([math.cos(th), math.sin(th), 0.0])))
    return out


def _rotation(g):
    q, _ = np.linalg.qr(g.standard_normal((3, 3)))
    return q


@pytest.mark.parametrize("init", [0, 1])
def test_step_criterion_circular_orbit_closed_form(init):
    """On a circular orbit every derivative of the acceleration has magnitude
    |a| omega^k, so the sixth-order Aarseth criterion gives eta / omega exactly and the
    start rule gives eta_init / omega (the orbital time scale, whatever the radius).
    The step is the largest power of two not above that. Time scales are placed
    0.15 and 0.85 of an octave above a power of two, so a factor of 2^(1/3) either
    way (a dropped term, a swapped derivative) or a wrong power of omega moves the
    level."""
    g = ni.rng(41)
    eta_init = 0.01
    for e in (4.15, 4.85, 7.5, 12.15, 12.85, 21.15, 21.85, 33.15, 36.85):
        for radius in (1e-3, 1.0, 250.0):
            # time scale 2^-e of the tested rule
            omega = (eta_init if init else ETA) * 2.0 ** e
            a, j, s, c, a4, a5 = _circular_derivatives(omega, radius, float(g.uniform(0, 6.3)),
                                                       _rotation(g))
            st = _ts_state(a, j, s, c, np.linalg.norm(a4), np.linalg.norm(a5), tick=0, level=0)
            oracle.timesteps(st, [0], init, ETA, eta_init, -3, DT_MIN_LOG2)
            # largest 2^(-3-k) <= 2^-e
            assert st.level[0] == math.ceil(e) - 3, (e, radius, init)


def test_active_set_brute_force():
    g = ni.rng(40)
    Lt = 20
    for trial in range(20):
        n = int(g.integers(1, 300))
        level = g.integers(0, 8, n).astype(np.int32)
        # a valid block state: each body's time is a multiple of its step
        tick = np.array([int(g.integers(0, 64)) * (1 << (Lt - k)) for k in level], np.int64)
        idx, tn = oracle.active(tick, level, Lt)
        ends = tick + (1 << (Lt - level.astype(np.int64)))
        assert tn == ends.min()
        assert np.array_equal(idx, np.nonzero(ends == tn)[0].astype(np.int32))


def test_energy_two_body_closed_form():
    m = np.array([0.25, 0.75])
    x = np.array([[0.1, -0.4], [0.2, 0.3], [-0.3, 0.0]])
    v = np.array([[0.5, -0.1], [0.0, 0.2], [0.3, -0.4]])
    eps = 0.05
    ek, ep = oracle.energy(m, x, v, eps)
    d2 = ((x[:, 0] - x[:, 1]) ** 2).sum() + eps * eps
    assert ek == pytest.approx(0.5 * (m * (v ** 2).sum(0)).sum(), rel=1e-15)
    assert ep == pytest.approx(-m[0] * m[1] / math.sqrt(d2), rel=1e-15)


# ----------------------------------------------------------------- Kepler ----
def _kepler_state(e=0.5):
    """Two bodies of mass 1/2 on an orbit with a = 1, eccentricity e, at pericentre."""
    rp = 1.0 - e
    vp = math.sqrt((1.0 + e) / (1.0 - e))
    m = np.array([0.5, 0.5])
    x = np.array([[-rp / 2, rp / 2], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-vp / 2, vp / 2], [0.0, 0.0]])
    return oracle.State(m=m, x=x, v=v)


def _kepler_exact(t, e=0.5):
    M = t  # mean motion sqrt(G M / a^3) = 1
    E = M
    for _ in range(60):
        E = E - (E - e * math.sin(E) - M) / (1.0 - e * math.cos(E))
    rx = math.cos(E) - e
    ry = math.sqrt(1 - e * e) * math.sin(E)
    return np.array([[-rx / 2, rx / 2], [-ry / 2, ry / 2], [0.0, 0.0]])


@pytest.mark.parametrize("eta,tol", [(0.45, 2e-6), (0.1, 1e-9)])
def test_kepler_orbit_block_steps(eta, tol):
    st = _kepler_state()
    t_end_ticks = 2 * (1 << 40)      # t = 2
    steps, stt, sna, _ = oracle.integrate(st, 0.0, eta, 0.01, -3, DT_MIN_LOG2, t_end_ticks)
    assert steps > 10
    assert np.all(st.tick == t_end_ticks)
    ref = _kepler_exact(2.0)
    assert np.abs(st.x - ref).max() < tol
    e0 = sum(oracle.energy(np.array([0.5, 0.5]), _kepler_state().x, _kepler_state().v, 0.0))
    e1 = sum(oracle.energy(st.m, st.x, st.v, 0.0))
    assert abs(e1 - e0) < 1e3 * tol * abs(e0)


def test_sixth_order_convergence():
    errs = []
    for k in (4, 5, 6):
        st = _kepler_state()
        # eta and eta_init huge: every step is the fixed dt_max = 2^-k
        oracle.integrate(st, 0.0, 1e9, 1e9, -k, DT_MIN_LOG2, 2 * (1 << 40))
        errs.append(np.abs(st.x - _kepler_exact(2.0)).max())
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 5.3 < r1 < 6.8 and 5.3 < r2 < 6.8, errs


def test_block_invariants_plummer():
    ic = ni.plummer(128, 3)
    st = oracle.State(m=ic.m, x=ic.x, v=ic.v)
    t_end = 1 << 37                 # t = 0.125 = dt_max: every body must land on it
    steps, stt, sna, inter = oracle.integrate(st, 1e-4, 0.45, 0.01, -3, DT_MIN_LOG2, t_end)
    assert steps >= 1
    assert np.all(np.diff(stt) > 0)
    assert np.all(st.tick == t_end)
    assert np.all((st.level >= 0) & (st.level <= L))
    assert inter == pytest.approx(2 * 128 * 128 + sna.sum() * 128)


def test_crackle_start_matches_kepler_third_derivative():
    """On the closed-form Kepler orbit (e = 0.5, at pericentre) the crackle start
    sets c to the third time derivative of each body's acceleration, taken by
    40-digit differentiation of the exact solution."""
    import mpmath as mp
    mp.mp.dps = 40
    e = mp.mpf("0.5")

    def accel2(t):
        E = mp.findroot(lambda E: E - e * mp.sin(E) - t, t)
        rx, ry = mp.cos(E) - e, mp.sqrt(1 - e * e) * mp.sin(E)
        r3 = (rx * rx + ry * ry) ** mp.mpf(1.5)
        # body 2 sits at +r/2; its acceleration from body 1 (mass 1/2) is -r / (2 |r|^3)
        return [-rx / (2 * r3), -ry / (2 * r3)]

    st = _kepler_state()
    oracle.integrate(st, 0.0, 0.45, 0.01, -3, DT_MIN_LOG2, 0, start_crackle=True)
    for k in range(2):
        ref = mp.diff(lambda t: accel2(t)[k], 0, 3)
        assert abs(st.c[k, 1] - float(ref)) <= 1e-12 * max(1.0, abs(float(ref))), (k, st.c[:, 1], ref)
        assert st.c[k, 0] == pytest.approx(-st.c[k, 1], rel=1e-14, abs=1e-14)


def test_crackle_start_sets_the_evaluated_crackle():
    """With the crackle start the initial c is the crackle evaluated from the
    start-up passes' a and j (zero steps taken)."""
    import nbody_inputs as ni
    ic = ni.plummer(64, 5)
    st = oracle.State(m=ic.m, x=ic.x, v=ic.v)
    oracle.integrate(st, 1e-3, 0.45, 0.01, -3, -40, 0, start_crackle=True)
    # reference: the two start-up passes by hand, then the crackle evaluation
    p1 = oracle.evaluate(ic.m, ic.x, ic.v, np.zeros((3, 64)), 1e-3)
    p2 = oracle.evaluate(ic.m, ic.x, ic.v, p1[0:3], 1e-3)
    ref = oracle.evaluate_crackle(ic.m, ic.x, ic.v, p1[0:3], p2[3:6], 1e-3)
    assert np.array_equal(st.c, ref[9:12]) and np.array_equal(st.j, p2[3:6])
    assert np.any(st.c != 0.0)
