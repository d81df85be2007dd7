"""Pins of the oracle's pairwise evaluation (acceleration, jerk, snap, potential).

None of these re-types the oracle's jerk/snap formulas:
  * the acceleration is checked against minus the gradient of the potential, both
    taken in 40-digit arithmetic from the definition of the softened potential;
  * jerk and snap are checked against the first and second time derivatives of
    that acceleration along the bodies' quadratic trajectories x(t) = x + v t + a t^2/2
    (numerical differentiation at 40 digits);
  * Newton's third law (sum m a = sum m j = sum m s = 0, zero net torque) and
    translation/Galilean invariance must hold to round-off;
  * a two-body case is compared with its closed form.
The error metric is the per-body relative error of the 3-vector (Euclidean norm).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import nbody_inputs as ni
import oracle

mp.mp.dps = 40


def _random_system(n, seed, spread=1.0):
    g = ni.rng(seed)
    m = g.uniform(0.2, 1.0, n)
    m /= m.sum()
    x = g.normal(0, spread, (3, n))
    v = g.normal(0, 0.7, (3, n))
    a = g.normal(0, 1.5, (3, n))
    return m, x, v, a


def _mp_phi_i(i, m, X, eps):
    """Potential at body i from the definition, X a list of mp 3-vectors."""
    tot = mp.mpf(0)
    for j in range(len(m)):
        if j == i:
            continue
        d2 = sum((X[j][k] - X[i][k]) ** 2 for k in range(3)) + mp.mpf(eps) ** 2
        tot -= mp.mpf(m[j]) / mp.sqrt(d2)
    return tot


def _mp_acc_i(i, m, X, eps):
    """Acceleration of body i as minus the gradient of its potential w.r.t. x_i."""
    g = []
    for k in range(3):
        def f(h, k=k):
            Y = [list(p) for p in X]
            Y[i][k] = Y[i][k] + h
            return _mp_phi_i(i, m, Y, eps)
        g.append(-mp.diff(f, 0))
    return g


def _traj(x, v, a, t):
    n = x.shape[1]
    return [[mp.mpf(x[k, j]) + mp.mpf(v[k, j]) * t + mp.mpf(a[k, j]) * t * t / 2
             for k in range(3)] for j in range(n)]


def _mp_acc_direct(i, m, X, eps):
    """Softened Newtonian acceleration of body i (definition), for differentiation."""
    out = [mp.mpf(0)] * 3
    for j in range(len(m)):
        if j == i:
            continue
        r = [X[j][k] - X[i][k] for k in range(3)]
        R = sum(c * c for c in r) + mp.mpf(eps) ** 2
        f = mp.mpf(m[j]) / (R * mp.sqrt(R))
        out = [out[k] + f * r[k] for k in range(3)]
    return out


def _rel(vec_test, vec_ref):
    d = math.sqrt(sum((float(a) - float(b)) ** 2 for a, b in zip(vec_test, vec_ref)))
    nrm = math.sqrt(sum(float(b) ** 2 for b in vec_ref))
    return d / nrm


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_acceleration_is_minus_grad_potential(eps):
    m, x, v, a = _random_system(7, 11)
    out = oracle.evaluate(m, x, v, a, eps)
    X = [[mp.mpf(x[k, j]) for k in range(3)] for j in range(7)]
    for i in range(7):
        ref = _mp_acc_i(i, m, X, eps)
        assert _rel(out[0:3, i], ref) < 1e-14
        phi = _mp_phi_i(i, m, X, eps)
        assert abs(out[9, i] - float(phi)) <= 1e-15 * abs(float(phi))


@pytest.mark.parametrize("eps", [0.0, 3e-2])
def test_jerk_and_snap_are_time_derivatives(eps):
    n = 6
    m, x, v, a = _random_system(n, 12)
    out = oracle.evaluate(m, x, v, a, eps)
    for i in range(n):
        jref, sref = [], []
        for k in range(3):
            def comp(t, k=k):
                return _mp_acc_direct(i, m, _traj(x, v, a, t), eps)[k]
            jref.append(mp.diff(comp, 0, 1))
            sref.append(mp.diff(comp, 0, 2))
        assert _rel(out[3:6, i], jref) < 1e-13, ("jerk", i)
        assert _rel(out[6:9, i], sref) < 1e-13, ("snap", i)


def test_extended_precision_brute_force():
    """All ten outputs against a 40-digit evaluation of the same definitions for
    N = 16: the compensated FP64 oracle stays within a few ulp times the
    condition number sum_j |q_ij| / |q_i|."""
    n = 16
    eps = 1e-3
    m, x, v, a = _random_system(n, 13)
    out = oracle.evaluate(m, x, v, a, eps)
    for i in range(n):
        X = _traj(x, v, a, mp.mpf(0))
        Ai = _mp_acc_direct(i, m, X, eps)
        phi = _mp_phi_i(i, m, X, eps)
        # magnitude sum for the condition number of the acceleration
        kap = mp.mpf(0)
        for j in range(n):
            if j == i:
                continue
            r = [X[j][k] - X[i][k] for k in range(3)]
            R = sum(c * c for c in r) + mp.mpf(eps) ** 2
            kap += mp.mpf(m[j]) / R
        kappa = float(kap / mp.sqrt(sum(c * c for c in Ai)))
        assert _rel(out[0:3, i], Ai) < 8 * 2.0**-53 * max(1.0, kappa)
        assert abs(out[9, i] - float(phi)) <= 4 * 2.0**-53 * abs(float(phi))


def test_newton_third_law_and_torque():
    ic = ni.plummer(512, 5)
    g = ni.rng(6)
    ap = g.normal(0, 1.0, (3, 512))
    out = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-4)
    m = ic.m
    for c0 in (0, 3, 6):
        q = out[c0:c0 + 3]
        net = np.abs((q * m).sum(axis=1)).max()
        scale = (np.linalg.norm(q, axis=0) * m).sum()
        assert net < 1e-14 * scale
    torque = np.cross(ic.x.T, out[0:3].T) * m[:, None]
    scale = (np.linalg.norm(ic.x, axis=0) * np.linalg.norm(out[0:3], axis=0) * m).sum()
    assert np.abs(torque.sum(axis=0)).max() < 1e-14 * scale


def test_translation_and_galilean_invariance():
    ic = ni.plummer(256, 7)
    ap = ni.rng(8).normal(0, 1.0, (3, 256))
    base = oracle.evaluate(ic.m, ic.x, ic.v, ap, 1e-3)
    shifted = oracle.evaluate(ic.m, ic.x + np.array([[0.25], [-0.5], [0.125]]),
                              ic.v + np.array([[0.5], [0.25], [-1.0]]),
                              ap + np.array([[0.0], [2.0], [0.0]]), 1e-3)
    for c0 in (0, 3, 6):
        d = np.linalg.norm(shifted[c0:c0 + 3] - base[c0:c0 + 3], axis=0)
        assert (d / np.linalg.norm(base[c0:c0 + 3], axis=0)).max() < 1e-11
    assert np.allclose(shifted[9], base[9], rtol=1e-12, atol=0)


def test_two_body_closed_form():
    # body 1 at distance d on x, moving perpendicular (circular-type relative velocity)
    d, eps, m1 = 0.75, 0.1, 0.3
    m = np.array([0.7, m1])
    x = np.array([[0.0, d], [0.0, 0.0], [0.0, 0.0]])
    w = 0.4
    v = np.array([[0.0, 0.0], [0.0, w], [0.0, 0.0]])
    a = np.zeros((3, 2))
    out = oracle.evaluate(m, x, v, a, eps, idx=np.array([0], dtype=np.int32))
    R = d * d + eps * eps
    # A = m1 r / R^1.5, r.v = 0 so alpha = 0 and J = m1 v / R^1.5
    assert out[0, 0] == pytest.approx(m1 * d / R**1.5, rel=1e-15)
    assert out[1, 0] == 0.0 and out[2, 0] == 0.0
    assert out[4, 0] == pytest.approx(m1 * w / R**1.5, rel=1e-15)
    # snap: beta = w^2/R, S = -3 beta A (along x)
    assert out[6, 0] == pytest.approx(-3 * (w * w / R) * m1 * d / R**1.5, rel=1e-14)
    assert out[9, 0] == pytest.approx(-m1 / math.sqrt(R), rel=1e-15)


def test_self_pair_excluded_and_subset_consistent():
    ic = ni.plummer(300, 9)
    ap = ni.rng(10).normal(0, 1.0, (3, 300))
    full = oracle.evaluate(ic.m, ic.x, ic.v, ap, 0.0)
    assert np.all(np.isfinite(full))
    idx = ni.active_subset(300, 17, 3)
    sub = oracle.evaluate(ic.m, ic.x, ic.v, ap, 0.0, idx=idx)
    assert np.array_equal(sub, full[:, idx])


def test_single_body_has_no_force():
    out = oracle.evaluate(np.array([1.0]), np.zeros((3, 1)), np.zeros((3, 1)),
                          np.zeros((3, 1)), 0.0)
    assert np.array_equal(out, np.zeros((10, 1)))


# ------------------------------------------------------------------ crackle --
def _traj3(x, v, a, jk, t):
    n = x.shape[1]
    return [[mp.mpf(x[k, j]) + mp.mpf(v[k, j]) * t + mp.mpf(a[k, j]) * t * t / 2
             + mp.mpf(jk[k, j]) * t * t * t / 6 for k in range(3)] for j in range(n)]


@pytest.mark.parametrize("eps", [0.0, 3e-2])
def test_crackle_is_third_time_derivative(eps):
    """Crackle against the third time derivative of the softened acceleration
    along the cubic trajectories x(t) = x + v t + a t^2/2 + j t^3/6 (40 digits);
    a, j, s of the same call against the first two derivatives as well."""
    n = 6
    m, x, v, a = _random_system(n, 13)
    jk = ni.rng(14).normal(0, 2.0, (3, n))
    out = oracle.evaluate_crackle(m, x, v, a, jk, eps)
    for i in range(n):
        ref = [[], [], [], []]
        for k in range(3):
            def comp(t, k=k):
                return _mp_acc_direct(i, m, _traj3(x, v, a, jk, t), eps)[k]
            for d in range(4):
                ref[d].append(mp.diff(comp, 0, d))
        assert _rel(out[0:3, i], ref[0]) < 1e-14, ("acc", i)
        assert _rel(out[3:6, i], ref[1]) < 1e-13, ("jerk", i)
        assert _rel(out[6:9, i], ref[2]) < 1e-13, ("snap", i)
        assert _rel(out[9:12, i], ref[3]) < 1e-12, ("crackle", i)


def test_crackle_newton_third_law_and_consistency():
    n = 40
    m, x, v, a = _random_system(n, 15)
    jk = ni.rng(16).normal(0, 2.0, (3, n))
    out = oracle.evaluate_crackle(m, x, v, a, jk, 1e-3)
    scale = np.abs(m[None, :] * out[9:12]).sum()
    assert np.abs((m[None, :] * out[9:12]).sum(axis=1)).max() < 1e-13 * scale
    # the a, j, s, phi rows are the plain evaluation's (same arithmetic, same order)
    ref = oracle.evaluate(m, x, v, a, 1e-3)
    assert np.array_equal(out[0:9], ref[0:9]) and np.array_equal(out[12], ref[9])
    # crackle does not depend on the jerk of the body itself only through j_j - j_i:
    # a common jerk added to every body changes nothing
    out2 = oracle.evaluate_crackle(m, x, v, a, jk + np.array([[0.3], [-1.2], [0.7]]), 1e-3)
    assert np.allclose(out2[9:12], out[9:12], rtol=1e-12, atol=1e-12 * np.abs(out[9:12]).max())
