"""Checks of the seeded synthetic inputs (Plummer spheres, Kroupa masses,
parabolic pairs) against closed-form properties of those distributions."""
import math

import numpy as np

import nbody_inputs as ni
import oracle


def test_plummer_is_seeded_and_centred():
    a = ni.plummer(2000, 17)
    b = ni.plummer(2000, 17)
    c = ni.plummer(2000, 18)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert not np.array_equal(a.x, c.x)
    assert abs(a.m.sum() - 1.0) < 1e-14
    assert np.abs(a.x @ a.m).max() < 1e-15 and np.abs(a.v @ a.m).max() < 1e-15


def test_plummer_henon_units():
    ic = ni.plummer(4096, 1)
    ek, ep = oracle.energy(ic.m, ic.x, ic.v, 0.0)
    # Henon units: E = -1/4, virial ratio E_kin/|E_pot| = 1/2 (sampling noise ~ N^-1/2)
    assert abs((ek + ep) + 0.25) < 0.02
    assert abs(ek / -ep - 0.5) < 0.03
    # half-mass radius of a Plummer sphere in these units: 1.305 * 3 pi / 16 = 0.7686
    r = np.linalg.norm(ic.x, axis=0)
    assert abs(np.median(r) - 1.30476 * 3 * math.pi / 16) < 0.03


def test_kroupa_fraction_below_break():
    n = 200000
    m = ni.kroupa_masses(n, 3)
    scale = 1.0 / m.min() * 0.08   # undo the normalisation to total mass 1
    raw = m * scale
    assert raw.min() >= 0.08 * (1 - 1e-12) and raw.max() <= 100.0 * (1 + 1e-12)
    p = ni.kroupa_fraction_below(0.5)
    frac = np.mean(raw < 0.5)
    sigma = math.sqrt(p * (1 - p) / n)
    assert abs(frac - p) < 5 * sigma
    p1 = ni.kroupa_fraction_below(2.0)
    assert abs(np.mean(raw < 2.0) - p1) < 5 * math.sqrt(p1 * (1 - p1) / n)
    assert abs(m.sum() - 1.0) < 1e-12


def test_parabolic_pair_orbit():
    ic = ni.parabolic_pair(4000, 5)
    h = 2000
    m1, m2 = ic.m[:h], ic.m[h:]
    assert abs(m1.sum() - 0.5) < 1e-14 and abs(m2.sum() - 0.5) < 1e-14
    c1, c2 = ic.x[:, :h] @ m1 / 0.5, ic.x[:, h:] @ m2 / 0.5
    u1, u2 = ic.v[:, :h] @ m1 / 0.5, ic.v[:, h:] @ m2 / 0.5
    d = c2 - c1
    w = u2 - u1
    assert abs(np.linalg.norm(d) - 10.0) < 1e-12
    # zero two-body orbital energy (parabolic) with total mass 1, reduced mass 1/4
    e_orb = 0.5 * 0.25 * (w @ w) - 0.25 / np.linalg.norm(d)
    assert abs(e_orb) < 1e-14
    # pericentre from the angular momentum: q = |d x w|^2 / (2 G M)
    lz = np.cross(d, w)
    assert abs((lz @ lz) / 2.0 - 1.0) < 1e-12


def test_active_subset():
    idx = ni.active_subset(65536, 1024, 22)
    assert idx.dtype == np.int32 and idx.shape == (1024,)
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < 65536
    assert np.array_equal(ni.active_subset(10, 10, 1), np.arange(10))
