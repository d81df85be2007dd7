"""Seeded synthetic inputs for the Hermite-6 N-body path.

This module only draws initial conditions and index sets. It holds none of the
integrator's arithmetic (no forces, no predictor, no corrector, no time steps),
so both the CPU oracle's tests and the GPU path can take their inputs from it.

Every generator takes an explicit seed and uses NumPy's PCG64 bit generator, so a
(seed, size) pair always yields the same arrays. Arrays are float64, positions and
velocities as structure-of-arrays ``[3][n]`` (component-major), masses ``[n]``.

Units are Henon units (G = 1, total mass 1, total energy close to -1/4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "ICs",
    "rng",
    "plummer",
    "kroupa_masses",
    "kroupa_fraction_below",
    "parabolic_pair",
    "log_uniform_n",
    "active_subset",
    "plummer_mean_field_acc",
    "block_state",
]

# Mass fraction at which the Plummer radius draw is truncated (the tail beyond it
# holds 0.1 % of the mass and would put a few bodies at very large radii).
PLUMMER_MASS_CUT = 0.999
# Kroupa (2001) broken power law used for the mass function.
KROUPA_M_LO = 0.08
KROUPA_M_BREAK = 0.5
KROUPA_M_HI = 100.0
KROUPA_ALPHA_LO = 1.3
KROUPA_ALPHA_HI = 2.3


@dataclass
class ICs:
    """Initial conditions: masses m[n], positions x[3][n], velocities v[3][n]."""

    m: np.ndarray
    x: np.ndarray
    v: np.ndarray

    @property
    def n(self) -> int:
        return int(self.m.shape[0])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(g: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Vectors of length r with uniformly distributed directions, shape [3][n]."""
    n = r.shape[0]
    cz = 1.0 - 2.0 * g.random(n)
    ph = 2.0 * math.pi * g.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([r * sz * np.cos(ph), r * sz * np.sin(ph), r * cz])


def plummer(n: int, seed: int, masses: np.ndarray | None = None) -> ICs:
    """Plummer sphere in Henon units (Aarseth, Henon & Wielen 1974 sampling).

    Radius from the inverted cumulative mass, r = (X^(-2/3) - 1)^(-1/2), with X
    uniform below the mass cut; isotropic directions; speed q * v_esc with
    v_esc = sqrt(2) (1 + r^2)^(-1/4) and q drawn by rejection from
    g(q) = q^2 (1 - q^2)^(7/2). Lengths are scaled by 3 pi / 16 and speeds by
    sqrt(16 / (3 pi)) so that the virial radius is 1, then the centre of mass is
    moved to rest at the origin. Equal masses 1/n unless ``masses`` is given.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    g = rng(seed)
    X = g.random(n) * PLUMMER_MASS_CUT
    X = np.maximum(X, 1e-300)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(g, r)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        q_try = g.random(todo.size)
        y = 0.1 * g.random(todo.size)
        ok = y < q_try * q_try * (1.0 - q_try * q_try) ** 3.5
        q[todo[ok]] = q_try[ok]
        todo = todo[~ok]
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = _isotropic(g, speed)
    pos *= 3.0 * math.pi / 16.0
    vel *= math.sqrt(16.0 / (3.0 * math.pi))
    if masses is None:
        m = np.full(n, 1.0 / n)
    else:
        m = np.asarray(masses, dtype=np.float64).copy()
        if m.shape != (n,):
            raise ValueError("masses must have shape (n,)")
    mt = m.sum()
    pos -= (pos @ m / mt)[:, None]
    vel -= (vel @ m / mt)[:, None]
    return ICs(m=m, x=np.ascontiguousarray(pos), v=np.ascontiguousarray(vel))


def _kroupa_segments():
    # Unnormalised density k1 m^-1.3 below the break and k2 m^-2.3 above it,
    # continuous at the break: k2 = k1 * m_break.
    k1 = 1.0
    k2 = k1 * KROUPA_M_BREAK
    a1 = 1.0 - KROUPA_ALPHA_LO  # -0.3 ... exponent of the integral
    a2 = 1.0 - KROUPA_ALPHA_HI  # -1.3
    w1 = k1 * (KROUPA_M_BREAK ** a1 - KROUPA_M_LO ** a1) / a1
    w2 = k2 * (KROUPA_M_HI ** a2 - KROUPA_M_BREAK ** a2) / a2
    return a1, a2, w1, w2


def kroupa_fraction_below(m: float) -> float:
    """Closed-form fraction of stars (by number) with mass below m."""
    a1, a2, w1, w2 = _kroupa_segments()
    m = min(max(m, KROUPA_M_LO), KROUPA_M_HI)
    if m <= KROUPA_M_BREAK:
        return (m ** a1 - KROUPA_M_LO ** a1) / a1 / (w1 + w2)
    k2 = KROUPA_M_BREAK
    return (w1 + k2 * (m ** a2 - KROUPA_M_BREAK ** a2) / a2) / (w1 + w2)


def kroupa_masses(n: int, seed: int) -> np.ndarray:
    """n masses from the Kroupa (2001) IMF on [0.08, 100] by piecewise inverse CDF,
    normalised to total mass 1."""
    a1, a2, w1, w2 = _kroupa_segments()
    g = rng(seed)
    u = g.random(n) * (w1 + w2)
    m = np.empty(n)
    lo = u < w1
    # segment 1: u = (m^a1 - mlo^a1)/a1
    m[lo] = (KROUPA_M_LO ** a1 + a1 * u[lo]) ** (1.0 / a1)
    # segment 2: u - w1 = k2 (m^a2 - mb^a2)/a2 with k2 = m_break
    k2 = KROUPA_M_BREAK
    m[~lo] = (KROUPA_M_BREAK ** a2 + a2 * (u[~lo] - w1) / k2) ** (1.0 / a2)
    np.clip(m, KROUPA_M_LO, KROUPA_M_HI, out=m)
    return m / m.sum()


def parabolic_pair(n: int, seed: int, separation: float = 10.0,
                   pericentre: float = 1.0) -> ICs:
    """Two Plummer spheres of n/2 bodies each on a parabolic orbit.

    Each sphere is drawn in Henon units, then its masses are halved and its speeds
    scaled by sqrt(1/2) so it stays in virial equilibrium at mass 1/2. The centres
    start ``separation`` apart on the x axis, approaching, with the relative speed
    of a zero-energy two-body orbit of total mass 1 and the given pericentre.
    """
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    g = rng(seed)
    s1, s2 = (int(s) for s in g.integers(0, 2**31 - 1, size=2))
    a = plummer(n // 2, s1)
    b = plummer(n // 2, s2)
    d = float(separation)
    v2 = 2.0 / d                       # parabolic: v^2 = 2 G M / d with M = 1
    vt = math.sqrt(2.0 * pericentre) / d   # angular momentum sqrt(2 G M q) / d
    vr = math.sqrt(max(0.0, v2 - vt * vt))
    rel_x = np.array([d, 0.0, 0.0])
    rel_v = np.array([-vr, vt, 0.0])
    m = np.concatenate([a.m * 0.5, b.m * 0.5])
    x = np.concatenate([a.x - 0.5 * rel_x[:, None], b.x + 0.5 * rel_x[:, None]], axis=1)
    sv = math.sqrt(0.5)
    v = np.concatenate([a.v * sv - 0.5 * rel_v[:, None], b.v * sv + 0.5 * rel_v[:, None]],
                       axis=1)
    return ICs(m=m, x=np.ascontiguousarray(x), v=np.ascontiguousarray(v))


def log_uniform_n(g: np.random.Generator, lo: int, hi: int, even: bool = False) -> int:
    n = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    n = min(max(n, lo), hi)
    if even and n % 2:
        n += 1 if n < hi else -1
    return n


def active_subset(n: int, n_act: int, seed: int) -> np.ndarray:
    """Sorted random subset of n_act distinct indices in [0, n), as int32.
    n_act == n returns every index."""
    if not 0 <= n_act <= n:
        raise ValueError("need 0 <= n_act <= n")
    if n_act == n:
        return np.arange(n, dtype=np.int32)
    g = rng(seed)
    return np.sort(g.choice(n, size=n_act, replace=False)).astype(np.int32)


def plummer_mean_field_acc(x: np.ndarray, mass: float = 1.0) -> np.ndarray:
    """Acceleration of the smooth Plummer potential at positions x[3][n], in the
    Henon-unit scaling used by ``plummer`` (scale radius 3 pi / 16):
    a = -M x / (|x|^2 + b^2)^(3/2). A closed-form stand-in, with the right
    magnitudes and directions, for the predicted accelerations of a Plummer sphere."""
    b = 3.0 * math.pi / 16.0
    r2 = (x * x).sum(axis=0) + b * b
    return -mass * x / r2 ** 1.5


def block_state(n: int, seed: int, L: int, max_level: int = 10, span: int = 64):
    """A random, valid block-time-step bookkeeping state: levels in [0, max_level]
    and each body's tick a multiple of its own step 2^(L - level)."""
    g = rng(seed)
    level = g.integers(0, max_level + 1, n).astype(np.int32)
    mult = g.integers(0, span, n).astype(np.int64)
    tick = mult * (np.int64(1) << (L - level.astype(np.int64)))
    return tick, level


def serving_requests(count: int, rate: float, seed: int, lo: int = 1024, hi: int = 65536,
                     pair_fraction: float = 0.1, separation: float = 10.0):
    """A seeded stream of integration requests: Poisson arrivals at `rate` per second
    (exponential gaps, the first at 0) of single Plummer clusters with N log-uniform in
    [lo, hi], a `pair_fraction` of them replaced by two equal Plummer spheres of N/2
    each on a parabolic orbit `separation` apart. Returns a list of dicts
    {arrival, kind, n, ic}."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        if k:
            t += float(g.exponential(1.0 / rate))
        pair = bool(g.random() < pair_fraction)
        n = log_uniform_n(g, lo, hi, even=pair)
        s = int(g.integers(0, 2**31 - 1))
        ic = parabolic_pair(n, s, separation=separation) if pair else plummer(n, s)
        out.append({"arrival": t, "kind": "pair" if pair else "cluster", "n": n, "ic": ic})
    return out
