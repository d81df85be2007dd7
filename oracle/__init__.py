"""CPU oracle for the Hermite 6th-order block-step N-body method.

TEST INFRASTRUCTURE ONLY: the plain, slow FP64 reference that the GPU library is
checked against. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the GPU library never does, and this module imports
nothing from it. The arithmetic lives in ``nbody_oracle.c`` (built with
``gcc -O2 -ffp-contract=off -fopenmp``); this file only marshals NumPy arrays.

Parity status of each function (what pins it is in the tests under ``tests/``):
  evaluate   pinned  (finite differences, -grad phi, Newton's third law, closed forms)
  evaluate_crackle  pinned  (third time derivative by finite differences, Newton's law)
  predict    pinned  (exact on polynomial motion of degree <= 5)
  correct    pinned  (exact on polynomial accelerations; interpolation exact)
  timesteps  pinned  (block rules by hand cases; the step criterion and the start
             rule by the circular-orbit closed form: dt = eta / omega,
             eta_init / omega). Which criterion the method uses is a reading of
             the literature, since the paper prints none.
  active     pinned  (brute force by definition on small random cases)
  energy     pinned  (closed form two-body, Plummer virial values)
  integrate  pinned  (closed-form Kepler orbit, 6th-order convergence)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "libnbody_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc. Returns its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = configure(ctypes.CDLL(_LIB))
    return _lib


def configure(lib):
    """Declare the C signatures on a loaded oracle library (also used by the tests
    that load deliberately broken copies of it)."""
    lib.nbo_evaluate.argtypes = [_i64, _d, _d, _d, _d, _dbl, _i64, _i32p, _d, _int]
    lib.nbo_evaluate.restype = _int
    lib.nbo_evaluate_crackle.argtypes = [_i64, _d, _d, _d, _d, _d, _dbl, _i64, _i32p, _d, _int]
    lib.nbo_evaluate_crackle.restype = _int
    lib.nbo_predict.argtypes = [_i64, _i64p, _i64, _int, _d, _d, _d, _d, _d, _d, _d, _d, _d]
    lib.nbo_predict.restype = _int
    lib.nbo_correct.argtypes = [_i64, _i64, _i32p, _i64, _int, _d, _i64p, _d, _d, _d, _d,
                                _d, _d, _d, _d]
    lib.nbo_correct.restype = _int
    lib.nbo_timesteps.argtypes = [_i64, _i64, _i32p, _int, _i64p, _i32p, _d, _d, _d, _d,
                                  _d, _d, _dbl, _dbl, _int, _int]
    lib.nbo_timesteps.restype = _int
    lib.nbo_active.argtypes = [_i64, _i64p, _i32p, _int, _i32p, _i64p]
    lib.nbo_active.restype = _i64
    lib.nbo_energy.argtypes = [_i64, _d, _d, _d, _dbl, _d, _d, _int]
    lib.nbo_energy.restype = _int
    lib.nbo_integrate.argtypes = [_i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i64p, _i32p,
                                  _dbl, _dbl, _dbl, _int, _int, _i64, _i64, _i64p, _i64p,
                                  _d, _int, _int]
    lib.nbo_integrate.restype = _i64
    return lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_d)


def _p(a, ctype):
    return a.ctypes.data_as(ctype)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc == 1:
        raise OracleError(f"{what}: bad argument")
    if rc == 2:
        raise OracleError(f"{what}: numeric failure")
    if rc:
        raise OracleError(f"{what}: code {rc}")


def evaluate(m, xp, vp, ap, eps, idx=None, nthreads=None):
    """Acceleration, jerk, snap and potential of the bodies ``idx`` against all
    bodies. Returns out[10][n_act] (ax ay az jx jy jz sx sy sz phi)."""
    lib = _load()
    m, pm = _f64(m)
    n = m.shape[0]
    xp, px = _f64(np.reshape(xp, (3, n)))
    vp, pv = _f64(np.reshape(vp, (3, n)))
    ap, pa = _f64(np.reshape(ap, (3, n)))
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.zeros((10, idx.shape[0]))
    rc = lib.nbo_evaluate(n, pm, px, pv, pa, float(eps), idx.shape[0], _p(idx, _i32p),
                          _p(out, _d), nthreads or default_threads())
    _check(rc, "evaluate")
    return out


def evaluate_crackle(m, xp, vp, ap, jp, eps, idx=None, nthreads=None):
    """evaluate() plus crackle (third derivative of the acceleration) from the
    predicted jerks jp. Returns out[13][n_act] (a, j, s, crackle, phi)."""
    lib = _load()
    m, pm = _f64(m)
    n = m.shape[0]
    xp, px = _f64(np.reshape(xp, (3, n)))
    vp, pv = _f64(np.reshape(vp, (3, n)))
    ap, pa = _f64(np.reshape(ap, (3, n)))
    jp, pj = _f64(np.reshape(jp, (3, n)))
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.zeros((13, idx.shape[0]))
    rc = lib.nbo_evaluate_crackle(n, pm, px, pv, pa, pj, float(eps), idx.shape[0], _p(idx, _i32p),
                                  _p(out, _d), nthreads or default_threads())
    _check(rc, "evaluate_crackle")
    return out


def predict(tick, tick_next, dt_min_log2, x, v, a, j, s, c):
    lib = _load()
    tick = np.ascontiguousarray(tick, dtype=np.int64)
    n = tick.shape[0]
    arrs = [_f64(np.reshape(q, (3, n))) for q in (x, v, a, j, s, c)]
    xp, vp, ap = (np.zeros((3, n)) for _ in range(3))
    rc = lib.nbo_predict(n, _p(tick, _i64p), int(tick_next), int(dt_min_log2),
                         *[p for _, p in arrs], _p(xp, _d), _p(vp, _d), _p(ap, _d))
    _check(rc, "predict")
    return xp, vp, ap


@dataclass
class State:
    """Full integrator state, FP64 structure-of-arrays."""

    m: np.ndarray
    x: np.ndarray
    v: np.ndarray
    a: np.ndarray = None
    j: np.ndarray = None
    s: np.ndarray = None
    c: np.ndarray = None
    a4n: np.ndarray = None
    a5n: np.ndarray = None
    tick: np.ndarray = None
    level: np.ndarray = None
    records: dict = field(default_factory=dict)

    def __post_init__(self):
        n = self.m.shape[0]
        self.m = np.ascontiguousarray(self.m, dtype=np.float64)
        self.x = np.ascontiguousarray(np.reshape(self.x, (3, n)), dtype=np.float64).copy()
        self.v = np.ascontiguousarray(np.reshape(self.v, (3, n)), dtype=np.float64).copy()
        for name in ("a", "j", "s", "c"):
            val = getattr(self, name)
            val = np.zeros((3, n)) if val is None else np.array(val, dtype=np.float64).reshape(3, n)
            setattr(self, name, np.ascontiguousarray(val))
        for name in ("a4n", "a5n"):
            val = getattr(self, name)
            val = np.zeros(n) if val is None else np.array(val, dtype=np.float64)
            setattr(self, name, np.ascontiguousarray(val))
        self.tick = (np.zeros(n, dtype=np.int64) if self.tick is None
                     else np.array(self.tick, dtype=np.int64))
        self.level = (np.zeros(n, dtype=np.int32) if self.level is None
                      else np.array(self.level, dtype=np.int32))

    @property
    def n(self):
        return self.m.shape[0]

    def copy(self):
        return State(m=self.m.copy(), x=self.x.copy(), v=self.v.copy(), a=self.a.copy(),
                     j=self.j.copy(), s=self.s.copy(), c=self.c.copy(), a4n=self.a4n.copy(),
                     a5n=self.a5n.copy(), tick=self.tick.copy(), level=self.level.copy())


def correct(st: State, idx, tick_next, dt_min_log2, anew):
    """Corrector for the active bodies ``idx`` (in place on ``st``)."""
    lib = _load()
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    anew = np.ascontiguousarray(anew, dtype=np.float64)
    assert anew.shape == (10, idx.shape[0]) or anew.shape == (9, idx.shape[0])
    if anew.shape[0] == 9:
        anew = np.concatenate([anew, np.zeros((1, idx.shape[0]))])
    rc = lib.nbo_correct(st.n, idx.shape[0], _p(idx, _i32p), int(tick_next), int(dt_min_log2),
                         _p(anew, _d), _p(st.tick, _i64p), _p(st.x, _d), _p(st.v, _d),
                         _p(st.a, _d), _p(st.j, _d), _p(st.s, _d), _p(st.c, _d),
                         _p(st.a4n, _d), _p(st.a5n, _d))
    _check(rc, "correct")


def timesteps(st: State, idx, init, eta, eta_init, dt_max_log2, dt_min_log2, check=True):
    """New block levels for the active bodies ``idx`` (in place on ``st.level``).
    Returns the status code (0 ok, 2 numeric) when check is False."""
    lib = _load()
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    rc = lib.nbo_timesteps(st.n, idx.shape[0], _p(idx, _i32p), int(bool(init)),
                           _p(st.tick, _i64p), _p(st.level, _i32p), _p(st.a, _d),
                           _p(st.j, _d), _p(st.s, _d), _p(st.c, _d), _p(st.a4n, _d),
                           _p(st.a5n, _d), float(eta), float(eta_init), int(dt_max_log2),
                           int(dt_min_log2))
    if check:
        _check(rc, "timesteps")
    return rc


def active(tick, level, L):
    """(idx[int32], tick_next) of the next block step."""
    lib = _load()
    tick = np.ascontiguousarray(tick, dtype=np.int64)
    level = np.ascontiguousarray(level, dtype=np.int32)
    n = tick.shape[0]
    idx = np.zeros(n, dtype=np.int32)
    tn = ctypes.c_int64(0)
    cnt = lib.nbo_active(n, _p(tick, _i64p), _p(level, _i32p), int(L), _p(idx, _i32p),
                         ctypes.byref(tn))
    if cnt < 0:
        raise OracleError("active: bad argument")
    return idx[:cnt].copy(), int(tn.value)


def energy(m, x, v, eps, nthreads=None):
    """(E_kin, E_pot) with Plummer softening eps."""
    lib = _load()
    m, pm = _f64(m)
    n = m.shape[0]
    x, px = _f64(np.reshape(x, (3, n)))
    v, pv = _f64(np.reshape(v, (3, n)))
    ek, ep = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib.nbo_energy(n, pm, px, pv, float(eps), ctypes.byref(ek), ctypes.byref(ep),
                        nthreads or default_threads())
    _check(rc, "energy")
    return ek.value, ep.value


def integrate(st: State, eps, eta, eta_init, dt_max_log2, dt_min_log2, tick_end,
              max_steps=1 << 20, nthreads=None, start_crackle=False):
    """Block-step integration of a synchronised state to tick_end (in place).
    start_crackle: start from the evaluated crackle instead of c = 0.
    Returns (steps, step_tick[steps], step_nact[steps], interactions)."""
    lib = _load()
    stt = np.zeros(max_steps, dtype=np.int64)
    sna = np.zeros(max_steps, dtype=np.int64)
    inter = ctypes.c_double(0)
    steps = lib.nbo_integrate(st.n, _p(st.m, _d), _p(st.x, _d), _p(st.v, _d), _p(st.a, _d),
                              _p(st.j, _d), _p(st.s, _d), _p(st.c, _d), _p(st.a4n, _d),
                              _p(st.a5n, _d), _p(st.tick, _i64p), _p(st.level, _i32p),
                              float(eps), float(eta), float(eta_init), int(dt_max_log2),
                              int(dt_min_log2), int(tick_end), max_steps, _p(stt, _i64p),
                              _p(sna, _i64p), ctypes.byref(inter), int(bool(start_crackle)),
                              nthreads or default_threads())
    if steps < 0:
        _check(-steps, "integrate")
    k = min(steps, max_steps)
    return int(steps), stt[:k].copy(), sna[:k].copy(), inter.value
