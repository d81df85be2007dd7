"""MI355X-native Hermite 6th-order block-step direct N-body evaluation path.

Python binding over the C ABI of libnbody.so (include/nbody.h). PyTorch supplies
device memory (the workspace and the caller's arrays) and the stream; every step
of the method runs in the library's HIP kernels. There is no CPU fallback: on a
machine without a GPU or without the built library, creating a Simulation raises.

Typical use (time in ticks of 2^dt_min_log2):

    sim = Simulation(n, eps=1e-4)
    sim.set_state(m, x, v)          # torch float64 tensors on the GPU, x, v [3][n]
    sim.start()
    while True:
        n_act, tick = sim.step(tick_end)
        if n_act == 0: break
"""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import NB_FLAG_START_CRACKLE, NB_FP64, NB_SPLIT, NBodyError

__all__ = ["Simulation", "Batch", "NBodyError", "NB_FP64", "NB_SPLIT", "NB_FLAG_START_CRACKLE",
           "workspace_bytes", "evaluate_static",
           "batch_workspace_bytes"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def workspace_bytes(n, precision=NB_FP64, partial_slots=0, eps=1e-4, eta=0.45, eta_init=0.01,
                    dt_max_log2=-3, dt_min_log2=-40):
    lib = _abi.load()
    p = _abi.Params(n=n, eps=eps, eta=eta, eta_init=eta_init, dt_max_log2=dt_max_log2,
                    dt_min_log2=dt_min_log2, precision=precision, flags=0,
                    partial_slots=partial_slots, stream=None)
    out = ctypes.c_size_t(0)
    rc = lib.nb_workspace_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise NBodyError(rc, "invalid parameters")
    return out.value


class Simulation:
    """One N-body system resident on one GPU."""

    def __init__(self, n, eps=1e-4, eta=0.45, eta_init=0.01, dt_max_log2=-3, dt_min_log2=-40,
                 precision=NB_FP64, partial_slots=0, device=None, stream=None, flags=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1812_00367_amd needs a ROCm GPU; none is visible")
        self._lib = _abi.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n = int(n)
        self.eps = float(eps)
        self.dt_min_log2 = int(dt_min_log2)
        self.dt_max_log2 = int(dt_max_log2)
        self.precision = int(precision)
        self._params = _abi.Params(n=self.n, eps=self.eps, eta=float(eta),
                                   eta_init=float(eta_init), dt_max_log2=self.dt_max_log2,
                                   dt_min_log2=self.dt_min_log2, precision=self.precision,
                                   flags=int(flags), partial_slots=int(partial_slots),
                                   stream=ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = ctypes.c_size_t(0)
        rc = self._lib.nb_workspace_bytes(ctypes.byref(self._params), ctypes.byref(nbytes))
        if rc:
            raise NBodyError(rc, "invalid parameters")
        self.workspace_bytes = nbytes.value
        with torch.cuda.device(self.device):
            raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self._ws = raw[off:off + nbytes.value]
        ctx = ctypes.c_void_p(0)
        rc = self._lib.nb_create(ctypes.byref(self._params), _ptr(self._ws), nbytes.value,
                                 ctypes.byref(ctx))
        if rc:
            raise NBodyError(rc, "nb_create failed")
        self._ctx = ctx
        self._idx = torch.empty(self.n, dtype=torch.int32, device=self.device)

    # ----------------------------------------------------------------- helpers --
    @property
    def tick_size(self):
        return 2.0 ** self.dt_min_log2

    def ticks(self, t):
        """Ticks of time t (must be a whole number of ticks)."""
        k = t / self.tick_size
        if k != int(k):
            raise ValueError("time is not a whole number of ticks")
        return int(k)

    def _check(self, rc):
        if rc:
            msg = self._lib.nb_last_error(self._ctx).decode()
            raise NBodyError(rc, msg)

    def _dev(self, t, dtype, shape):
        torch = _torch()
        if t is None:
            return None
        t = torch.as_tensor(t, dtype=dtype, device=self.device).reshape(shape).contiguous()
        return t

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.nb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------------- state --
    def set_state(self, m, x, v, tick0=0, a=None, j=None, s=None, c=None, a4n=None, a5n=None,
                  tick=None, level=None):
        torch = _torch()
        n = self.n
        f = torch.float64
        keep = dict(m=self._dev(m, f, (n,)), x=self._dev(x, f, (3, n)), v=self._dev(v, f, (3, n)),
                    a=self._dev(a, f, (3, n)), j=self._dev(j, f, (3, n)),
                    s=self._dev(s, f, (3, n)), c=self._dev(c, f, (3, n)),
                    a4n=self._dev(a4n, f, (n,)), a5n=self._dev(a5n, f, (n,)),
                    tick=self._dev(tick, torch.int64, (n,)),
                    level=self._dev(level, torch.int32, (n,)))
        view = _abi.State(**{k: (v_.data_ptr() if v_ is not None else None)
                             for k, v_ in keep.items()})
        self._check(self._lib.nb_set_state(self._ctx, ctypes.byref(view), int(tick0)))
        # the copies are ordered on the stream; keeping the sources referenced until the
        # next call is enough because torch reuses freed memory in stream order
        self._keepalive = keep

    def set_times(self, tick, level):
        """Reload every body's time (ticks) and step level; the physical state is kept."""
        torch = _torch()
        tick = self._dev(tick, torch.int64, (self.n,))
        level = self._dev(level, torch.int32, (self.n,))
        self._check(self._lib.nb_set_times(self._ctx, _ptr(tick), _ptr(level)))
        self._times_keep = (tick, level)

    def get_state(self):
        torch = _torch()
        n = self.n
        f = torch.float64
        out = dict(m=torch.empty(n, dtype=f, device=self.device))
        for k in ("x", "v", "a", "j", "s", "c"):
            out[k] = torch.empty((3, n), dtype=f, device=self.device)
        for k in ("a4n", "a5n", "phi"):
            out[k] = torch.empty(n, dtype=f, device=self.device)
        out["tick"] = torch.empty(n, dtype=torch.int64, device=self.device)
        out["level"] = torch.empty(n, dtype=torch.int32, device=self.device)
        view = _abi.State(**{k: v_.data_ptr() for k, v_ in out.items()})
        self._check(self._lib.nb_get_state(self._ctx, ctypes.byref(view)))
        return out

    # ---------------------------------------------------------------- the path --
    def start(self):
        self._check(self._lib.nb_start(self._ctx))

    def active(self, out=None):
        """(idx tensor[int32, n_act] (view of out), tick_next)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        na, tn = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self._lib.nb_active(self._ctx, _ptr(out), ctypes.byref(na), ctypes.byref(tn)))
        return out[:na.value], tn.value

    def predict(self, tick):
        self._check(self._lib.nb_predict(self._ctx, int(tick)))

    def get_predicted(self):
        torch = _torch()
        xp, vp, ap = (torch.empty((3, self.n), dtype=torch.float64, device=self.device)
                      for _ in range(3))
        self._check(self._lib.nb_get_predicted(self._ctx, _ptr(xp), _ptr(vp), _ptr(ap)))
        return xp, vp, ap

    def evaluate(self, idx, out=None):
        """a, j, s, phi of the bodies idx: returns out[10][n_act] (float64)."""
        torch = _torch()
        idx = self._dev(idx, torch.int32, (-1,))
        n_act = idx.shape[0]
        if out is None:
            out = torch.empty((10, n_act), dtype=torch.float64, device=self.device)
        self._check(self._lib.nb_evaluate(self._ctx, _ptr(idx), n_act, _ptr(out)))
        self._eval_idx = idx
        return out

    def evaluate_into(self, idx, out):
        """nb_evaluate with caller tensors as they are (no conversion; for timing)."""
        self._check(self._lib.nb_evaluate(self._ctx, _ptr(idx), idx.shape[0], _ptr(out)))

    def set_evaluation(self, idx, values):
        """Provide the evaluation values[10][n_act] of idx for the next correct()."""
        torch = _torch()
        idx = self._dev(idx, torch.int32, (-1,))
        values = self._dev(values, torch.float64, (10, idx.shape[0]))
        self._check(self._lib.nb_set_evaluation(self._ctx, _ptr(idx), idx.shape[0], _ptr(values)))
        self._eval_idx = idx
        self._eval_in = values

    def evaluate_crackle(self, idx, out=None):
        """a, j, s, crackle, phi of the bodies idx: returns out[13][n_act] (float64)."""
        torch = _torch()
        idx = self._dev(idx, torch.int32, (-1,))
        n_act = idx.shape[0]
        if out is None:
            out = torch.empty((13, n_act), dtype=torch.float64, device=self.device)
        self._check(self._lib.nb_evaluate_crackle(self._ctx, _ptr(idx), n_act, _ptr(out)))
        self._crk_idx = idx
        return out

    def eval_config(self, cfg=None, n_act=None):
        """Force (ipl, waves, tile, splits) or restore the default (cfg None); returns the
        shape {ipl, waves, tile, jchunk, splits, iblocks, fused} used for n_act bodies."""
        arr = (ctypes.c_int32 * 4)(*(cfg if cfg is not None else (0, 0, 0, 0)))
        shape = (ctypes.c_int32 * 7)()
        self._check(self._lib.nb_eval_config(self._ctx, arr, int(n_act or self.n), shape))
        return dict(zip(("ipl", "waves", "tile", "jchunk", "splits", "iblocks", "fused"),
                        list(shape)))

    def eval_table(self, rows=None):
        """Install a launch-shape table: rows of (n_act_max, ipl, waves, tile, target_waves);
        None restores the built-in table."""
        rows = list(rows or [])
        flat = (ctypes.c_int32 * max(1, 5 * len(rows)))(*[int(v) for r in rows for v in r])
        self._check(self._lib.nb_eval_table(self._ctx, flat, len(rows)))

    def correct(self, idx, tick):
        torch = _torch()
        idx = self._dev(idx, torch.int32, (-1,))
        if getattr(self, "_eval_idx", None) is not None and idx.data_ptr() != self._eval_idx.data_ptr():
            if torch.equal(idx, self._eval_idx):
                idx = self._eval_idx
        self._check(self._lib.nb_correct(self._ctx, _ptr(idx), idx.shape[0], int(tick)))

    def timesteps(self, idx, init=False):
        torch = _torch()
        idx = self._dev(idx, torch.int32, (-1,))
        self._check(self._lib.nb_timesteps(self._ctx, _ptr(idx), idx.shape[0], int(bool(init))))
        self._ts_idx = idx

    def step(self, tick_limit=-1):
        """One block step; returns (n_act, tick_next). n_act == 0: next time beyond limit."""
        na, tn = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self._lib.nb_step(self._ctx, int(tick_limit), ctypes.byref(na), ctypes.byref(tn)))
        return na.value, tn.value

    def energy(self, tick):
        ek, ep = ctypes.c_double(0), ctypes.c_double(0)
        self._check(self._lib.nb_energy(self._ctx, int(tick), ctypes.byref(ek), ctypes.byref(ep)))
        return ek.value, ep.value

    def integrate(self, tick_end, record=None):
        """Block steps until every body reaches tick_end. Returns (steps, [(tick, n_act)], interactions)."""
        steps, log, inter = 0, [], 0
        while True:
            na, tn = self.step(tick_end)
            if na == 0:
                break
            steps += 1
            inter += na * self.n
            log.append((tn, na))
            if record is not None:
                record(tn, na)
        return steps, log, inter


def evaluate_static(m, xp, vp, ap, eps, idx, out=None, stream=None):
    """nb_evaluate_static: a, j, s, phi of the bodies idx against all n predicted bodies
    (m[n], xp / vp / ap [3][n], float64 tensors on the GPU) without a context or
    workspace; the library's fixed device array holds its intermediates. Returns
    out[10][n_act]. Enqueued on `stream` (torch's current stream by default)."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1812_00367_amd needs a ROCm GPU; none is visible")
    lib = _abi.load()
    n = int(m.shape[0])
    idx = torch.as_tensor(idx, dtype=torch.int32, device=m.device).reshape(-1).contiguous()
    n_act = int(idx.shape[0])
    if out is None:
        out = torch.empty((10, n_act), dtype=torch.float64, device=m.device)
    if stream is None:
        stream = torch.cuda.current_stream(m.device)
    rc = lib.nb_evaluate_static(n, _ptr(m), _ptr(xp), _ptr(vp), _ptr(ap), float(eps), _ptr(idx),
                                n_act, _ptr(out), ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise NBodyError(rc, "nb_evaluate_static failed (arguments, or more than "
                             f"{_abi.NB_STATIC_SCRATCH_BYTES} bytes of device memory needed)")
    return out


from .batch import Batch, batch_workspace_bytes  # noqa: E402
