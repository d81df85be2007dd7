"""Python binding of the batch entry points (nb_batch_* in include/nbody.h).

Many independent N-body systems ("jobs") live in one pool on one GPU and advance
together: each Batch.step() gives every job its own next block step, with one
kernel launch per stage for all jobs. Argument marshalling only; no CPU fallback.
"""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import NB_ERR_SPACE, NB_FP64, NBodyError


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def batch_workspace_bytes(capacity, max_jobs, precision=NB_FP64, eps=1e-4, eta=0.45,
                          eta_init=0.01, dt_max_log2=-3, dt_min_log2=-40, jchunk=0,
                          items_per_job=0, partial_slots=0, chunk_tile=0, chunk_wide=0,
                          chunk_direct=0):
    lib = _abi.load()
    p = _abi.BatchParams(capacity=capacity, max_jobs=max_jobs, precision=precision, eps=eps,
                         eta=eta, eta_init=eta_init, dt_max_log2=dt_max_log2,
                         dt_min_log2=dt_min_log2, jchunk=jchunk, items_per_job=items_per_job,
                         chunk_tile=chunk_tile, chunk_wide=chunk_wide, chunk_direct=chunk_direct,
                         partial_slots=partial_slots, stream=None)
    out = ctypes.c_size_t(0)
    rc = lib.nb_batch_workspace_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise NBodyError(rc, "invalid batch parameters")
    return out.value


class Batch:
    """A pool of `capacity` bodies shared by at most `max_jobs` jobs on one GPU.

    jchunk, items_per_job and chunk_tile / chunk_wide / chunk_direct set the work
    split (the fields of nb_batch_params; 0 = the library defaults)."""

    def __init__(self, capacity, max_jobs, eps=1e-4, eta=0.45, eta_init=0.01, dt_max_log2=-3,
                 dt_min_log2=-40, precision=NB_FP64, jchunk=0, items_per_job=0, partial_slots=0,
                 device=None, stream=None, chunk_tile=0, chunk_wide=0, chunk_direct=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1812_00367_amd needs a ROCm GPU; none is visible")
        self._lib = _abi.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        # a stream of its own by default (default priority): a multi-step call replays a
        # captured HIP graph of one batch step, and the null stream cannot be captured
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.capacity = int(capacity)
        self.max_jobs = int(max_jobs)
        self.dt_min_log2 = int(dt_min_log2)
        self.dt_max_log2 = int(dt_max_log2)
        self.precision = int(precision)
        self._params = _abi.BatchParams(
            capacity=self.capacity, max_jobs=self.max_jobs, precision=self.precision,
            eps=float(eps), eta=float(eta), eta_init=float(eta_init),
            dt_max_log2=self.dt_max_log2, dt_min_log2=self.dt_min_log2, jchunk=int(jchunk),
            items_per_job=int(items_per_job), partial_slots=int(partial_slots),
            chunk_tile=int(chunk_tile), chunk_wide=int(chunk_wide), chunk_direct=int(chunk_direct),
            stream=ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = ctypes.c_size_t(0)
        rc = self._lib.nb_batch_workspace_bytes(ctypes.byref(self._params), ctypes.byref(nbytes))
        if rc:
            raise NBodyError(rc, "invalid batch parameters")
        self.workspace_bytes = nbytes.value
        raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self._ws = raw[off:off + nbytes.value]
        ctx = ctypes.c_void_p(0)
        self._order()
        rc = self._lib.nb_batch_create(ctypes.byref(self._params), _ptr(self._ws), nbytes.value,
                                       ctypes.byref(ctx))
        if rc:
            raise NBodyError(rc, "nb_batch_create failed")
        self._ctx = ctx
        J = self.max_jobs
        self._nact = (ctypes.c_int64 * J)()
        self._tnext = (ctypes.c_int64 * J)()
        self._err = (ctypes.c_int32 * J)()
        self.jobs = {}  # job id -> n

    def _check(self, rc):
        if rc:
            raise NBodyError(rc, self._lib.nb_batch_last_error(self._ctx).decode())

    def _order(self):
        """The batch's stream waits for torch's current stream (tensors the call reads
        or writes were made there); every call waits for its own stream on return."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.nb_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, dtype, shape):
        torch = _torch()
        if t is None:
            return None
        return torch.as_tensor(t, dtype=dtype, device=self.device).reshape(shape).contiguous()

    # ------------------------------------------------------------------- jobs --
    def add(self, m, x, v, tick_end, tick0=0, a=None, j=None, s=None, c=None, a4n=None, a5n=None,
            tick=None, level=None):
        """Admit a job; returns its id, or None when the pool has no room (NB_ERR_SPACE).
        Without `tick` the job starts synchronised at tick0 with the Hermite start-up."""
        torch = _torch()
        f = torch.float64
        m = self._dev(m, f, (-1,))
        n = m.shape[0]
        keep = dict(m=m, x=self._dev(x, f, (3, n)), v=self._dev(v, f, (3, n)),
                    a=self._dev(a, f, (3, n)), j=self._dev(j, f, (3, n)),
                    s=self._dev(s, f, (3, n)), c=self._dev(c, f, (3, n)),
                    a4n=self._dev(a4n, f, (n,)), a5n=self._dev(a5n, f, (n,)),
                    tick=self._dev(tick, torch.int64, (n,)),
                    level=self._dev(level, torch.int32, (n,)))
        view = _abi.State(**{k: (t.data_ptr() if t is not None else None) for k, t in keep.items()})
        job = ctypes.c_int32(-1)
        self._order()
        rc = self._lib.nb_batch_add(self._ctx, n, ctypes.byref(view), int(tick0), int(tick_end),
                                    ctypes.byref(job))
        if rc == NB_ERR_SPACE:
            return None
        self._check(rc)
        self.jobs[job.value] = n
        return job.value

    def remove(self, job):
        self._check(self._lib.nb_batch_remove(self._ctx, int(job)))
        self.jobs.pop(int(job), None)

    def info(self, job):
        off, n = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self._lib.nb_batch_info(self._ctx, int(job), ctypes.byref(off), ctypes.byref(n)))
        return off.value, n.value

    # ------------------------------------------------------------------- steps --
    def step(self):
        """One block step of every live job. Returns (n_act, tick_next, err, interactions):
        per-job lists indexed by job id, and the total n_act x n of the step."""
        inter = ctypes.c_int64(0)
        self._check(self._lib.nb_batch_step(self._ctx, self._nact, self._tnext, self._err,
                                            ctypes.byref(inter)))
        return list(self._nact), list(self._tnext), list(self._err), inter.value

    def run_steps(self, steps):
        """`steps` batch steps with no host wait in between (nb_batch_run). Returns
        (n_act, tick_next, err, interactions, steps_taken); the per-job lists describe
        the last step."""
        inter, taken = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self._lib.nb_batch_run(self._ctx, int(steps), self._nact, self._tnext, self._err,
                                           ctypes.byref(inter), ctypes.byref(taken)))
        return list(self._nact), list(self._tnext), list(self._err), inter.value, taken.value

    def run(self, max_steps=1 << 40, record=None):
        """Batch steps until no job advances. Returns (batch steps, interactions,
        {job: [(tick_next, n_act), ...]})."""
        logs = {k: [] for k in self.jobs}
        steps = inter = 0
        while steps < max_steps:
            nact, tnext, err, it = self.step()
            moved = False
            for k in self.jobs:
                if nact[k] > 0:
                    logs[k].append((tnext[k], nact[k]))
                    moved = True
            if not moved:
                break
            steps += 1
            inter += it
            if record is not None:
                record(nact, tnext, err)
        return steps, inter, logs

    def get(self, job):
        torch = _torch()
        n = self.info(job)[1]
        f = torch.float64
        out = dict(m=torch.empty(n, dtype=f, device=self.device))
        for k in ("x", "v", "a", "j", "s", "c"):
            out[k] = torch.empty((3, n), dtype=f, device=self.device)
        for k in ("a4n", "a5n", "phi"):
            out[k] = torch.empty(n, dtype=f, device=self.device)
        out["tick"] = torch.empty(n, dtype=torch.int64, device=self.device)
        out["level"] = torch.empty(n, dtype=torch.int32, device=self.device)
        view = _abi.State(**{k: t.data_ptr() for k, t in out.items()})
        self._order()
        self._check(self._lib.nb_batch_get(self._ctx, int(job), ctypes.byref(view)))
        return out

    def energy(self, job, tick):
        ek, ep = ctypes.c_double(0), ctypes.c_double(0)
        self._check(self._lib.nb_batch_energy(self._ctx, int(job), int(tick), ctypes.byref(ek),
                                              ctypes.byref(ep)))
        return ek.value, ep.value
