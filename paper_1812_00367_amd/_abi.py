"""ctypes declarations of the C ABI in include/nbody.h (argument marshalling only).

Loading fails loudly if libnbody.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnbody.so")

NB_OK, NB_ERR_ARG, NB_ERR_SPACE, NB_ERR_DEVICE, NB_ERR_STATE, NB_ERR_NUMERIC = range(6)
NB_FP64, NB_SPLIT = 0, 1
NB_FLAG_START_CRACKLE = 1
NB_STATIC_SCRATCH_BYTES = 128 << 20
STATUS_NAMES = {0: "NB_OK", 1: "NB_ERR_ARG", 2: "NB_ERR_SPACE", 3: "NB_ERR_DEVICE",
                4: "NB_ERR_STATE", 5: "NB_ERR_NUMERIC"}

# Every function the header declares (checked against include/nbody.h by the tests).
EXPORTS = ["nb_workspace_bytes", "nb_create", "nb_destroy", "nb_last_error", "nb_set_state",
           "nb_set_times", "nb_get_state", "nb_start", "nb_active", "nb_predict", "nb_get_predicted",
           "nb_evaluate", "nb_evaluate_static", "nb_evaluate_crackle", "nb_set_evaluation", "nb_eval_config", "nb_eval_table", "nb_correct", "nb_timesteps",
           "nb_step", "nb_energy",
           "nb_batch_workspace_bytes", "nb_batch_create", "nb_batch_destroy", "nb_batch_last_error",
           "nb_batch_add", "nb_batch_remove", "nb_batch_step", "nb_batch_run", "nb_batch_get", "nb_batch_energy",
           "nb_batch_info"]


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("eps", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("eta_init", ctypes.c_double),
        ("dt_max_log2", ctypes.c_int32),
        ("dt_min_log2", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("partial_slots", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


class State(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("m", "x", "v", "a", "j", "s", "c", "a4n", "a5n", "phi", "tick", "level")]


class BatchParams(ctypes.Structure):
    _fields_ = [
        ("capacity", ctypes.c_int64),
        ("max_jobs", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("eta_init", ctypes.c_double),
        ("dt_max_log2", ctypes.c_int32),
        ("dt_min_log2", ctypes.c_int32),
        ("jchunk", ctypes.c_int32),
        ("items_per_job", ctypes.c_int32),
        ("chunk_tile", ctypes.c_int32),
        ("chunk_wide", ctypes.c_int32),
        ("chunk_direct", ctypes.c_int32),
        ("partial_slots", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


class NBodyError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libnbody.so and declare its signatures. Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1812_00367_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i64, i32, dbl, c = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int
    lib.nb_workspace_bytes.argtypes = [P(Params), P(ctypes.c_size_t)]
    lib.nb_create.argtypes = [P(Params), vp, ctypes.c_size_t, P(vp)]
    lib.nb_destroy.argtypes = [vp]
    lib.nb_destroy.restype = None
    lib.nb_last_error.argtypes = [vp]
    lib.nb_last_error.restype = ctypes.c_char_p
    lib.nb_set_state.argtypes = [vp, P(State), i64]
    lib.nb_set_times.argtypes = [vp, vp, vp]
    lib.nb_get_state.argtypes = [vp, P(State)]
    lib.nb_start.argtypes = [vp]
    lib.nb_active.argtypes = [vp, vp, P(i64), P(i64)]
    lib.nb_predict.argtypes = [vp, i64]
    lib.nb_get_predicted.argtypes = [vp, vp, vp, vp]
    lib.nb_evaluate.argtypes = [vp, vp, i64, vp]
    lib.nb_evaluate_static.argtypes = [i64, vp, vp, vp, vp, dbl, vp, i64, vp, vp]
    lib.nb_evaluate_crackle.argtypes = [vp, vp, i64, vp]
    lib.nb_set_evaluation.argtypes = [vp, vp, i64, vp]
    lib.nb_eval_config.argtypes = [vp, vp, i64, vp]
    lib.nb_eval_table.argtypes = [vp, vp, i32]
    lib.nb_correct.argtypes = [vp, vp, i64, i64]
    lib.nb_timesteps.argtypes = [vp, vp, i64, c]
    lib.nb_step.argtypes = [vp, i64, P(i64), P(i64)]
    lib.nb_energy.argtypes = [vp, i64, P(dbl), P(dbl)]
    lib.nb_batch_workspace_bytes.argtypes = [P(BatchParams), P(ctypes.c_size_t)]
    lib.nb_batch_create.argtypes = [P(BatchParams), vp, ctypes.c_size_t, P(vp)]
    lib.nb_batch_destroy.argtypes = [vp]
    lib.nb_batch_destroy.restype = None
    lib.nb_batch_last_error.argtypes = [vp]
    lib.nb_batch_last_error.restype = ctypes.c_char_p
    lib.nb_batch_add.argtypes = [vp, i64, P(State), i64, i64, P(i32)]
    lib.nb_batch_remove.argtypes = [vp, i32]
    lib.nb_batch_step.argtypes = [vp, vp, vp, vp, P(i64)]
    lib.nb_batch_run.argtypes = [vp, i32, vp, vp, vp, P(i64), P(i64)]
    lib.nb_batch_get.argtypes = [vp, i32, P(State)]
    lib.nb_batch_energy.argtypes = [vp, i32, i64, P(dbl), P(dbl)]
    lib.nb_batch_info.argtypes = [vp, i32, P(i64), P(i64)]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("nb_destroy", "nb_last_error", "nb_batch_destroy", "nb_batch_last_error"):
            fn.restype = c
    if path == LIB_PATH:
        _lib = lib
    return lib
