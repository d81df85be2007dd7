"""Host-side checks of the C-ABI library that need no GPU: the library builds and
loads, exports every function include/nbody.h declares, and rejects bad arguments
before touching a device. No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_1812_00367_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1812_00367_amd import build
        build.build()
    return _abi.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert set(_declared()) == set(_abi.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def _params(**kw):
    p = dict(n=1024, eps=1e-4, eta=0.45, eta_init=0.01, dt_max_log2=-3, dt_min_log2=-40,
             precision=0, flags=0, partial_slots=0, stream=None)
    p.update(kw)
    return _abi.Params(**p)


def test_workspace_bytes_and_argument_checks(lib):
    out = ctypes.c_size_t(0)
    assert lib.nb_workspace_bytes(ctypes.byref(_params()), ctypes.byref(out)) == 0
    fp64 = out.value
    # state (19 doubles + 2 ints) + j-records + evaluation + partials at least
    assert fp64 >= 1024 * (8 * 19 + 12 + 80 + 80) + 80 * (1 << 20)
    assert lib.nb_workspace_bytes(ctypes.byref(_params(precision=1)), ctypes.byref(out)) == 0
    assert out.value >= fp64 + 64 * 1024
    bad = [dict(n=0), dict(n=(1 << 30) + 1), dict(eps=-1.0), dict(eps=float("nan")),
           dict(eta=0.0), dict(eta_init=-1.0), dict(dt_max_log2=-3, dt_min_log2=-70),
           dict(dt_max_log2=-3, dt_min_log2=-2), dict(precision=2), dict(flags=2),
           dict(partial_slots=-1)]
    for kw in bad:
        assert lib.nb_workspace_bytes(ctypes.byref(_params(**kw)), ctypes.byref(out)) == 1, kw
    assert lib.nb_workspace_bytes(None, ctypes.byref(out)) == 1


def test_create_rejects_bad_workspace_without_a_device(lib):
    ctx = ctypes.c_void_p(0)
    p = _params()
    assert lib.nb_create(ctypes.byref(p), None, 1 << 30, ctypes.byref(ctx)) == 1
    assert lib.nb_create(ctypes.byref(p), ctypes.c_void_p(0x1001), 1 << 30, ctypes.byref(ctx)) == 1
    assert lib.nb_create(ctypes.byref(p), ctypes.c_void_p(0x100000), 16, ctypes.byref(ctx)) == 2
    assert not ctx.value


def test_null_context_is_safe(lib):
    lib.nb_destroy(None)
    assert lib.nb_last_error(None) == b"null context"
    assert lib.nb_predict(None, 0) == 1
    assert lib.nb_evaluate(None, None, 0, None) == 1


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1812_00367_amd import Simulation
    with pytest.raises(RuntimeError):
        Simulation(16)


def _bparams(**kw):
    p = dict(capacity=4096, max_jobs=16, precision=0, eps=1e-4, eta=0.45, eta_init=0.01,
             dt_max_log2=-3, dt_min_log2=-40, jchunk=0, items_per_job=0, partial_slots=0, stream=None)
    p.update(kw)
    return _abi.BatchParams(**p)


def test_batch_workspace_bytes_and_argument_checks(lib):
    out = ctypes.c_size_t(0)
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams()), ctypes.byref(out)) == 0
    fp64 = out.value
    # pool state + j-records + the partial-sum bound 2 capacity + 128 (2048 + 1) max_jobs
    bound = 2 * 4096 + 128 * 2049 * 16
    assert fp64 >= 4096 * (8 * 19 + 12 + 80) + 80 * bound
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(precision=1)), ctypes.byref(out)) == 0
    assert out.value >= fp64 + 64 * 4096
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(partial_slots=bound + (1 << 20))),
                                        ctypes.byref(out)) == 0
    assert out.value >= fp64 + 80 * (1 << 20)
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(partial_slots=16)), ctypes.byref(out)) == 0
    assert out.value == fp64  # raised to the bound
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(items_per_job=64)), ctypes.byref(out)) == 0
    assert out.value < fp64
    # the chunk factors change the split, not the workspace
    assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(chunk_tile=1, chunk_wide=8, chunk_direct=64)),
                                        ctypes.byref(out)) == 0
    assert out.value == fp64
    bad = [dict(capacity=0), dict(capacity=(1 << 30) + 1), dict(max_jobs=0),
           dict(max_jobs=(1 << 16) + 1), dict(eps=-1.0), dict(eta=float("inf")),
           dict(dt_min_log2=-70), dict(precision=3), dict(jchunk=100), dict(jchunk=-64),
           dict(items_per_job=-1), dict(items_per_job=(1 << 14) + 1), dict(partial_slots=-5),
           dict(chunk_tile=-1), dict(chunk_wide=65), dict(chunk_direct=-2)]
    for kw in bad:
        assert lib.nb_batch_workspace_bytes(ctypes.byref(_bparams(**kw)), ctypes.byref(out)) == 1, kw
    b = ctypes.c_void_p(0)
    p = _bparams()
    assert lib.nb_batch_create(ctypes.byref(p), None, 1 << 30, ctypes.byref(b)) == 1
    assert lib.nb_batch_create(ctypes.byref(p), ctypes.c_void_p(0x1080), 1 << 30, ctypes.byref(b)) == 1
    assert lib.nb_batch_create(ctypes.byref(p), ctypes.c_void_p(0x100000), 64, ctypes.byref(b)) == 2
    assert not b.value
    lib.nb_batch_destroy(None)
    assert lib.nb_batch_last_error(None) == b"null batch"
    assert lib.nb_batch_step(None, None, None, None, None) == 1
    assert lib.nb_batch_run(None, 1, None, None, None, None, None) == 1
    assert lib.nb_batch_remove(None, 0) == 1
    assert lib.nb_batch_info(None, 0, None, None) == 1


def test_batch_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1812_00367_amd import Batch
    with pytest.raises(RuntimeError):
        Batch(64, 2)
