"""nb_evaluate_static, the entry point for callers that cannot allocate device
memory, through the C ABI: its output is bitwise that of nb_evaluate on the same
predicted state, on two calls in a row (the second smaller, so the library's fixed
device array holds the first call's contents), then the first again; an index out
of range makes every output NaN and the next good call is clean again; a size
beyond the array is refused with NB_ERR_SPACE."""
import sys

import numpy as np
import pytest

import nbody_inputs as ni

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_00367_amd as nb
    return nb


def reference(nb, n, seed, n_act, act_seed, eps=1e-4):
    """nb_evaluate of n_act bodies of a Plummer sphere, and the predicted arrays it
    evaluated (read back with nb_get_predicted)."""
    ic = ni.plummer(n, seed)
    ap = ni.plummer_mean_field_acc(ic.x)
    sim = nb.Simulation(n, eps=eps)
    sim.set_state(ic.m, ic.x, ic.v, a=ap)
    sim.predict(0)
    idx = torch.as_tensor(ni.active_subset(n, n_act, act_seed), device="cuda")
    want = sim.evaluate(idx).clone()
    xp, vp, apr = (t.clone() for t in sim.get_predicted())
    m = torch.as_tensor(ic.m, device="cuda")
    shape = sim.eval_config(None, n_act)
    sim.close()
    return m, xp, vp, apr, idx, want, shape


def test_static_matches_evaluate_on_two_calls(nb):
    cases = [(20000, 41, 5000, 42), (3001, 43, 100, 44)]
    refs = [reference(nb, *c) for c in cases]
    for (n, _, n_act, _), (m, xp, vp, ap, idx, want, shape) in zip(cases + cases[:1], refs + refs[:1]):
        say("nb_evaluate_static n", n, "n_act", n_act, "shape", shape)
        got = nb.evaluate_static(m, xp, vp, ap, 1e-4, idx)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, n_act)


def test_static_bad_index_gives_nan_then_recovers(nb):
    m, xp, vp, ap, idx, want, _ = reference(nb, 3001, 45, 300, 46)
    bad = idx.clone()
    bad[7] = 3001
    out = nb.evaluate_static(m, xp, vp, ap, 1e-4, bad)
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
    got = nb.evaluate_static(m, xp, vp, ap, 1e-4, idx)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_static_refuses_sizes_beyond_its_array(nb):
    from paper_1812_00367_amd import _abi
    lib = _abi.load()
    n = 1 << 21  # 80 n bytes of j-records alone exceed the array
    assert 80 * n > _abi.NB_STATIC_SCRATCH_BYTES
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = dummy.data_ptr()
    rc = lib.nb_evaluate_static(n, p, p, p, p, 1e-4, idx.data_ptr(), 1, p, None)
    assert rc == _abi.NB_ERR_SPACE
    rc = lib.nb_evaluate_static(100, p, p, p, p, -1.0, idx.data_ptr(), 1, p, None)
    assert rc == _abi.NB_ERR_ARG
