"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle (a dropped term, a wrong sign, coefficient or index, a transposed operand;
in every function that writes the formula out) makes at least one pin fail. The mutants are compiled on the CPU into a temporary
directory and swapped in for the real oracle library for the duration of a check.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_inputs as ti
import test_oracle_eval as te
import test_oracle_integrator as tg

SRC = os.path.join(os.path.dirname(oracle.__file__), "nbody_oracle.c")

# (name, exact text in the oracle, replacement)
MUTANTS = [
    ("jerk: sign of the alpha term", "J[k] = m3 * v[k] - 3.0 * alpha * A[k];",
     "J[k] = m3 * v[k] + 3.0 * alpha * A[k];"),
    ("snap: coefficient of the alpha term", "- 6.0 * alpha * J[k]", "- 3.0 * alpha * J[k]"),
    ("snap: dropped alpha^2 in beta", "                                + alpha * alpha;",
     "                                ;"),
    ("snap: wrong index in relative acceleration",
     "a[k] = ap[k * n + j] - ap[k * n + i];", "a[k] = ap[k * n + j] - ap[k * n + j];"),
    ("snap: dropped r.a in beta", "+ r[0] * a[0] + r[1] * a[1] + r[2] * a[2]) / R",
     "+ r[0] * a[0] + r[1] * a[1]) / R"),
    ("acceleration: transposed difference", "r[k] = xp[k * n + j] - xp[k * n + i];",
     "r[k] = xp[k * n + i] - xp[k * n + j];"),
    ("potential: wrong power", "cs_add(&acc[9], -(m[j] / sqR));",
     "cs_add(&acc[9], -(m[j] / R));"),
    ("predictor: wrong factorial", "const double f4 = h * h * h * h / 24.0;",
     "const double f4 = h * h * h * h / 12.0;"),
    ("predictor: dropped crackle term in v", "f3 * s[e] + f4 * c[e];", "f3 * s[e];"),
    ("corrector: sign of the jerk term", "- h2 / 10.0 * (j1 - j0)", "+ h2 / 10.0 * (j1 - j0)"),
    ("corrector: x uses old velocity twice", "h / 2.0 * (v0 + v1)", "h / 2.0 * (v0 + v0)"),
    ("interpolation: swapped jerk weights", "h * (36.0 * j1 + 24.0 * j0)",
     "h * (24.0 * j1 + 36.0 * j0)"),
    ("interpolation: a4 snap weights", "h2 * (36.0 * s1 - 24.0 * s0)",
     "h2 * (24.0 * s1 - 36.0 * s0)"),
    ("block rule: growth without the even-time test",
     "(t % ((int64_t)1 << (L - kold + 1))) == 0", "(t % ((int64_t)1 << (L - kold))) == 0"),
    ("block rule: cube missing", "ldexp(1.0, 3 * (dt_max_log2 - k)) <= qv",
     "ldexp(1.0, 2 * (dt_max_log2 - k)) <= qv"),
    ("step criterion: dropped sqrt(|a||s|) term", "const double num = sqrt(an * sn) + jn;",
     "const double num = jn;"),
    ("step criterion: 4th and 5th derivatives swapped",
     "const double den = sqrt(cn * a5n[i]) + a4n[i];",
     "const double den = sqrt(cn * a4n[i]) + a5n[i];"),
    ("start rule: snap time scale without its square root", "sqrt(an / sn)", "(an / sn)"),
    ("start rule: max instead of min", "d0 = eta_init * (ra < rs ? ra : rs);",
     "d0 = eta_init * (ra > rs ? ra : rs);"),
    ("active set: max instead of min", "if (e < tn)", "if (e > tn || tn == INT64_MAX)"),
    ("energy: potential double counted", "cs_add(&ep, -0.5 * m[i] * phi[i]);",
     "cs_add(&ep, -1.0 * m[i] * phi[i]);"),
    ("crackle: v.a weight in gamma", "(3.0 * va + rj) / R", "(2.0 * va + rj) / R"),
    ("crackle: alpha^3 weight in gamma", "(3.0 * beta - 4.0 * alpha * alpha)",
     "(3.0 * beta - 3.0 * alpha * alpha)"),
    ("crackle: beta J weight", "- 9.0 * beta * J[k]", "- 6.0 * beta * J[k]"),
    ("crackle: wrong index in relative jerk", "jj[k] = jp[k * n + j] - jp[k * n + i];",
     "jj[k] = jp[k * n + j] - jp[k * n + j];"),
    ("crackle: dropped r.j", "(3.0 * va + rj) / R", "(3.0 * va) / R"),
]

PINS = [
    lambda: te.test_acceleration_is_minus_grad_potential(1e-2),
    lambda: te.test_jerk_and_snap_are_time_derivatives(3e-2),
    lambda: te.test_crackle_is_third_time_derivative(3e-2),
    lambda: te.test_newton_third_law_and_torque(),
    lambda: te.test_two_body_closed_form(),
    lambda: tg.test_predictor_exact_on_degree5_motion(),
    lambda: tg.test_corrector_polynomial_exactness(5, -1),
    lambda: tg.test_corrector_polynomial_exactness(4, -7),
    lambda: tg.test_block_rule_shrink_is_free(),
    lambda: tg.test_block_rule_grow_one_level_only_at_even_time(),
    lambda: tg.test_initial_step_rule(),
    lambda: tg.test_step_criterion_circular_orbit_closed_form(0),
    lambda: tg.test_step_criterion_circular_orbit_closed_form(1),
    lambda: tg.test_active_set_brute_force(),
    lambda: tg.test_energy_two_body_closed_form(),
    lambda: ti.test_plummer_henon_units(),
    lambda: tg.test_sixth_order_convergence(),
]


def _killed():
    for pin in PINS:
        try:
            pin()
        except Exception:  # an assertion or an oracle error: the mutant is caught
            return True
    return False


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_real_oracle_passes_every_pin():
    assert not _killed()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, name, old, new):
    # a formula written out in more than one function gets the mistake everywhere
    assert source.count(old) >= 1, f"mutation site not found: {old!r}"
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(source.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(so), str(mutant_src), "-lm"], check=True)
    saved = oracle._lib
    oracle._lib = oracle.configure(ctypes.CDLL(str(so)))
    try:
        assert _killed(), f"no pin caught the mutant: {name}"
    finally:
        oracle._lib = saved
