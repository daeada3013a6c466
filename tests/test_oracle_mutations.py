"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU, in
memory; the files on disk are untouched) and checks that a pin that holds for
the real oracle fails for the mutant. Mistakes that full reorthogonalization
silently repairs (a wrong sign on a term that the Gram-Schmidt projection
removes anyway) are not listed: they do not change the result.
"""
import importlib
import inspect
import types

import numpy as np
import pytest

from oracle import checks, gk, rank
from paper_2104_10785_amd import inputs


def mutant(modname, old, new):
    mod = importlib.import_module(modname)
    src = inspect.getsource(mod)
    assert src.count(old) == 1, f"mutation anchor not unique in {modname}: {old!r}"
    m = types.ModuleType(modname + "_mutant")
    m.__package__ = "oracle"
    exec(compile(src.replace(old, new), modname + "_mutant", "exec"), m.__dict__)
    return m


def _restart_pin(g):
    s = np.concatenate([np.geomspace(1.0, 0.5, 8), np.geomspace(0.45, 0.01, 92)])
    A, _, _ = inputs.svd_matrix(300, 100, s, seed=21)
    out = g.partial_svd(A, 8, 14, 1e-11, 200, inputs.start_vector(300, seed=22))
    err = np.max(np.abs(out["sigma"] - s[: out["sigma"].size]) / s[: out["sigma"].size])
    return out["status"] == gk.OK and out["sigma"].size == 8 and err < 1e-12


def _c1_like_pin(g):
    s = np.geomspace(1.0, 1e-4, 120)
    A, Q1, Q2 = inputs.svd_matrix(240, 120, s, seed=3)
    out = g.partial_svd(A, 6, 20, 1e-10, 40, inputs.start_vector(240, seed=4))
    if out["sigma"].size != 6:
        return False
    ok_s = np.max(np.abs(out["sigma"] - s[:6]) / s[:6]) < 1e-12
    ok_v = np.min(checks.alignment(Q1[:, :6], Q2[:, :6], out["U"], out["V"])) > 1 - 1e-8
    r1, r2 = checks.triplet_residuals(A, out["sigma"], out["U"], out["V"])
    ok_r = np.max(np.abs(r2 - out["res_est"])) < 1e-12 and np.max(r1) < 1e-12
    return bool(ok_s and ok_v and ok_r)


def _sturm_pin(r):
    e = np.abs(np.random.default_rng(3).standard_normal(30)) + 0.1
    T = np.diag(e, 1) + np.diag(e, -1)
    lam = np.linalg.eigvalsh(T)
    return all(r.count_above(e, t) == int(np.count_nonzero(lam > t)) for t in [0.05, 0.5, 1.5])


def test_pins_hold_for_real_oracle():
    assert _restart_pin(gk) and _c1_like_pin(gk) and _sturm_pin(rank)


MUTATIONS = [
    ("oracle.gk", "rho = fac.alpha_res * X[nq - 1, :l]", "rho = fac.alpha_res * X[0, :l]", _restart_pin),
    ("oracle.gk", "H[j + 1, j] = betas[j]", "H[j, j + 1] = betas[j] if j + 1 < np_ else 0.0", _c1_like_pin),
    ("oracle.gk", "V = fac.P @ Y[:, :r_eff]", "V = fac.P @ X[: fac.P.shape[1], :r_eff]", _c1_like_pin),
    ("oracle.gk", "res = fac.alpha_res * np.abs(X[nq - 1, :])", "res = fac.alpha_res * np.abs(X[0, :])", _c1_like_pin),
    ("oracle.gk", "Q[:, 0] = q / beta1", "Q[:, 0] = q", _c1_like_pin),
    ("oracle.gk", "H[j, j + 1] = alpha", "H[j + 1, j] = alpha", _restart_pin),
    ("oracle.gk", "Pn[:, l] = fac.p_res", "Pn[:, l] = fac.P[:, np_ - 1]", _restart_pin),
    ("oracle.rank", "d = -tau - e[i] * e[i] / d", "d = -tau + e[i] * e[i] / d", _sturm_pin),
]


@pytest.mark.parametrize("modname,old,new,pin", MUTATIONS, ids=[m[2][:40] for m in MUTATIONS])
def test_planted_mistake_is_caught(modname, old, new, pin):
    m = mutant(modname, old, new)
    try:
        held = pin(m)
    except (ValueError, FloatingPointError, IndexError, np.linalg.LinAlgError, ZeroDivisionError):
        held = False
    assert not held


# ------------------------------------------- in-cycle test, refinement, metrics
def _holds(fn):
    try:
        fn()
        return True
    except AssertionError:
        return False


def _first_cycle_stop_pin(g, every=1):
    from tests.test_oracle_checks import check_against_brute_force
    s = np.geomspace(1.0, 1e-8, 200)
    A, _, _ = inputs.svd_matrix(400, 200, s, seed=41)
    return _holds(lambda: check_against_brute_force(A, inputs.start_vector(400, seed=42), s, 5, 60, 1e-10, every,
                                                    solver=g))


def _restart_stop_pin(g):
    from tests.test_oracle_checks import check_against_brute_force
    s = inputs.decade_spectrum(1000)
    A, _, _ = inputs.svd_matrix(2000, 1000, s, seed=0)
    return _holds(lambda: check_against_brute_force(A, inputs.start_vector(2000, seed=1), s, 10, 30, 1e-10, 1,
                                                    solver=g))


def _sharp_pin(g, case):
    from tests.test_oracle_checks import sharp_stop_check
    if case == "first":
        s = np.geomspace(1.0, 1e-8, 200)
        A, Q1, Q2 = inputs.svd_matrix(400, 200, s, seed=41)
        data, r, k, cyc = (A, Q1, Q2, s, inputs.start_vector(400, seed=42)), 5, 60, 0
    else:
        s = inputs.decade_spectrum(1000)
        A, Q1, Q2 = inputs.svd_matrix(2000, 1000, s, seed=0)
        data, r, k, cyc = (A, Q1, Q2, s, inputs.start_vector(2000, seed=1)), 10, 30, 2
    return _holds(lambda: sharp_stop_check(data, r, k, cyc, solver=g))


def _np_equal_r_pin(g):
    from tests.test_oracle_checks import check_against_brute_force
    s = np.concatenate([[4.0, 3.0, 2.0], np.full(57, 1e-9)])
    A, _, _ = inputs.svd_matrix(90, 60, s, seed=5)

    def run():
        out, np_ = check_against_brute_force(A, inputs.start_vector(90, seed=6), s, 3, 20, 1e-8, 1, solver=g)
        assert np_ == 3 and out["checks"] == 1
    return _holds(run)


def _refine_exact_pin(b):
    import tests.test_oracle_checks as t
    orig = t.bf16
    t.bf16 = b
    try:
        return _holds(t.test_refined_on_bfloat16_exact_matrix_gives_exact_triplets) and \
            _holds(t.test_refined_dimension_is_as_stated)
    finally:
        t.bf16 = orig


def _err_res_pin(c):
    import tests.test_oracle_checks as t
    orig = t.checks
    t.checks = c
    try:
        return _holds(t.test_err_res_is_the_eckart_young_tail)
    finally:
        t.checks = orig


def test_new_pins_hold_for_real_oracle():
    from oracle import bf16
    assert _first_cycle_stop_pin(gk) and _first_cycle_stop_pin(gk, 3) and _restart_stop_pin(gk)
    assert _np_equal_r_pin(gk) and _refine_exact_pin(bf16) and _err_res_pin(checks)
    assert _sharp_pin(gk, "first") and _sharp_pin(gk, "restart")


STOP_MUTATIONS = [
    # the in-cycle test fed the residual coefficient of the previous step
    ("oracle.gk", "if stop(H, alpha):", "if stop(H, alphas[-2]):", lambda g: _sharp_pin(g, "first")),
    ("oracle.gk", "if stop(Hp, alpha):", "if stop(Hp, alpha_prev):", lambda g: _sharp_pin(g, "restart")),
    # an early stop that returns the previous step's residual coefficient
    ("oracle.gk", "H, alpha, P[:, np_].copy(), None,", "H, alphas[-2], P[:, np_].copy(), None,",
     _first_cycle_stop_pin),
    # the schedule off by one, in either direction
    ("oracle.gk", "np_ % self.every == 0", "(np_ + 1) % self.every == 0",
     lambda g: _first_cycle_stop_pin(g, 3)),
    ("oracle.gk", "np_ >= self.r and", "np_ > self.r and", _np_equal_r_pin),
    # refinement subspace: wrong default size, wrong Ritz vectors
    ("oracle.bf16", "else 2 * r", "else r", _refine_exact_pin),
    ("oracle.bf16", "Vd = fac.P @ Y[:, :d]", "Vd = fac.P[:, :d]", _refine_exact_pin),
    # the residual metric without the singular values
    ("oracle.checks", "np.linalg.norm(A - (U * sigma[None, :]) @ V.T)", "np.linalg.norm(A - U @ V.T)",
     _err_res_pin),
]


@pytest.mark.parametrize("modname,old,new,pin", STOP_MUTATIONS, ids=[m[2][:40] for m in STOP_MUTATIONS])
def test_planted_stop_refine_metric_mistake_is_caught(modname, old, new, pin):
    m = mutant(modname, old, new)
    try:
        held = pin(m)
    except (ValueError, FloatingPointError, IndexError, np.linalg.LinAlgError, ZeroDivisionError):
        held = False
    assert not held
