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
