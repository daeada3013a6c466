"""The one-pass oracle (both products from one reading of A): pinned to the
two-product recurrence of `gk.first_cycle`, to G = A^T Q computed directly,
to the relations of eq. (2.4), to the exact breakdown of a low-rank matrix,
and to a closed-form spectrum; plus a planted mistake in the recovery."""
import numpy as np
import pytest

from oracle import checks, gk, onepass


def _matrix(m, n, decay, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    V, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    s = decay ** np.arange(min(m, n))
    return (U * s) @ V.T, s


@pytest.mark.parametrize("m,n,decay", [(300, 200, 0.9), (300, 200, 0.5), (120, 250, 0.95), (80, 80, 0.99)])
def test_same_factorization_as_two_products(m, n, decay):
    A, _ = _matrix(m, n, decay, seed=m + n)
    q = np.random.default_rng(1).standard_normal(m)
    k = 30
    f1 = gk.first_cycle(A, q, k, gk.BreakThreshold(1e-12, True))
    f2, G = onepass.first_cycle(A, q, k, gk.BreakThreshold(1e-12, True))
    assert f1.breakdown is None and f2.breakdown is None
    assert f2.matvecs == f1.matvecs + len(f2.coeffs["refreshed"])
    assert np.max(np.abs(f1.H - f2.H)) < 1e-11
    # basis vectors are compared while beta stays above 1e-4 sigma_1: past that
    # a new vector is w / beta with w small relative to sigma_1, so rounding is
    # amplified by sigma_1 / beta and two runs that round differently
    # legitimately disagree in it (the relations below still hold)
    betas = np.diag(f1.H, -1)
    good = int(np.argmax(np.append(betas, 0.0) < 1e-4 * f1.H[0, 0]))
    assert np.max(np.abs(f1.P[:, :good] - f2.P[:, :good])) < 1e-9
    assert np.max(np.abs(f1.Q[:, : good + 1] - f2.Q[:, : good + 1])) < 1e-9
    assert np.max(np.abs(gk.ritz(f1.H)[1][:10] - gk.ritz(f2.H)[1][:10])) < 1e-12
    # the stored column images are A^T Q itself, to the guard's tolerance
    assert np.max(np.abs(G - A.T @ f2.Q)) < onepass.TAU
    # eq. (2.4)
    assert checks.relation_error(A, f2.P, f2.Q, f2.H) < 1e-12
    assert checks.transpose_relation_error(A, f2.P, f2.Q, f2.H, f2.alpha_res, f2.p_res) < 1e-12


def test_closed_form_spectrum():
    """A diagonal matrix: after enough steps the largest Ritz values are its diagonal."""
    s = 0.8 ** np.arange(60)
    A = np.zeros((90, 60))
    A[np.arange(60), np.arange(60)] = s
    q = np.random.default_rng(2).standard_normal(90)
    fac, _ = onepass.first_cycle(A, q, 59, gk.BreakThreshold(1e-14, True))
    _, sv, _ = gk.ritz(fac.H)
    assert np.max(np.abs(sv[:5] - s[:5])) < 1e-12


def test_low_rank_breakdown_matches():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((100, 6)) @ rng.standard_normal((6, 70))
    q = rng.standard_normal(100)
    f1 = gk.first_cycle(A, q, 20, gk.BreakThreshold(1e-10, True))
    f2, _ = onepass.first_cycle(A, q, 20, gk.BreakThreshold(1e-10, True))
    assert f1.breakdown == f2.breakdown and f1.breakdown is not None
    assert f1.H.shape == f2.H.shape
    assert np.max(np.abs(gk.ritz(f1.H)[1] - gk.ritz(f2.H)[1])) < 1e-10
    assert np.allclose(np.sort(gk.ritz(f2.H)[1])[::-1][:6], np.linalg.svd(A, compute_uv=False)[:6], rtol=1e-10)


def test_recovery_needs_the_recurrence_term():
    """Planted mistake: leaving alpha_t out of c breaks A^T q_{t+1} = recover(...)."""
    A, _ = _matrix(200, 150, 0.9, seed=5)
    q = np.random.default_rng(6).standard_normal(200)
    fac, G = onepass.first_cycle(A, q, 10, gk.BreakThreshold(1e-12, True))
    t = 5
    p = fac.P[:, t]
    w0 = A @ p
    y = A.T @ w0
    Qt = fac.Q[:, : t + 1]
    alpha = fac.H[t, t]
    w = w0 - alpha * Qt[:, t]
    h = Qt.T @ w
    w = w - Qt @ h
    beta = gk.vnorm(w)
    c = h.copy()
    c[t] += alpha
    good = onepass.recover(y, G[:, : t + 1], c, beta)
    assert np.max(np.abs(good - A.T @ (w / beta))) < 1e-12
    bad = onepass.recover(y, G[:, : t + 1], h, beta)
    assert np.max(np.abs(bad - A.T @ (w / beta))) > 1e-3


def test_guard_bounds_the_recovery_error():
    """Flat spectrum: alpha_t / beta_{t+1} is about 3, so the unguarded recovery
    loses about half a digit per step; the guard recomputes a column when its
    error bound passes tau * sigma and keeps the relations at the float64 level."""
    A, _ = _matrix(80, 80, 0.99, seed=160)
    q = np.random.default_rng(1).standard_normal(80)
    k = 30
    ref = gk.first_cycle(A, q, k, gk.BreakThreshold(1e-12, True))
    raw, Graw = onepass.first_cycle(A, q, k, gk.BreakThreshold(1e-12, True), tau=None)
    guarded, G = onepass.first_cycle(A, q, k, gk.BreakThreshold(1e-12, True))
    assert raw.coeffs["refreshed"] == []
    assert np.max(np.abs(Graw - A.T @ raw.Q)) > 1e-8
    assert 1 <= len(guarded.coeffs["refreshed"]) <= 5
    assert guarded.matvecs == ref.matvecs + len(guarded.coeffs["refreshed"])
    assert np.max(np.abs(G - A.T @ guarded.Q)) < 1e-11
    assert np.max(np.abs(guarded.H - ref.H)) < 1e-11
    assert checks.transpose_relation_error(A, guarded.P, guarded.Q, guarded.H, guarded.alpha_res,
                                           guarded.p_res) < 1e-11


def test_error_bound_dominates_the_actual_error():
    """The tracked bound is above the measured column error at every step."""
    for decay, seed in [(0.99, 160), (0.9, 500), (0.7, 77)]:
        A, _ = _matrix(120, 90, decay, seed=seed)
        q = np.random.default_rng(seed).standard_normal(120)
        m, n = A.shape
        eps0 = 2.0 ** -52 * np.sqrt(m + n)
        fac, G = onepass.first_cycle(A, q, 25, gk.BreakThreshold(1e-12, True), tau=None)
        actual = np.linalg.norm(G - A.T @ fac.Q, axis=0)
        # rebuild the bound from the returned coefficients (full reorthogonalisation:
        # the Gram-Schmidt parts of c are at rounding level, so c ~ alpha_t e_t)
        seen = max(np.max(np.diag(fac.H)), np.max(np.diag(fac.H, -1)))
        e = eps0 * seen
        for t in range(24):
            alpha, beta = fac.H[t, t], fac.H[t + 1, t]
            e = (alpha * e + eps0 * (seen * seen + seen * alpha)) / beta
            assert actual[t + 1] <= 10 * e


@pytest.mark.parametrize("decay,seed", [(0.9, 500), (0.99, 160)])
def test_restart_cycle_matches_two_products(decay, seed):
    """A thick restart on the one-sweep factorisation: the restarted cycle
    equals `gk.restart_cycle` on the two-product factorisation, and the stored
    columns are still A^T Q (A^T Q~ = (A^T Q) X_l for the kept ones)."""
    A, _ = _matrix(160, 120, decay, seed=seed)
    q = np.random.default_rng(seed + 1).standard_normal(160)
    k, l = 24, 10
    e1 = gk.BreakThreshold(1e-12, True)
    e2 = gk.BreakThreshold(1e-12, True)
    f1 = gk.first_cycle(A, q, k, e1)
    f2, G = onepass.first_cycle(A, q, k, e2)
    X1, s1, Y1 = gk.ritz(f1.H)
    X2, s2, Y2 = gk.ritz(f2.H)
    e1.seen(s1[0])
    e2.seen(s2[0])
    r1 = gk.restart_cycle(A, f1, X1, s1, Y1, l, k, e1)
    r2, G2, err2 = onepass.restart_cycle(A, f2, G, f2.coeffs["err"], X2, s2, Y2, l, k, e2)
    assert r1.breakdown is None and r2.breakdown is None
    assert r2.matvecs == r1.matvecs + len(f2.coeffs["refreshed"]) + len(r2.coeffs["refreshed"])
    assert np.max(np.abs(r1.H - r2.H)) < 1e-10
    assert np.max(np.abs(gk.ritz(r1.H)[1][:l] - gk.ritz(r2.H)[1][:l])) < 1e-12
    assert np.max(np.abs(G2 - A.T @ r2.Q)) < onepass.TAU
    assert np.all(np.linalg.norm(G2 - A.T @ r2.Q, axis=0) <= 10 * err2 + 1e-300)
    assert checks.relation_error(A, r2.P, r2.Q, r2.H) < 1e-12
