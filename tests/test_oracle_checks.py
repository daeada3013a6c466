"""Pins for the oracle's in-cycle convergence test, its early-stop branches,
the bfloat16 refinement and the error metrics of the experiments section.

Nothing here touches the GPU.  The in-cycle test (`gk.ConvergenceCheck`) and
the early returns of `gk.first_cycle` / `gk.restart_cycle` are checked by
brute force: every cycle is rerun to its full Krylov dimension without the
test, and at every scheduled column count np the top-r Ritz triplets of the
truncated factorization are formed explicitly (U = Q X, V = P Y) and their
true residuals ||A^T u_i - sigma_i v_i|| computed with products by A.  The
solve with the in-cycle test must stop at the first np whose true residuals
all pass, in the same cycle, after the same number of tests, with residual
estimates equal to the true residuals of what it returns (the third relation
of eq. (2.4)) and singular values equal to the prescribed spectrum.
"""
import numpy as np
import pytest

from oracle import bf16, checks, gk
from paper_2104_10785_amd import inputs


def true_residuals(A, Q, P, H, r):
    """Top-r Ritz triplets of the projected matrix H (LAPACK SVD), their vectors
    formed explicitly, and ||A^T u_i - sigma_i v_i|| by products with A."""
    X, s, Yt = np.linalg.svd(H, full_matrices=False)
    U = Q @ X[:, :r]
    V = P @ Yt.T[:, :r]
    return np.linalg.norm(A.T @ U - V * s[None, :r], axis=0), s


def prefix_first(fac, np_):
    """The first cycle after np_ right vectors, read off a longer run: the
    recurrence does not look ahead, so a run stopped at np_ is this prefix."""
    a, b = fac.coeffs["alpha"], fac.coeffs["beta"]
    H = np.zeros((np_ + 1, np_))
    for j in range(np_):
        H[j, j] = a[j]
        H[j + 1, j] = b[j]
    return fac.Q[:, : np_ + 1], fac.P[:, :np_], H


def prefix_restart(fac, np_):
    """A restarted cycle after np_ right vectors (prefix of a longer run)."""
    return fac.Q[:, :np_], fac.P[:, :np_], fac.H[:np_, :np_].copy()


def brute_force_stop(A, q, r, k, tol, every, max_restarts, eps_break=1e-12):
    """Where the solve with in-cycle tests must stop, found without them.

    The schedule: after np right vectors with np >= r, np % every == 0 and
    np < k, plus the end-of-cycle test at np = k.  Returns (cycle, np, tests
    before and at the stop) and the margins |res - tol sigma_1| / (tol sigma_1)
    seen at every test (a decision on a knife edge would make the comparison
    meaningless)."""
    eps = gk.BreakThreshold(eps_break, True)
    fac = gk.first_cycle(A, q, k, eps, 2)
    l = gk.default_keep(r, k)
    tests = 0
    margins = []
    for cycle in range(max_restarts + 1):
        first = cycle == 0
        lo = r if first else l + 1
        for np_ in range(lo, k):
            if np_ % every:
                continue
            Q, P, H = prefix_first(fac, np_) if first else prefix_restart(fac, np_)
            res, s = true_residuals(A, Q, P, H, r)
            tests += 1
            margins.append(np.min(np.abs(res - tol * s[0])) / (tol * s[0]))
            if np.all(res <= tol * s[0]):
                return cycle, np_, tests, margins
        # end of the cycle: the full factorization
        res, s = true_residuals(A, fac.Q[:, : fac.H.shape[0]], fac.P[:, : fac.H.shape[1]], fac.H, r)
        margins.append(np.min(np.abs(res - tol * s[0])) / (tol * s[0]))
        if np.all(res <= tol * s[0]):
            return cycle, k, tests, margins
        X, sv, Y = gk.ritz(fac.H)
        eps.seen(sv[0])
        fac = gk.restart_cycle(A, fac, X, sv, Y, l, k, eps, 2)
    raise AssertionError("brute force: no convergence within the restarts")


def check_against_brute_force(A, q, s, r, k, tol, every, max_restarts=50, solver=gk):
    out = solver.partial_svd(A, r, k, tol, max_restarts, q, check_every=every, eps_break=1e-12)
    cycle, np_, tests, margins = brute_force_stop(A, q, r, k, tol, every, max_restarts)
    assert min(margins) > 1e-6, "test case sits on a decision boundary"
    assert out["status"] == gk.OK and out["nconv"] == r
    assert out["restarts"] == cycle
    assert out["factorization"].H.shape[1] == np_
    assert out["checks"] == tests
    # the returned triplets: closed-form singular values, residual estimates
    # equal to the true residuals (eq. (2.4), third relation), A v = sigma u
    sig = out["sigma"]
    assert np.max(np.abs(sig - s[:r]) / s[:r]) < 1e-12
    r1, r2 = checks.triplet_residuals(A, sig, out["U"], out["V"])
    assert np.max(np.abs(r2 - out["res_est"])) < 1e-13 * s[0]
    assert np.max(r2) <= tol * sig[0] * (1 + 1e-9)
    assert np.max(r1) < 1e-13 * s[0]
    return out, np_


@pytest.fixture(scope="module")
def fast_decay():
    s = np.geomspace(1.0, 1e-8, 200)
    A, Q1, Q2 = inputs.svd_matrix(400, 200, s, seed=41)
    return A, Q1, Q2, s, inputs.start_vector(400, seed=42)


@pytest.mark.parametrize("every", [1, 3, 5])
def test_first_cycle_early_stop_matches_brute_force(fast_decay, every):
    A, Q1, Q2, s, q = fast_decay
    out, np_ = check_against_brute_force(A, q, s, 5, 60, 1e-10, every)
    assert out["restarts"] == 0 and np_ < 60          # stopped inside the first cycle
    assert np.min(checks.alignment(Q1[:, :5], Q2[:, :5], out["U"], out["V"])) > 1 - 1e-12


@pytest.fixture(scope="module")
def c1():
    s = inputs.decade_spectrum(1000)
    A, Q1, Q2 = inputs.svd_matrix(2000, 1000, s, seed=0)
    return A, Q1, Q2, s, inputs.start_vector(2000, seed=1)


@pytest.mark.parametrize("every", [1, 5])
def test_c1_in_cycle_checks_match_brute_force(c1, every):
    """The CPU-sized workload (2000 x 1000, s_i = 10^(-i/100), top 10, k = 30,
    tol 1e-10) with tests every 1 or 5 vectors: it needs restarts, so the stop
    lies in a restarted cycle (every 1: inside it; every 5: at its end)."""
    A, Q1, Q2, s, q = c1
    out, np_ = check_against_brute_force(A, q, s, 10, 30, 1e-10, every)
    assert out["restarts"] >= 1
    assert np.min(checks.alignment(Q1[:, :10], Q2[:, :10], out["U"], out["V"])) > 1 - 1e-8


def test_stop_at_np_equal_r():
    """A matrix whose r leading values sit far above a flat 1e-9 floor: the
    test due at np = r (the first column count the schedule allows) passes."""
    rng = np.random.default_rng(3)
    s = np.concatenate([[4.0, 3.0, 2.0], np.full(57, 1e-9)])
    A, _, _ = inputs.svd_matrix(90, 60, s, seed=5)
    q = inputs.start_vector(90, seed=6)
    out, np_ = check_against_brute_force(A, q, s, 3, 20, 1e-8, 1)
    assert np_ == 3 and out["checks"] == 1 and out["matvecs"] == 1 + 2 * 3
    del rng


def examined_points(A, q, r, k, every, cycles, eps_break=1e-12):
    """Every scheduled test of a solve that never stops (tol = 0), in order:
    (cycle, np, max_i true residual / sigma_1, alpha_res at np, the residual
    coefficient of the step before).  The run for any tol is a prefix of this
    one, so the stop for tol T is at the first point whose ratio is <= T."""
    eps = gk.BreakThreshold(eps_break, True)
    fac = gk.first_cycle(A, q, k, eps, 2)
    l = gk.default_keep(r, k)
    pts = []
    for cycle in range(cycles):
        first = cycle == 0
        for np_ in range(r if first else l + 1, k + 1):
            if np_ < k and np_ % every:
                continue
            if np_ == k:
                Q, P, H = fac.Q[:, : fac.H.shape[0]], fac.P, fac.H
            else:
                Q, P, H = prefix_first(fac, np_) if first else prefix_restart(fac, np_)
            res, s = true_residuals(A, Q, P, H, r)
            if first:
                a_now, a_prev = fac.coeffs["alpha"][np_], fac.coeffs["alpha"][np_ - 1]
            else:
                a_now = fac.alpha_res if np_ == k else fac.H[np_ - 1, np_]
                a_prev = fac.H[np_ - 2, np_ - 1] if np_ - 1 > l else 0.0
            pts.append((cycle, np_, np.max(res) / s[0], a_now, a_prev))
        X, sv, Y = gk.ritz(fac.H)
        eps.seen(sv[0])
        fac = gk.restart_cycle(A, fac, X, sv, Y, l, k, eps, 2)
    return pts


def sharp_tolerance(pts, cycle):
    """A tol 0.1 % above the true residual ratio of a point in `cycle` that is a
    clear new minimum (every earlier point is > 0.4 % above it) and where the
    residual coefficients of the step and the step before differ by > 1 %:
    the solve must stop exactly there, and a test fed the previous step's
    coefficient would not."""
    for i, (c, np_, rho, a_now, a_prev) in enumerate(pts):
        if c != cycle or np_ == pts[-1][1] or i == 0:
            continue
        if min(p[2] for p in pts[:i]) > rho * 1.004 and a_prev > 1.01 * a_now:
            return rho * 1.001, c, np_
    raise AssertionError("no suitable point")


def sharp_stop_check(data, r, k, cyc, solver=gk):
    A, _, _, s, q = data
    pts = examined_points(A, q, r, k, 1, cyc + 1)
    tol, c, np_ = sharp_tolerance(pts, cyc)
    out = solver.partial_svd(A, r, k, tol, 50, q, check_every=1, eps_break=1e-12)
    assert out["restarts"] == c and out["factorization"].H.shape[1] == np_
    r1, r2 = checks.triplet_residuals(A, out["sigma"], out["U"], out["V"])
    assert np.max(np.abs(r2 - out["res_est"])) < 1e-13 * s[0]


@pytest.mark.parametrize("case", ["first_cycle", "restarted_cycle"])
def test_stop_decision_is_sharp(fast_decay, c1, case):
    if case == "first_cycle":
        sharp_stop_check(fast_decay, 5, 60, 0)
    else:
        sharp_stop_check(c1, 10, 30, 2)


def test_early_stopped_factorization_satisfies_eq_2_4(fast_decay):
    """What an early stop returns is a valid factorization: A P = Q H and
    A^T Q = P H^T + alpha_res p_res e_last^T with orthonormal bases."""
    A, _, _, s, q = fast_decay
    out = gk.partial_svd(A, 5, 60, 1e-10, 0, q, check_every=2, eps_break=1e-12)
    fac = out["factorization"]
    assert fac.H.shape[1] < 60 and fac.coeffs.get("early")
    assert checks.relation_error(A, fac.P, fac.Q, fac.H) < 1e-14
    assert checks.transpose_relation_error(A, fac.P, fac.Q, fac.H, fac.alpha_res, fac.p_res) < 1e-14
    assert checks.orth_error(np.column_stack([fac.P, fac.p_res])) < 1e-13
    assert checks.orth_error(fac.Q) < 1e-13


# ------------------------------------------------ bfloat16 + float32 refinement
def bf16_exact_matrix(m, n, vals, seed):
    """A = Pi_1 diag(vals) Pi_2 with random row/column permutations and signs;
    every entry is 0 or +-vals[i], so it is exact in bfloat16 when vals are."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, n), dtype=np.float32)
    rows = rng.permutation(m)[: vals.size]
    cols = rng.permutation(n)[: vals.size]
    sg = rng.choice([-1.0, 1.0], vals.size)
    A[rows, cols] = (sg * vals).astype(np.float32)
    return A, rows, cols, sg


def test_refined_on_bfloat16_exact_matrix_gives_exact_triplets():
    # values that bfloat16 holds exactly (8 significant bits), all distinct
    vals = np.array([2.0 ** (-0.125 * i) for i in range(40)], dtype=np.float32)
    vals = bf16.from_bf16_bits(bf16.to_bf16_bits(vals))
    vals = np.unique(vals)[::-1]
    A, rows, cols, sg = bf16_exact_matrix(70, 50, vals, seed=3)
    assert np.array_equal(bf16.from_bf16_bits(bf16.to_bf16_bits(A)), A.astype(np.float64))
    r = 4
    q = inputs.start_vector(70, seed=4)
    Ue = np.zeros((70, r))
    Ve = np.zeros((50, r))
    Ue[rows[:r], np.arange(r)] = sg[:r]
    Ve[cols[:r], np.arange(r)] = 1.0
    # restarted solve (k = 20), and one cycle run to the breakdown at the 40th
    # step, where the basis is a Krylov basis rather than kept Ritz vectors
    for k, restarts in ((20, 30), (40, 0)):
        out, (sig, U, V), d = bf16.refined_partial_svd(A, r, k, 1e-12, restarts, q, eps_break=1e-12)
        assert out["status"] == gk.OK
        assert d == 2 * r
        assert np.max(np.abs(sig - vals[:r]) / vals[:r]) < 1e-13
        assert np.min(checks.alignment(Ue, Ve, U, V)) > 1 - 1e-13


def test_refined_dimension_is_as_stated():
    s = np.geomspace(1.0, 1e-3, 30)
    A, _, _ = inputs.svd_matrix(60, 30, s, seed=8)
    q = inputs.start_vector(60, seed=9)
    A32 = A.astype(np.float32)
    # default d = 2 r when the Krylov dimension allows it
    assert bf16.refined_partial_svd(A32, 3, 12, 1e-6, 0, q)[2] == 6
    # capped by the Krylov dimension of the final projected matrix (fixed k = 8)
    assert bf16.refined_partial_svd(A32, 5, 8, 1e-6, 0, q)[2] == 8
    # explicit refine_dim, and never below r
    assert bf16.refined_partial_svd(A32, 3, 12, 1e-6, 0, q, refine_dim=4)[2] == 4
    assert bf16.refined_partial_svd(A32, 3, 12, 1e-6, 0, q, refine_dim=1)[2] == 3


def test_refinement_within_the_rayleigh_ritz_bound():
    """Noisy float32 matrix: the unrefined bfloat16 values lie within Weyl's
    bound ||A16 - A32||_2 of sigma(A32) (LAPACK on the float64 upcast); the
    refined ones within the quadratic Rayleigh-Ritz bound
    (||A16 - A32||_2 + tol sigma_1)^2 / gap, gap = sigma_r - sigma_{d+1} of A32."""
    s = np.concatenate([np.geomspace(1.0, 0.3, 6), np.geomspace(0.2, 1e-3, 74)])
    A, _, _ = inputs.svd_matrix(300, 80, s, seed=12)
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    A16 = bf16.from_bf16_bits(bf16.to_bf16_bits(A32))
    sl = np.linalg.svd(A64, compute_uv=False)
    E2 = np.linalg.norm(A16 - A64, 2)
    r, k, tol = 6, 30, 1e-8
    out, (sig, U, V), d = bf16.refined_partial_svd(A32, r, k, tol, 20, inputs.start_vector(300, seed=2),
                                                   eps_break=1e-12)
    assert out["status"] == gk.OK and d == 12
    un = out["sigma"]
    assert np.all(np.abs(un - sl[:r]) <= E2 + tol * sl[0] + 1e-14)
    gap = sl[r - 1] - sl[d]
    bound = (E2 + tol * sl[0]) ** 2 / gap
    err = np.abs(sig - sl[:r])
    assert np.all(err <= bound + 1e-14)
    assert np.max(err) < 0.1 * np.max(np.abs(un - sl[:r]))   # the refinement helps
    r1, _ = checks.triplet_residuals(A64, sig, U, V)
    assert np.max(r1) < 1e-13                                    # A32 v = sigma u by construction


# ------------------------------------------------------------- error metrics
def test_err_res_is_the_eckart_young_tail():
    """||A - U_r S_r V_r^T||_F of the exact top-r triplets is the norm of the
    discarded singular values (Eckart-Young); err_rel of exact triplets is 0."""
    s = np.geomspace(5.0, 0.01, 25)
    A, Q1, Q2 = inputs.svd_matrix(40, 25, s, seed=14)
    for r in (1, 7, 25):
        want = np.sqrt(np.sum(s[r:] ** 2))
        got = checks.err_res(A, s[:r], Q1[:, :r], Q2[:, :r])
        assert abs(got - want) < 1e-13 * s[0] * 10
        assert checks.err_rel(A, s[:r], Q1[:, :r], Q2[:, :r]) < 1e-14 * 10
    # a wrong singular value shows up in both metrics by exactly its error
    bad = s[:3].copy()
    bad[1] += 1e-3
    got = checks.err_res(A, bad, Q1[:, :3], Q2[:, :3])
    assert abs(got - np.sqrt(np.sum(s[3:] ** 2) + 1e-6)) < 1e-12
    assert abs(checks.err_rel(A, bad, Q1[:, :3], Q2[:, :3]) - 1e-3 / np.linalg.norm(bad)) < 1e-12


def test_alignment_and_canonical_signs():
    """Figure 1's metric is 1 for the same triplets whatever the signs of the
    pairs, 0 for orthogonal ones; canonical signs make the largest-magnitude
    entry of each v positive and flip u with it."""
    rng = np.random.default_rng(2)
    U = np.linalg.qr(rng.standard_normal((30, 4)))[0]
    V = np.linalg.qr(rng.standard_normal((20, 4)))[0]
    f = np.array([1.0, -1.0, -1.0, 1.0])
    assert np.allclose(checks.alignment(U, V, U * f, V * f), 1.0, atol=1e-15)
    assert np.allclose(checks.alignment(U, V, np.roll(U, 1, axis=1), V), 0.0, atol=1e-15)
    Uc, Vc = checks.canonical_signs(U * f, V * f)
    idx = np.argmax(np.abs(Vc), axis=0)
    assert np.all(Vc[idx, np.arange(4)] > 0)
    assert np.allclose(checks.alignment(U, V, Uc, Vc), 1.0, atol=1e-15)
    assert np.allclose(Uc * Vc[idx, np.arange(4)], U * V[idx, np.arange(4)], atol=1e-15)
