"""Partial SVD and numerical rank through the C ABI against the float64 oracle.

Both sides get the same seeded inputs (the input generator module) and the
same start vector.  Float64 mode: singular values within 1e-10 relative of
the oracle; vectors compared with the sign-invariant alignment metric of
Figure 1; ranks exactly equal.
"""
import numpy as np
import pytest

from oracle import checks, gk, philox
from oracle import rank as orank
from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu


def run_gpu(A, r, k, tol, restarts, q=None, dtype=None, **kw):
    import torch
    Ad = to_dev(A) if dtype is None else to_dev(A).to(dtype)
    qd = to_dev(q) if q is not None else None
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(Ad, r, k, tol, restarts, q1=qd, **kw)
    torch.cuda.synchronize()
    return sigma, to_host(Ut).T.astype(np.float64), to_host(Vt).T.astype(np.float64), status, stats


@pytest.fixture(scope="module")
def c1():
    s = inputs.decade_spectrum(1000)
    A, Q1, Q2 = inputs.svd_matrix(2000, 1000, s, seed=0)
    q = inputs.start_vector(2000, seed=1)
    return A, Q1, Q2, s, q


U32 = 2.0 ** -24


def sigma_tolerance_f32(sigma1):
    """First-order tolerance for float32 products against the float64 oracle on
    the exact upcast of the same matrix.  A perturbation E moves a simple
    singular value by u_i^T E v_i (plus O(||E||^2 / gap)).  Here E collects
    the float32 roundings of the basis vectors and of the products' sums,
    each a relative perturbation of about u32 of a vector of size at most
    sigma_1; their projections on one singular pair add without a common
    direction, so the sum stays at the scale u32 sigma_1 (measured 0.01 u32
    sigma_1 at 50000 x 20000)."""
    return U32 * sigma1


def vector_tolerance_f32(sigma, gaps):
    """Davis-Kahan with the perturbation of sigma_tolerance_f32: sin(angle)
    <= ||E|| / gap_i, times 1.5 for the 32-column sketch estimate of a
    distance (chi-square(32) ratio below 1.49 with probability 1 - 1e-4) and
    sqrt(2) from angle to distance."""
    return 1.5 * np.sqrt(2.0) * sigma_tolerance_f32(sigma[0]) / gaps


def test_c1_partial_svd_f64(c1):
    device()
    A, Q1, Q2, s, q = c1
    banner("c1 2000x1000 f64 r=10 k=30 tol=1e-10")
    ref = gk.partial_svd(A, 10, 30, 1e-10, 50, q)
    sigma, U, V, status, stats = run_gpu(A, 10, 30, 1e-10, 50, q)
    assert status == 0 and stats["nconv"] == 10
    assert np.max(np.abs(sigma - ref["sigma"]) / ref["sigma"]) <= 1e-10
    assert np.max(np.abs(sigma - s[:10]) / s[:10]) <= 1e-10
    assert np.min(checks.alignment(ref["U"], ref["V"], U, V)) >= 1 - 1e-8
    r1, r2 = checks.triplet_residuals(A, sigma, U, V)
    assert np.max(r1) < 1e-12 and np.max(r2) <= 1.01e-10 * sigma[0]
    assert abs(stats["restarts"] - ref["restarts"]) <= 1
    assert checks.orth_error(U) < 1e-12 and checks.orth_error(V) < 1e-12


def test_c1_one_shot_algorithm2(c1):
    device()
    A, Q1, Q2, s, q = c1
    banner("c1 f64 max_restarts=0 k=60")
    ref = gk.partial_svd(A, 10, 60, 1e-10, 0, q)
    sigma, U, V, status, stats = run_gpu(A, 10, 60, 1e-10, 0, q)
    assert status == ref["status"] and stats["nconv"] == ref["nconv"]
    assert np.max(np.abs(sigma - ref["sigma"]) / ref["sigma"]) <= 1e-10
    assert stats["matvecs"] == 121 and stats["restarts"] == 0


def test_many_restarts_match_oracle():
    device()
    banner("300x100 f64 r=8 k=14 many restarts")
    s = np.concatenate([np.geomspace(1.0, 0.5, 8), np.geomspace(0.45, 0.01, 92)])
    A, Q1, Q2 = inputs.svd_matrix(300, 100, s, seed=21)
    q = inputs.start_vector(300, seed=22)
    ref = gk.partial_svd(A, 8, 14, 1e-11, 200, q)
    sigma, U, V, status, stats = run_gpu(A, 8, 14, 1e-11, 200, q)
    assert status == 0 and ref["status"] == 0
    assert abs(stats["restarts"] - ref["restarts"]) <= 1
    assert np.max(np.abs(sigma - s[:8]) / s[:8]) <= 1e-10
    assert np.min(checks.alignment(Q1[:, :8], Q2[:, :8], U, V)) >= 1 - 1e-8


@pytest.mark.parametrize("tau,want", [(10 ** -6.005, 601), (10 ** -5.995, 600)])
def test_c1_rank(c1, tau, want):
    device()
    A, _, _, s, q = c1
    banner(f"c1 rank tau={tau:.3e}")
    ref = orank.numerical_rank(A, tau, q)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(A), tau, q1=to_dev(q))
    assert rank == want and rank_s == want and ref["rank"] == want
    assert sig.size == ref["sigma"].size
    top = ref["sigma"] > 1e-6
    assert np.max(np.abs(sig[top] - ref["sigma"][top]) / ref["sigma"][top]) < 1e-10


@pytest.mark.parametrize("l", [1, 5, 37, 100])
def test_rank_exact_products(l):
    device()
    banner(f"rank of product l={l}")
    A = inputs.product_matrix(600, 400, l, seed=5)
    q = inputs.start_vector(600, seed=2)
    ref = orank.numerical_rank(A, 1e-8, q)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(A), 1e-8, q1=to_dev(q))
    assert rank == l and rank_s == l and ref["rank"] == l
    assert abs(sig.size - ref["steps"]) <= 1


def test_rank_one_and_zero():
    device()
    banner("rank-1 and zero matrices")
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(300), rng.standard_normal(200)
    A = np.outer(x, y)
    q = inputs.start_vector(300, seed=2)
    sigma, U, V, status, stats = run_gpu(A, 1, 3, 1e-12, 0, q)
    assert status == 0
    assert abs(sigma[0] - np.linalg.norm(x) * np.linalg.norm(y)) < 1e-13 * sigma[0]
    assert abs(abs(U[:, 0] @ x) / np.linalg.norm(x) - 1) < 1e-13
    Z = np.zeros((50, 40))
    sigma, U, V, status, stats = run_gpu(Z, 2, 4, 1e-10, 1, inputs.start_vector(50, seed=1))
    assert status == 2 and stats["returned"] == 0 and np.all(sigma == 0)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(Z), 1e-6, q1=to_dev(inputs.start_vector(50, 1)))
    assert rank == 0


@pytest.mark.parametrize("shape", [(7, 1, 1), (1, 9, 1), (1, 1, 1), (2, 2, 2), (3, 2, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_degenerate_shapes(shape, dtype):
    """A single row or column, a 1 x 1 matrix and k = min(m, n) on 2 x 2 and 3 x 2:
    the recurrence ends after one or two steps (by breakdown or at k = min(m, n))
    and the triplets are exact; the same status and matvec count as the oracle."""
    import torch
    device()
    m, n, r = shape
    banner(f"degenerate shape {shape} {dtype}")
    rng = np.random.default_rng(m * 10 + n)
    A = rng.standard_normal((m, n))
    q = inputs.start_vector(m, seed=4)
    ref = gk.partial_svd(A, r, r, 1e-12, 0, q)
    if dtype == "bf16":   # bfloat16 cycles, float32 Rayleigh-Ritz refinement
        A32 = to_dev(A).to(torch.float32)
        sigma, U, V, status, stats = run_gpu(A, r, r, 1e-6, 0, q, dtype=torch.bfloat16, refine=A32)
        assert stats["refined"] == 1
    else:
        sigma, U, V, status, stats = run_gpu(A, r, r, 1e-12 if dtype == "f64" else 1e-6, 0, q,
                                             dtype=None if dtype == "f64" else torch.float32)
    assert status == ref["status"] == 0
    A32 = A.astype(np.float32).astype(np.float64)
    sl = np.linalg.svd(A32 if dtype != "f64" else A, compute_uv=False)[:r]
    tol = 1e-13 if dtype == "f64" else 1e-6
    r1, r2 = checks.triplet_residuals(A32 if dtype != "f64" else A, sigma, U, V)
    if dtype == "bf16":
        # the refinement works inside the bfloat16 Krylov subspace: sigma within
        # ||A16 - A32||_2^2 / sigma_1 + sqrt(n) u32 ||A||_F, A^T u - sigma v within ||A16 - A32||_2
        A16 = torch.from_numpy(A32).to(torch.bfloat16).to(torch.float64).numpy()
        dA = np.linalg.norm(A16 - A32, 2)
        bound = dA ** 2 / sl[0] + np.sqrt(max(m, n)) * 2.0 ** -24 * np.linalg.norm(A32)
        assert np.max(np.abs(sigma - sl)) <= 2 * bound + 1e-7 * sl[0]
        assert r1.max() <= 1e-5 * sl[0] and r2.max() <= 2 * dA + 1e-5 * sl[0]
    else:
        assert np.max(np.abs(sigma - sl)) <= tol * sl[0]
        assert max(r1.max(), r2.max()) <= 10 * tol * sl[0]
    if dtype == "f64":
        assert stats["matvecs"] == ref["matvecs"]


@pytest.mark.parametrize("shape", [(9, 4, 2, 4), (1, 8, 1, 1), (4, 4, 4, 4)])
def test_degenerate_shapes_one_sweep(shape):
    """The one-sweep step (float32 A, n a multiple of 4) at k = min(m, n): exact
    triplets, the oracle's status."""
    import torch
    device()
    m, n, r, k = shape
    banner(f"degenerate shape one-sweep {shape}")
    rng = np.random.default_rng(m * 10 + n + 1)
    A = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    q = inputs.start_vector(m, seed=4)
    ref = gk.partial_svd(A, r, k, 1e-6, 0, q, eps_break=1e-6)
    sigma, U, V, status, stats = run_gpu(A, r, k, 1e-6, 0, q, dtype=torch.float32, one_pass=True)
    assert status == ref["status"] == 0
    sl = np.linalg.svd(A, compute_uv=False)[:r]
    assert np.max(np.abs(sigma - sl)) <= 1e-6 * sl[0]
    r1, r2 = checks.triplet_residuals(A, sigma, U, V)
    assert max(r1.max(), r2.max()) <= 1e-5 * sl[0]


@pytest.mark.parametrize("shape", [(7, 1), (1, 9), (1, 1)])
def test_rank_degenerate_shapes(shape):
    """Numerical rank of a single row, a single column and a 1 x 1 matrix (1), and
    of the zero matrix of that shape (0)."""
    device()
    m, n = shape
    banner(f"rank of degenerate shape {shape}")
    A = np.random.default_rng(m + 2 * n).standard_normal((m, n))
    q = to_dev(inputs.start_vector(m, seed=1))
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(A), 1e-6, q1=q)
    assert rank == rank_s == 1
    assert abs(sig[0] - np.linalg.norm(A)) <= 1e-13 * np.linalg.norm(A)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(np.zeros((m, n))), 1e-6, q1=q)
    assert rank == 0


def test_rank_deficient_returns_exact_triplets():
    device()
    banner("rank-3 product with r=5")
    A = inputs.product_matrix(500, 300, 3, seed=4)
    q = inputs.start_vector(500, seed=5)
    ref = gk.partial_svd(A, 5, 10, 1e-10, 3, q)
    sigma, U, V, status, stats = run_gpu(A, 5, 10, 1e-10, 3, q)
    assert status == 2 and ref["status"] == 2 and stats["returned"] == 3
    assert np.max(np.abs(sigma[:3] - ref["sigma"]) / ref["sigma"]) < 1e-12
    r1, r2 = checks.triplet_residuals(A, sigma[:3], U[:, :3], V[:, :3])
    assert max(r1.max(), r2.max()) < 1e-11 * sigma[0]


def test_wide_and_full_dimension():
    device()
    banner("wide 40x90 and k=min(m,n)")
    s = np.geomspace(3.0, 0.1, 40)
    A, Q1, Q2 = inputs.svd_matrix(40, 90, s, seed=31)
    q = inputs.start_vector(40, seed=1)
    sigma, U, V, status, stats = run_gpu(A, 5, 25, 1e-12, 50, q)
    assert status == 0 and np.max(np.abs(sigma - s[:5]) / s[:5]) < 1e-12
    sigma, U, V, status, stats = run_gpu(A, 40, 40, 1e-12, 0, q)
    assert np.max(np.abs(sigma - s) / s) < 1e-12


def test_nan_input_reports_numeric_error():
    device()
    banner("NaN input")
    A = np.ones((64, 32))
    A[3, 5] = np.nan
    with pytest.raises(gkb.GkbError) as ei:
        run_gpu(A, 2, 4, 1e-8, 0, np.ones(64))
    assert ei.value.status == -3


def test_device_start_vector_path(c1):
    device()
    A, Q1, Q2, s, q = c1
    banner("c1 with device Philox start (q1=NULL)")
    qp = philox.start_vector(2000, 12345)
    ref = gk.partial_svd(A, 10, 30, 1e-10, 50, qp)
    sigma, U, V, status, stats = run_gpu(A, 10, 30, 1e-10, 50, None, seed=12345)
    assert status == 0
    assert np.max(np.abs(sigma - ref["sigma"]) / ref["sigma"]) <= 1e-10
    assert np.min(checks.alignment(ref["U"], ref["V"], U, V)) >= 1 - 1e-8


def test_f32_lowrank_noise_midsize():
    import torch
    device()
    m, n = 6000, 2500
    banner(f"f32 low-rank+noise {m}x{n} r=20 k=60")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 200, 0.95, 1e-6, seed=7, dtype=np.float32)
    q = inputs.start_vector(m, seed=8)
    ref = gk.partial_svd(A32.astype(np.float64), 20, 60, 1e-6, 20, q, eps_break=1e-6)
    sigma, U, V, status, stats = run_gpu(A32, 20, 60, 1e-6, 20, q)
    assert status == 0
    # first-order float32 tolerance (sigma_tolerance_f32); the norm-wise bound
    # (about sqrt(n) u ||A|| per matvec, Weyl) stays as a sanity check
    err = np.abs(sigma - ref["sigma"])
    tight = sigma_tolerance_f32(ref["sigma"][0])
    print(f"f32 sigma abs err max {err.max():.3e} = {err.max() / (U32 * ref['sigma'][0]):.4f} u32 sigma_1, "
          f"rel {(err / ref['sigma']).max():.3e}", flush=True)
    bound = 8.0 * np.sqrt(max(m, n)) * 2.0 ** -24 * ref["sigma"][0]
    assert np.all(err <= tight) and np.all(err <= bound)
    al = checks.alignment(ref["U"], ref["V"], U, V)
    print("f32 alignment min", al.min(), flush=True)
    r1, r2 = checks.triplet_residuals(A32.astype(np.float64), sigma, U, V)
    assert np.max(r1) <= bound * 10 and np.max(r2) <= 1e-6 * sigma[0] + bound * 10


def test_determinism(c1):
    device()
    A, Q1, Q2, s, q = c1
    banner("determinism: two runs bitwise equal")
    a = run_gpu(A, 10, 30, 1e-10, 50, q)
    b = run_gpu(A, 10, 30, 1e-10, 50, q)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("every", [1, 5])
def test_c1_in_cycle_checks_match_oracle(c1, every):
    """In-cycle convergence test (eq. (2.4), third relation): same stop point as
    the oracle, sigma against the prescribed spectrum, and the residual the
    test relies on checked directly: ||A^T u - sigma v|| <= tol sigma_1 for
    every returned triplet, the device's residual estimate equal to the true
    residual, and A v = sigma u to rounding (U = Q X with eq. (2.4))."""
    device()
    A, Q1, Q2, s, q = c1
    tol = 1e-10
    banner(f"c1 f64 with check_every={every}")
    ref = gk.partial_svd(A, 10, 30, tol, 50, q, check_every=every)
    sigma, U, V, status, stats = run_gpu(A, 10, 30, tol, 50, q, check_every=every)
    assert status == 0 and ref["status"] == 0
    assert np.max(np.abs(sigma - ref["sigma"]) / ref["sigma"]) <= 1e-10
    assert np.max(np.abs(sigma - s[:10]) / s[:10]) <= 1e-10
    assert np.min(checks.alignment(ref["U"], ref["V"], U, V)) >= 1 - 1e-8
    assert np.min(checks.alignment(Q1[:, :10], Q2[:, :10], U, V)) >= 1 - 1e-8
    assert stats["krylov_dim"] == ref["factorization"].H.shape[1]
    assert stats["matvecs"] == ref["matvecs"] and stats["restarts"] == ref["restarts"]
    assert stats["checks"] == ref["checks"] and stats["checks"] > 0
    r1, r2 = checks.triplet_residuals(A, sigma, U, V)
    print(f"c1 every={every}: ||Av-su|| max {r1.max():.3e}, ||A^T u-sv|| max {r2.max():.3e}, "
          f"device estimate {stats['max_res_est']:.3e}, oracle estimate {ref['res_est'].max():.3e}", flush=True)
    assert r2.max() <= tol * sigma[0]
    assert r1.max() <= 1e-12 * sigma[0]
    # the estimate alpha_res |X[last, i]| is the true residual (eq. (2.4)), to rounding
    assert abs(stats["max_res_est"] - r2.max()) <= 1e-13 * sigma[0]
    assert abs(stats["max_res_est"] - ref["res_est"].max()) <= 1e-13 * sigma[0]


def test_restarted_cycle_with_checks():
    device()
    banner("300x100 f64 r=8 k=20 check_every=3 with restarts")
    s = np.concatenate([np.geomspace(1.0, 0.5, 8), np.geomspace(0.45, 0.01, 92)])
    A, Q1, Q2 = inputs.svd_matrix(300, 100, s, seed=21)
    q = inputs.start_vector(300, seed=22)
    ref = gk.partial_svd(A, 8, 20, 1e-11, 200, q, check_every=3)
    sigma, U, V, status, stats = run_gpu(A, 8, 20, 1e-11, 200, q, check_every=3)
    assert status == 0 and ref["status"] == 0 and ref["restarts"] > 0
    assert abs(stats["restarts"] - ref["restarts"]) <= 1
    assert np.max(np.abs(sigma - s[:8]) / s[:8]) <= 1e-10
    assert np.min(checks.alignment(Q1[:, :8], Q2[:, :8], U, V)) >= 1 - 1e-8
    r1, r2 = checks.triplet_residuals(A, sigma, U, V)
    print(f"restarted with checks: ||A^T u-sv|| max {r2.max():.3e}, device estimate {stats['max_res_est']:.3e}",
          flush=True)
    assert r2.max() <= 1e-11 * sigma[0] and r1.max() <= 1e-12 * sigma[0]
    assert abs(stats["max_res_est"] - r2.max()) <= 1e-13 * sigma[0]


def _host_residuals(A32, sigma, U, V, rows=2000):
    """||A v_i - sigma_i u_i|| and ||A^T u_i - sigma_i v_i|| in float64, A in row blocks."""
    m, n = A32.shape
    AV = np.zeros((m, V.shape[1]))
    ATU = np.zeros((n, U.shape[1]))
    for r0 in range(0, m, rows):
        blk = A32[r0:r0 + rows].astype(np.float64)
        AV[r0:r0 + rows] = blk @ V
        ATU += blk.T @ U[r0:r0 + rows]
    return (np.linalg.norm(AV - U * sigma[None, :], axis=0),
            np.linalg.norm(ATU - V * sigma[None, :], axis=0))


@pytest.mark.parametrize("check_every", [0, 10])
def test_c2_fullsize_f32_against_stored_oracle(check_every):
    """50000 x 20000 float32 at the benchmark's launch configuration.

    Expected values: tests/golden/c2_oracle_top50.json, written by
    tests/golden/make_c2_reference.py from the float64 oracle on the exact
    upcast of the same float32 matrix, with the same test schedule.  sigma
    within the first-order float32 tolerance (sigma_tolerance_f32), the
    norm-wise bound sqrt(n) u32 ||A||_F kept as a sanity check; singular vectors
    against the oracle's through its stored Gaussian sketches.
    """
    import json
    import os
    import torch
    from .gpu_util import sketch_distances
    device()
    ref_all = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_top50.json")))
    ref = ref_all if check_every == 0 else ref_all["check_every_10"]
    banner(f"c2 full size 50000x20000 f32 r=50 k=120 check_every={check_every}")
    A32, s, _, _ = inputs.lowrank_noise(50000, 20000, 200, 0.95, 1e-6, seed=2, dtype=np.float32)
    q = inputs.start_vector(50000, seed=1)
    Ad = torch.from_numpy(A32).to("cuda:0")
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(Ad, 50, 120, 1e-6, 20, q1=to_dev(q),
                                                       check_every=check_every)
    torch.cuda.synchronize()
    del Ad
    assert status == 0 and stats["nconv"] == 50
    want = np.array(ref["sigma"])
    fro = float(np.sqrt(np.sum(s ** 2) + 1e-12 * A32.size))
    loose = np.sqrt(20000) * U32 * fro
    tight = sigma_tolerance_f32(want[0])
    err = np.abs(sigma - want)
    print(f"c2 sigma max abs err {err.max():.3e} = {err.max() / (U32 * want[0]):.4f} u32 sigma_1 "
          f"(tolerance {tight:.3e}, norm-wise {loose:.3e}), max rel {np.max(err / want):.3e}, "
          f"matvecs {stats['matvecs']} (oracle {ref['matvecs']}), checks {stats['checks']} "
          f"(oracle {ref['checks']})", flush=True)
    assert np.all(err <= tight) and np.all(err <= loose)
    assert stats["matvecs"] == ref["matvecs"] and stats["checks"] == ref["checks"]
    assert stats["krylov_dim"] == ref["krylov_dim"] and stats["restarts"] == ref["restarts"]
    U = to_host(Ut).T.astype(np.float64)
    V = to_host(Vt).T.astype(np.float64)
    sp = np.concatenate([want, [s[50]]])
    gaps = np.minimum(np.abs(np.diff(np.concatenate([[np.inf], sp])))[:50], np.abs(np.diff(sp)))
    du, dv = sketch_distances(ref, U, V)
    vt = vector_tolerance_f32(want, gaps)
    print(f"c2 vector distances (sketch): u max {du.max():.3e}, v max {dv.max():.3e}; "
          f"max ratio to tolerance {np.max(np.maximum(du, dv) / vt):.3f}", flush=True)
    assert np.all(du <= vt) and np.all(dv <= vt)
    idx = [0, 1, 24, 48, 49]
    r1, r2 = _host_residuals(A32, sigma[idx], U[:, idx], V[:, idx])
    print(f"c2 residuals ||Av-su|| {r1.max():.3e} ||A^T u - s v|| {r2.max():.3e}", flush=True)
    assert np.max(r1) <= 10 * loose and np.max(r2) <= 1e-6 * sigma[0] + 10 * loose
    assert checks.orth_error(V[:, idx]) < 1e-5 and checks.orth_error(U[:, idx]) < 1e-5


def test_c2_fullsize_f64_against_stored_oracle():
    """The 50000 x 20000 workload in float64: the exact upcast of the float32
    matrix is the very matrix the stored oracle run used, so the float64 path
    must reproduce it to the float64 bar: sigma within 1e-10 relative, the
    same number of products and tests, and singular vectors (through the
    stored sketches) within the Davis-Kahan bound that a 1e-10 sigma_1
    perturbation allows."""
    import json
    import os
    import torch
    from .gpu_util import sketch_distances
    device()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_top50.json")))["check_every_10"]
    banner("c2 full size 50000x20000 f64 r=50 k=120 check_every=10")
    A32, s, _, _ = inputs.lowrank_noise(50000, 20000, 200, 0.95, 1e-6, seed=2, dtype=np.float32)
    q = inputs.start_vector(50000, seed=1)
    Ad = torch.from_numpy(A32).to("cuda:0").double()
    del A32
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(Ad, 50, 120, 1e-6, 20, q1=to_dev(q), check_every=10)
    torch.cuda.synchronize()
    del Ad
    want = np.array(ref["sigma"])
    rel = np.abs(sigma - want) / want
    print(f"c2 f64 sigma max rel err {rel.max():.3e}, matvecs {stats['matvecs']} (oracle {ref['matvecs']}), "
          f"checks {stats['checks']} (oracle {ref['checks']})", flush=True)
    assert status == 0 and stats["nconv"] == 50
    assert rel.max() <= 1e-10
    assert stats["matvecs"] == ref["matvecs"] and stats["checks"] == ref["checks"]
    U = to_host(Ut).T
    V = to_host(Vt).T
    sp = np.concatenate([want, [s[50]]])
    gaps = np.minimum(np.abs(np.diff(np.concatenate([[np.inf], sp])))[:50], np.abs(np.diff(sp)))
    du, dv = sketch_distances(ref, U, V)
    vt = 1.5 * np.sqrt(2.0) * 1e-10 * want[0] / gaps
    print(f"c2 f64 vector distances (sketch): u max {du.max():.3e}, v max {dv.max():.3e}; "
          f"max ratio to tolerance {np.max(np.maximum(du, dv) / vt):.3e}", flush=True)
    assert np.all(du <= vt) and np.all(dv <= vt)


@pytest.mark.parametrize("one_pass", [False, True])
def test_bf16_storage_with_refinement_midsize(one_pass):
    """bfloat16 storage + float32 Rayleigh-Ritz refinement, per-triplet errors
    against the float64 oracle on the float32 matrix, with two sweeps of the
    bfloat16 A per step or one.

    Unrefined (bfloat16 solve): Weyl, |sigma_i(A16) - sigma_i(A32)| <= ||A16 - A32||_2.
    Refined: the Rayleigh-Ritz values from a subspace at angle ~ ||E||/gap from
    the exact one are off by ~ ||E||^2 / gap (gap = sigma_r - sigma_{d+1}),
    plus the float32 product rounding sqrt(n) u ||A||_F.
    """
    import torch
    from oracle import bf16 as obf16
    device()
    # the one-sweep form needs n a multiple of 8 for bfloat16 rows
    m, n, r, k = 6000, (2496 if one_pass else 2500), 20, 60
    banner(f"bf16 + refinement {m}x{n} r={r} k={k} one_pass={one_pass}")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 200, 0.95, 1e-6, seed=7, dtype=np.float32)
    q = inputs.start_vector(m, seed=8)
    exact = gk.partial_svd(A32.astype(np.float64), 60, 120, 1e-13, 50, q)["sigma"]
    ref_un, (ref_sig, ref_U, ref_V), d = obf16.refined_partial_svd(A32, r, k, 1e-6, 20, q)
    A16 = obf16.from_bf16_bits(obf16.to_bf16_bits(A32))
    E = A16 - A32.astype(np.float64)
    normE = gk.partial_svd(E, 1, 30, 1e-8, 20, inputs.start_vector(m, 3))["sigma"][0]
    A32d = torch.from_numpy(A32).to("cuda:0")
    A16d = gkb.gkb_cast_bf16(A32d)
    qd = to_dev(q)
    sig_u, Ut_u, Vt_u, st_u, stats_u = gkb.gkb_partial_svd(A16d, r, k, 1e-6, 20, q1=qd, one_pass=one_pass)
    sig, Ut, Vt, status, stats = gkb.gkb_partial_svd(A16d, r, k, 1e-6, 20, q1=qd, refine=A32d, one_pass=one_pass)
    torch.cuda.synchronize()
    assert st_u == 0 and status == 0 and stats["refined"] == 1
    err_un = np.abs(sig_u - exact[:r])
    err_ref = np.abs(sig - exact[:r])
    gap = exact[r - 1] - exact[d]
    fp32 = np.sqrt(n) * 2.0 ** -24 * np.sqrt(np.sum(exact ** 2))
    print(f"bf16 ||E||_2={normE:.3e}; unrefined max err {err_un.max():.3e}; refined max err "
          f"{err_ref.max():.3e} (bound {normE ** 2 / gap + fp32:.3e}); oracle refined err "
          f"{np.max(np.abs(ref_sig - exact[:r])):.3e}", flush=True)
    for i in range(r):
        print(f"  triplet {i}: sigma {exact[i]:.6e} unrefined {err_un[i]:.2e} refined {err_ref[i]:.2e}",
              flush=True)
    assert np.all(err_un <= normE + fp32)
    assert np.all(err_ref <= normE ** 2 / gap + fp32)
    U = to_host(Ut).T.astype(np.float64)
    V = to_host(Vt).T.astype(np.float64)
    assert np.min(checks.alignment(ref_U, ref_V, U, V)) >= 1 - 1e-6
    r1, r2 = checks.triplet_residuals(A32.astype(np.float64), sig, U, V)
    r1u, r2u = checks.triplet_residuals(A32.astype(np.float64), sig_u, to_host(Ut_u).T.astype(np.float64),
                                        to_host(Vt_u).T.astype(np.float64))
    print(f"  residual ||A^T u - s v|| max: unrefined {r2u.max():.3e}, refined {r2.max():.3e}", flush=True)
    # Rayleigh-Ritz fixes the values to second order; the vectors keep the
    # subspace's first-order error ~ ||E|| / gap, so the residual does not grow
    assert r2.max() <= 1.05 * r2u.max()


@pytest.mark.parametrize("one_pass", [False, True])
def test_c3_fullsize_bf16_refined_against_stored_oracle(one_pass):
    """bfloat16 storage of the 50000 x 20000 matrix (two sweeps of it per step,
    or one), float32 refinement; the
    refined singular values against the oracle's values for the float32 matrix
    (tests/golden/c2_oracle_top50.json).  Bound: ||E||^2/gap + sqrt(n) u ||A||_F,
    E = A16 - A32 with entries uniform in [-u|a|, u|a|], u = 2^-8, so
    ||E||_2 ~ (u/sqrt(3)) rms(A) (sqrt(m) + sqrt(n)) (iid-like rounding errors;
    this estimate matched the oracle's exact ||E||_2 to 1% at 6000 x 2500),
    taken with a 1.2 margin."""
    import json
    import os
    import torch
    device()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_top50.json")))
    banner(f"c3 full size 50000x20000 bf16 + f32 refinement r=50 k=120 check_every=10 one_pass={one_pass}")
    A32, s, _, _ = inputs.lowrank_noise(50000, 20000, 200, 0.95, 1e-6, seed=2, dtype=np.float32)
    q = inputs.start_vector(50000, seed=1)
    A32d = torch.from_numpy(A32).to("cuda:0")
    A16d = gkb.gkb_cast_bf16(A32d)
    qd = to_dev(q)
    sig_u, _, _, st_u, stats_u = gkb.gkb_partial_svd(A16d, 50, 120, 1e-6, 20, q1=qd, check_every=10,
                                                     one_pass=one_pass)
    sig, Ut, Vt, status, stats = gkb.gkb_partial_svd(A16d, 50, 120, 1e-6, 20, q1=qd, check_every=10, refine=A32d,
                                                     one_pass=one_pass)
    torch.cuda.synchronize()
    del A32d, A16d
    want = np.array(ref["sigma"])
    fro = float(np.sqrt(np.sum(s ** 2)))
    rms = fro / np.sqrt(A32.size)
    normE = 1.2 * 2.0 ** -8 / np.sqrt(3.0) * rms * (np.sqrt(50000) + np.sqrt(20000))
    gap = want[-1] * (1 - 0.95 ** 50)  # sigma_50 - sigma_100 of the 0.95^i spectrum
    bound = normE ** 2 / gap + np.sqrt(20000) * 2.0 ** -24 * fro
    err_u = np.abs(sig_u - want)
    err = np.abs(sig - want)
    print(f"c3 bf16 unrefined max err {err_u.max():.3e}; refined max err {err.max():.3e} (bound {bound:.3e}); "
          f"matvecs {stats['matvecs']} refine {stats['ms_refine']:.2f} ms", flush=True)
    assert status == 0 and stats["refined"] == 1
    assert np.all(err <= bound) and np.all(err_u <= normE)
    assert err.max() < err_u.max()


@pytest.mark.parametrize("one_pass", [False, True])
def test_c2_gapped_rank_fullsize(one_pass):
    """Numerical rank at the gap after index 200 (50000 x 20000 float32, noise
    std 1e-10 so the noise edge ~ 3.7e-8 is far below s_200 = 0.95^200 ~ 3.5e-5;
    threshold 1e-6 sigma_1): both counts must be exactly 200, with two sweeps
    of A per step or one."""
    import torch
    device()
    banner(f"c2 gapped rank 50000x20000 f32 one_pass={one_pass}")
    A32, s, _, _ = inputs.lowrank_noise(50000, 20000, 200, 0.95, 1e-10, seed=2, dtype=np.float32)
    Ad = torch.from_numpy(A32).to("cuda:0")
    del A32
    q = to_dev(inputs.start_vector(50000, seed=1))
    rank, rank_s, sig, status, st = gkb.gkb_numerical_rank(Ad, 1e-6, k_max=400, q1=q, one_pass=one_pass)
    print(f"gapped rank {rank} sturm {rank_s} steps {len(sig)} breakdown {st['breakdown']} "
          f"products {st['matvecs']} recomputed {st['refreshes']}", flush=True)
    assert rank == 200 and rank_s == 200
    assert np.max(np.abs(sig[:200] - s) / s) < 1e-3


@pytest.mark.parametrize("one_pass", [False, True])
def test_phase_timing_stats(one_pass):
    """Per-phase device times (opt.phase_timing): the events change no result,
    the five phases add up to the call's wall time (to 5 %: the host's launch
    time before the first event and after the last one is outside them), and
    bytes_A counts the passes over A."""
    device()
    m, n = 6000, 2500
    banner(f"phase timing {m}x{n} f32 r=20 k=60 one_pass={one_pass}")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 200, 0.95, 1e-6, seed=7, dtype=np.float32)
    q = inputs.start_vector(m, seed=8)
    plain = run_gpu(A32, 20, 60, 1e-6, 20, q, check_every=5, one_pass=one_pass)
    timed = run_gpu(A32, 20, 60, 1e-6, 20, q, check_every=5, one_pass=one_pass, phase_timing=True)
    for a, b in zip(plain[:3], timed[:3]):
        assert np.array_equal(a, b)
    st = timed[4]
    phases = [st[f] for f in ("ms_matvec", "ms_reorth", "ms_sync", "ms_ritz", "ms_other")]
    print(f"phases {phases} sum {sum(phases):.3f} ms, total {st['ms_total']:.3f} ms, bytes_A {st['bytes_A']:.4e}",
          flush=True)
    assert min(phases) >= 0 and st["ms_matvec"] > 0 and st["ms_reorth"] > 0 and st["ms_ritz"] > 0
    assert abs(sum(phases) - st["ms_total"]) <= 0.05 * st["ms_total"]
    assert plain[4]["ms_matvec"] == 0 and plain[4]["ms_reorth"] == 0
    passes = st["matvecs"] if not one_pass else (st["matvecs"] - st["refreshes"] - 1) // 2 + 1 + st["refreshes"]
    assert st["bytes_A"] == passes * m * n * 4 and plain[4]["bytes_A"] == st["bytes_A"]
