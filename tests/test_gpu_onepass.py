"""The one-pass step (option one_pass: A read once per Golub-Kahan step)
through the C ABI against the float64 oracle.

The oracle runs the standard two-product recurrence on the exact float64
upcast of the same float32 matrix with the same start vector; the one-pass
path computes the same factorisation (see oracle.onepass and its pins), so
the Ritz values must agree to the float32 storage level: the only float32
rounding left is that of p before the product (float64 bases, float64 sums),
a relative perturbation of about u32 of each p.  To first order a
perturbation E moves a simple singular value by u_i^T E v_i; the roundings of
the k steps have no common direction, so their projections on one singular
pair stay at the scale of one of them: tolerance u32 sigma_1 (measured
0.002-0.04 u32 sigma_1).  The norm-wise bound 8 sqrt(k) u32 sigma_1 (Weyl,
one u32 ||A|| per step) is kept as a sanity check.  Vectors are compared with
the sign-invariant alignment metric of Figure 1.
"""
import json
import os

import numpy as np
import pytest

from oracle import checks, gk
from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, sketch_distances, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def run(A32, r, k, tol, restarts, q, **kw):
    import torch
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(to_dev(A32), r, k, tol, restarts, q1=to_dev(q), **kw)
    torch.cuda.synchronize()
    return sigma, to_host(Ut).T.astype(np.float64), to_host(Vt).T.astype(np.float64), status, stats


def _check_against(ref, sigma, U, V, k, align=1 - 1e-5):
    loose = 8.0 * np.sqrt(k) * U32 * ref["sigma"][0]
    tight = U32 * ref["sigma"][0]
    err = np.abs(sigma - ref["sigma"])
    print(f"one-pass sigma max abs err {err.max():.3e} = {err.max() / tight:.4f} u32 sigma_1 "
          f"(norm-wise bound {loose:.3e})", flush=True)
    assert np.all(err <= tight) and np.all(err <= loose)
    al = checks.alignment(ref["U"], ref["V"], U, V)
    print(f"one-pass alignment min {al.min():.9f}", flush=True)
    assert np.min(al) >= align


def test_onepass_lowrank_noise_midsize():
    device()
    m, n = 6000, 2500
    banner(f"one-pass f32 low-rank+noise {m}x{n} r=20 k=60")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 200, 0.95, 1e-6, seed=7, dtype=np.float32)
    q = inputs.start_vector(m, seed=8)
    ref = gk.partial_svd(A32.astype(np.float64), 20, 60, 1e-6, 20, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 20, 60, 1e-6, 20, q, one_pass=True)
    print("stats", stats, flush=True)
    assert status == 0 and ref["status"] == 0
    _check_against(ref, sigma, U, V, 60)
    assert abs(stats["restarts"] - ref["restarts"]) <= 1
    # two products per sweep, plus one per recomputed column
    two = run(A32, 20, 60, 1e-6, 20, q)
    assert stats["matvecs"] - stats["refreshes"] == two[4]["matvecs"] or stats["restarts"] != two[4]["restarts"]
    r1, r2 = checks.triplet_residuals(A32.astype(np.float64), sigma, U, V)
    assert np.max(r2) <= 1e-6 * sigma[0] + 1e-5 * sigma[0]


def test_onepass_flat_spectrum_recomputes_columns():
    """Square, ten separated values above a bulk in [0.5, 1]: there
    alpha_t / beta_{t+1} is about 3, an unguarded recovery loses half a digit
    per step (oracle.onepass pins this), and the guard must recompute columns."""
    device()
    s = np.concatenate([np.linspace(2.0, 1.1, 10), np.linspace(1.0, 0.5, 990)])
    A, _, _ = inputs.svd_matrix(1000, 1000, s, seed=31)
    A32 = A.astype(np.float32)
    q = inputs.start_vector(1000, seed=32)
    banner("one-pass square, flat bulk 1000x1000 r=10 k=40")
    ref = gk.partial_svd(A32.astype(np.float64), 10, 40, 1e-6, 40, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 10, 40, 1e-6, 40, q, one_pass=True)
    print("stats", stats, flush=True)
    assert stats["refreshes"] >= 2
    assert status == ref["status"] == 0
    _check_against(ref, sigma, U, V, 40)


@pytest.mark.parametrize("shape,r,k,check_every", [((100, 64), 4, 20, 0), ((333, 1000), 5, 30, 4),
                                                   ((5000, 4), 2, 4, 0), ((1200, 840), 8, 24, 5)])
def test_onepass_shapes(shape, r, k, check_every):
    """Fewer rows than workgroups, a wide matrix, n = 4 (k = n: the exact
    bidiagonalisation), in-cycle checks with restarts."""
    device()
    m, n = shape
    banner(f"one-pass {m}x{n} r={r} k={k} check_every={check_every}")
    rng = np.random.default_rng(m + n)
    p = min(m, n)
    s = np.geomspace(1.0, 1e-3, p)
    A, _, _ = inputs.svd_matrix(m, n, s, seed=m * 3 + n)
    A32 = A.astype(np.float32)
    q = rng.standard_normal(m) + 2.0
    ref = gk.partial_svd(A32.astype(np.float64), r, k, 1e-6, 200, q, eps_break=1e-6, check_every=check_every)
    sigma, U, V, status, stats = run(A32, r, k, 1e-6, 200, q, one_pass=True, check_every=check_every)
    print("stats", stats, flush=True)
    assert status == ref["status"]
    _check_against(ref, sigma, U, V, k, align=1 - 1e-4)


@pytest.mark.parametrize("check_every", [0, 3])
def test_onepass_many_restarts(check_every):
    """Thick restarts carry A^T Q~ = (A^T Q) X_l and the error bounds of the kept
    columns; a slowly converging spectrum forces many of them."""
    device()
    banner(f"one-pass 300x100 r=8 k=12 many restarts, check_every={check_every}")
    s = np.concatenate([np.geomspace(1.0, 0.5, 8), np.geomspace(0.45, 0.01, 92)])
    A, Q1, Q2 = inputs.svd_matrix(300, 100, s, seed=21)
    A32 = A.astype(np.float32)
    q = inputs.start_vector(300, seed=22)
    ref = gk.partial_svd(A32.astype(np.float64), 8, 12, 1e-8, 200, q, eps_break=1e-6, check_every=check_every)
    sigma, U, V, status, stats = run(A32, 8, 12, 1e-8, 200, q, one_pass=True, check_every=check_every)
    print("stats", stats, "oracle restarts", ref["restarts"], flush=True)
    assert status == ref["status"] == 0
    assert ref["restarts"] >= 8 and abs(stats["restarts"] - ref["restarts"]) <= 1
    _check_against(ref, sigma, U, V, 12)


def test_onepass_rank_deficient():
    device()
    banner("one-pass exact rank 6")
    rng = np.random.default_rng(3)
    A32 = (rng.standard_normal((400, 6)) @ rng.standard_normal((6, 300))).astype(np.float32)
    q = rng.standard_normal(400)
    ref = gk.partial_svd(A32.astype(np.float64), 8, 20, 1e-6, 5, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 8, 20, 1e-6, 5, q, one_pass=True)
    assert ref["status"] == 2 and len(ref["sigma"]) == 6
    assert status == 2 and stats["returned"] == 6
    assert np.max(np.abs(sigma[:6] - ref["sigma"])) <= U32 * ref["sigma"][0]
    assert np.all(sigma[6:] == 0.0)
    assert np.all(U[:, 6:] == 0.0) and np.all(V[:, 6:] == 0.0)


@pytest.mark.parametrize("l,shape", [(1, (600, 400)), (5, (600, 400)), (37, (600, 400)), (100, (600, 400)),
                                     (5, (300, 30000)), (37, (200, 50000))])
def test_onepass_rank_exact_products(l, shape):
    """Exact-rank products M N (float32): the one-sweep rank equals l, the
    oracle's rank and the two-sweep rank; the singular values of B agree with
    the two-sweep run to the float32 level (rows of 30000 and 50000 entries:
    the team sweep)."""
    from oracle import rank as orank
    device()
    m, n = shape
    banner(f"one-pass rank of product l={l} {m}x{n}")
    A32 = inputs.product_matrix(m, n, l, seed=5).astype(np.float32)
    q = inputs.start_vector(m, seed=2)
    ref = orank.numerical_rank(A32.astype(np.float64), 1e-5, q)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(A32), 1e-5, q1=to_dev(q), one_pass=True)
    rank2, _, sig2, _, _ = gkb.gkb_numerical_rank(to_dev(A32), 1e-5, q1=to_dev(q))
    print(f"l={l} rank {rank} sturm {rank_s} steps {sig.size} (two-sweep {sig2.size}, oracle {ref['steps']}) "
          f"recomputed {stats['refreshes']}", flush=True)
    assert stats["one_pass_used"] == 1
    assert rank == l and rank_s == l and rank2 == l and ref["rank"] == l
    top = min(l, sig.size, sig2.size)
    assert np.max(np.abs(sig[:top] - sig2[:top])) <= 8 * np.sqrt(l + 1) * U32 * sig2[0]


def test_onepass_zero_and_nan():
    """Degenerate inputs: A = 0 (A^T q_1 = 0 at the start: nothing to return)
    and a NaN entry (numeric error), as in the two-sweep path."""
    device()
    banner("one-pass zero matrix and NaN entry")
    Z = np.zeros((48, 40), dtype=np.float32)
    sigma, U, V, status, stats = run(Z, 2, 4, 1e-6, 1, inputs.start_vector(48, seed=1), one_pass=True)
    assert status == 2 and stats["returned"] == 0 and np.all(sigma == 0)
    rank, rank_s, sig, st, _ = gkb.gkb_numerical_rank(to_dev(Z), 1e-6, q1=to_dev(inputs.start_vector(48, 1)),
                                                      one_pass=True)
    assert rank == 0
    A = np.ones((64, 32), dtype=np.float32)
    A[3, 5] = np.nan
    with pytest.raises(gkb.GkbError) as ei:
        run(A, 2, 4, 1e-6, 0, np.ones(64), one_pass=True)
    assert ei.value.status == -3


def test_onepass_deterministic():
    device()
    banner("one-pass determinism")
    A32, _, _, _ = inputs.lowrank_noise(3000, 1500, 100, 0.9, 1e-6, seed=11, dtype=np.float32)
    q = inputs.start_vector(3000, seed=12)
    a = run(A32, 10, 30, 1e-6, 10, q, one_pass=True)
    b = run(A32, 10, 30, 1e-6, 10, q, one_pass=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_onepass_falls_back_to_two_products():
    """Where the one-sweep step is not available (n not a multiple of 4, a
    float64 A of odd n, rows longer than the team sweep takes) a one_pass request runs
    the two-product step: bitwise the same results as without the request, and
    stats say which step ran."""
    device()
    banner("one-pass fallback to the two-product step")
    rng = np.random.default_rng(0)
    cases = [rng.standard_normal((50, 30)).astype(np.float32), rng.standard_normal((50, 31)),
             rng.standard_normal((40, 262148)).astype(np.float32)]
    for A in cases:
        Ad = to_dev(A)
        q = to_dev(rng.standard_normal(A.shape[0]))
        a = gkb.gkb_partial_svd(Ad, 2, 6, 1e-6, 2, q1=q, one_pass=True)
        b = gkb.gkb_partial_svd(Ad, 2, 6, 1e-6, 2, q1=q)
        assert a[4]["one_pass_used"] == 0 and b[4]["one_pass_used"] == 0
        assert a[3] == b[3] and np.array_equal(a[0], b[0])
        assert np.array_equal(to_host(a[1]), to_host(b[1])) and np.array_equal(to_host(a[2]), to_host(b[2]))
        ra = gkb.gkb_numerical_rank(Ad, 1e-3, q1=q, one_pass=True)
        rb = gkb.gkb_numerical_rank(Ad, 1e-3, q1=q)
        assert ra[0] == rb[0] and np.array_equal(ra[2], rb[2]) and ra[4]["one_pass_used"] == 0
    A = rng.standard_normal((64, 48)).astype(np.float32)
    assert gkb.gkb_partial_svd(to_dev(A), 2, 6, 1e-6, 2, one_pass=True)[4]["one_pass_used"] == 1
    # rows longer than one workgroup holds: the team sweep, for both entry points
    A = to_dev(rng.standard_normal((64, 30000)).astype(np.float32))
    assert gkb.gkb_partial_svd(A, 2, 6, 1e-6, 2, one_pass=True)[4]["one_pass_used"] == 1
    assert gkb.gkb_numerical_rank(A, 1e-3, one_pass=True)[4]["one_pass_used"] == 1


@pytest.mark.parametrize("check_every", [0, 10])
def test_c2_fullsize_onepass_against_stored_oracle(check_every):
    """50000 x 20000 float32, r=50, k=120 with one sweep of A per step (with
    check_every=10: the benchmark's launch configuration), against the stored
    float64 oracle values (tests/golden/c2_oracle_top50.json, written by
    tests/golden/make_c2_reference.py)."""
    import torch
    device()
    ref_all = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle_top50.json")))
    ref = ref_all if check_every == 0 else ref_all["check_every_10"]
    banner(f"c2 full size 50000x20000 f32 r=50 k=120 one_pass check_every={check_every}")
    A32, s, _, _ = inputs.lowrank_noise(50000, 20000, 200, 0.95, 1e-6, seed=2, dtype=np.float32)
    q = inputs.start_vector(50000, seed=1)
    Ad = torch.from_numpy(A32).to("cuda:0")
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(Ad, 50, 120, 1e-6, 20, q1=to_dev(q), one_pass=True,
                                                       check_every=check_every)
    torch.cuda.synchronize()
    del Ad
    print("stats", stats, flush=True)
    assert status == 0 and stats["nconv"] == 50
    want = np.array(ref["sigma"])
    loose = 8.0 * np.sqrt(120) * U32 * want[0]
    tight = U32 * want[0]
    err = np.abs(sigma - want)
    print(f"c2 one-pass sigma max abs err {err.max():.3e} = {err.max() / tight:.4f} u32 sigma_1 "
          f"(norm-wise {loose:.3e}); matvecs {stats['matvecs']} (oracle {ref['matvecs']}), "
          f"refreshes {stats['refreshes']}, checks {stats['checks']} (oracle {ref['checks']})", flush=True)
    assert np.all(err <= tight) and np.all(err <= loose)
    # one sweep = two products; a recomputed column adds one direct product
    assert stats["matvecs"] - stats["refreshes"] == ref["matvecs"]
    assert stats["checks"] == ref["checks"] and stats["krylov_dim"] == ref["krylov_dim"]
    U = to_host(Ut).T.astype(np.float64)
    V = to_host(Vt).T.astype(np.float64)
    idx = [0, 1, 24, 48, 49]
    # residuals of sampled triplets against the float32 matrix, in float64 row blocks
    AV = np.zeros((50000, len(idx)))
    ATU = np.zeros((20000, len(idx)))
    for r0 in range(0, 50000, 2000):
        blk = A32[r0:r0 + 2000].astype(np.float64)
        AV[r0:r0 + 2000] = blk @ V[:, idx]
        ATU += blk.T @ U[r0:r0 + 2000, idx]
    r1 = np.linalg.norm(AV - U[:, idx] * sigma[idx][None, :], axis=0)
    r2 = np.linalg.norm(ATU - V[:, idx] * sigma[idx][None, :], axis=0)
    print(f"c2 one-pass residuals ||Av-su|| {r1.max():.3e} ||A^T u - s v|| {r2.max():.3e}", flush=True)
    assert np.max(r1) <= 1e-6 * want[0] and np.max(r2) <= 2e-6 * want[0]
    # singular vectors against the oracle's, through its stored sketches
    sp = np.concatenate([want, [s[50]]])
    gaps = np.minimum(np.abs(np.diff(np.concatenate([[np.inf], sp])))[:50], np.abs(np.diff(sp)))
    du, dv = sketch_distances(ref, U, V)
    vt = 1.5 * np.sqrt(2.0) * tight / gaps
    print(f"c2 one-pass vector distances (sketch): u max {du.max():.3e}, v max {dv.max():.3e}; "
          f"max ratio to tolerance {np.max(np.maximum(du, dv) / vt):.3f}", flush=True)
    assert np.all(du <= vt) and np.all(dv <= vt)


@pytest.mark.parametrize("shape", [(2000, 30000), (600, 80000), (257, 24580)])
def test_onepass_on_rows_longer_than_one_workgroup_holds(shape):
    """Rows of 24580, 30000 and 80000 entries are longer than one workgroup's
    registers hold (24576): the one-sweep step runs on teams of workgroups
    (4, 4 and 10 members with slices of at most 8192 columns), with the same
    tolerance against the float64 oracle on the exact upcast; the product
    count equals the two-product run's, and a second solve is bitwise equal
    (the team exchange keeps a fixed order)."""
    device()
    m, n = shape
    banner(f"one-pass team sweep {m}x{n} f32")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 100, 0.9, 1e-6, seed=m + n, dtype=np.float32)
    q = inputs.start_vector(m, seed=3)
    ref = gk.partial_svd(A32.astype(np.float64), 6, 24, 1e-6, 20, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 6, 24, 1e-6, 20, q, one_pass=True)
    print("stats", stats, flush=True)
    assert stats["one_pass_used"] == 1
    assert status == ref["status"] == 0
    _check_against(ref, sigma, U, V, 24)
    two = run(A32, 6, 24, 1e-6, 20, q)
    assert two[4]["one_pass_used"] == 0
    assert stats["matvecs"] - stats["refreshes"] == two[4]["matvecs"] or stats["restarts"] != two[4]["restarts"]
    again = run(A32, 6, 24, 1e-6, 20, q, one_pass=True)
    assert np.array_equal(again[0], sigma) and np.array_equal(again[1], U) and np.array_equal(again[2], V)


def test_onepass_team_sweep_with_checks_and_restarts():
    """The team sweep through in-cycle checks and a thick restart (k = 2 r),
    against the oracle with the same schedule."""
    device()
    m, n = 1500, 40000
    banner(f"one-pass team sweep {m}x{n} f32, checks every 4, restarts")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 60, 0.9, 1e-6, seed=11, dtype=np.float32)
    q = inputs.start_vector(m, seed=5)
    ref = gk.partial_svd(A32.astype(np.float64), 8, 16, 1e-6, 40, q, eps_break=1e-6, check_every=4)
    sigma, U, V, status, stats = run(A32, 8, 16, 1e-6, 40, q, one_pass=True, check_every=4)
    print("stats", stats, "oracle restarts", ref["restarts"], flush=True)
    assert stats["one_pass_used"] == 1 and stats["restarts"] >= 1
    assert status == ref["status"] == 0
    assert abs(stats["restarts"] - ref["restarts"]) <= 1
    _check_against(ref, sigma, U, V, 16)


def test_onepass_request_past_the_team_limit():
    """Rows longer than 262144 entries (32 members of 8192 columns) have no
    team form: the request runs the two-product step, against the oracle."""
    device()
    m, n = 64, 262148
    banner(f"one_pass request on {m}x{n} f32 (past the team limit)")
    A32, s, _, _ = inputs.lowrank_noise(m, n, 30, 0.8, 1e-6, seed=4, dtype=np.float32)
    q = inputs.start_vector(m, seed=6)
    ref = gk.partial_svd(A32.astype(np.float64), 4, 16, 1e-6, 20, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 4, 16, 1e-6, 20, q, one_pass=True)
    assert stats["one_pass_used"] == 0
    assert status == ref["status"] == 0
    _check_against(ref, sigma, U, V, 16)


ONEPASS_TAU = 1e-10   # the recovery guard: a column past tau sigma_1 is recomputed directly


def _check_f64(ref, sigma, U, V, k):
    """float64 A: every stored A^T q column is within ONEPASS_TAU sigma_1 of the
    exact one (or recomputed), so the factorisation is that of A + E with
    ||E|| <= sqrt(k) tau sigma_1 (one column error per step) and, by Weyl,
    each singular value moves by at most that much."""
    bound = np.sqrt(k) * ONEPASS_TAU * ref["sigma"][0]
    err = np.abs(sigma - ref["sigma"])
    print(f"float64 one-pass sigma max abs err {err.max():.3e} ({err.max() / ref['sigma'][0]:.2e} sigma_1; "
          f"bound {bound:.3e})", flush=True)
    assert np.all(err <= bound)
    al = checks.alignment(ref["U"], ref["V"], U, V)
    print(f"float64 one-pass alignment min {al.min():.12f}", flush=True)
    assert np.min(al) >= 1 - 1e-8


@pytest.mark.parametrize("shape", [(3000, 1500), (400, 20000)])
def test_onepass_float64(shape):
    """float64 A through the team sweep (4096-column slices: 1 and 5 members),
    against the float64 oracle: the singular values within the recovery bound,
    the same product count as the two-product run, U and V float64."""
    import torch
    device()
    m, n = shape
    banner(f"one-pass float64 {m}x{n}")
    A, s, _, _ = inputs.lowrank_noise(m, n, 100, 0.9, 1e-6, seed=m + n, dtype=np.float64)
    q = inputs.start_vector(m, seed=9)
    ref = gk.partial_svd(A, 10, 30, 1e-6, 20, q, eps_break=1e-12)
    sigma, Ut, Vt, status, stats = gkb.gkb_partial_svd(to_dev(A), 10, 30, 1e-6, 20, q1=to_dev(q), one_pass=True)
    torch.cuda.synchronize()
    print("stats", stats, flush=True)
    assert stats["one_pass_used"] == 1 and Ut.dtype == torch.float64
    assert status == ref["status"] == 0
    _check_f64(ref, sigma, to_host(Ut).T, to_host(Vt).T, 30)
    two = gkb.gkb_partial_svd(to_dev(A), 10, 30, 1e-6, 20, q1=to_dev(q))
    assert two[4]["one_pass_used"] == 0
    assert stats["matvecs"] - stats["refreshes"] == two[4]["matvecs"] or stats["restarts"] != two[4]["restarts"]


def test_onepass_float64_cpu_sized_config():
    """The CPU-sized float64 workload (2000 x 1000, Q1 diag(10^(-i/100)) Q2^T,
    top 10, k 30, tol 1e-10) with the one-sweep step: the singular values
    within the recovery bound of the prescribed spectrum and of the oracle."""
    device()
    banner("one-pass float64 2000x1000 prescribed spectrum")
    s = inputs.decade_spectrum(1000)
    A, _, _ = inputs.svd_matrix(2000, 1000, s, seed=0)
    q = inputs.start_vector(2000, seed=2)
    ref = gk.partial_svd(A, 10, 30, 1e-10, 50, q, eps_break=1e-12)
    sigma, U, V, status, stats = run(A, 10, 30, 1e-10, 50, q, one_pass=True)
    print("stats", stats, "oracle restarts", ref["restarts"], flush=True)
    assert stats["one_pass_used"] == 1 and status == ref["status"] == 0
    _check_f64(ref, sigma, U, V, 30)
    assert np.max(np.abs(sigma - s[:10])) <= np.sqrt(30) * ONEPASS_TAU * s[0]


@pytest.mark.parametrize("l", [5, 37])
def test_onepass_float64_rank(l):
    """Exact-rank float64 products through the one-sweep rank: rank l, as the
    oracle and the two-product rank."""
    from oracle import rank as orank
    device()
    banner(f"one-pass float64 rank l={l}")
    A = inputs.product_matrix(600, 400, l, seed=7)
    q = inputs.start_vector(600, seed=3)
    ref = orank.numerical_rank(A, 1e-8, q)
    rank, rank_s, sig, status, stats = gkb.gkb_numerical_rank(to_dev(A), 1e-8, q1=to_dev(q), one_pass=True)
    rank2, _, _, _, st2 = gkb.gkb_numerical_rank(to_dev(A), 1e-8, q1=to_dev(q))
    assert stats["one_pass_used"] == 1 and st2["one_pass_used"] == 0
    assert rank == l and rank_s == l and rank2 == l and ref["rank"] == l


def test_team_sweep_timeout_path(monkeypatch):
    """The team sweep's bounded wait, forced from the host: with
    GKB_TEAM_STALL_POLLS set every wait gives up after a few polls (as when a
    member never runs) while every kernel runs to its end.  The solve returns
    GKB_ERR_TIMEOUT, the product pair returns NaN; without the setting the
    next solve on the same matrix is normal (the mailbox is reset per solve)."""
    import torch
    device()
    banner("team sweep timeout path (forced from the host)")
    A32, s, _, _ = inputs.lowrank_noise(300, 30000, 40, 0.9, 1e-6, seed=21, dtype=np.float32)
    q = inputs.start_vector(300, seed=4)
    Ad = to_dev(A32)
    monkeypatch.setenv("GKB_TEAM_STALL_POLLS", "8")
    with pytest.raises(gkb.GkbError) as ei:
        gkb.gkb_partial_svd(Ad, 4, 12, 1e-6, 5, q1=to_dev(q), one_pass=True)
    assert ei.value.status == -5
    w, y = gkb.gkb_matvec_fused(Ad, to_dev(np.ones(30000, dtype=np.float32)))
    torch.cuda.synchronize()
    assert torch.isnan(w).all().item() and torch.isnan(y).all().item()
    monkeypatch.delenv("GKB_TEAM_STALL_POLLS")
    ref = gk.partial_svd(A32.astype(np.float64), 4, 12, 1e-6, 5, q, eps_break=1e-6)
    sigma, U, V, status, stats = run(A32, 4, 12, 1e-6, 5, q, one_pass=True)
    assert status == ref["status"] == 0 and stats["one_pass_used"] == 1
    _check_against(ref, sigma, U, V, 12)
