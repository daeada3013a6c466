"""Sparse A: the binned CSR products and the partial SVD against the float64
oracle (scipy CSR), through the C ABI."""
import numpy as np
import pytest

from oracle import checks, gk
from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("scipy.sparse")

U32 = 2.0 ** -24


def csr_of(S):
    return sp.csr_matrix((S["val"].astype(np.float64), S["col_idx"], S["row_ptr"]), shape=(S["m"], S["n"]))


def one_long_row(m, n, seed):
    """Power-law rows plus one full row and one full column (the medium-row
    wave path, and the chunked path when a row has more than 4096 entries)."""
    S = inputs.sparse_powerlaw(m, n, 4 * m, seed=seed)
    A = csr_of(S).tolil()
    A[m // 2, :] = np.linspace(-1, 1, n)
    A[:, n // 3] = np.linspace(1, 2, m)[:, None]
    A = A.tocsr().astype(np.float32)
    A.sort_indices()
    T = A.T.tocsr()
    T.sort_indices()
    return {"m": m, "n": n, "nnz": A.nnz, "row_ptr": A.indptr.astype(np.int64), "col_idx": A.indices.astype(np.int32),
            "val": A.data.astype(np.float32), "col_ptr": T.indptr.astype(np.int64),
            "row_idx": T.indices.astype(np.int32), "val_t": T.data.astype(np.float32)}


def empty_matrix(m, n):
    z32 = np.zeros(0, dtype=np.int32)
    zf = np.zeros(0, dtype=np.float32)
    return {"m": m, "n": n, "nnz": 0, "row_ptr": np.zeros(m + 1, np.int64), "col_idx": z32, "val": zf,
            "col_ptr": np.zeros(n + 1, np.int64), "row_idx": z32, "val_t": zf}


CASES = {
    "powerlaw": lambda: inputs.sparse_powerlaw(5000, 2000, 100000, seed=1),
    "wide": lambda: inputs.sparse_powerlaw(700, 3000, 40000, seed=2),
    "permuted_diagonal": lambda: inputs.sparse_permuted_diagonal(3000, 1000, np.geomspace(1, 1e-3, 800), seed=3),
    "long_rows": lambda: one_long_row(2500, 3000, seed=4),
    "huge_row": lambda: one_long_row(600, 10000, seed=6),
    "empty": lambda: empty_matrix(300, 200),
    # several column panels (28672 columns each) in A p, in A^T q, and a full
    # row of 70000 entries whose panel segments are cut into chunks
    "multipanel": lambda: inputs.sparse_powerlaw(300, 100000, 60000, seed=9),
    "multipanel_tall": lambda: inputs.sparse_powerlaw(100000, 300, 400000, seed=10),
    "multipanel_long": lambda: one_long_row(600, 70000, seed=12),
}


@pytest.mark.parametrize("layout", ["csr", "panels"])
@pytest.mark.parametrize("name", list(CASES))
def test_sparse_matvec(name, layout):
    device()
    S = CASES[name]()
    banner(f"sparse matvec {name} {S['m']}x{S['n']} nnz={S['nnz']} {layout}")
    plan = gkb.SparsePlan(S["m"], S["n"], S, panels=layout == "panels")
    assert plan.panels == (3 if layout == "panels" else 0), plan.panels
    A = csr_of(S)
    rng = np.random.default_rng(7)
    for trans in (0, 1):
        x = rng.standard_normal(S["m"] if trans else S["n"]).astype(np.float32)
        y = to_host(plan.matvec(to_dev(x), trans))
        M = A.T if trans else A
        ref = M @ x.astype(np.float64)
        # recursive-summation bound over the stored entries (duplicates
        # included): (length + 1) u32 sum_j |val_j x_idx_j| per row
        ptr, idx, val = ((S["col_ptr"], S["row_idx"], S["val_t"]) if trans else
                         (S["row_ptr"], S["col_idx"], S["val"]))
        lens = np.diff(ptr)
        rows = np.repeat(np.arange(lens.size), lens)
        absum = np.bincount(rows, weights=np.abs(val.astype(np.float64) * x[idx].astype(np.float64)),
                            minlength=lens.size)
        bound = (lens + 1) * U32 * absum + 1e-300
        assert np.all(np.abs(y - ref) <= bound), (trans, np.max(np.abs(y - ref) - bound))
        y2 = to_host(plan.matvec(to_dev(x), trans))
        assert np.array_equal(y, y2)
    plan.close()


def test_sparse_plan_rejects_invalid_arrays():
    device()
    banner("sparse plan validation")
    S = inputs.sparse_powerlaw(400, 300, 5000, seed=5)
    bad = dict(S, col_idx=S["col_idx"].copy())
    bad["col_idx"][17] = 300                     # column out of range
    with pytest.raises(gkb.GkbError):
        gkb.SparsePlan(400, 300, bad)
    bad = dict(S, row_idx=S["row_idx"].copy())
    bad["row_idx"][5] = -1                       # row of A^T out of range
    with pytest.raises(gkb.GkbError):
        gkb.SparsePlan(400, 300, bad)
    bad = dict(S, row_ptr=S["row_ptr"].copy())
    bad["row_ptr"][10], bad["row_ptr"][11] = bad["row_ptr"][11] + 5, bad["row_ptr"][10]   # decreasing
    with pytest.raises(gkb.GkbError):
        gkb.SparsePlan(400, 300, bad)
    bad = dict(S, col_ptr=S["col_ptr"].copy())
    bad["col_ptr"][-1] -= 1                      # does not end at nnz
    with pytest.raises(gkb.GkbError):
        gkb.SparsePlan(400, 300, bad)


def bound32(A):
    return np.sqrt(max(A.shape)) * U32 * sp.linalg.norm(A)


@pytest.mark.parametrize("name,r,k,check_every,layout", [
    ("powerlaw", 10, 40, 0, "panels"), ("powerlaw", 10, 40, 5, "panels"), ("powerlaw", 10, 40, 5, "csr"),
    ("wide", 6, 30, 3, "panels"), ("permuted_diagonal", 5, 20, 0, "panels"), ("long_rows", 8, 30, 4, "panels"),
    ("huge_row", 6, 25, 0, "panels"), ("huge_row", 6, 25, 0, "csr"), ("multipanel", 6, 30, 0, "panels"),
    ("multipanel_tall", 6, 30, 5, "panels"), ("multipanel_long", 6, 25, 0, "panels")])
def test_sparse_partial_svd_against_oracle(name, r, k, check_every, layout):
    import scipy.sparse.linalg  # noqa: F401  (sp.linalg.norm)
    device()
    S = CASES[name]()
    banner(f"sparse partial svd {name} r={r} k={k} check_every={check_every} {layout}")
    A = csr_of(S)
    q = inputs.start_vector(S["m"], seed=11)
    ref = gk.partial_svd(A, r, k, 1e-6, 30, q, eps_break=1e-6, check_every=check_every)
    plan = gkb.SparsePlan(S["m"], S["n"], S, panels=layout == "panels")
    assert plan.panels == (3 if layout == "panels" else 0), plan.panels
    sig, Ut, Vt, status, st = plan.partial_svd(r, k, 1e-6, 30, q1=to_dev(q), check_every=check_every)
    ne = ref["sigma"].size
    assert status == ref["status"], (status, ref["status"])
    assert abs(st["restarts"] - ref["restarts"]) <= 1
    err = np.max(np.abs(sig[:ne] - ref["sigma"]))
    print(f"  sigma err {err:.2e} (bound {bound32(A):.2e}), matvecs {st['matvecs']} (oracle {ref['matvecs']})",
          flush=True)
    assert err <= bound32(A)
    U = to_host(Ut).T[:, :ne].astype(np.float64)
    V = to_host(Vt).T[:, :ne].astype(np.float64)
    r1 = np.linalg.norm(A @ V - U * sig[:ne], axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sig[:ne], axis=0)
    assert np.max(r1) <= 100 * bound32(A) and np.max(r2) <= 1e-6 * sig[0] + 100 * bound32(A)
    al = checks.alignment(U, V, ref["U"], ref["V"])
    assert np.min(al) > 1 - 1e-4, np.min(al)
    if name == "permuted_diagonal":
        want = np.geomspace(1, 1e-3, 800)[:r]
        assert np.max(np.abs(sig - want) / want) < 1e-6
    plan.close()


def test_sparse_fullsize_against_stored_oracle():
    """The full sparse workload (1000000 x 200000, 5e7 entries, power-law
    degrees) against the oracle's stored top 20 (written by
    tests/golden/make_sparse_reference.py from oracle code only), plus the
    residuals of the returned triplets computed in float64 on the host."""
    import json
    import os
    import scipy.sparse.linalg  # noqa: F401
    device()
    path = os.path.join(os.path.dirname(__file__), "golden", "sparse_oracle_top20.json")
    ref = json.load(open(path))
    banner("sparse full size 1000000x200000 nnz 5e7, r=20 k=60 check_every=5")
    S = inputs.sparse_powerlaw(1000000, 200000, 50000000, seed=7)
    plan = gkb.SparsePlan(1000000, 200000, S)
    assert plan.panels == 3, plan.panels
    q = inputs.start_vector(1000000, seed=8)
    sig, Ut, Vt, status, st = plan.partial_svd(20, 60, 1e-6, 50, q1=to_dev(q), check_every=5)
    A = csr_of(S)
    del S
    want = np.array(ref["sigma"])
    bound = bound32(A)
    err = np.max(np.abs(sig - want))
    print(f"  sparse full size: sigma err {err:.2e} (bound {bound:.2e}), matvecs {st['matvecs']} "
          f"(oracle {ref['matvecs']}), restarts {st['restarts']} (oracle {ref['restarts']})", flush=True)
    assert status == ref["status"] == 0
    assert err <= bound
    assert abs(st["restarts"] - ref["restarts"]) <= 1
    U = to_host(Ut).T.astype(np.float64)
    V = to_host(Vt).T.astype(np.float64)
    r1 = np.linalg.norm(A @ V - U * sig, axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sig, axis=0)
    print(f"  residuals ||Av - su|| {r1.max():.2e}, ||A^T u - s v|| {r2.max():.2e} (tol s1 {1e-6 * sig[0]:.2e})",
          flush=True)
    assert r1.max() <= 100 * bound and r2.max() <= 1e-6 * sig[0] + 100 * bound
    plan.close()
