"""The oracle on sparse matrices (scipy CSR kept sparse): pinned to a sparse
matrix with a known spectrum, to the same oracle on the dense form, and to
the summed matrix when entries repeat; plus the transpose built by the input
generator."""
import numpy as np
import pytest

from oracle import gk
from paper_2104_10785_amd import inputs

sp = pytest.importorskip("scipy.sparse")


def csr_of(S, transpose=False):
    if transpose:
        return sp.csr_matrix((S["val_t"].astype(np.float64), S["row_idx"], S["col_ptr"]), shape=(S["n"], S["m"]))
    return sp.csr_matrix((S["val"].astype(np.float64), S["col_idx"], S["row_ptr"]), shape=(S["m"], S["n"]))


def test_permuted_diagonal_spectrum_in_closed_form():
    s = np.geomspace(1.0, 1e-2, 150).astype(np.float32)
    S = inputs.sparse_permuted_diagonal(300, 200, s, seed=4)
    A = csr_of(S)
    assert A.nnz == 150
    q = inputs.start_vector(300, seed=1)
    res = gk.partial_svd(A, 10, 40, 1e-10, 20, q)
    want = np.sort(np.abs(s.astype(np.float64)))[::-1][:10]
    assert res["status"] == 0
    assert np.max(np.abs(res["sigma"] - want) / want) < 1e-12
    # the vectors are signed unit vectors on the permuted coordinates
    U, V = res["U"], res["V"]
    assert np.allclose(np.sort(np.abs(U).max(axis=0)), 1.0, atol=1e-8)
    assert np.allclose(np.sort(np.abs(V).max(axis=0)), 1.0, atol=1e-8)


def test_sparse_equals_dense():
    S = inputs.sparse_powerlaw(600, 300, 6000, seed=2)
    A = csr_of(S)
    q = inputs.start_vector(600, seed=3)
    a = gk.partial_svd(A, 8, 30, 1e-10, 30, q, check_every=5)
    b = gk.partial_svd(A.toarray(), 8, 30, 1e-10, 30, q, check_every=5)
    assert a["status"] == b["status"] == 0
    assert a["restarts"] == b["restarts"] and a["matvecs"] == b["matvecs"]
    assert np.max(np.abs(a["sigma"] - b["sigma"]) / b["sigma"]) < 1e-12


def test_repeated_entries_are_summed():
    rng = np.random.default_rng(0)
    m, n, nnz = 200, 120, 3000
    rows = np.sort(rng.integers(0, m, nnz))
    cols = rng.integers(0, n, nnz).astype(np.int32)
    cols[1::7] = cols[0::7][: len(cols[1::7])]   # force repeats of (row, col) pairs within rows
    rows[1::7] = rows[0::7][: len(rows[1::7])]
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    vals = rng.standard_normal(nnz)
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=ptr[1:])
    A = sp.csr_matrix((vals, cols, ptr), shape=(m, n))          # keeps the repeats
    D = np.zeros((m, n))
    np.add.at(D, (rows, cols), vals)
    q = inputs.start_vector(m, seed=5)
    a = gk.partial_svd(A, 5, 25, 1e-10, 30, q)
    b = gk.partial_svd(D, 5, 25, 1e-10, 30, q)
    assert np.max(np.abs(a["sigma"] - b["sigma"]) / b["sigma"]) < 1e-12


def test_generator_transpose_and_degrees():
    S = inputs.sparse_powerlaw(5000, 2000, 100000, seed=1)
    A, AT = csr_of(S), csr_of(S, transpose=True)
    assert abs(A.T - AT).max() == 0
    deg = np.diff(S["row_ptr"])
    assert deg.sum() == 100000 and deg.max() > 1024 and (deg <= 16).sum() > 1000
    # rows of A^T list their entries in increasing row order of A
    for j in range(0, 2000, 97):
        seg = S["row_idx"][S["col_ptr"][j]:S["col_ptr"][j + 1]]
        assert np.all(np.diff(seg) >= 0)
