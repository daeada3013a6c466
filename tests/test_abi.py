"""Host-side checks of the C ABI (no GPU): the library loads and exports every
declared symbol, arguments are rejected before any device work, and the
host float64 pieces (small SVD, inertia count) are right."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

from oracle import philox, rank as orank
from paper_2104_10785_amd import gkb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gkb_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = gkb.lib()
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert names <= set(gkb.EXPORTS)


def test_status_strings():
    L = gkb.lib()
    for code, name in gkb.STATUS.items():
        assert L.gkb_status_string(code).decode() == name


def _fake_matrix(m=100, n=50, dtype=gkb.GKB_F32, lda=None, data=0x1000):
    return gkb.GkbMatrix(m, n, lda or n, dtype, data, None, 0)


def _call_svd(mat, r, k, tol=1e-6, restarts=0, ws=None, wsb=0, sigma=True, U=0x2000, V=0x3000):
    L = gkb.lib()
    o = gkb.GkbOptions()
    L.gkb_default_options(C.byref(o))
    sig = (C.c_double * max(r, 1))() if sigma else None
    return L.gkb_partial_svd(C.byref(mat) if mat is not None else None, r, k, tol, restarts, C.byref(o), ws, wsb,
                             sig, U, V, None, None)


def test_validation_before_device_work():
    # All of these must be rejected on the host: no GPU is touched here.
    ERR = -1
    assert _call_svd(None, 2, 4) == ERR
    assert _call_svd(_fake_matrix(m=0), 2, 4) == ERR
    assert _call_svd(_fake_matrix(lda=10), 2, 4) == ERR
    assert _call_svd(_fake_matrix(dtype=7), 2, 4) == ERR
    assert _call_svd(_fake_matrix(data=None), 2, 4) == ERR
    assert _call_svd(_fake_matrix(), 0, 4) == ERR
    assert _call_svd(_fake_matrix(), 5, 4) == ERR
    assert _call_svd(_fake_matrix(), 2, 51) == ERR  # k > min(m, n)
    assert _call_svd(_fake_matrix(), 2, 4, tol=-1.0) == ERR
    assert _call_svd(_fake_matrix(), 2, 4, tol=float("nan")) == ERR
    assert _call_svd(_fake_matrix(), 2, 4, restarts=-1) == ERR
    assert _call_svd(_fake_matrix(), 2, 4, sigma=False) == ERR
    assert "k <= min(m, n)" in gkb.last_error() or gkb.last_error()
    # workspace errors
    assert _call_svd(_fake_matrix(), 2, 4, ws=None) == -4
    assert _call_svd(_fake_matrix(), 2, 4, ws=0x10001, wsb=1 << 40) == -4  # misaligned
    assert _call_svd(_fake_matrix(), 2, 4, ws=0x10000, wsb=16) == -4       # too small


def test_rank_validation():
    L = gkb.lib()
    mat = _fake_matrix()
    rk = C.c_int64()
    assert L.gkb_numerical_rank(C.byref(mat), 0.0, 1, 0, None, None, 0, C.byref(rk), None, None, None, None,
                                None) == -1
    assert L.gkb_numerical_rank(C.byref(mat), 1e-6, 1, 51, None, None, 0, C.byref(rk), None, None, None, None,
                                None) == -1
    assert L.gkb_numerical_rank(C.byref(mat), 1e-6, 1, 0, None, None, 0, None, None, None, None, None,
                                None) == -1


def test_workspace_size_query():
    L = gkb.lib()
    mat = _fake_matrix(50000, 20000, gkb.GKB_F32)
    ws = L.gkb_workspace_size(C.byref(mat), 50, 120, None)
    # two copies of each basis (restart) dominate: 2 * 121 * (50048 + 20032) * 4 bytes
    basis = 2 * 121 * (50048 + 20032) * 4
    assert basis < ws < basis + 64 * 2**20
    assert L.gkb_workspace_size(C.byref(mat), 50, 20001, None) == 0
    assert L.gkb_rank_workspace_size(C.byref(mat), 0, None) > 20001 * 50000 * 4


@pytest.mark.parametrize("shape", [(121, 120), (120, 120), (30, 45), (1, 1), (7, 1), (1, 9), (200, 3)])
def test_host_dense_svd_against_lapack(shape):
    rng = np.random.default_rng(sum(shape))
    H = rng.standard_normal(shape)
    X, s, Y = gkb.gkb_host_dense_svd(H)
    sl = np.linalg.svd(H, compute_uv=False)
    assert np.max(np.abs(s - sl)) < 1e-13 * sl[0]
    assert np.max(np.abs((X * s) @ Y.T - H)) < 1e-13 * sl[0]
    kk = min(shape)
    assert np.max(np.abs(X.T @ X - np.eye(kk))) < 1e-13
    assert np.max(np.abs(Y.T @ Y - np.eye(kk))) < 1e-13


def test_host_dense_svd_structured():
    # lower bidiagonal (first cycle) and arrowhead-triangular (restarted cycle)
    rng = np.random.default_rng(0)
    k, l = 60, 40
    B = np.zeros((k + 1, k))
    B[np.arange(k), np.arange(k)] = np.geomspace(1, 1e-12, k)
    B[np.arange(1, k + 1), np.arange(k)] = np.geomspace(0.5, 1e-13, k)
    H = np.zeros((k, k))
    H[:l, :l] = np.diag(np.sort(rng.uniform(0.1, 1, l))[::-1])
    H[:l, l] = rng.standard_normal(l) * 1e-3
    H[np.arange(l, k), np.arange(l, k)] = rng.uniform(0.01, 0.1, k - l)
    H[np.arange(l, k - 1), np.arange(l + 1, k)] = rng.uniform(0.01, 0.1, k - l - 1)
    for M in (B, H, np.zeros((5, 4))):
        X, s, Y = gkb.gkb_host_dense_svd(M)
        sl = np.linalg.svd(M, compute_uv=False)
        assert np.max(np.abs(s - sl)) <= 1e-14 * max(sl[0], 1e-300) * 10
        assert np.max(np.abs((X * s) @ Y.T - M)) <= 1e-14 * max(sl[0], 1e-300) * 10


@pytest.mark.parametrize("n", [1, 2, 5, 50, 70, 121])
def test_host_bidiag_lastrow_against_lapack(n):
    """The screening step of the in-cycle test: singular values and the last
    row of the left singular vectors of a first-cycle lower bidiagonal, against
    LAPACK's SVD of the same matrix (graded spectrum, distinct values)."""
    rng = np.random.default_rng(n)
    alpha = np.geomspace(1.0, 1e-3, n) * (1 + 0.05 * rng.random(n))
    beta = 0.4 * rng.random(n)
    B = np.zeros((n + 1, n))
    B[np.arange(n), np.arange(n)] = alpha
    B[np.arange(1, n + 1), np.arange(n)] = beta
    s, last = gkb.gkb_host_bidiag_lastrow(alpha, beta)
    U, sl, _ = np.linalg.svd(B, full_matrices=False)
    assert np.max(np.abs(s - sl)) < 1e-13 * sl[0]
    assert np.max(np.abs(np.abs(last) - np.abs(U[-1]))) < 1e-12
    # the same numbers as the full host SVD the driver falls back to
    X, sd, _ = gkb.gkb_host_dense_svd(B)
    assert np.max(np.abs(np.abs(last) - np.abs(X[-1]))) < 1e-12


def test_host_bidiag_lastrow_rejects_nan():
    with pytest.raises(gkb.GkbError):
        gkb.gkb_host_bidiag_lastrow([1.0, np.nan], [0.5, 0.5])


def test_host_dense_svd_rejects_nan():
    H = np.ones((3, 3))
    H[1, 1] = np.nan
    with pytest.raises(gkb.GkbError):
        gkb.gkb_host_dense_svd(H)


def test_host_inertia_count_matches_oracle_and_eigen():
    rng = np.random.default_rng(2)
    for np_ in [1, 2, 17, 90]:
        for nq in [np_, np_ + 1]:
            a = np.abs(rng.standard_normal(np_)) * np.geomspace(1, 1e-7, np_)
            b = np.abs(rng.standard_normal(max(nq - 1, 0))) * np.geomspace(1, 1e-7, max(nq - 1, 0))
            B = np.zeros((nq, np_))
            B[np.arange(np_), np.arange(np_)] = a
            if nq > 1:
                B[np.arange(1, nq), np.arange(nq - 1)] = b
            s = np.linalg.svd(B, compute_uv=False)
            for tau in [1e-8, 1e-5, 1e-2, 0.3]:
                want = int(np.count_nonzero(s > tau))
                assert gkb.gkb_host_bidiag_count_above(a, b, nq, tau) == want
                assert orank.count_above(orank.gk_tridiagonal_offdiag(B), tau) == want


def test_oracle_philox_known_answers():
    path = os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        words = philox.philox4x32_10([np.array([x], dtype=np.uint64) for x in v[:4]], (v[4], v[5]))
        assert [int(w[0]) for w in words] == v[6:]
    q = philox.start_vector(200000, 3)
    assert abs(q.mean() - 2.0) < 0.01 and abs(q.std() - 1.0) < 0.01


def _options(**kw):
    o = gkb.GkbOptions()
    gkb.lib().gkb_default_options(C.byref(o))
    for k2, v in kw.items():
        setattr(o, k2, v)
    return o


def test_one_pass_availability_and_workspace():
    """The one-sweep step needs float32 with n and lda multiples of 4 (bfloat16:
    8, float64: 2), n <= 262144 (float64: 131072; float32 rows longer than 24576
    and all float64 rows: team sweeps, with their exchange area in the
    workspace) and a 16-byte aligned A; for any other A a one_pass request
    takes the two-product step, so it passes the option checks (and here stops
    at the missing workspace) and its workspace is the two-product one.  The
    one-sweep workspace holds float64 bases and A^T Q."""
    L = gkb.lib()
    one = _options(one_pass=1)
    two = _options()
    sig = (C.c_double * 2)()

    def svd(mat):
        return L.gkb_partial_svd(C.byref(mat), 2, 4, 1e-6, 0, C.byref(one), None, 0, sig, 0x2000, 0x3000, None,
                                 None)
    others = [_fake_matrix(n=50),                       # n % 4
              _fake_matrix(n=52, lda=54),               # lda % 4
              _fake_matrix(n=52, data=0x1004),          # alignment
              _fake_matrix(n=51, dtype=gkb.GKB_F64),    # float64 needs n % 2
              _fake_matrix(n=131074, dtype=gkb.GKB_F64),  # float64 n > 131072
              _fake_matrix(n=52, dtype=gkb.GKB_BF16),   # bfloat16 needs n % 8
              _fake_matrix(m=100, n=262148)]            # n > 262144
    for bad in others:
        assert svd(bad) == -4 and "workspace" in gkb.last_error()
        assert L.gkb_workspace_size(C.byref(bad), 2, 4, C.byref(one)) == \
            L.gkb_workspace_size(C.byref(bad), 2, 4, C.byref(two)) > 0
        assert L.gkb_rank_workspace_size(C.byref(bad), 0, C.byref(one)) == \
            L.gkb_rank_workspace_size(C.byref(bad), 0, C.byref(two)) > 0
    good = _fake_matrix(50000, 20000, gkb.GKB_F32)
    w1 = L.gkb_workspace_size(C.byref(good), 50, 120, C.byref(one))
    w2 = L.gkb_workspace_size(C.byref(good), 50, 120, C.byref(two))
    # float64 bases (two copies) + two copies of A^T Q dominate
    assert w1 > 2 * 121 * (50048 + 20032) * 8 + 2 * 121 * 20032 * 8
    assert w1 > w2 > 0
    bf = _fake_matrix(100, 48, gkb.GKB_BF16)
    assert L.gkb_workspace_size(C.byref(bf), 2, 4, C.byref(one)) > 0
    # rows longer than one workgroup holds: team sweeps, whose exchange area
    # (one entry of two words per row and member) is in the workspace
    wide = _fake_matrix(20000, 80000, gkb.GKB_F32)
    assert L.gkb_workspace_size(C.byref(wide), 10, 40, C.byref(one)) > \
        L.gkb_workspace_size(C.byref(wide), 10, 40, C.byref(two)) + 20000 * 10 * 16
    # the building block takes the same shapes
    assert L.gkb_matvec_fused_workspace_size(C.byref(_fake_matrix(n=50))) == 0
    assert L.gkb_matvec_fused_workspace_size(C.byref(_fake_matrix(n=52))) > 0
    assert L.gkb_matvec_fused_workspace_size(C.byref(_fake_matrix(n=262148))) == 0
    # float64 A: the one-sweep step through teams, but not the float32-input building block
    f64 = _fake_matrix(2000, 1000, gkb.GKB_F64)
    assert L.gkb_workspace_size(C.byref(f64), 10, 30, C.byref(one)) > \
        L.gkb_workspace_size(C.byref(f64), 10, 30, C.byref(two)) > 0
    assert L.gkb_matvec_fused_workspace_size(C.byref(f64)) == 0
    assert L.gkb_matvec_fused_workspace_size(C.byref(wide)) >= 20000 * 10 * 16 + 80000 * 8


def test_embedded_heuristic_initialisation_reproduces_the_heuristic():
    """The network initialised by `_embedded_heuristic_init` computes exactly the
    heuristic start (its output equals the 2r-unit heuristic network's) for any
    features, before any training."""
    from paper_2104_10785_amd import learned

    def forward(params, hidden, X, n_in):
        W1 = params[: hidden * n_in].reshape(hidden, n_in)
        b1 = params[hidden * n_in: hidden * n_in + hidden]
        w2 = params[hidden * n_in + hidden: hidden * n_in + 2 * hidden]
        return np.maximum(X @ W1.T + b1, 0.0) @ w2 + params[-1]
    ws, r, hidden = 32, 30, 256
    n_in = ws + r
    p = learned._embedded_heuristic_init(ws, r, n_in, hidden, seed=5, scale=0.1).astype(np.float64)
    hp, hh = learned._heuristic_params(ws, r, n_in)
    X = np.random.default_rng(0).standard_normal((500, n_in))
    z = forward(p, hidden, X, n_in)
    zh = forward(hp.astype(np.float64), hh, X, n_in)
    assert np.max(np.abs(z - zh)) <= 1e-12 * np.max(np.abs(zh))
    # the heuristic network is sum_j x_{ws+j}: relu(x) - relu(-x) = x
    assert np.allclose(zh, X[:, ws:].sum(axis=1))
