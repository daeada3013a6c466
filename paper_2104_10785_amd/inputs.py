"""Seeded synthetic inputs for the partial-SVD / numerical-rank workloads.

This module only draws random numbers and builds test matrices; it holds none
of the Golub-Kahan arithmetic. Both the CPU oracle side and the GPU side of the
tests and of the benchmark take their inputs from here, so that the two are
always fed bit-identical data.

Workloads (all synthetic, every seed fixed):

* ``svd_matrix``      A = Q1 diag(s) Q2^T with Haar-random orthonormal factors
                      (a matrix with a prescribed spectrum, so every singular
                      value is known in closed form).
* ``product_matrix``  A = M N with Gaussian M (m x l), N (l x n): the exact
                      rank-l inputs of the paper's experiments (Section 5).
* ``lowrank_noise``   A = U_f diag(decay^i) V_f^T + E, E iid Gaussian: the
                      large low-rank-plus-noise matrix, built in row blocks
                      with one child seed per block so the result does not
                      depend on the number of threads.
* ``start_vector``    the N(2, 1) start vector of Algorithm 1.
* ``batch_problems``  many small uneven matrices with geometric spectra.
* ``drift_sequence``  a slowly changing matrix sequence A_t = A_{t-1} + dA_t.
* ``sparse_powerlaw``  a sparse matrix with power-law row and column degrees
                      (CSR of A and of A^T); ``sparse_permuted_diagonal`` a
                      sparse matrix with a known spectrum.
* ``similarity_pairs`` labelled pairs (x, v, y) from two synthetic domains
                      for the similarity-learning workload, and
                      ``rank_r_point`` a point W = U diag(s) V^T of the
                      rank-r manifold.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """m x n (n <= m) matrix with orthonormal columns, Haar-distributed.

    QR of a Gaussian matrix with each column multiplied by the sign of the
    matching diagonal entry of R (Mezzadri's correction), so the distribution
    is exactly Haar and the result is a deterministic function of the draw.
    """
    if n > m:
        raise ValueError("haar: need n <= m")
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def geometric_spectrum(count: int, ratio: float, first_power: int = 1) -> np.ndarray:
    """s_i = ratio ** (i - 1 + first_power) for i = 1..count."""
    return ratio ** np.arange(first_power, first_power + count, dtype=np.float64)


def decade_spectrum(count: int = 1000, per_decade: float = 100.0) -> np.ndarray:
    """s_i = 10 ** (-i / per_decade), i = 1..count (1-based index)."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return 10.0 ** (-i / per_decade)


def svd_matrix(m: int, n: int, s: np.ndarray, seed: int):
    """A = Q1 diag(s) Q2^T in float64, with Q1 (m x p), Q2 (n x p), p = len(s).

    Returns (A, Q1, Q2). The singular values of A are s (up to rounding) and
    its singular vectors are the columns of Q1 and Q2.
    """
    s = np.asarray(s, dtype=np.float64)
    p = s.shape[0]
    if p > min(m, n):
        raise ValueError("svd_matrix: len(s) > min(m, n)")
    rng = _rng(seed)
    q1 = haar(rng, m, p)
    q2 = haar(rng, n, p)
    a = (q1 * s[None, :]) @ q2.T
    return a, q1, q2


def product_matrix(m: int, n: int, l: int, seed: int) -> np.ndarray:
    """A = M N, M (m x l) and N (l x n) iid standard Gaussian: rank exactly l."""
    rng = _rng(seed)
    mm = rng.standard_normal((m, l))
    nn = rng.standard_normal((l, n))
    return mm @ nn


def start_vector(m: int, seed: int, mean: float = 2.0, std: float = 1.0) -> np.ndarray:
    """The start vector q ~ N(2, 1)^m of Algorithm 1 (float64, unnormalised)."""
    return _rng(seed).normal(mean, std, m)


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def lowrank_noise(m: int, n: int, rank: int, decay: float, noise_std: float,
                  seed: int, dtype=np.float32, block_rows: int = 1000,
                  threads: int | None = None):
    """A = U_f diag(decay^i)_{i=1..rank} V_f^T + E, stored in `dtype`.

    U_f (m x rank) and V_f (n x rank) are Haar; E has iid N(0, noise_std^2)
    entries. The low-rank part and the noise are formed in float64 row block
    by row block, then rounded once to `dtype`. Each row block draws its noise
    from its own child seed, so the matrix is the same for any thread count.

    Returns (A, s, U_f, V_f) with s the prescribed spectrum of the low-rank
    part.
    """
    root = np.random.SeedSequence(seed)
    kid_factors, kid_noise = root.spawn(2)
    frng = np.random.default_rng(kid_factors)
    uf = haar(frng, m, rank)
    vf = haar(frng, n, rank)
    s = decay ** np.arange(1, rank + 1, dtype=np.float64)
    us = uf * s[None, :]
    vft = np.ascontiguousarray(vf.T)
    nblk = (m + block_rows - 1) // block_rows
    seeds = kid_noise.spawn(nblk)
    out = np.empty((m, n), dtype=dtype)

    def work(b):
        r0 = b * block_rows
        r1 = min(m, r0 + block_rows)
        blk = us[r0:r1] @ vft
        if noise_std != 0.0:
            g = np.random.default_rng(seeds[b]).standard_normal((r1 - r0, n))
            blk += noise_std * g
        out[r0:r1] = blk.astype(dtype)

    nt = threads or _threads()
    if nt == 1:
        for b in range(nblk):
            work(b)
    else:
        with _cf.ThreadPoolExecutor(nt) as ex:
            list(ex.map(work, range(nblk)))
    return out, s, uf, vf


def batch_problems(count: int, seed: int, m_range=(500, 4000), n_range=(200, 2000),
                   ratio_range=(0.8, 0.99), r_range=(5, 20), dtype=np.float32,
                   materialize: bool = True):
    """Many small uneven dense problems with geometric spectra.

    Problem i has m_i ~ U{m_range}, n_i ~ U{n_range}, ratio rho_i ~ U[ratio_range),
    r_i ~ U{r_range}, and A_i = Q1 diag(rho_i^(j-1))_{j=1..n_i} Q2^T (m_i >= n_i is
    not required; the spectrum has min(m_i, n_i) entries).

    Returns a list of dicts {m, n, rho, r, seed, A (if materialize)}.
    """
    rng = _rng(seed)
    specs = []
    for i in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        rho = float(rng.uniform(ratio_range[0], ratio_range[1]))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        specs.append({"m": m, "n": n, "rho": rho, "r": r, "seed": seed * 100003 + i})
    if materialize:
        for sp in specs:
            sp["A"] = batch_matrix(sp, dtype)
    return specs


def batch_matrix(spec, dtype=np.float32) -> np.ndarray:
    """Materialise one problem of `batch_problems`."""
    m, n, rho = spec["m"], spec["n"], spec["rho"]
    p = min(m, n)
    s = rho ** np.arange(p, dtype=np.float64)
    a, _, _ = svd_matrix(m, n, s, spec["seed"])
    return a.astype(dtype)


def drift_base(m: int, n: int, ratio: float, seed: int, dtype=np.float32):
    """A_0 = Q1 diag(ratio^(i-1))_{i=1..n} Q2^T (float64 factors, rounded once)."""
    s = ratio ** np.arange(min(m, n), dtype=np.float64)
    a, _, _ = svd_matrix(m, n, s, seed)
    return a.astype(dtype), s


def drift_update(m: int, n: int, rank: int, scale: float, seed: int, step: int) -> np.ndarray:
    """dA_t = scale * G1 G2^T with G1 ~ N(0, 1/m) (m x rank), G2 ~ N(0, 1/n) (n x rank).

    The 1/m and 1/n variances make ||dA_t||_2 about `scale`, so the sequence
    changes slowly relative to a unit top singular value.
    """
    ss = np.random.SeedSequence([seed, step])
    rng = np.random.default_rng(ss)
    g1 = rng.standard_normal((m, rank)) / np.sqrt(m)
    g2 = rng.standard_normal((n, rank)) / np.sqrt(n)
    return scale * (g1 @ g2.T)


def sketch_matrix(n: int, width: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Gaussian test matrix Omega (n x width) for the sketch A Omega."""
    return _rng(seed).standard_normal((n, width)).astype(dtype)


def batch_matrix_torch(spec, device, dtype=None):
    """Materialise one problem of `batch_problems` on a GPU with torch.

    Same construction as `batch_matrix` (Haar factors from the QR of a
    Gaussian with the sign correction, spectrum rho^(j-1)), drawn from torch's
    device generator seeded with the problem's seed, in float64, rounded once
    to float32.  Used where hundreds of large problems must be generated
    quickly; the matrix is a deterministic function of (seed, device type).
    """
    import torch
    dtype = dtype or torch.float32
    m, n, rho = spec["m"], spec["n"], spec["rho"]
    p = min(m, n)
    g = torch.Generator(device=device)
    g.manual_seed(int(spec["seed"]))

    def haar_t(rows):
        z = torch.randn(rows, p, generator=g, device=device, dtype=torch.float64)
        q, r = torch.linalg.qr(z)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    q1 = haar_t(m)
    q2 = haar_t(n)
    s = rho ** torch.arange(p, device=device, dtype=torch.float64)
    return ((q1 * s[None, :]) @ q2.T).to(dtype).contiguous()


def drift_base_torch(m: int, n: int, ratio: float, seed: int, device, dtype=None):
    """A_0 = Q1 diag(ratio^(i-1))_{i=1..min(m,n)} Q2^T on a GPU (Haar factors
    from torch's seeded device generator, float64, rounded once)."""
    import torch
    dtype = dtype or torch.float32
    p = min(m, n)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))

    def haar_t(rows):
        z = torch.randn(rows, p, generator=g, device=device, dtype=torch.float64)
        q, r = torch.linalg.qr(z)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d[None, :]

    q1 = haar_t(m)
    q2 = haar_t(n)
    s = ratio ** torch.arange(p, device=device, dtype=torch.float64)
    return ((q1 * s[None, :]) @ q2.T).to(dtype).contiguous()


def drift_update_torch(m: int, n: int, rank: int, scale: float, seed: int, step: int, device, dtype=None):
    """dA_t = scale * G1 G2^T with G1 ~ N(0, 1/m) (m x rank), G2 ~ N(0, 1/n)
    (n x rank), drawn on a GPU from a generator seeded by (seed, step)."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + int(step))
    g1 = torch.randn(m, rank, generator=g, device=device, dtype=torch.float64) / np.sqrt(m)
    g2 = torch.randn(n, rank, generator=g, device=device, dtype=torch.float64) / np.sqrt(n)
    return (scale * (g1 @ g2.T)).to(dtype)


def mlp_init(n_in: int, hidden: int, seed: int) -> np.ndarray:
    """Initial network parameters [W1 | b1 | w2 | b2] (float32): W1 ~ N(0, 2/n_in)
    (He), w2 ~ N(0, 1/hidden), biases 0."""
    rng = _rng(seed)
    w1 = rng.standard_normal(hidden * n_in) * np.sqrt(2.0 / n_in)
    w2 = rng.standard_normal(hidden) * np.sqrt(1.0 / hidden)
    return np.concatenate([w1, np.zeros(hidden), w2, [0.0]]).astype(np.float32)


def _csr_transpose(m: int, n: int, row_ptr: np.ndarray, col_idx: np.ndarray, val: np.ndarray):
    """CSR arrays of A^T from those of A (entries of a row of A^T in increasing
    row order of A, repeats kept; pure data movement by a counting sort)."""
    try:
        import scipy.sparse as sp
        A = sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n))
        T = A.tocsc()          # stable counting sort; keeps repeated entries
        return T.indptr.astype(np.int64), T.indices.astype(np.int32), T.data.astype(np.float32)
    except ImportError:
        rows = np.repeat(np.arange(m, dtype=np.int32), np.diff(row_ptr))
        order = np.argsort(col_idx, kind="stable")
        col_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(col_idx, minlength=n), out=col_ptr[1:])
        return col_ptr, rows[order].astype(np.int32), val[order]


def sparse_powerlaw(m: int, n: int, nnz: int, seed: int, row_exp: float = 0.6, col_exp: float = 0.5):
    """A sparse m x n float32 matrix with power-law degrees, as CSR of A and of A^T.

    Row i (in a random order) gets about nnz * w_i / sum(w) entries with
    w_i = (rank + 1)^-row_exp (rounded down, so some rows are empty; the
    remainder goes to the heaviest rows); the column of each entry is drawn
    independently from the continuous power law with density proportional to
    (x + 1)^-col_exp on [0, n) (inverse CDF, rounded down) mapped through a
    random order of the columns; values are N(0, 1).  Duplicate (row, column)
    pairs can occur and stand for their sum.  Returns a dict with m, n, nnz,
    row_ptr (int64), col_idx (int32), val (float32), col_ptr, row_idx, val_t.
    """
    rng = _rng(seed)
    w = (np.arange(1, m + 1, dtype=np.float64)) ** (-row_exp)
    deg = np.floor(nnz * w / w.sum()).astype(np.int64)
    short = nnz - int(deg.sum())
    deg[:short] += 1
    deg = deg[rng.permutation(m)]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    g = 1.0 - col_exp                       # col_exp < 1
    span = (n + 1.0) ** g - 1.0
    col_perm = rng.permutation(n).astype(np.int32)
    col_idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float32)
    step = 1 << 24
    for a in range(0, nnz, step):
        b = min(nnz, a + step)
        x = (1.0 + rng.random(b - a) * span) ** (1.0 / g) - 1.0
        col_idx[a:b] = col_perm[np.minimum(x.astype(np.int64), n - 1)]
        val[a:b] = rng.standard_normal(b - a, dtype=np.float32)
    col_ptr, row_idx, val_t = _csr_transpose(m, n, row_ptr, col_idx, val)
    return {"m": m, "n": n, "nnz": nnz, "row_ptr": row_ptr, "col_idx": col_idx, "val": val,
            "col_ptr": col_ptr, "row_idx": row_idx, "val_t": val_t}


def sparse_permuted_diagonal(m: int, n: int, s: np.ndarray, seed: int):
    """A = P diag(s) Q^T with random permutations P, Q (s of length <= min(m, n)):
    sparse, one entry per row and column at most, singular values |s| exactly."""
    rng = _rng(seed)
    s = np.asarray(s, dtype=np.float32)
    k = s.size
    rows = rng.permutation(m)[:k]
    cols = rng.permutation(n)[:k].astype(np.int32)
    order = np.argsort(rows, kind="stable")
    rows, cols, vals = rows[order], cols[order], s[order]
    deg = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col_ptr, row_idx, val_t = _csr_transpose(m, n, row_ptr, cols, vals)
    return {"m": m, "n": n, "nnz": k, "row_ptr": row_ptr, "col_idx": cols, "val": vals,
            "col_ptr": col_ptr, "row_idx": row_idx, "val_t": val_t}


def similarity_pairs(count: int, d1: int, d2: int, seed: int, proto_seed: int = 0, classes: int = 10,
                     same: float = 0.5, noise: float = 1.0):
    """Labelled pairs from two domains with shared classes (a synthetic stand-in
    for two image datasets of different sizes).  Class c has a prototype with
    N(0, 1/d) entries in each domain; a sample of class c is its prototype plus
    noise * N(0, 1/d) per entry.  A pair takes a class for x and, with
    probability `same`, the same class for v (label +1), else another class
    (label -1).  The prototypes come from `proto_seed` (shared by a training
    and a held-out draw), the samples from `seed`.  Returns X (count x d1),
    V (count x d2), y (count,) as float32 and the two class vectors."""
    prng = _rng(proto_seed)
    px = prng.standard_normal((classes, d1)) / np.sqrt(d1)
    pv = prng.standard_normal((classes, d2)) / np.sqrt(d2)
    rng = _rng(seed)
    cx = rng.integers(0, classes, count)
    is_same = rng.random(count) < same
    cv = np.where(is_same, cx, (cx + rng.integers(1, classes, count)) % classes)
    X = px[cx] + noise * rng.standard_normal((count, d1)) / np.sqrt(d1)
    V = pv[cv] + noise * rng.standard_normal((count, d2)) / np.sqrt(d2)
    y = np.where(is_same, 1.0, -1.0)
    return X.astype(np.float32), V.astype(np.float32), y.astype(np.float32), cx, cv


def rank_r_point(d1: int, d2: int, r: int, seed: int, scale: float = 1.0):
    """W = U diag(s) V^T on the rank-r manifold: Haar U (d1 x r), V (d2 x r),
    s = scale * sorted |N(0, 1)| + scale (distinct, descending)."""
    rng = _rng(seed)
    U = haar(rng, d1, r)
    V = haar(rng, d2, r)
    s = scale * (np.sort(np.abs(rng.standard_normal(r)))[::-1] + 1.0)
    return U, s, V
