"""Numerical rank from the Golub-Kahan bidiagonal (Section 3.2, Algorithm 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 3 runs Algorithm 1 with k = min(m, n) and counts the eigenvalues of
B^T B above epsilon. Readings used here:
* the threshold tau is on singular values (B^T B's eigenvalues are sigma**2),
  relative to sigma_1(B) unless `tau_relative` is False, and the comparison is
  strict (values that exceed tau);
* k_max is a parameter (default min(m, n)); the breakdown test of the
  bidiagonalization stops the recurrence near the rank on gapped spectra.

Two independent counts are produced: the number of singular values of B above
tau (LAPACK SVD of the small matrix) and a Sylvester-inertia count on the
Golub-Kahan tridiagonal, whose eigenvalues are +-sigma_i(B) (and zeros), so the
number of its eigenvalues above tau is the number of sigma_i(B) above tau.
"""
from __future__ import annotations

import numpy as np

from . import gk


def gk_tridiagonal_offdiag(H: np.ndarray) -> np.ndarray:
    """Off-diagonal (alpha_1, beta_2, alpha_2, beta_3, ...) of the zero-diagonal
    symmetric tridiagonal that is the perfect-shuffle permutation of
    [[0, B], [B^T, 0]] for a lower bidiagonal B (nq x np, nq in {np, np+1})."""
    nq, np_ = H.shape
    e = []
    for j in range(np_):
        e.append(H[j, j])
        if j + 1 < nq:
            e.append(H[j + 1, j])
    return np.asarray(e, dtype=np.float64)


def count_above(offdiag: np.ndarray, tau: float) -> int:
    """Number of eigenvalues > tau (tau > 0) of the symmetric tridiagonal T
    with zero diagonal and the given off-diagonal.

    Sylvester's law of inertia on T - tau I = L D L^T: the number of negative
    pivots d_i equals the number of eigenvalues below tau. A zero pivot is
    replaced by a tiny negative number (the usual Sturm-sequence convention).
    """
    if tau <= 0:
        raise ValueError("tau must be positive")
    e = np.asarray(offdiag, dtype=np.float64)
    order = e.size + 1
    tiny = np.finfo(np.float64).tiny
    below = 0
    d = -tau
    if d < 0:
        below += 1
    for i in range(e.size):
        if d == 0.0:
            d = -tiny
        d = -tau - e[i] * e[i] / d
        if d < 0:
            below += 1
    return order - below


def numerical_rank(A, tau: float, q, k_max: int = 0, eps_break: float | None = None,
                   eps_relative: bool = True, tau_relative: bool = True, passes: int = 2):
    """Numerical rank #{sigma_i > tau} via Golub-Kahan (Algorithm 3, reading above).

    Returns a dict with rank (SVD count), rank_sturm (inertia count), sigma
    (all singular values of B), steps (completed Bidiag 1 steps), breakdown and
    the threshold actually used.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    k = k_max if k_max else min(m, n)
    if not (1 <= k <= min(m, n)):
        raise ValueError("need 1 <= k_max <= min(m, n)")
    eps = gk.BreakThreshold(gk.default_eps_break() if eps_break is None else eps_break,
                            eps_relative)
    fac = gk.first_cycle(A, np.asarray(q, dtype=np.float64), k, eps, passes)
    H = fac.H
    if H.shape[1] == 0:
        return {"rank": 0, "rank_sturm": 0, "sigma": np.zeros(0), "steps": 0,
                "breakdown": fac.breakdown, "threshold": tau, "H": H}
    s = np.linalg.svd(H, compute_uv=False)
    thr = tau * s[0] if tau_relative else tau
    rank_svd = int(np.count_nonzero(s > thr))
    rank_sturm = count_above(gk_tridiagonal_offdiag(H), thr)
    return {"rank": rank_svd, "rank_sturm": rank_sturm, "sigma": s, "steps": H.shape[1],
            "breakdown": fac.breakdown, "threshold": thr, "H": H}
