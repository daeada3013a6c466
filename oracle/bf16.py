"""bfloat16 storage and the float32 Rayleigh-Ritz refinement.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``to_bf16_bits``: IEEE float32 -> bfloat16 (upper 16 bits) rounded to
  nearest, ties to even; NaN stays a quiet NaN.
* ``from_bf16_bits``: exact widening back to float64.
* ``rayleigh_ritz``: the Rayleigh-Ritz projection of eq. (5) for A^T A on the
  subspace spanned by the orthonormal columns of Vl: with A Vl = Q_W R (thin
  QR), the eigenvectors of Vl^T A^T A Vl = R^T R are the right singular
  vectors Y of R = X diag(s) Y^T, so the Ritz values are s, the right Ritz
  vectors Vl Y, and the left ones A Vl Y / s = Q_W X.
"""
from __future__ import annotations

import numpy as np


def to_bf16_bits(x) -> np.ndarray:
    """Round float32 values to bfloat16, returned as uint16 bit patterns."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    is_nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    q = ((u >> 16) | 0x0040) & 0xFFFF
    return np.where(is_nan, q, r).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    """Widen bfloat16 bit patterns to float64 exactly."""
    u = (np.asarray(b, dtype=np.uint32) << 16).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def rayleigh_ritz(A, Vl, r: int):
    """Top-r Ritz triplets of A from the right subspace span(Vl) (eq. (5))."""
    A = np.asarray(A, dtype=np.float64)
    W = A @ Vl
    Qw, R = np.linalg.qr(W)
    X, s, Yt = np.linalg.svd(R)
    return s[:r], Qw @ X[:, :r], Vl @ Yt.T[:, :r]


def refined_partial_svd(A32, r: int, k: int, tol: float, max_restarts: int, q, refine_dim: int = 0,
                        check_every: int = 0, eps_break: float = 1e-6):
    """The bfloat16 storage form followed by the float32 refinement.

    Golub-Kahan partial SVD (oracle.gk.partial_svd, float64 arithmetic) of the
    bfloat16 rounding of A32; the top d Ritz vectors of its final projected
    matrix (d = refine_dim, default 2 r, at most the Krylov dimension) then
    span the Rayleigh-Ritz projection with A32 itself (eq. (5)).
    Returns (unrefined result dict, (sigma, U, V) refined, d).
    """
    from . import gk
    A32 = np.asarray(A32, dtype=np.float32)
    A16 = from_bf16_bits(to_bf16_bits(A32))
    out = gk.partial_svd(A16, r, k, tol, max_restarts, q, eps_break=eps_break, check_every=check_every)
    fac = out["factorization"]
    X, s, Y = gk.ritz(fac.H)
    d = refine_dim if refine_dim > 0 else 2 * r
    d = max(out["sigma"].size, min(d, s.size))
    Vd = fac.P @ Y[:, :d]
    return out, rayleigh_ritz(A32.astype(np.float64), Vd, out["sigma"].size), d
