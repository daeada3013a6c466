"""Brute-force one-sided Jacobi SVD (Hestenes), the pin for tiny inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Columns of the working matrix are rotated in pairs until every pair is
orthogonal to working precision; the column norms are then the singular values
(Demmel and Veselic, "Jacobi's method is more accurate than QR", 1992). Plain
Python loops: meant for matrices up to a few dozen rows and columns.
"""
from __future__ import annotations

import numpy as np


def jacobi_svd(A, tol: float = 1e-15, max_sweeps: int = 60):
    """Thin SVD A = U diag(s) V^T, s descending. Returns (U, s, V)."""
    A = np.array(A, dtype=np.float64)
    transposed = A.shape[0] < A.shape[1]
    if transposed:
        A = A.T.copy()
    m, n = A.shape
    W = A.copy()
    V = np.eye(n)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(n - 1):
            for j in range(i + 1, n):
                a = float(W[:, i] @ W[:, i])
                b = float(W[:, j] @ W[:, j])
                c = float(W[:, i] @ W[:, j])
                if c == 0.0 or abs(c) <= tol * np.sqrt(a * b):
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * c)
                t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                if zeta == 0.0:
                    t = 1.0
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = cs * t
                wi = W[:, i].copy()
                W[:, i] = cs * wi - sn * W[:, j]
                W[:, j] = sn * wi + cs * W[:, j]
                vi = V[:, i].copy()
                V[:, i] = cs * vi - sn * V[:, j]
                V[:, j] = sn * vi + cs * V[:, j]
        if not rotated:
            break
    s = np.sqrt(np.einsum("ij,ij->j", W, W))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    W = W[:, order]
    V = V[:, order]
    U = np.zeros_like(W)
    for j in range(n):
        if s[j] > 0:
            U[:, j] = W[:, j] / s[j]
    if transposed:
        return V, s, U
    return U, s, V
