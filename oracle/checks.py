"""Invariants and error metrics of the Golub-Kahan factorization.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def relation_error(A, P, Q, H) -> float:
    """||A P - Q H||_F / ||A||_F  (second relation of eq. 2.4)."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A @ P - Q @ H) / max(np.linalg.norm(A), 1e-300))


def transpose_relation_error(A, P, Q, H, alpha_res, p_res) -> float:
    """||A^T Q - P H^T - alpha_res p_res e_last^T||_F / ||A||_F  (third relation of eq. 2.4)."""
    A = np.asarray(A, dtype=np.float64)
    R = A.T @ Q - P @ H.T
    if p_res is not None and alpha_res != 0.0:
        R[:, -1] -= alpha_res * p_res
    return float(np.linalg.norm(R) / max(np.linalg.norm(A), 1e-300))


def orth_error(X) -> float:
    """max |X^T X - I| (eq. 2.5, orthonormality of the bases)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.max(np.abs(X.T @ X - np.eye(X.shape[1])))) if X.shape[1] else 0.0


def triplet_residuals(A, sigma, U, V):
    """Per triplet: (||A v_i - sigma_i u_i||, ||A^T u_i - sigma_i v_i||)."""
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    r1 = np.linalg.norm(A @ V - U * sigma[None, :], axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sigma[None, :], axis=0)
    return r1, r2


def err_rel(A, sigma, U, V) -> float:
    """Relative error of the experiments section: ||A^T U - V Sigma||_F / ||Sigma||_F."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A.T @ U - V * sigma[None, :]) / np.linalg.norm(sigma))


def err_res(A, sigma, U, V) -> float:
    """Residual error of the experiments section: ||A - U Sigma V^T||_F."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - (U * sigma[None, :]) @ V.T))


def alignment(U1, V1, U2, V2) -> np.ndarray:
    """Figure 1's triplet-quality vector diag(U1^T U2) * diag(V1^T V2).

    Invariant to flipping the sign of a pair (u_i, v_i) on either side; a value
    of 1 means both vectors of triplet i agree.
    """
    return np.einsum("ij,ij->j", U1, U2) * np.einsum("ij,ij->j", V1, V2)


def canonical_signs(U, V):
    """Flip each pair (u_i, v_i) so that v_i's largest-magnitude entry (lowest
    index on ties) is positive."""
    U = np.array(U, dtype=np.float64, copy=True)
    V = np.array(V, dtype=np.float64, copy=True)
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] *= -1.0
            U[:, i] *= -1.0
    return U, V
