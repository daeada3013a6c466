"""Riemannian mini-batch gradient descent for similarity learning (Algorithm 4), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Section 4): f_W(x, v) = x^T W v with W of rank r (the manifold M_r).
One step on a batch {(x_i, v_i, y_i)}:

* Euclidean gradient of the batch objective.  Reading of Algorithm 4 (its
  signs are inconsistent as printed): the objective is
  F(W) = -(1/b) sum_i y_i x_i^T W v_i + (lam/2) ||W||_F^2, whose gradient is
  G = -(1/b) sum_i y_i x_i v_i^T + lam W; the step descends F.
* Riemannian gradient: the projection of G onto the tangent space at
  W = U S V^T (Section 4, with P^H_X = X X^T, P^V_X = I - X X^T):
  Z = P^H_U G P^H_V + P^V_U G P^H_V + P^H_U G P^V_V.  Reading: U, V are the
  factors of W (Algorithm 4 takes them from an SVD of the gradient, but the
  tangent space is that of W).
* Retraction: W_new = R_W(-eta Z) = the best rank-r approximation of W - eta Z,
  i.e. its first r singular triplets (the closed form of the retraction).

The retraction's SVD is numpy's full SVD truncated (the plain definition).
"""
from __future__ import annotations

import numpy as np


def euclidean_gradient(X, V, y, W, lam):
    """G = -(1/b) sum_i y_i x_i v_i^T + lam W for the batch (X: b x d1, V: b x d2)."""
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return -(X.T * y[None, :]) @ V / X.shape[0] + lam * np.asarray(W, dtype=np.float64)


def project(G, U, Vf):
    """Tangent-space projection at W = U S Vf^T (orthonormal U, Vf)."""
    G = np.asarray(G, dtype=np.float64)
    PU = U @ U.T
    PV = Vf @ Vf.T
    I1 = np.eye(U.shape[0])
    I2 = np.eye(Vf.shape[0])
    return PU @ G @ PV + (I1 - PU) @ G @ PV + PU @ G @ (I2 - PV)


def retract(Y, r):
    """First r singular triplets of Y (descending): (U, s, Vf) with Y ~ U diag(s) Vf^T."""
    Uf, s, Vt = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    return Uf[:, :r], s[:r], Vt[:r].T


def step(X, V, y, U, s, Vf, eta, lam):
    """One step from W = U diag(s) Vf^T; returns (U', s', Vf', W', Y = W - eta Z)."""
    W = (U * s[None, :]) @ Vf.T
    G = euclidean_gradient(X, V, y, W, lam)
    Z = project(G, U, Vf)
    Y = W - eta * Z
    U2, s2, V2 = retract(Y, U.shape[1])
    return U2, s2, V2, (U2 * s2[None, :]) @ V2.T, Y


def objective(X, V, y, W, lam):
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    f = np.einsum("ij,jk,ik->i", X, np.asarray(W, dtype=np.float64), V)
    return float(-np.mean(np.asarray(y, dtype=np.float64) * f) + 0.5 * lam * np.sum(np.asarray(W) ** 2))


def accuracy(X, V, y, W):
    """Fraction of pairs whose similarity sign x^T W v matches the label."""
    f = np.einsum("ij,jk,ik->i", np.asarray(X, np.float64), np.asarray(W, np.float64), np.asarray(V, np.float64))
    return float(np.mean(np.sign(f) == np.sign(y)))
