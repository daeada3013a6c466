"""The Riemannian gradient step of Algorithm 4 in the oracle, pinned to what the
geometry fixes: the tangent projection is an idempotent projection onto the
tangent space, the retraction fixes points of the manifold and agrees with
W + xi to first order, the Euclidean gradient matches finite differences of
the objective, and a small step descends."""
import numpy as np

from oracle import rsgd
from paper_2104_10785_amd import inputs

D1, D2, R = 60, 40, 4


def point(seed=3):
    return inputs.rank_r_point(D1, D2, R, seed=seed)


def tangent(U, V, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((R, R))
    Up = rng.standard_normal((D1, R))
    Up -= U @ (U.T @ Up)
    Vp = rng.standard_normal((D2, R))
    Vp -= V @ (V.T @ Vp)
    return U @ M @ V.T + Up @ V.T + U @ Vp.T


def test_projection_is_the_tangent_projection():
    U, s, V = point()
    G = np.random.default_rng(0).standard_normal((D1, D2))
    Z = rsgd.project(G, U, V)
    assert np.allclose(rsgd.project(Z, U, V), Z, atol=1e-12)                       # idempotent
    PU, PV = np.eye(D1) - U @ U.T, np.eye(D2) - V @ V.T
    assert np.abs(PU @ Z @ PV).max() < 1e-12                                       # no normal part
    xi = tangent(U, V, 1)
    assert np.allclose(rsgd.project(xi, U, V), xi, atol=1e-12)                     # fixes tangents
    assert abs(np.sum(G * xi) - np.sum(Z * xi)) < 1e-10                            # <G, xi> = <P G, xi>
    W = (U * s) @ V.T
    assert np.allclose(rsgd.project(W, U, V), W, atol=1e-12)                       # W is its own tangent


def test_retraction_fixes_the_manifold_and_is_first_order():
    U, s, V = point()
    W = (U * s) @ V.T
    U2, s2, V2 = rsgd.retract(W, R)
    assert np.allclose((U2 * s2) @ V2.T, W, atol=1e-12) and np.allclose(s2, s)
    xi = tangent(U, V, 2)
    errs = []
    for t in (1e-2, 5e-3):
        U3, s3, V3 = rsgd.retract(W + t * xi, R)
        errs.append(np.linalg.norm((U3 * s3) @ V3.T - (W + t * xi)))
    assert 3.0 < errs[0] / errs[1] < 5.0                                           # O(t^2)


def test_euclidean_gradient_matches_finite_differences():
    X, V, y, _, _ = inputs.similarity_pairs(32, D1, D2, seed=5)
    U, s, Vf = point()
    W = (U * s) @ Vf.T
    lam = 0.1
    G = rsgd.euclidean_gradient(X, V, y, W, lam)
    rng = np.random.default_rng(7)
    for _ in range(3):
        E = rng.standard_normal((D1, D2))
        h = 1e-5
        fd = (rsgd.objective(X, V, y, W + h * E, lam) - rsgd.objective(X, V, y, W - h * E, lam)) / (2 * h)
        assert abs(fd - np.sum(G * E)) < 1e-6 * max(1.0, abs(fd))


def test_small_step_descends_and_stays_rank_r():
    X, V, y, _, _ = inputs.similarity_pairs(64, D1, D2, seed=6)
    U, s, Vf = point()
    W = (U * s) @ Vf.T
    lam = 1e-3
    U2, s2, V2, W2, Y = rsgd.step(X, V, y, U, s, Vf, 1e-2, lam)
    assert rsgd.objective(X, V, y, W2, lam) < rsgd.objective(X, V, y, W, lam)
    assert np.linalg.matrix_rank(W2, tol=1e-10) == R
    assert np.linalg.matrix_rank(Y, tol=1e-9 * np.linalg.norm(Y)) <= 2 * R       # W - eta Z has rank <= 2r
    assert np.allclose(U2.T @ U2, np.eye(R), atol=1e-12) and np.allclose(V2.T @ V2, np.eye(R), atol=1e-12)
