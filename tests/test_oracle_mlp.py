"""Pins for the float64 start-vector network of the oracle."""
import numpy as np

from oracle import mlp


def setup(m=60, ws=4, r=3, hidden=7, seed=0):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((m, ws))
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    Up = np.linalg.qr(rng.standard_normal((m, r)))[0]
    n_in = ws + r
    params = rng.standard_normal(hidden * n_in + 2 * hidden + 1) * 0.5
    X = mlp.features(S, Up)
    return params, n_in, hidden, X, U


def test_gradient_matches_central_differences():
    params, n_in, hidden, X, U = setup()
    g = mlp.grad(params, n_in, hidden, X, U)
    h = 1e-6
    fd = np.zeros_like(params)
    for i in range(params.size):
        e = np.zeros_like(params)
        e[i] = h
        fd[i] = (mlp.loss(params + e, n_in, hidden, X, U) - mlp.loss(params - e, n_in, hidden, X, U)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_loss_special_cases():
    m, r = 40, 3
    rng = np.random.default_rng(2)
    ones = np.ones((m, 1)) / np.sqrt(m)
    U = np.linalg.qr(np.concatenate([ones, rng.standard_normal((m, r - 1))], axis=1))[0]
    n_in, hidden = 5, 4
    X = np.concatenate([rng.standard_normal((m, n_in)), np.ones((m, 1))], axis=1)
    p = np.zeros(hidden * n_in + 2 * hidden + 1)
    p[-1] = 2.5                            # z = b2 * 1: inside span(U)
    assert abs(mlp.loss(p, n_in, hidden, X, U)) < 1e-14
    V = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V = V - ones @ (ones.T @ V)            # orthogonal to the constant vector
    V = np.linalg.qr(V)[0]
    assert abs(mlp.loss(p, n_in, hidden, X, V) - 1.0) < 1e-14
    # scale invariance of the normalised energy
    params, n_in, hidden, X, U = setup(seed=3)
    q = params.copy()
    q[hidden * n_in + hidden:] *= 3.0
    assert abs(mlp.loss(params, n_in, hidden, X, U) - mlp.loss(q, n_in, hidden, X, U)) < 1e-13


def test_features_sign_canonical_and_scaled():
    rng = np.random.default_rng(4)
    m = 50
    S = rng.standard_normal((m, 3)) * 7.0
    Up = np.linalg.qr(rng.standard_normal((m, 2)))[0]
    X = mlp.features(S, Up)
    Xf = mlp.features(S, Up * np.array([-1.0, 1.0]))
    assert np.allclose(X, Xf)
    assert abs(np.sqrt(np.mean(X[:, :3] ** 2)) - 1.0) < 1e-12
    for j in range(2):
        col = X[:, 3 + j]
        assert col[np.argmax(np.abs(col))] > 0
        assert abs(np.linalg.norm(col) - np.sqrt(m)) < 1e-10
    assert np.all(X[:, 5] == 1.0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(20)
    g = rng.standard_normal(20)
    new, m1, m2 = mlp.adam_step(p, g, np.zeros(20), np.zeros(20), 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(new, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_logtan_gradient_matches_central_differences():
    params, n_in, hidden, X, U = setup(seed=5)
    g = mlp.grad(params, n_in, hidden, X, U, kind=1)
    h = 1e-6
    fd = np.zeros_like(params)
    for i in range(params.size):
        e = np.zeros_like(params)
        e[i] = h
        fd[i] = (mlp.loss(params + e, n_in, hidden, X, U, kind=1)
                 - mlp.loss(params - e, n_in, hidden, X, U, kind=1)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_logtan_loss_closed_forms():
    """z at 45 degrees to every target vector: tan^2 = ... computed by hand;
    z along one target vector only: the other angles are right angles
    (log((1+d)/d)); scale invariance."""
    m, r = 30, 3
    rng = np.random.default_rng(6)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    n_in, hidden = 4, 3
    d = mlp.LOGTAN_DELTA
    # a network whose output is the constant b2 * 1: choose U so that 1 has known projections
    ones = np.ones(m) / np.sqrt(m)
    W = np.linalg.qr(np.concatenate([ones[:, None], rng.standard_normal((m, r))], axis=1))[0]
    u = (ones + W[:, 1]) / np.sqrt(2.0)          # 45 degrees to the constant vector
    Uc = np.stack([u, W[:, 2], W[:, 3]], axis=1)  # 90 degrees for the other two
    X = np.concatenate([rng.standard_normal((m, n_in)), np.ones((m, 1))], axis=1)
    p = np.zeros(hidden * n_in + 2 * hidden + 1)
    p[-1] = 1.7
    zz = 1.7 ** 2 * m
    c2 = zz / 2.0
    want = (np.log(((1 + d) * zz - c2) / (c2 + d * zz)) + 2 * np.log((1 + d) / d)) / 3
    assert abs(mlp.loss(p, n_in, hidden, X, Uc, kind=1) - want) < 1e-12
    params, n_in, hidden, X, U = setup(seed=7)
    q = params.copy()
    q[hidden * n_in + hidden:] *= 2.5
    assert abs(mlp.loss(params, n_in, hidden, X, U, kind=1) - mlp.loss(q, n_in, hidden, X, U, kind=1)) < 1e-12
