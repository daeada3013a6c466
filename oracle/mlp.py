"""The start-vector network, its loss, gradient and optimiser in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not in the paper (Algorithm 2 only says the start vector q is arbitrary).
Features of row i: [S_i / c_S, sqrt(m) s_j U_prev[i, j], 1] with S the sketch
(m x ws), c_S its RMS, U_prev (m x r) the previous left vectors and s_j the sign
making column j's largest-magnitude entry (lowest index on ties) positive.
Network: z_i = w2 . relu(W1 x_i + b1) + b2.  Loss: L = 1 - ||U^T z||^2 / ||z||^2.
Parameters are packed as [W1 (hidden x in, row-major) | b1 | w2 | b2].
"""
from __future__ import annotations

import numpy as np


def unpack(params, n_in: int, hidden: int):
    p = np.asarray(params, dtype=np.float64)
    W1 = p[: hidden * n_in].reshape(hidden, n_in)
    b1 = p[hidden * n_in: hidden * n_in + hidden]
    w2 = p[hidden * n_in + hidden: hidden * n_in + 2 * hidden]
    b2 = p[hidden * n_in + 2 * hidden]
    return W1, b1, w2, b2


def features(S, U_prev):
    """X (m x (ws + r + 1)) from the sketch S (m x ws) and U_prev (m x r)."""
    S = np.asarray(S, dtype=np.float64)
    U = np.asarray(U_prev, dtype=np.float64)
    m = S.shape[0]
    cs = np.sqrt(np.mean(S * S))
    sgn = np.ones(U.shape[1])
    for j in range(U.shape[1]):
        idx = int(np.argmax(np.abs(U[:, j])))  # first index of the maximum
        sgn[j] = -1.0 if U[idx, j] < 0 else 1.0
    return np.concatenate([S / cs if cs > 0 else S * 0, np.sqrt(m) * U * sgn[None, :], np.ones((m, 1))], axis=1)


def forward(params, n_in, hidden, X):
    """z and the hidden activations H (m x hidden)."""
    W1, b1, w2, b2 = unpack(params, n_in, hidden)
    A = X[:, :n_in] @ W1.T + b1[None, :]
    H = np.maximum(A, 0.0)
    return H @ w2 + b2, H, A


LOGTAN_DELTA = 1e-6


def loss(params, n_in, hidden, X, U, kind=0):
    """kind 0: energy of z outside span(U), 1 - ||U^T z||^2 / ||z||^2.
    kind 1: mean over the columns u_j of U of log tan^2(angle(z, u_j)),
    regularised: log(((1 + d) ||z||^2 - (u_j.z)^2) / ((u_j.z)^2 + d ||z||^2))."""
    z, _, _ = forward(params, n_in, hidden, X)
    c = U.T @ z
    zz = float(z @ z)
    if kind == 0:
        return 1.0 - float(c @ c) / zz
    d = LOGTAN_DELTA
    return float(np.mean(np.log(((1.0 + d) * zz - c * c) / (c * c + d * zz))))


def grad(params, n_in, hidden, X, U, kind=0):
    """Analytic gradient of `loss` (chain rule through the loss in terms of z)."""
    W1, b1, w2, b2 = unpack(params, n_in, hidden)
    z, H, A = forward(params, n_in, hidden, X)
    c = U.T @ z
    zz = float(z @ z)
    if kind == 0:
        cc = float(c @ c)
        dz = (2.0 / zz) * (-(U @ c) + (cc / zz) * z)
    else:
        d = LOGTAN_DELTA
        r = U.shape[1]
        a = (1.0 + d) * zz - c * c
        b = c * c + d * zz
        # d log a_j / dz = (2 (1 + d) z - 2 c_j u_j) / a_j ; d log b_j / dz = (2 c_j u_j + 2 d z) / b_j
        dz = (np.sum(2.0 * (1.0 + d) / a - 2.0 * d / b) / r) * z - U @ ((2.0 / r) * c * (1.0 / a + 1.0 / b))
    dW2 = H.T @ dz
    db2 = dz.sum()
    dH = np.outer(dz, w2) * (A > 0)
    dW1 = dH.T @ X[:, :n_in]
    db1 = dH.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2, [db2]])


def adam_step(p, g, m1, m2, lr, beta1, beta2, eps, step):
    """One Adam update (Kingma and Ba 2015) with bias correction; returns new (p, m1, m2)."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mh = m1 / (1 - beta1 ** step)
    vh = m2 / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2
