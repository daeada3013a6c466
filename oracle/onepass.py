"""Golub-Kahan steps that read A once per step: the float64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain numpy float64.

Bidiag 1 (eq. 2.2) with reorthogonalisation forms, at step t,
    beta_{t+1} q_{t+1} = A p_t - alpha_t q_t - Q_{t+1} h
where h collects the Gram-Schmidt coefficients of all passes. Writing
c = alpha_t e_t + h, this is beta_{t+1} q_{t+1} = A p_t - Q_{t+1} c, so
    A^T q_{t+1} = (A^T A p_t - (A^T Q_{t+1}) c) / beta_{t+1}.
If G = A^T Q is kept column by column, both products of a step come from one
reading of A: w = A p_t and y = A^T w are formed together, and the second
product of the recurrence is recovered from y, G and c. The factorisation is
the one of `gk.first_cycle` (same coefficients and bases, up to rounding); the
only new step is the recovery, whose error is the rounding error of y and G c
divided by beta_{t+1}.

The recovery is not self-correcting: an error d_t in the stored A^T q_t enters
A^T q_{t+1} multiplied by alpha_t / beta_{t+1} (through c), so errors grow
geometrically whenever alpha_t > beta_{t+1}, e.g. for a flat spectrum. The
guard tracks a bound e_j on the error of each stored column,
    e_{t+1} = (sum_j |c_j| e_j + eps0 (s^2 + s sum_j |c_j|)) / beta_{t+1},
with s the largest coefficient seen so far (a lower bound on sigma_1, standing
in for ||A||) and eps0 = 2^-52 sqrt(m + n) the typical relative rounding of a
float64 product of that length; a column whose bound exceeds tau * s is
recomputed by a direct product A^T q_{t+1} (error bound eps0 * s again). With
tau = 1e-10 the relations of eq. (2.4) hold to about 1e-10 sigma_1, far below
the float32 rounding of A itself.

A thick restart (see `gk.restart_cycle`) keeps the identity: with
Q~ = Q X_l the kept columns have A^T Q~ = G X_l, and the first step after it
subtracts Q~ rho instead of alpha_t q_t (c = rho + h).
"""
from __future__ import annotations

import numpy as np

from . import gk


def recover(y: np.ndarray, G: np.ndarray, c: np.ndarray, beta: float) -> np.ndarray:
    """A^T q_{t+1} from y = A^T A p_t, G = A^T Q_{t+1} and the coefficients c."""
    return (y - G @ c) / beta


TAU = 1e-10


def error_bound(c: np.ndarray, e: np.ndarray, beta: float, s: float, eps0: float) -> float:
    """Bound on the error of a recovered column (see the module docstring)."""
    ac = np.abs(c)
    return float((ac @ e + eps0 * (s * s + s * ac.sum())) / beta)


def first_cycle(A: np.ndarray, q: np.ndarray, k: int, eps: gk.BreakThreshold, passes: int = 2,
                tau: float | None = TAU):
    """k steps of Bidiag 1 with one product sweep per step.

    Returns (Factorization, G) with G = A^T Q (m x (np + 1) columns used);
    Factorization.coeffs["refreshed"] lists the steps whose column was
    recomputed directly (tau=None: never, the unguarded recovery). Same
    breakdown rules and matrices as `gk.first_cycle` without in-cycle checks;
    matvecs counts products (two per sweep, one per direct recomputation).
    """
    m, n = A.shape
    eps0 = 2.0 ** -52 * np.sqrt(m + n)
    Q = np.zeros((m, k + 1))
    P = np.zeros((n, k + 1))
    G = np.zeros((n, k + 1))
    err = np.zeros(k + 1)
    refreshed: list[int] = []
    alphas: list[float] = []
    betas: list[float] = []
    Q[:, 0] = q / gk.vnorm(q)
    G[:, 0] = A.T @ Q[:, 0]
    matvecs = 1
    alpha = gk.vnorm(G[:, 0])
    if alpha == 0.0:
        return gk.Factorization(P[:, :0], Q[:, :1], np.zeros((1, 0)), 0.0, None, "alpha", matvecs), G[:, :1]
    eps.seen(alpha)
    alphas.append(alpha)
    P[:, 0] = G[:, 0] / alpha
    seen = alpha
    err[0] = eps0 * seen

    def bidiag(nq, np_):
        H = np.zeros((nq, np_))
        for j in range(np_):
            H[j, j] = alphas[j]
            if j + 1 < nq:
                H[j + 1, j] = betas[j]
        return H

    for t in range(k):
        # one sweep of A: w = A p_t and y = A^T w
        w = A @ P[:, t]
        y = A.T @ w
        matvecs += 2
        c = np.zeros(t + 1)
        c[t] = alphas[t]
        w = w - alphas[t] * Q[:, t]
        for _ in range(passes):
            h = Q[:, : t + 1].T @ w
            w = w - Q[:, : t + 1] @ h
            c += h
        beta = gk.vnorm(w)
        if beta <= eps():
            return (gk.Factorization(P[:, : t + 1], Q[:, : t + 1], bidiag(t + 1, t + 1), 0.0, None, "beta",
                                     matvecs - 1, {"refreshed": refreshed}), G[:, : t + 1])
        eps.seen(beta)
        seen = max(seen, beta)
        betas.append(beta)
        Q[:, t + 1] = w / beta
        G[:, t + 1] = recover(y, G[:, : t + 1], c, beta)
        err[t + 1] = error_bound(c, err[: t + 1], beta, seen, eps0)
        if tau is not None and err[t + 1] > tau * seen:
            G[:, t + 1] = A.T @ Q[:, t + 1]
            matvecs += 1
            err[t + 1] = eps0 * seen
            refreshed.append(t)
        z = gk.reorthogonalize(P[:, : t + 1], G[:, t + 1] - beta * P[:, t], passes)
        alpha = gk.vnorm(z)
        if alpha <= eps():
            return (gk.Factorization(P[:, : t + 1], Q[:, : t + 2], bidiag(t + 2, t + 1), 0.0, None, "alpha",
                                     matvecs, {"refreshed": refreshed}), G[:, : t + 2])
        eps.seen(alpha)
        seen = max(seen, alpha)
        alphas.append(alpha)
        P[:, t + 1] = z / alpha
    return (gk.Factorization(P[:, :k], Q[:, : k + 1], bidiag(k + 1, k), alphas[k], P[:, k].copy(), None, matvecs,
                             {"refreshed": refreshed, "err": err}), G)


def restart_cycle(A: np.ndarray, fac: gk.Factorization, G: np.ndarray, err: np.ndarray, X: np.ndarray,
                  s: np.ndarray, Y: np.ndarray, l: int, k: int, eps: gk.BreakThreshold, passes: int = 2,
                  tau: float | None = TAU):
    """`gk.restart_cycle` with one product sweep per step.

    G holds A^T Q of the previous factorisation (its nq columns) and err their
    error bounds. The kept columns are Q~ = Q X_l, so A^T Q~ = G X_l, each with
    the bound sqrt(nq) max(err) (the X columns are orthonormal). The first new
    step subtracts Q~ rho, so c = rho + h on the kept columns; later steps
    subtract alpha_j q_{j-1} as in the first cycle. Returns (Factorization, G, err).
    """
    m, n = A.shape
    eps0 = 2.0 ** -52 * np.sqrt(m + n)
    nq, np_ = fac.H.shape
    Pn = np.zeros((n, k + 1))
    Qn = np.zeros((m, k + 1))
    Gn = np.zeros((n, k + 1))
    en = np.zeros(k + 1)
    Pn[:, :l] = fac.P[:, :np_] @ Y[:, :l]
    Qn[:, :l] = fac.Q[:, :nq] @ X[:, :l]
    Gn[:, :l] = G[:, :nq] @ X[:, :l]
    en[:l] = np.sqrt(nq) * np.max(err[:nq])
    Pn[:, l] = fac.p_res
    rho = fac.alpha_res * X[nq - 1, :l]
    H = np.zeros((k, k))
    H[:l, :l] = np.diag(s[:l])
    H[:l, l] = rho
    seen = eps.scale
    matvecs = 0
    refreshed: list[int] = []
    alpha_prev = 0.0
    for j in range(l, k):
        w = A @ Pn[:, j]
        y = A.T @ w
        matvecs += 2
        c = np.zeros(j)
        if j == l:
            w = w - Qn[:, :l] @ rho
            c[:l] = rho
        else:
            w = w - alpha_prev * Qn[:, j - 1]
            c[j - 1] = alpha_prev
        for _ in range(passes):
            h = Qn[:, :j].T @ w
            w = w - Qn[:, :j] @ h
            c += h
        beta = gk.vnorm(w)
        if beta <= eps():
            return (gk.Factorization(Pn[:, : j + 1], Qn[:, :j], H[:j, : j + 1].copy(), 0.0, None, "beta",
                                     fac.matvecs + matvecs - 1, {"refreshed": refreshed}), Gn[:, :j], en[:j])
        eps.seen(beta)
        seen = max(seen, beta)
        Qn[:, j] = w / beta
        H[j, j] = beta
        Gn[:, j] = recover(y, Gn[:, :j], c, beta)
        en[j] = error_bound(c, en[:j], beta, seen, eps0)
        if tau is not None and en[j] > tau * seen:
            Gn[:, j] = A.T @ Qn[:, j]
            matvecs += 1
            en[j] = eps0 * seen
            refreshed.append(j)
        z = gk.reorthogonalize(Pn[:, : j + 1], Gn[:, j] - beta * Pn[:, j], passes)
        alpha = gk.vnorm(z)
        if alpha <= eps():
            return (gk.Factorization(Pn[:, : j + 1], Qn[:, : j + 1], H[: j + 1, : j + 1].copy(), 0.0, None, "alpha",
                                     fac.matvecs + matvecs, {"refreshed": refreshed}), Gn[:, : j + 1], en[: j + 1])
        eps.seen(alpha)
        seen = max(seen, alpha)
        Pn[:, j + 1] = z / alpha
        if j + 1 < k:
            H[j, j + 1] = alpha
        alpha_prev = alpha
    return (gk.Factorization(Pn[:, :k], Qn[:, :k], H, alpha_prev, Pn[:, k].copy(), None, fac.matvecs + matvecs,
                             {"refreshed": refreshed}), Gn[:, :k], en[:k])
