"""Golub-Kahan bidiagonalization with Ritz extraction: the float64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain numpy float64.

What the paper fixes and what is read into it
---------------------------------------------
* Bidiag 1 (eq. 2.1-2.2): beta_1 q_1 = q, alpha_1 p_1 = A^T q_1, then
  beta_{i+1} q_{i+1} = A p_i - alpha_i q_i and
  alpha_{i+1} p_{i+1} = A^T q_{i+1} - beta_{i+1} p_i, with alpha, beta >= 0.
* Every new vector is re-orthogonalised against all previous ones (Algorithm 1,
  the two projection steps; Section 3 says so in words). The paper does one
  classical Gram-Schmidt pass; the default here is two passes (CGS2), the
  paper-faithful functions at the bottom do one.
* Matrix relations (eq. 2.4): A P_k = Q_{k+1} B_{k+1,k} and
  A^T Q_{k+1} = P_k B^T + alpha_{k+1} p_{k+1} e_{k+1}^T, B lower bidiagonal
  (eq. 2.3).
* Ritz extraction (eq. 2.13 and the formula for the left vectors that follows
  it): the right Ritz vectors are P_k times eigenvectors of B^T B, the Ritz
  values are the square roots of its eigenvalues, and u_i = A v_i / sigma_i.
  Reading used by default: the SVD of B itself, B = X diag(s) Y^T, which gives
  the same s and Y without squaring the condition number, and U = Q X, which
  equals A V diag(s)^-1 by the second relation of eq. 2.4.
* Breakdown (Algorithm 1, the norm test; Section 3.2): the paper stops when the
  new q has norm below epsilon. Reading: test the norm before normalisation,
  and test the alpha side as well (for an exactly rank-deficient A the alpha
  side vanishes first). A threshold is relative to the largest coefficient
  seen so far unless `eps_relative` is False (the paper's absolute epsilon).
* Convergence and thick restart are not in the paper (it runs a fixed k).
  Triplet i is converged when alpha_res |X[last, i]| <= tol * sigma_1(H),
  which is the exact residual ||A^T u_i - sigma_i v_i|| by the third relation
  of eq. 2.4. A restart keeps l Ritz pairs (Ritz vectors as basis, in the spirit
  of augmented/restarted bidiagonalization) and continues the recurrence; see
  `restart_cycle`.
"""
from __future__ import annotations

import numpy as np

OK = 0
NOT_CONVERGED = 1
RANK_DEFICIENT = 2


def vnorm(x: np.ndarray) -> float:
    """Euclidean norm."""
    return float(np.sqrt(np.dot(x, x)))


def reorthogonalize(basis: np.ndarray, x: np.ndarray, passes: int) -> np.ndarray:
    """x <- x - basis (basis^T x), `passes` times (classical Gram-Schmidt).

    Algorithm 1 projects the new q against Q and the new p against P once;
    passes=2 repeats the projection (CGS2).
    """
    for _ in range(passes):
        if basis.shape[1] == 0:
            break
        x = x - basis @ (basis.T @ x)
    return x


class BreakThreshold:
    """The breakdown threshold epsilon_b.

    Absolute: eps_break itself (the paper's user-chosen epsilon).
    Relative: eps_break times the largest alpha, beta or Ritz value seen so far
    (a running lower bound on sigma_1(A)).
    """

    def __init__(self, eps_break: float, relative: bool):
        self.eps_break = float(eps_break)
        self.relative = bool(relative)
        self.scale = 0.0

    def seen(self, value: float) -> None:
        self.scale = max(self.scale, float(value))

    def __call__(self) -> float:
        return self.eps_break * self.scale if self.relative else self.eps_break


class Factorization:
    """A P = Q H and A^T Q = P H^T + alpha_res p_res e_last^T.

    P: n x np orthonormal, Q: m x nq orthonormal, H: nq x np.
    breakdown: None, 'alpha' or 'beta' (then alpha_res = 0: the relations are
    exact and every Ritz triplet of H is a singular triplet of A).
    """

    def __init__(self, P, Q, H, alpha_res, p_res, breakdown, matvecs, coeffs=None):
        self.P = P
        self.Q = Q
        self.H = H
        self.alpha_res = float(alpha_res)
        self.p_res = p_res
        self.breakdown = breakdown
        self.matvecs = matvecs
        self.coeffs = coeffs or {}


def first_cycle(A: np.ndarray, q: np.ndarray, k: int, eps: BreakThreshold,
                passes: int = 2, stop=None) -> Factorization:
    """k steps of Bidiag 1 from the start vector q (eq. 2.1-2.3, Algorithm 1).

    Step t (1-based) uses p_t, alpha_t, q_t and produces beta_{t+1} q_{t+1} and
    then alpha_{t+1} p_{t+1}. After k steps, H = B_{k+1,k} and p_{k+1} with
    alpha_{k+1} is the residual direction. Matvecs: 1 + 2k.

    `stop`, if given, is called as stop(H, alpha_res) after steps whose
    column count np satisfies its schedule (see `ConvergenceCheck`); when it
    returns True the cycle ends there with H = B_{np+1,np}.
    """
    m, n = A.shape
    Q = np.zeros((m, k + 1))
    P = np.zeros((n, k + 1))
    alphas: list[float] = []
    betas: list[float] = []
    beta1 = vnorm(q)
    Q[:, 0] = q / beta1
    z = A.T @ Q[:, 0]
    matvecs = 1
    alpha = vnorm(z)
    if not np.isfinite(alpha):
        raise FloatingPointError("non-finite alpha_1")
    if alpha == 0.0:
        # A^T q_1 = 0: nothing to extract (A = 0 or q_1 orthogonal to range(A)).
        return Factorization(P[:, :0], Q[:, :1], np.zeros((1, 0)), 0.0, None, "alpha", matvecs,
                             {"alpha": [0.0], "beta": []})
    eps.seen(alpha)
    alphas.append(alpha)
    P[:, 0] = z / alpha

    def bidiag(nq, np_):
        H = np.zeros((nq, np_))
        for j in range(np_):
            H[j, j] = alphas[j]
            if j + 1 < nq:
                H[j + 1, j] = betas[j]
        return H

    for t in range(k):  # t is 0-based: P[:, t] = p_{t+1}, Q[:, t] = q_{t+1}
        w = A @ P[:, t] - alphas[t] * Q[:, t]
        matvecs += 1
        w = reorthogonalize(Q[:, : t + 1], w, passes)
        beta = vnorm(w)
        if not np.isfinite(beta):
            raise FloatingPointError("non-finite beta")
        if beta <= eps():
            # A P_{t+1} lies in span(Q_{t+1}): square B_{t+1,t+1}, exact.
            return Factorization(P[:, : t + 1], Q[:, : t + 1], bidiag(t + 1, t + 1), 0.0, None,
                                 "beta", matvecs, {"alpha": alphas, "beta": betas})
        eps.seen(beta)
        betas.append(beta)
        Q[:, t + 1] = w / beta
        z = A.T @ Q[:, t + 1] - beta * P[:, t]
        matvecs += 1
        z = reorthogonalize(P[:, : t + 1], z, passes)
        alpha = vnorm(z)
        if not np.isfinite(alpha):
            raise FloatingPointError("non-finite alpha")
        if alpha <= eps():
            # A^T Q_{t+2} lies in span(P_{t+1}): B_{t+2,t+1}, exact.
            return Factorization(P[:, : t + 1], Q[:, : t + 2], bidiag(t + 2, t + 1), 0.0, None,
                                 "alpha", matvecs, {"alpha": alphas, "beta": betas})
        eps.seen(alpha)
        alphas.append(alpha)
        P[:, t + 1] = z / alpha
        np_ = t + 1
        if stop is not None and np_ < k and stop.due(np_):
            H = bidiag(np_ + 1, np_)
            if stop(H, alpha):
                return Factorization(P[:, :np_], Q[:, : np_ + 1], H, alpha, P[:, np_].copy(), None,
                                     matvecs, {"alpha": alphas, "beta": betas, "early": True})
    return Factorization(P[:, :k], Q[:, : k + 1], bidiag(k + 1, k), alphas[k], P[:, k].copy(),
                         None, matvecs, {"alpha": alphas, "beta": betas})


def ritz(H: np.ndarray):
    """SVD of the projected matrix, H = X diag(s) Y^T, s descending.

    Reading of Algorithm 2's eigendecomposition of B^T B (eq. 2.13): the right
    singular vectors Y of H are the eigenvectors of H^T H and s**2 its
    eigenvalues.
    """
    X, s, Yt = np.linalg.svd(H, full_matrices=False)
    return X, s, Yt.T


def restart_cycle(A: np.ndarray, fac: Factorization, X: np.ndarray, s: np.ndarray,
                  Y: np.ndarray, l: int, k: int, eps: BreakThreshold,
                  passes: int = 2, stop=None) -> Factorization:
    """Thick restart keeping l Ritz pairs, then continue to k vectors.

    With P~ = P Y_l, Q~ = Q X_l, rho = alpha_res X[last, :l] and p_{l+1} = p_res:
      A P~ = Q~ diag(s_l),  A^T Q~ = P~ diag(s_l) + p_{l+1} rho^T,
    so Q~^T A p_{l+1} = rho. The recurrence resumes with
      beta_{l+1} q_{l+1} = A p_{l+1} - Q~ rho,
      alpha_{l+2} p_{l+2} = A^T q_{l+1} - beta_{l+1} p_{l+1},
    and for j > l+1 the usual pair
      beta_j q_j = A p_j - alpha_j q_{j-1},  alpha_{j+1} p_{j+1} = A^T q_j - beta_j p_j,
    each vector re-orthogonalised as in Algorithm 1. The new H (k x k) is upper
    triangular: diag(s_l) with rho in column l+1, then an upper-bidiagonal
    block with beta_j on the diagonal and alpha_j above it.
    Matvecs: 2 (k - l).
    """
    m, n = A.shape
    nq, np_ = fac.H.shape
    Pn = np.zeros((n, k + 1))
    Qn = np.zeros((m, k + 1))
    Pn[:, :l] = fac.P[:, :np_] @ Y[:, :l]
    Qn[:, :l] = fac.Q[:, :nq] @ X[:, :l]
    Pn[:, l] = fac.p_res
    rho = fac.alpha_res * X[nq - 1, :l]
    H = np.zeros((k, k))
    H[:l, :l] = np.diag(s[:l])
    H[:l, l] = rho
    matvecs = 0
    alpha_prev = 0.0
    for j in range(l, k):  # 0-based: produce Q[:, j] from P[:, j], then P[:, j+1]
        if j == l:
            w = A @ Pn[:, l] - Qn[:, :l] @ rho
        else:
            w = A @ Pn[:, j] - alpha_prev * Qn[:, j - 1]
        matvecs += 1
        w = reorthogonalize(Qn[:, :j], w, passes)
        beta = vnorm(w)
        if not np.isfinite(beta):
            raise FloatingPointError("non-finite beta")
        if beta <= eps():
            return Factorization(Pn[:, : j + 1], Qn[:, :j], H[:j, : j + 1].copy(), 0.0, None,
                                 "beta", fac.matvecs + matvecs)
        eps.seen(beta)
        Qn[:, j] = w / beta
        H[j, j] = beta
        z = A.T @ Qn[:, j] - beta * Pn[:, j]
        matvecs += 1
        z = reorthogonalize(Pn[:, : j + 1], z, passes)
        alpha = vnorm(z)
        if not np.isfinite(alpha):
            raise FloatingPointError("non-finite alpha")
        if alpha <= eps():
            return Factorization(Pn[:, : j + 1], Qn[:, : j + 1], H[: j + 1, : j + 1].copy(), 0.0,
                                 None, "alpha", fac.matvecs + matvecs)
        eps.seen(alpha)
        Pn[:, j + 1] = z / alpha
        np_ = j + 1
        if stop is not None and np_ < k and stop.due(np_):
            Hp = H[:np_, :np_].copy()
            if stop(Hp, alpha):
                return Factorization(Pn[:, :np_], Qn[:, :np_], Hp, alpha, Pn[:, np_].copy(), None,
                                     fac.matvecs + matvecs, {"early": True})
        if j + 1 < k:
            H[j, j + 1] = alpha
        alpha_prev = alpha
    return Factorization(Pn[:, :k], Qn[:, :k], H, alpha_prev, Pn[:, k].copy(), None,
                         fac.matvecs + matvecs)


def top_r_converged(H: np.ndarray, alpha_res: float, r: int, tol: float, thr: float):
    """The convergence test on a projected matrix H (nq x np).

    Ritz values above the breakdown threshold `thr` count as available; the r
    largest must all be available and satisfy alpha_res |X[last, i]| <=
    tol * sigma_1(H). Returns (converged, r_eff, nconv, X, s, Y, res).
    """
    nq, np_ = H.shape
    if np_ == 0:
        return False, 0, 0, np.zeros((nq, 0)), np.zeros(0), np.zeros((0, 0)), np.zeros(0)
    X, s, Y = ritz(H)
    res = alpha_res * np.abs(X[nq - 1, :])
    avail = int(np.count_nonzero(s > thr))
    r_eff = min(r, avail)
    conv = res[:r_eff] <= tol * s[0]
    nconv = int(np.count_nonzero(conv))
    return (r_eff == r and nconv == r), r_eff, nconv, X, s, Y, res


class ConvergenceCheck:
    """In-cycle convergence test (not in the paper, which runs a fixed k).

    Due after every `every` right basis vectors once there are at least r of
    them (np >= r and np % every == 0); the cycle then stops as soon as the r
    largest Ritz triplets pass the residual test.
    """

    def __init__(self, r: int, tol: float, every: int, eps: BreakThreshold):
        self.r, self.tol, self.every, self.eps = r, tol, every, eps
        self.checks = 0

    def due(self, np_: int) -> bool:
        return self.every > 0 and np_ >= self.r and np_ % self.every == 0

    def __call__(self, H, alpha_res) -> bool:
        self.checks += 1
        return top_r_converged(H, alpha_res, self.r, self.tol, self.eps())[0]


def default_keep(r: int, k: int) -> int:
    """Restart size l = r + floor((k - r) / 2), at most k - 1."""
    return min(r + (k - r) // 2, k - 1)


def as_operator(A):
    """A in float64: a dense array, or a scipy.sparse matrix kept sparse (the
    method touches A only through the products A x and A^T y, eq. (2.1)-(2.2),
    so a sparse A goes through unchanged; the paper allows either kind)."""
    try:
        import scipy.sparse as sp
        if sp.issparse(A):
            return sp.csr_matrix(A, dtype=np.float64)
    except ImportError:
        pass
    return np.asarray(A, dtype=np.float64)


def default_eps_break(dtype_name: str = "f64") -> float:
    """Relative breakdown threshold: 1e-12 for float64 work, 1e-6 for float32."""
    return 1e-12 if dtype_name == "f64" else 1e-6


def partial_svd(A, r: int, k: int, tol: float, max_restarts: int, q: np.ndarray,
                keep: int = 0, eps_break: float | None = None, eps_relative: bool = True,
                passes: int = 2, left_from_matvec: bool = False, record: bool = False,
                check_every: int = 0):
    """Top-r singular triplets of A by restarted Golub-Kahan (Algorithm 2 + restart).

    Algorithm 2 is the case max_restarts = 0: run Algorithm 1 for k steps, take
    the Ritz triplets of B. With max_restarts > 0 the factorization is restarted
    (keeping `keep` Ritz pairs) until the r largest Ritz triplets all pass the
    residual test or the restarts are used up.

    check_every > 0 adds the in-cycle convergence test of `ConvergenceCheck`.

    Returns a dict: sigma (r'), U (m x r'), V (n x r'), res_est (r'), nconv,
    restarts, matvecs, status, breakdown, cycles (per-cycle H if `record`).
    r' = r unless A has fewer than r singular values above the breakdown
    threshold (status RANK_DEFICIENT).
    """
    A = as_operator(A)
    q = np.asarray(q, dtype=np.float64)
    m, n = A.shape
    if not (1 <= r <= k <= min(m, n)):
        raise ValueError("need 1 <= r <= k <= min(m, n)")
    if tol < 0 or max_restarts < 0:
        raise ValueError("need tol >= 0 and max_restarts >= 0")
    l = keep if keep else default_keep(r, k)
    if max_restarts > 0 and not (r <= l < k):
        if k == r:
            max_restarts = 0
        else:
            raise ValueError("need r <= keep < k")
    eps = BreakThreshold(default_eps_break() if eps_break is None else eps_break, eps_relative)
    stop = ConvergenceCheck(r, tol, check_every, eps) if check_every > 0 else None
    fac = first_cycle(A, q, k, eps, passes, stop)
    restarts = 0
    cycles = []
    while True:
        nq, np_ = fac.H.shape
        if np_ == 0:
            X = np.zeros((nq, 0))
            s = np.zeros(0)
            Y = np.zeros((0, 0))
        else:
            X, s, Y = ritz(fac.H)
        if record:
            cycles.append({"H": fac.H.copy(), "P": fac.P.copy(), "Q": fac.Q.copy(),
                           "alpha_res": fac.alpha_res,
                           "p_res": None if fac.p_res is None else fac.p_res.copy(),
                           "breakdown": fac.breakdown})
        res = fac.alpha_res * np.abs(X[nq - 1, :]) if s.size else np.zeros(0)
        thr = eps()
        avail = int(np.count_nonzero(s > thr)) if s.size else 0
        r_eff = min(r, avail)
        conv = res[:r_eff] <= tol * (s[0] if s.size else 0.0)
        done = (fac.breakdown is not None) or (r_eff == r and bool(conv.all()))
        if done or restarts >= max_restarts:
            break
        eps.seen(s[0])
        fac = restart_cycle(A, fac, X, s, Y, l, k, eps, passes, stop)
        restarts += 1
    sigma = s[:r_eff].copy()
    V = fac.P @ Y[:, :r_eff] if r_eff else np.zeros((n, 0))
    if left_from_matvec:
        U = (A @ V) / sigma[None, :] if r_eff else np.zeros((m, 0))
    else:
        U = fac.Q @ X[:, :r_eff] if r_eff else np.zeros((m, 0))
    nconv = int(np.count_nonzero(conv))
    if r_eff < r:
        status = RANK_DEFICIENT
    elif nconv == r:
        status = OK
    else:
        status = NOT_CONVERGED
    return {"sigma": sigma, "U": U, "V": V, "res_est": res[:r_eff].copy(), "nconv": nconv,
            "restarts": restarts, "matvecs": fac.matvecs, "status": status,
            "breakdown": fac.breakdown, "keep": l, "cycles": cycles, "factorization": fac,
            "checks": stop.checks if stop else 0}


# ---------------------------------------------------------------------------
# Paper-faithful forms (one Gram-Schmidt pass, absolute epsilon on the q side
# only, eigendecomposition of B^T B, U = A V / sigma, fixed k, no restart).
# ---------------------------------------------------------------------------

def paper_algorithm1(A, q, k: int, eps: float):
    """Algorithm 1 as printed, with the index readings noted in the module doc.

    The break test uses beta before normalisation. Returns (B, P, Q, kprime,
    alpha_next) where B is (k'+1) x k' on a normal stop and square on a break.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Q = np.zeros((m, k + 1))
    P = np.zeros((n, k + 1))
    Q[:, 0] = q / vnorm(q)
    z = A.T @ Q[:, 0]
    alphas = [vnorm(z)]
    betas = []
    P[:, 0] = z / alphas[0]
    kp = 0
    broke = False
    while kp < k:
        w = A @ P[:, kp] - alphas[kp] * Q[:, kp]
        w = reorthogonalize(Q[:, : kp + 1], w, 1)
        beta = vnorm(w)
        if beta < eps:
            broke = True
            break
        betas.append(beta)
        Q[:, kp + 1] = w / beta
        z = A.T @ Q[:, kp + 1] - beta * P[:, kp]
        z = reorthogonalize(P[:, : kp + 1], z, 1)
        alpha = vnorm(z)
        alphas.append(alpha)
        P[:, kp + 1] = z / alpha if alpha > 0 else 0.0
        kp += 1
    if broke:
        nb = kp + 1
        B = np.zeros((nb, nb))
        for j in range(nb):
            B[j, j] = alphas[j]
            if j + 1 < nb:
                B[j + 1, j] = betas[j]
        return B, P[:, :nb], Q[:, :nb], kp, 0.0
    B = np.zeros((kp + 1, kp))
    for j in range(kp):
        B[j, j] = alphas[j]
        B[j + 1, j] = betas[j]
    return B, P[:, :kp], Q[:, : kp + 1], kp, alphas[kp]


def paper_fsvd(A, q, k: int, r: int, eps: float = 1e-8):
    """Algorithm 2 (F-SVD) as printed: eig(B^T B), V = P V1, sigma = sqrt, U = A V / sigma."""
    A = np.asarray(A, dtype=np.float64)
    B, P, Q, kp, _ = paper_algorithm1(A, q, k, eps)
    lam, V1 = np.linalg.eigh(B.T @ B)
    order = np.argsort(lam)[::-1][:r]
    V = P @ V1[:, order]
    sigma = np.sqrt(np.maximum(lam[order], 0.0))
    U = (A @ V) / sigma[None, :]
    return sigma, U, V, kp


def paper_rank(A, q, eps: float = 1e-8):
    """Algorithm 3 as printed: k = min(m, n), Algorithm 1, count eig(B^T B) > eps.

    Note that the count is over eigenvalues of B^T B, i.e. sigma**2 > eps.
    Returns (rank, kprime).
    """
    A = np.asarray(A, dtype=np.float64)
    k = min(A.shape)
    B, _, _, kp, _ = paper_algorithm1(A, q, k, eps)
    lam = np.linalg.eigvalsh(B.T @ B)
    return int(np.count_nonzero(lam > eps)), kp
