"""Learned start vectors on a drifting matrix sequence: training and evaluation.

Sequence: A_0 = Q1 diag(ratio^(i-1)) Q2^T, A_t = A_{t-1} + scale * G1 G2^T
(rank-`rank` Gaussian update with entries of G1 ~ N(0, 1/m), G2 ~ N(0, 1/n), so
||dA_t||_2 ~ scale).  For each t the top r triplets are computed by
gkb_partial_svd (Krylov dimension k, tolerance tol, in-cycle checks every
`check_every` vectors).  All arithmetic runs in the library's kernels; this
module only sequences the calls.

Training (t = 1..t_train): solve with the random start q ~ N(2, 1) (device
Philox, key t); the pair (features from S_t = A_t Omega and U_{t-1}, target
U_t) is kept.  The network is trained with the library's forward/backward and
Adam kernels.  Evaluation (t = t_train+1 .. t_train+t_eval): three solves per t
from the same A_t -- random start, learned start (one sketch product counted as
one matvec, random-start fallback if the learned start does not converge) and
the heuristic q = sum_j s_j u_j(t-1) -- and their matvec counts.
"""
from __future__ import annotations

import time

import numpy as np

from . import gkb, inputs


def _heuristic_params(ws: int, r: int, n_in: int):
    """Parameters under which the network computes z = sum of the previous-vector
    features: hidden units relu(+x_j) and relu(-x_j), output weights +1 / -1."""
    hidden = 2 * r
    W1 = np.zeros((hidden, n_in), dtype=np.float32)
    for j in range(r):
        W1[2 * j, ws + j] = 1.0
        W1[2 * j + 1, ws + j] = -1.0
    w2 = np.tile(np.array([1.0, -1.0], dtype=np.float32), r)
    return np.concatenate([W1.ravel(), np.zeros(hidden, np.float32), w2, [0.0]]).astype(np.float32), hidden


class DriftSequence:
    def __init__(self, m, n, ratio, rank, scale, seed, device):
        self.m, self.n, self.rank, self.scale, self.seed, self.device = m, n, rank, scale, seed, device
        self.A = inputs.drift_base_torch(m, n, ratio, seed, device)
        self.t = 0

    def advance(self):
        self.t += 1
        self.A += inputs.drift_update_torch(self.m, self.n, self.rank, self.scale, self.seed, self.t, self.device)
        return self.A


def _embedded_heuristic_init(ws: int, r: int, n_in: int, hidden: int, seed: int, scale: float):
    """Initial parameters whose output equals the heuristic start: its 2r hidden
    units in the first rows (output weights +1 / -1), the other units drawn as
    in `inputs.mlp_init` times `scale` with zero output weights, so training
    starts from the heuristic and can only add to it what lowers the loss."""
    hp, hh = _heuristic_params(ws, r, n_in)
    base = inputs.mlp_init(n_in, hidden, seed)
    W1 = base[: hidden * n_in].reshape(hidden, n_in) * scale
    W1[:hh] = hp[: hh * n_in].reshape(hh, n_in)
    b1 = np.zeros(hidden, np.float32)
    w2 = np.zeros(hidden, np.float32)
    w2[:hh] = hp[hh * n_in + hh: hh * n_in + 2 * hh]
    return np.concatenate([W1.ravel(), b1, w2, [0.0]]).astype(np.float32)


def run(m=20000, n=5000, r=30, k=70, tol=1e-8, ratio=0.97, rank=4, scale=1e-3, t_train=100, t_eval=100,
        ws=32, hidden=256, epochs=20, lr=1e-3, lr_final=0.02, check_every=2, max_restarts=50, seed=3,
        device="cuda:0", log=None, init="random", loss_kind=0, t_val=None, eval_every=2, prev="U"):
    """init: "random" (He initialisation) or "heuristic" (the heuristic start
    embedded in the network, see `_embedded_heuristic_init`); loss_kind: 0
    (energy outside the target subspace) or 1 (mean log tan^2 of the angles
    to the target vectors), see gkb_mlp_loss_grad_kind.

    Of the t_train training solves, the last t_val (default t_train // 5) are
    held out: the network is trained on the others, and the parameters it
    starts from and those after every eval_every-th epoch are scored by the
    mean number of products the held-out solves need from the network's start
    vector (the convergence test decides); the best-scoring parameters
    (the earliest on a tie) are the ones evaluated.  Adam's step size decays from lr to lr * lr_final along a
    cosine over the epochs, so the updates shrink as the loss flattens.

    prev: what the network gets besides the sketch.  "U": the previous left
    vectors U_{t-1} (their span drifts away from the target's, so no function
    of them alone reaches the current vectors).  "AV": the previous right
    vectors taken through the current matrix, A_t V_{t-1} (one more block
    product, counted as one more matvec like the sketch): since A_t v_j(t-1) =
    sigma_j u_j(t) + O(drift), these columns already point into span(U_t).
    The heuristic start (sum of the previous left vectors, no extra product)
    is reported either way; with "AV" also the sum of the A_t V_{t-1} columns."""
    import torch
    say = log or (lambda msg: None)
    t0 = time.time()
    seq = DriftSequence(m, n, ratio, rank, scale, seed, device)
    omega_t = torch.from_numpy(np.ascontiguousarray(inputs.sketch_matrix(n, ws, seed + 1).T)).to(device)
    n_in = ws + r
    ws_svd = torch.empty(gkb.gkb_workspace_size(seq.A, r, k), dtype=torch.uint8, device=device)

    def solve(q1=None, key=0):
        return gkb.gkb_partial_svd(seq.A, r, k, tol, max_restarts, q1=q1, seed=key, workspace=ws_svd,
                                   check_every=check_every)

    extra = 1 if prev == "AV" else 0   # block products besides the sketch

    def features(U_prev, V_prev):
        St = gkb.gkb_gemm_rowmajor(seq.A, omega_t)   # (ws, m) = m x ws column-major
        if prev == "AV":
            return gkb.gkb_mlp_features(St, gkb.gkb_gemm_rowmajor(seq.A, V_prev))
        return gkb.gkb_mlp_features(St, U_prev)

    # t = 0
    _, U_prev, V_prev, st0, _ = solve(key=10_000)
    data = []
    held = []       # (A_t, X_t) of the held-out training solves
    train_mv = []
    if t_val is None:
        t_val = t_train // 5
    t_fit = max(1, t_train - t_val)
    for t in range(1, t_train + 1):
        seq.advance()
        X = features(U_prev, V_prev)
        sig, Ut, Vt, status, stats = solve(key=t)
        train_mv.append(stats["matvecs"])
        if t <= t_fit:
            data.append((X, Ut.clone()))
        else:
            held.append((seq.A.clone(), X))
        U_prev, V_prev = Ut, Vt
    say(f"training data: {t_train} solves ({t_fit} to fit, {len(held)} held out), mean matvecs "
        f"{np.mean(train_mv):.1f}, {time.time() - t0:.1f} s")

    def held_out_matvecs(prm):
        """Mean products to tolerance over the held-out solves from the network's
        start vector (a start that fails counts its products plus a random-start
        solve's)."""
        if not held:
            return float("nan")
        A_keep = seq.A
        mv = []
        try:
            for A_h, X_h in held:
                seq.A = A_h
                q = gkb.gkb_mlp_start_vector(prm, n_in, hidden, X_h)
                try:
                    _, _, _, st_h, s_h = solve(q1=q)
                    cnt = s_h["matvecs"] + 1 + extra
                    if st_h != 0:
                        cnt += solve(key=1)[4]["matvecs"]
                except gkb.GkbError:
                    cnt = 1 + extra + solve(key=1)[4]["matvecs"]
                mv.append(cnt)
        finally:
            seq.A = A_keep
        return float(np.mean(mv))

    # ---- training on the device
    if init == "heuristic":
        params = torch.from_numpy(_embedded_heuristic_init(ws, r, n_in, hidden, seed + 2, 0.1)).to(device)
    else:
        params = torch.from_numpy(inputs.mlp_init(n_in, hidden, seed + 2)).to(device)
    m1 = torch.zeros_like(params)
    m2 = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device=device)
    wsp = torch.empty(gkb.lib().gkb_mlp_workspace_size(m, n_in, hidden, r), dtype=torch.uint8, device=device)
    rng = np.random.default_rng(seed + 3)
    losses = []
    step = 0
    t1 = time.time()
    scores = [(0, held_out_matvecs(params))]
    best_params, best_score, best_epoch = params.clone(), scores[0][1], 0
    for ep in range(epochs):
        ep_loss = []
        # cosine decay of the step size: lr at the first epoch, lr * lr_final at the last
        frac = ep / max(1, epochs - 1)
        lr_ep = lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + np.cos(np.pi * frac)))
        for t in rng.permutation(len(data)):
            X, Ut = data[t]
            gkb.gkb_mlp_loss_grad(params, n_in, hidden, X, Ut, grad=grad, loss=loss, workspace=wsp, kind=loss_kind)
            step += 1
            gkb.gkb_adam_step(params, grad, m1, m2, lr_ep, step)
            ep_loss.append(loss.clone())
        losses.append(float(torch.cat(ep_loss).mean().item()) if ep_loss else 0.0)
        if (ep + 1) % eval_every == 0 or ep + 1 == epochs:
            sc = held_out_matvecs(params)
            scores.append((ep + 1, sc))
            if sc < best_score:
                best_params, best_score, best_epoch = params.clone(), sc, ep + 1
    torch.cuda.synchronize()
    train_s = time.time() - t1
    say(f"trained {epochs} epochs in {train_s:.2f} s; loss by epoch {['%.3e' % x for x in losses]}; "
        f"held-out matvecs by epoch {[(e, round(v, 2)) for e, v in scores]}; kept epoch {best_epoch}")
    params = best_params
    del held

    # ---- evaluation
    hparams, hhidden = _heuristic_params(ws, r, n_in)
    hparams = torch.from_numpy(hparams).to(device)
    rows = []
    def clock():
        torch.cuda.synchronize()
        return time.perf_counter()

    for t in range(t_train + 1, t_train + t_eval + 1):
        seq.advance()
        c0 = clock()
        X = features(U_prev, V_prev)
        c1 = clock()
        # random start
        sig_r, Ut_r, _, st_r, s_r = solve(key=t)
        c2 = clock()
        # learned start (+1 matvec for the sketch, +1 for A_t V_{t-1}), random fallback
        q_l = gkb.gkb_mlp_start_vector(params, n_in, hidden, X)
        c3 = clock()
        fallback = False
        try:
            sig_l, Ut_l, Vt_l, st_l, s_l = solve(q1=q_l)
            mv_l = s_l["matvecs"] + 1 + extra
            ok = st_l == 0
        except gkb.GkbError:
            ok, mv_l = False, 1 + extra
        c4 = clock()
        if not ok:
            fallback = True
            sig_l, Ut_l, Vt_l, st_l, s_l2 = solve(key=t)
            mv_l += s_l2["matvecs"]
        # heuristic start: the previous left vectors summed (no extra product)
        XU = X if prev == "U" else gkb.gkb_mlp_features(gkb.gkb_gemm_rowmajor(seq.A, omega_t), U_prev)
        q_h = gkb.gkb_mlp_start_vector(hparams, n_in, hhidden, XU)
        try:
            sig_h, _, _, st_h, s_h = solve(q1=q_h)
            mv_h = s_h["matvecs"]
        except gkb.GkbError:
            st_h, mv_h = -1, -1
        mv_hav = None
        if prev == "AV":  # the A_t V_{t-1} columns summed (the heuristic on the network's inputs)
            try:
                mv_hav = solve(q1=gkb.gkb_mlp_start_vector(hparams, n_in, hhidden, X))[4]["matvecs"] + extra
            except gkb.GkbError:
                mv_hav = -1
        rows.append({"t": t, "random": s_r["matvecs"], "learned": mv_l, "heuristic": mv_h, "heuristic_av": mv_hav,
                     "fallback": fallback,
                     "ms_features": (c1 - c0) * 1e3, "ms_random": (c2 - c1) * 1e3, "ms_network": (c3 - c2) * 1e3,
                     "ms_learned_solve": (c4 - c3) * 1e3,
                     "status_random": st_r, "status_learned": st_l, "status_heuristic": st_h,
                     "sigma_diff": float(np.max(np.abs(sig_l - sig_r)))})
        U_prev, V_prev = Ut_l, Vt_l
    mv_r = np.array([x["random"] for x in rows], dtype=float)
    mv_l = np.array([x["learned"] for x in rows], dtype=float)
    mv_h = np.array([x["heuristic"] for x in rows], dtype=float)
    out = {
        "m": m, "n": n, "r": r, "k": k, "tol": tol, "t_train": t_train, "t_eval": t_eval, "hidden": hidden,
        "sketch_width": ws, "epochs": epochs, "check_every": check_every, "init": init, "loss_kind": loss_kind,
        "train_loss_by_epoch": losses, "train_seconds": train_s, "lr": lr, "lr_final": lr * lr_final,
        "held_out": t_train - t_fit, "held_out_matvecs_by_epoch": scores, "kept_epoch": best_epoch,
        "held_out_matvecs_kept": best_score, "held_out_matvecs_init": scores[0][1],
        "matvecs_random": {"mean": mv_r.mean(), "median": float(np.median(mv_r))},
        "matvecs_learned": {"mean": mv_l.mean(), "median": float(np.median(mv_l))},
        "matvecs_heuristic": {"mean": mv_h.mean(), "median": float(np.median(mv_h))},
        "prev": prev, "extra_block_products": extra,
        "learned_over_random_ratio_mean": float(np.mean(mv_l / mv_r)),
        # wall time to tolerance per held-out matrix (device synchronised): the
        # random start's solve; the learned start's sketch + features + network
        # + solve (a fallback solve, if any, is not in these figures)
        "ms_random": float(np.mean([x["ms_random"] for x in rows])),
        "ms_learned": float(np.mean([x["ms_features"] + x["ms_network"] + x["ms_learned_solve"] for x in rows])),
        "ms_learned_start": float(np.mean([x["ms_features"] + x["ms_network"] for x in rows])),
        "learned_win_fraction": float(np.mean(mv_l < mv_r)),
        "fallbacks": int(sum(x["fallback"] for x in rows)),
        "max_sigma_diff_learned_vs_random": float(max(x["sigma_diff"] for x in rows)),
        "seconds": time.time() - t0,
        "per_t": rows,
    }
    if prev == "AV":
        mv_ha = np.array([x["heuristic_av"] for x in rows], dtype=float)
        out["matvecs_heuristic_av"] = {"mean": mv_ha.mean(), "median": float(np.median(mv_ha))}
    return out
