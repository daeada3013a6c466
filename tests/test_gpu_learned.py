"""Learned start: the device network kernels against the float64 oracle, and
the trained network against the random start on held-out solves."""
import numpy as np
import pytest

from oracle import mlp
from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu


def _setup(m=3000, ws=32, r=30, hidden=256, seed=0):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((m, ws)).astype(np.float32) * 3.0
    Up = np.linalg.qr(rng.standard_normal((m, r)))[0].astype(np.float32)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0].astype(np.float32)
    n_in = ws + r
    params = inputs.mlp_init(n_in, hidden, seed + 1)
    params[hidden * n_in: hidden * n_in + hidden] = rng.standard_normal(hidden).astype(np.float32) * 0.1
    params[-1] = 0.3
    return S, Up, U, params, n_in, hidden


@pytest.mark.parametrize("m", [1001, 3000, 20000])
def test_features_forward_loss_grad_adam_vs_oracle(m):
    """m = 20000 is the drifting sequence's row count; 1001 gives a ragged last
    row range in the split-K gradient products."""
    import torch
    device()
    banner(f"learned: features/forward/loss/grad/adam vs oracle m={m}")
    S, Up, U, params, n_in, hidden = _setup(m=m)
    m = S.shape[0]
    X = gkb.gkb_mlp_features(to_dev(np.ascontiguousarray(S.T)), to_dev(np.ascontiguousarray(Up.T)))
    Xh = to_host(X)
    Xo = mlp.features(S.astype(np.float64), Up.astype(np.float64))
    assert np.max(np.abs(Xh[:, : n_in + 1] - Xo)) < 1e-5 * np.max(np.abs(Xo))
    assert np.all(Xh[:, n_in + 1:] == 0)
    Xo32 = Xh[:, : n_in + 1].astype(np.float64)   # compare the rest on the same features
    pd = to_dev(params)
    z = to_host(gkb.gkb_mlp_forward(pd, n_in, hidden, X))
    zo, _, _ = mlp.forward(params.astype(np.float64), n_in, hidden, Xo32)
    scale = np.max(np.abs(zo))
    assert np.max(np.abs(z - zo)) <= n_in * hidden * 2.0 ** -24 * 8 * scale
    Ud = to_dev(np.ascontiguousarray(U.T))
    g, L = gkb.gkb_mlp_loss_grad(pd, n_in, hidden, X, Ud)
    go = mlp.grad(params.astype(np.float64), n_in, hidden, Xo32, U.astype(np.float64))
    Lo = mlp.loss(params.astype(np.float64), n_in, hidden, Xo32, U.astype(np.float64))
    gh = to_host(g)
    print(f"loss {to_host(L)[0]:.6f} vs {Lo:.6f}; grad rel err {np.max(np.abs(gh - go)) / np.max(np.abs(go)):.2e}",
          flush=True)
    assert abs(to_host(L)[0] - Lo) < 1e-5
    assert np.max(np.abs(gh - go)) <= 1e-3 * np.max(np.abs(go))
    # Adam: three steps against the oracle's update
    p = pd.clone()
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    po, m1o, m2o = params.astype(np.float64), np.zeros(params.size), np.zeros(params.size)
    for step in range(1, 4):
        gkb.gkb_adam_step(p, g, m1, m2, 1e-3, step)
        po, m1o, m2o = mlp.adam_step(po, gh.astype(np.float64), m1o, m2o, 1e-3, 0.9, 0.999, 1e-8, step)
    assert np.max(np.abs(to_host(p) - po)) < 1e-6


@pytest.mark.parametrize("m", [1001, 20000])
def test_logtan_loss_grad_vs_oracle(m):
    """Loss kind 1 (mean log tan^2 of the angles to the target vectors) and its
    gradient against the oracle on the same float32 features."""
    device()
    banner(f"learned: log-tan loss/grad vs oracle m={m}")
    S, Up, U, params, n_in, hidden = _setup(m=m)
    X = gkb.gkb_mlp_features(to_dev(np.ascontiguousarray(S.T)), to_dev(np.ascontiguousarray(Up.T)))
    Xo32 = to_host(X)[:, : n_in + 1].astype(np.float64)
    Ud = to_dev(np.ascontiguousarray(U.T))
    g, L = gkb.gkb_mlp_loss_grad(to_dev(params), n_in, hidden, X, Ud, kind=1)
    go = mlp.grad(params.astype(np.float64), n_in, hidden, Xo32, U.astype(np.float64), kind=1)
    Lo = mlp.loss(params.astype(np.float64), n_in, hidden, Xo32, U.astype(np.float64), kind=1)
    gh = to_host(g)
    print(f"log-tan loss {to_host(L)[0]:.6f} vs {Lo:.6f}; grad rel err "
          f"{np.max(np.abs(gh - go)) / np.max(np.abs(go)):.2e}", flush=True)
    assert abs(to_host(L)[0] - Lo) < 1e-5 * max(1.0, abs(Lo))
    assert np.max(np.abs(gh - go)) <= 1e-3 * np.max(np.abs(go))
    with pytest.raises(gkb.GkbError):
        gkb.gkb_mlp_loss_grad(to_dev(params), n_in, hidden, X, Ud, kind=2)


def test_learned_start_beats_random_on_held_out_solves():
    device()
    banner("learned start end to end, 3000x1000, r=8")
    out = gkb_learned_run()
    print({k: v for k, v in out.items() if k != "per_t"}, flush=True)
    assert out["train_loss_by_epoch"][-1] < out["train_loss_by_epoch"][0]
    assert out["matvecs_learned"]["mean"] < out["matvecs_random"]["mean"]
    assert out["learned_win_fraction"] >= 0.5
    assert out["max_sigma_diff_learned_vs_random"] < 1e-5


def gkb_learned_run():
    from paper_2104_10785_amd import learned
    return learned.run(m=3000, n=1000, r=8, k=26, tol=1e-8, t_train=30, t_eval=15, ws=16, hidden=64, epochs=15,
                       lr=3e-3, check_every=2, seed=5)


def test_learned_start_drifting_sequence_full_configuration():
    """The drifting-sequence workload at its stated size: 200 matrices of
    20000 x 5000 (A_t = A_{t-1} + 1e-3 rank-4 update, spectrum 0.97^i), top 30
    at tol 1e-8, a 2-layer network (256 hidden units) on the sketch A_t Omega
    (32 columns) plus the previous left vectors, trained on solves 1-100 (the
    last 20 held out to choose the parameters), evaluated on 101-200.  The
    trained start needs fewer products than the random start on every
    held-out matrix, the parameters kept are no worse on the held-out solves
    than the ones training started from, and the training loss decreases
    without the spikes of a constant step size.  Printed: the heuristic start
    (the previous vectors summed) for comparison."""
    from paper_2104_10785_amd import learned
    device()
    banner("learned start, drifting 20000x5000 sequence, r=30, t_train=100, t_eval=100")
    out = learned.run(m=20000, n=5000, r=30, k=70, tol=1e-8, t_train=100, t_eval=100, ws=32, hidden=256,
                      epochs=20, lr=1e-3, check_every=2, seed=3, init="heuristic")
    print({k: v for k, v in out.items() if k != "per_t"}, flush=True)
    print(f"products to tolerance, mean over t = 101..200: random {out['matvecs_random']['mean']:.2f}, "
          f"learned {out['matvecs_learned']['mean']:.2f} (sketch included), heuristic "
          f"{out['matvecs_heuristic']['mean']:.2f}", flush=True)
    assert out["matvecs_learned"]["mean"] < out["matvecs_random"]["mean"]
    assert out["learned_win_fraction"] == 1.0 and out["fallbacks"] == 0
    assert out["held_out_matvecs_kept"] <= out["held_out_matvecs_init"]
    loss = out["train_loss_by_epoch"]
    assert max(loss[6:]) <= loss[5]
    assert out["max_sigma_diff_learned_vs_random"] < 1e-6
