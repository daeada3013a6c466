"""Riemannian gradient steps (Algorithm 4) on the GPU against the float64
oracle step by step, a short trajectory, learning on held-out pairs, and
graph replays."""
import numpy as np
import pytest

from oracle import rsgd
from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu

D1, D2, R, B = 784, 256, 5, 64
U32 = 2.0 ** -24


def state(plan):
    U = to_host(plan.U).T.astype(np.float64)
    s = to_host(plan.s).astype(np.float64)
    V = to_host(plan.Vt).T.astype(np.float64)
    return U, s, V


@pytest.mark.parametrize("k", [20, 35])
def test_single_steps_match_the_oracle(k):
    device()
    banner(f"rsgd single steps k={k}")
    X, V, y, _, _ = inputs.similarity_pairs(8 * B, D1, D2, seed=1)
    U0, s0, V0 = inputs.rank_r_point(D1, D2, R, seed=3, scale=1.0)
    plan = gkb.RsgdPlan(D1, D2, R, k, B, 0.5, 1e-3, U0, s0, V0)
    U, s, Vf = U0, s0, V0
    for t in range(4):
        sl = slice(t * B, (t + 1) * B)
        # the oracle step from the GPU's current state (float32 factors, exact upcast)
        U, s, Vf = state(plan)
        _, s_ref, _, W_ref, Y = rsgd.step(X[sl], V[sl], y[sl], U, s, Vf, 0.5, 1e-3)
        plan.step(to_dev(X[sl]), to_dev(V[sl]), to_dev(y[sl]))
        info = plan.info()
        W = to_host(plan.weights()).astype(np.float64)
        nY = np.linalg.norm(Y, 2)
        err_w = np.abs(W - W_ref).max()
        err_s = np.abs(to_host(plan.s) - s_ref).max()
        print(f"  step {t}: status {info[0]}, |W - W_ref| {err_w:.2e}, |s - s_ref| {err_s:.2e}, ||Y|| {nY:.3f}",
              flush=True)
        assert info[0] == 0
        # float32 Y and factors, float64 products: each entry of Y carries ~u32 ||Y|| of
        # rounding and the rank-r truncation (gap s_r >> s_{r+1} of Y) passes it on
        # unamplified; 16 u32 ||Y|| ~ 1e-6 ||Y|| leaves room for the Krylov rounding
        assert err_s <= 16 * U32 * nY and err_w <= 16 * U32 * nY
    plan.close()


def test_trajectory_and_learning():
    device()
    banner("rsgd trajectory 40 steps and held-out accuracy")
    X, V, y, _, _ = inputs.similarity_pairs(40 * B, D1, D2, seed=1)
    Xt, Vt, yt, _, _ = inputs.similarity_pairs(4000, D1, D2, seed=2)
    U0, s0, V0 = inputs.rank_r_point(D1, D2, R, seed=3, scale=0.01)
    plan = gkb.RsgdPlan(D1, D2, R, 20, B, 2.0, 1e-3, U0, s0, V0)
    U, s, Vf = U0, s0, V0
    acc0 = rsgd.accuracy(Xt, Vt, yt, (U * s) @ Vf.T)
    for t in range(40):
        sl = slice(t * B, (t + 1) * B)
        U, s, Vf, W_ref, _ = rsgd.step(X[sl], V[sl], y[sl], U, s, Vf, 2.0, 1e-3)
        plan.step(to_dev(X[sl]), to_dev(V[sl]), to_dev(y[sl]))
    W = to_host(plan.weights()).astype(np.float64)
    rel = np.linalg.norm(W - W_ref) / np.linalg.norm(W_ref)
    acc_gpu = rsgd.accuracy(Xt, Vt, yt, W)
    acc_ref = rsgd.accuracy(Xt, Vt, yt, W_ref)
    print(f"  after 40 steps: ||W - W_ref|| / ||W_ref|| = {rel:.2e}; held-out accuracy {acc0:.3f} -> "
          f"{acc_gpu:.4f} (oracle {acc_ref:.4f})", flush=True)
    assert rel < 1e-4
    assert acc_gpu > 0.75 and acc0 < 0.6
    assert abs(acc_gpu - acc_ref) < 0.005
    plan.close()


def test_replays_are_deterministic():
    device()
    banner("rsgd graph replays")
    X, V, y, _, _ = inputs.similarity_pairs(5 * B, D1, D2, seed=4)
    U0, s0, V0 = inputs.rank_r_point(D1, D2, R, seed=5)
    outs = []
    for _ in range(2):
        plan = gkb.RsgdPlan(D1, D2, R, 20, B, 1.0, 1e-3, U0, s0, V0)
        for t in range(5):
            sl = slice(t * B, (t + 1) * B)
            plan.step(to_dev(X[sl]), to_dev(V[sl]), to_dev(y[sl]))
        outs.append(to_host(plan.weights()))
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_rsgd_validation():
    device()
    banner("rsgd validation")
    U0, s0, V0 = inputs.rank_r_point(D1, D2, R, seed=5)
    with pytest.raises(gkb.GkbError):
        gkb.RsgdPlan(D1, D2, R, 80, B, 1.0, 1e-3, U0, s0, V0)      # k > 64
    with pytest.raises(gkb.GkbError):
        gkb.RsgdPlan(D1, D2, R, 20, B, -1.0, 1e-3, U0, s0, V0)     # eta <= 0
