"""Solve plans (gkb_svd_plan_*): the stretches of device work between host
synchronisations are captured as HIP graphs by the first solve that reaches
them and replayed by later ones.  Every solve must equal gkb_partial_svd on the
same inputs bitwise -- over several replays with other device work in between,
after the matrix has been changed in place, and with another start vector."""
import numpy as np
import pytest

from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a[3] == b[3]
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(to_host(a[1]), to_host(b[1])) and np.array_equal(to_host(a[2]), to_host(b[2]))
    for key in ("nconv", "restarts", "matvecs", "checks", "krylov_dim", "returned", "refreshes"):
        assert a[4][key] == b[4][key], key


@pytest.mark.parametrize("case", ["f64_restarts", "f64_checks", "f32_one_pass_checks", "f32_two_product",
                                  "f64_one_pass_restarts", "f32_team_one_pass_checks"])
def test_plan_matches_direct_solves(case):
    """The last two cases capture the team sweep (float64 rows; 30000-column
    float32 rows): its mailbox generation lives on the device, so replays
    advance it as the direct solves do."""
    import torch
    device()
    if case.startswith("f64"):
        s = inputs.decade_spectrum(1000)
        A, _, _ = inputs.svd_matrix(2000, 1000, s, seed=0)
        r, k, tol, every, one_pass = 10, 30, 1e-10, (5 if case == "f64_checks" else 0), "one_pass" in case
    elif case == "f32_team_one_pass_checks":
        A, _, _, _ = inputs.lowrank_noise(1500, 30000, 60, 0.9, 1e-6, seed=11, dtype=np.float32)
        r, k, tol, every, one_pass = 8, 24, 1e-6, 4, True
    else:
        A, _, _, _ = inputs.lowrank_noise(6000, 2500, 200, 0.95, 1e-6, seed=7, dtype=np.float32)
        r, k, tol, every, one_pass = 20, 60, 1e-6, (5 if "checks" in case else 0), case.endswith("checks")
    banner(f"solve plan {case}: {A.shape} r={r} k={k} check_every={every} one_pass={one_pass}")
    Ad = to_dev(A)
    q = to_dev(inputs.start_vector(A.shape[0], seed=1))
    q2 = to_dev(inputs.start_vector(A.shape[0], seed=2))
    plan = gkb.SvdPlan(Ad, r, k, tol, 50, q1=q, check_every=every, one_pass=one_pass)
    for rep in range(3):
        got = plan.run()
        want = gkb.gkb_partial_svd(Ad, r, k, tol, 50, q1=q, check_every=every, one_pass=one_pass)
        _same(got, want)
        assert got[3] == 0 and got[4]["one_pass_used"] == (1 if one_pass else 0)
        x = torch.randn(512, 512, device="cuda:0")
        (x @ x).sum().item()   # other device work between the replays
        torch.cuda.synchronize()
    got = plan.run(q1=q2)
    _same(got, gkb.gkb_partial_svd(Ad, r, k, tol, 50, q1=q2, check_every=every, one_pass=one_pass))
    Ad.mul_(2.0)   # the matrix changed in place: same buffer, new contents
    torch.cuda.synchronize()
    got = plan.run()
    want = gkb.gkb_partial_svd(Ad, r, k, tol, 50, q1=q, check_every=every, one_pass=one_pass)
    _same(got, want)
    print(f"{case}: sigma_1 {got[0][0]:.6f}, matvecs {got[4]['matvecs']}, restarts {got[4]['restarts']}", flush=True)
    plan.close()


def test_plan_validation():
    device()
    banner("solve plan argument checks")
    A = to_dev(np.random.default_rng(0).standard_normal((60, 40)))
    with pytest.raises(gkb.GkbError):
        gkb.SvdPlan(A, 5, 3, 1e-6, 1)
    with pytest.raises(gkb.GkbError) as ei:
        gkb.SvdPlan(A, 2, 6, 1e-6, 1, phase_timing=True)
    assert ei.value.status == -1
