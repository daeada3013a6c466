"""gkb_partial_svd_noalloc (the library's fixed device array as workspace)
against gkb_partial_svd with a caller workspace: same kernels, same layout,
so the results must be bitwise equal; two calls in a row, the second on a
smaller problem (the array keeps the first call's contents), the one-sweep
step on both the single-workgroup and the team sweep, plus the rejection of
a problem whose workspace exceeds the array."""
import numpy as np
import pytest

from paper_2104_10785_amd import gkb, inputs

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu


def _both(A, r, k, tol, restarts, q, **kw):
    import torch
    Ad, qd = to_dev(A), to_dev(q)
    ref = gkb.gkb_partial_svd(Ad, r, k, tol, restarts, q1=qd, **kw)
    bt = ref[1].dtype
    Ut = torch.full((r, A.shape[0]), np.nan, dtype=bt, device="cuda:0")
    Vt = torch.full((r, A.shape[1]), np.nan, dtype=bt, device="cuda:0")
    torch.cuda.synchronize()
    got = gkb.gkb_partial_svd_noalloc(Ad, r, k, tol, restarts, q1=qd, U=Ut, V=Vt, **kw)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got):
    assert got[3] == ref[3]
    assert np.array_equal(got[0], ref[0])
    assert np.array_equal(to_host(got[1]), to_host(ref[1]))
    assert np.array_equal(to_host(got[2]), to_host(ref[2]))
    for key in ("nconv", "restarts", "matvecs", "checks", "krylov_dim", "returned"):
        assert got[4][key] == ref[4][key], key


def test_noalloc_matches_workspace_entry_point():
    device()
    # first call: 3000 x 1200 float64 with restarts and in-cycle checks
    s = inputs.decade_spectrum(1200)
    A, _, _ = inputs.svd_matrix(3000, 1200, s, seed=41)
    q = inputs.start_vector(3000, seed=42)
    need = gkb.gkb_workspace_size(to_dev(A), 10, 40)
    banner(f"no-alloc 3000x1200 f64 r=10 k=40 (workspace {need} bytes)")
    assert 0 < need <= gkb.NOALLOC_SCRATCH_BYTES
    ref, got = _both(A, 10, 40, 1e-10, 30, q, check_every=5)
    _same(ref, got)
    # second call, smaller: 700 x 300 float32
    A2, _, _, _ = inputs.lowrank_noise(700, 300, 60, 0.9, 1e-6, seed=43, dtype=np.float32)
    q2 = inputs.start_vector(700, seed=44)
    banner("no-alloc 700x300 f32 r=5 k=20 after the larger call")
    ref2, got2 = _both(A2, 5, 20, 1e-6, 30, q2)
    _same(ref2, got2)
    # and the one-sweep step on the smaller problem
    ref3, got3 = _both(A2, 5, 20, 1e-6, 30, q2, one_pass=True)
    _same(ref3, got3)
    # the one-sweep step through the team sweep, whose mailbox is part of the
    # workspace: float64 rows, then float32 rows longer than one workgroup holds
    A4, _, _ = inputs.svd_matrix(800, 500, np.geomspace(1.0, 1e-3, 500), seed=45)
    q4 = inputs.start_vector(800, seed=46)
    A5, _, _, _ = inputs.lowrank_noise(200, 24580, 40, 0.9, 1e-6, seed=47, dtype=np.float32)
    q5 = inputs.start_vector(200, seed=48)
    for name, Ax, qx, r, k in (("800x500 f64", A4, q4, 5, 20), ("200x24580 f32", A5, q5, 3, 12)):
        need = gkb.gkb_workspace_size(to_dev(Ax), r, k, one_pass=True)
        banner(f"no-alloc {name} one-sweep (team sweep) r={r} k={k} (workspace {need} bytes)")
        assert 0 < need <= gkb.NOALLOC_SCRATCH_BYTES
        ref4, got4 = _both(Ax, r, k, 1e-6, 30, qx, one_pass=True)
        assert ref4[4]["one_pass_used"] == 1 and got4[4]["one_pass_used"] == 1
        _same(ref4, got4)


def test_noalloc_rejects_too_large():
    import torch
    device()
    banner("no-alloc rejects a workspace above the fixed array")
    A = torch.zeros((40000, 200), dtype=torch.float64, device="cuda:0")
    need = gkb.gkb_workspace_size(A, 10, 150)
    assert need > gkb.NOALLOC_SCRATCH_BYTES
    with pytest.raises(gkb.GkbError) as ei:
        gkb.gkb_partial_svd_noalloc(A, 10, 150, 1e-6, 1)
    assert ei.value.status == -4
    with pytest.raises(gkb.GkbError) as ei:
        gkb.gkb_partial_svd_noalloc(A, 10, 20, 1e-6, 1, phase_timing=True)
    assert ei.value.status == -1
