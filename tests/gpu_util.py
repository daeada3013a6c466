"""Helpers for the GPU tests: device handle, case banner, host/device copies."""
import sys

import numpy as np
import pytest


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_10785_amd import gkb
    gkb.lib()  # fail loudly if the library is missing
    return torch.device("cuda:0")


def banner(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy()


def sketch_distances(ref, U, V):
    """Distances between a solver's singular vectors and the oracle's, from the
    32-column Gaussian sketches stored with the oracle's reference
    (tests/golden/make_c2_reference.py): for unit vectors a, b,
    ||Omega^T (a - b)|| estimates ||a - b|| (entries of Omega N(0, 1/32)).
    `ref` is the stored run (dict with U_sketch, V_sketch); U, V are m x r and
    n x r float64.  Each pair's common sign is fixed by the sketches.
    Returns per-triplet (du, dv)."""
    from paper_2104_10785_amd import inputs
    width = 32
    m, n = U.shape[0], V.shape[0]
    om_u = inputs.sketch_matrix(m, width, 101, dtype=np.float64) / np.sqrt(width)
    om_v = inputs.sketch_matrix(n, width, 102, dtype=np.float64) / np.sqrt(width)
    su, sv = om_u.T @ U, om_v.T @ V
    ru, rv = np.array(ref["U_sketch"]), np.array(ref["V_sketch"])
    sign = np.sign(np.sum(su * ru, axis=0) + np.sum(sv * rv, axis=0))
    sign[sign == 0] = 1.0
    du = np.linalg.norm(su - ru * sign[None, :], axis=0)
    dv = np.linalg.norm(sv - rv * sign[None, :], axis=0)
    return du, dv
