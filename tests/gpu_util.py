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
