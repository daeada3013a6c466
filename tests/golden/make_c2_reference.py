"""Write the oracle's reference for the large float32 workload.

Workload: A = U_f diag(0.95^i)_{i=1..200} V_f^T + E, 50000 x 20000, E iid
N(0, (1e-6)^2), rounded once to float32 (paper_2104_10785_amd.inputs.lowrank_noise,
seed 2); start vector q ~ N(2, 1) (inputs.start_vector, seed 1).  The oracle
(float64 on the exact upcast of the float32 matrix) computes the top 50
triplets with Krylov dimension 120, tol 1e-6, up to 20 restarts, relative
breakdown threshold 1e-6 (the float32 default).

Only oracle/ and the input generator are used.  Output:
tests/golden/c2_oracle_top50.json.

    python tests/golden/make_c2_reference.py      # about 5 minutes, ~20 GB RAM
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import gk  # noqa: E402
from paper_2104_10785_amd import inputs  # noqa: E402

M, N, RANK, DECAY, NOISE, SEED, QSEED = 50000, 20000, 200, 0.95, 1e-6, 2, 1
R, K, TOL, RESTARTS = 50, 120, 1e-6, 20


def main():
    t0 = time.time()
    A32, s, _, _ = inputs.lowrank_noise(M, N, RANK, DECAY, NOISE, seed=SEED, dtype=np.float32)
    A = A32.astype(np.float64)
    del A32
    q = inputs.start_vector(M, seed=QSEED)
    t1 = time.time()
    out = gk.partial_svd(A, R, K, TOL, RESTARTS, q, eps_break=1e-6)
    t2 = time.time()
    ref = {
        "workload": "lowrank_noise 50000x20000 rank 200 decay 0.95 noise 1e-6 float32 seed 2; q seed 1",
        "r": R, "k": K, "tol": TOL, "max_restarts": RESTARTS, "eps_break": 1e-6,
        "sigma": out["sigma"].tolist(),
        "res_est": out["res_est"].tolist(),
        "nconv": out["nconv"], "restarts": out["restarts"], "matvecs": out["matvecs"],
        "status": out["status"],
        "oracle_seconds": t2 - t1, "generation_seconds": t1 - t0,
    }
    with open(os.path.join(HERE, "c2_oracle_top50.json"), "w") as f:
        json.dump(ref, f, indent=1)
    print(json.dumps({k: v for k, v in ref.items() if k not in ("sigma", "res_est")}))


if __name__ == "__main__":
    main()
