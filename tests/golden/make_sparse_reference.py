"""Write the oracle's reference for the large sparse workload.

Workload: paper_2104_10785_amd.inputs.sparse_powerlaw(1000000, 200000,
50000000, seed=7): power-law row degrees (exponent 0.6) and column
popularity (exponent 0.5), N(0, 1) float32 values; start vector q ~ N(2, 1)
(inputs.start_vector, seed 8).  The oracle (float64, scipy CSR of the exact
float32 values) computes the top 20 triplets with Krylov dimension 60, tol
1e-6, up to 50 restarts, relative breakdown threshold 1e-6 (the float32
default), convergence checked every 5 vectors.

Only oracle/ and the input generator are used.  Output:
tests/golden/sparse_oracle_top20.json.

    python tests/golden/make_sparse_reference.py      # several minutes, ~10 GB RAM
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import gk  # noqa: E402
from paper_2104_10785_amd import inputs  # noqa: E402

M, N, NNZ, SEED, QSEED = 1000000, 200000, 50000000, 7, 8
R, K, TOL, RESTARTS, EVERY = 20, 60, 1e-6, 50, 5


def main():
    t0 = time.time()
    S = inputs.sparse_powerlaw(M, N, NNZ, seed=SEED)
    A = sp.csr_matrix((S["val"].astype(np.float64), S["col_idx"], S["row_ptr"]), shape=(M, N))
    del S
    q = inputs.start_vector(M, seed=QSEED)
    t1 = time.time()
    out = gk.partial_svd(A, R, K, TOL, RESTARTS, q, eps_break=1e-6, check_every=EVERY)
    t2 = time.time()
    ref = {
        "workload": f"sparse_powerlaw {M}x{N} nnz {NNZ} seed {SEED}; q seed {QSEED}",
        "r": R, "k": K, "tol": TOL, "max_restarts": RESTARTS, "eps_break": 1e-6, "check_every": EVERY,
        "sigma": out["sigma"].tolist(),
        "res_est": out["res_est"].tolist(),
        "nconv": out["nconv"], "restarts": out["restarts"], "matvecs": out["matvecs"],
        "status": out["status"],
        "oracle_seconds": t2 - t1, "generation_seconds": t1 - t0,
    }
    with open(os.path.join(HERE, "sparse_oracle_top20.json"), "w") as f:
        json.dump(ref, f, indent=1)
    print(json.dumps({k: v for k, v in ref.items() if k not in ("sigma", "res_est")}))


if __name__ == "__main__":
    main()
