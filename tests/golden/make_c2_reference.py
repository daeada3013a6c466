"""Write the oracle's reference for the large float32 workload.

Workload: A = U_f diag(0.95^i)_{i=1..200} V_f^T + E, 50000 x 20000, E iid
N(0, (1e-6)^2), rounded once to float32 (paper_2104_10785_amd.inputs.lowrank_noise,
seed 2); start vector q ~ N(2, 1) (inputs.start_vector, seed 1).  The oracle
(float64 on the exact upcast of the float32 matrix) computes the top 50
triplets with Krylov dimension 120, tol 1e-6, up to 20 restarts, relative
breakdown threshold 1e-6 (the float32 default).

The solve is run twice: with the convergence test only at the end of each
cycle (fixed k) and with the in-cycle test every 10 right vectors (the
benchmark's schedule).  Besides the singular values, each run stores sketches
of its singular vectors, Omega_U^T U and Omega_V^T V with Gaussian Omega
(50000 x 32 and 20000 x 32, entries N(0, 1/32), seeds 101 and 102 of the input
generator): for any unit vectors a, b, ||Omega^T (a - b)|| estimates ||a - b||
(Johnson-Lindenstrauss), so a solver's vectors can be compared with the
oracle's without storing 70000 x 50 numbers.

Only oracle/ and the input generator are used.  Output:
tests/golden/c2_oracle_top50.json.

    python tests/golden/make_c2_reference.py      # about 10 minutes, ~20 GB RAM
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


SKETCH_WIDTH, SKETCH_SEED_U, SKETCH_SEED_V = 32, 101, 102


def sketches(m, n):
    """The fixed Gaussian sketch blocks for left and right vectors."""
    om_u = inputs.sketch_matrix(m, SKETCH_WIDTH, SKETCH_SEED_U, dtype=np.float64) / np.sqrt(SKETCH_WIDTH)
    om_v = inputs.sketch_matrix(n, SKETCH_WIDTH, SKETCH_SEED_V, dtype=np.float64) / np.sqrt(SKETCH_WIDTH)
    return om_u, om_v


def summary(out, seconds, om_u, om_v):
    return {
        "sigma": out["sigma"].tolist(),
        "res_est": out["res_est"].tolist(),
        "nconv": out["nconv"], "restarts": out["restarts"], "matvecs": out["matvecs"],
        "status": out["status"], "checks": out["checks"],
        "krylov_dim": int(out["factorization"].H.shape[1]),
        "U_sketch": (om_u.T @ out["U"]).tolist(),
        "V_sketch": (om_v.T @ out["V"]).tolist(),
        "oracle_seconds": seconds,
    }


def main():
    t0 = time.time()
    A32, s, _, _ = inputs.lowrank_noise(M, N, RANK, DECAY, NOISE, seed=SEED, dtype=np.float32)
    A = A32.astype(np.float64)
    del A32
    q = inputs.start_vector(M, seed=QSEED)
    om_u, om_v = sketches(M, N)
    t1 = time.time()
    out = gk.partial_svd(A, R, K, TOL, RESTARTS, q, eps_break=1e-6)
    t2 = time.time()
    out10 = gk.partial_svd(A, R, K, TOL, RESTARTS, q, eps_break=1e-6, check_every=10)
    t3 = time.time()
    ref = {
        "workload": "lowrank_noise 50000x20000 rank 200 decay 0.95 noise 1e-6 float32 seed 2; q seed 1",
        "r": R, "k": K, "tol": TOL, "max_restarts": RESTARTS, "eps_break": 1e-6,
        "sketch": {"width": SKETCH_WIDTH, "seed_u": SKETCH_SEED_U, "seed_v": SKETCH_SEED_V,
                   "scale": "1/sqrt(width)"},
        "generation_seconds": t1 - t0,
    }
    ref.update(summary(out, t2 - t1, om_u, om_v))
    ref["check_every_10"] = summary(out10, t3 - t2, om_u, om_v)
    with open(os.path.join(HERE, "c2_oracle_top50.json"), "w") as f:
        json.dump(ref, f, indent=1)
    print(json.dumps({k: v for k, v in ref.items() if k not in ("sigma", "res_est", "U_sketch", "V_sketch",
                                                                  "check_every_10")}))
    print(json.dumps({k: v for k, v in ref["check_every_10"].items()
                      if k not in ("sigma", "res_est", "U_sketch", "V_sketch")}))


if __name__ == "__main__":
    main()
