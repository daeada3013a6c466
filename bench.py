"""Benchmark: partial SVD of the large float32 low-rank-plus-noise matrix.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --kernels-only      # only the product kernels, the Ritz GEMMs and a 1 GiB copy

Workload: A = U_f diag(0.95^i)_{i=1..200} V_f^T + E, 50000 x 20000 float32,
E iid N(0, (1e-6)^2) (synthetic, seeded); top 50 triplets, Krylov dimension
120, tol 1e-6, up to 20 restarts, in-cycle convergence tests every 10
vectors.  One step = one gkb_partial_svd call (start vector, Golub-Kahan
cycles with one sweep of A per step -- --two-pass for the two-product step --
and CGS2, host small SVDs, restarts, Ritz GEMMs), with A already resident in
HBM.

Prints one JSON line: converged triplets per second (whole job), the
roofline of the dominant kernel (the one-sweep product pair), the float64
CPU oracle's full solves of the same workload, and the extra legs.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, N, RANK, DECAY, NOISE, SEED, QSEED = 50000, 20000, 200, 0.95, 1e-6, 2, 1
R, K, TOL, RESTARTS = 50, 120, 1e-6, 20
CHECK_EVERY = 10
HBM_PEAK_GBS = 8000.0
F32_MFMA_PEAK_TFLOPS = 157.3
# HBM traffic per launch of the A-streaming kernels, measured with hardware
# counters (FETCH_SIZE and WRITE_SIZE, calibrated against a 1 GiB copy); each
# summary is valid only for the kernel sources whose digest it records.
TRAFFIC = {
    "gemv_n": ("gemv_c2_f32_hbm_traffic.md", ["paper_2104_10785_amd/csrc/gemv.hip", "paper_2104_10785_amd/csrc/gemv.h",
                                              "paper_2104_10785_amd/csrc/device_common.h"]),
    "gemv_fused": ("gemv_fused_c2_f32_hbm_traffic.md", ["paper_2104_10785_amd/csrc/fused.hip",
                                                        "paper_2104_10785_amd/csrc/fused.h",
                                                        "paper_2104_10785_amd/csrc/fused_device.h"]),
}
TRAFFIC["gemv_t"] = TRAFFIC["gemv_n"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_kernel(fn, reps, stream):
    """Average device duration of fn() over reps launches, bracketed by HIP events
    recorded on the stream the launches go to."""
    import torch
    fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def kernel_source_digest(kernel="gemv_n"):
    h = hashlib.sha256()
    for rel in TRAFFIC[kernel][1]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` ("gemv_n", "gemv_t" or "gemv_fused") from
    the committed counter summary, or None when it is absent or was taken on
    other sources."""
    path = os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^\s*([a-z_]+):\s*(\S+)\s*$", line)
            if m:
                vals[m.group(1)] = m.group(2)
    if vals.get("source_digest") != kernel_source_digest(kernel) or f"{kernel}_bytes" not in vals:
        return None
    return float(vals[f"{kernel}_bytes"])


def matvec_operands(torch, Ad, dev):
    xn = torch.randn(N, dtype=torch.float32, device=dev)
    xm = torch.randn(M, dtype=torch.float32, device=dev)
    yn = torch.empty(M, dtype=torch.float64, device=dev)
    ym = torch.empty(N, dtype=torch.float64, device=dev)
    return xn, xm, yn, ym


def fused_operands(gkb, torch, Ad, dev):
    p = torch.randn(N, dtype=torch.float32, device=dev)
    w = torch.empty(M, dtype=torch.float64, device=dev)
    y = torch.empty(N, dtype=torch.float64, device=dev)
    ws = torch.empty(max(256, gkb.lib().gkb_matvec_fused_workspace_size(gkb.C.byref(gkb.make_matrix(Ad)))),
                     dtype=torch.uint8, device=dev)
    return p, w, y, ws


def kernels_only(gkb, torch, Ad, dev, stream, reps, f64=False, bf16=False, unaligned=False):
    """The A-streaming kernels alone (reps launches each: A p, A^T q, and the
    one-sweep pair A p, A^T A p) and a plain 1 GiB device copy (3 launches)
    whose counter readings calibrate the traffic figures.  f64: the same
    matrix upcast to float64 (8.0 GB), the two products only (the one-sweep
    pair holds float32 or bfloat16 rows).  bf16: the matrix rounded to
    bfloat16 (2.0 GB).  unaligned: the float32 matrix copied into rows of
    n + 1 elements (lda = 20001: rows not 16-byte aligned), the two products
    only."""
    if f64:
        Ad = Ad.double()
    elif bf16:
        Ad = gkb.gkb_cast_bf16(Ad)
    elif unaligned:
        buf = torch.zeros((M, N + 1), dtype=torch.float32, device=dev)
        buf[:, :N].copy_(Ad)
        Ad = buf[:, :N]
    mws = torch.empty(gkb.gkb_matvec_workspace_size(Ad), dtype=torch.uint8, device=dev)
    xn, xm, yn, ym = matvec_operands(torch, Ad, dev)
    if Ad.dtype == torch.float64:
        xn, xm = xn.double(), xm.double()
    ms_n = time_kernel(lambda: gkb.gkb_matvec(Ad, xn, 0, y=yn, stream=stream), reps, stream)
    ms_t = time_kernel(lambda: gkb.gkb_matvec(Ad, xm, 1, y=ym, workspace=mws, stream=stream), reps, stream)
    ms_f, ritz = None, None
    if not (f64 or unaligned):   # the one-sweep pair takes aligned float32 or bfloat16 rows only
        fp, fw, fy, fws = fused_operands(gkb, torch, Ad, dev)
        ms_f = time_kernel(lambda: gkb.gkb_matvec_fused(Ad, fp, fw, fy, fws, stream=stream), reps, stream)
        ritz = ritz_gemms(gkb, torch, dev, stream, reps)
    src = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    es = Ad.element_size()
    vs = 8 if Ad.dtype == torch.float64 else 4   # input vector element (basis type)
    dname = "f64" if Ad.dtype == torch.float64 else ("bf16" if bf16 else ("f32_lda20001" if unaligned else "f32"))
    print(json.dumps({"kernels_only": True, "dtype": dname, "gemv_n_ms": ms_n, "gemv_t_ms": ms_t,
                      "gemv_n_GBps": (M * N * es + N * vs + M * 8) / (ms_n * 1e-3) / 1e9,
                      "gemv_t_GBps": (M * N * es + M * vs + N * 8) / (ms_t * 1e-3) / 1e9, "gemv_fused_ms": ms_f,
                      "gemv_fused_GBps": None if ms_f is None else (M * N * es + N * 4 + M * 8 + N * 8) / (ms_f * 1e-3) / 1e9,
                      "reps": reps, "ritz_gemms": ritz, "copy_bytes": 2 ** 30,
                      "source_digest": kernel_source_digest("gemv_n"),
                      "fused_source_digest": kernel_source_digest("gemv_fused")}), flush=True)


def ritz_gemms(gkb, torch, dev, stream, reps):
    """The Ritz-vector products of the workload at their real shapes on the float32
    MFMA: U = Q_k X_r (m x k times k x r) and V = P_k Y_r (n x k times k x r)."""
    out = {}
    for name, rows in (("U=QX", M), ("V=PY", N)):
        Bt = torch.randn(K, rows, dtype=torch.float32, device=dev)   # basis, column-major rows x K
        Xt = torch.randn(R, K, dtype=torch.float32, device=dev)      # small factor, column-major K x R
        Ct = torch.empty(R, rows, dtype=torch.float32, device=dev)
        ms = time_kernel(lambda: gkb.gkb_gemm_tall(Bt, Xt, C_out=Ct, stream=stream), reps, stream)
        flops = 2.0 * rows * K * R
        byts = 4.0 * (rows * K + K * R + rows * R)
        out[name] = {"ms": ms, "TFLOPs": flops / (ms * 1e-3) / 1e12, "GBps": byts / (ms * 1e-3) / 1e9,
                     "mfma_frac_of_f32_peak": flops / (ms * 1e-3) / 1e12 / F32_MFMA_PEAK_TFLOPS,
                     "hbm_frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def headline_accuracy(sigma, Ut, Vt, check_every):
    """Per-triplet singular-value error of the timed solve against the float64
    oracle's solve of the same matrix with the same schedule (stored in
    tests/golden/c2_oracle_top50.json by an oracle-only script), and the
    distances of the singular vectors estimated through the oracle's stored
    32-column Gaussian sketches."""
    ref_path = os.path.join(ROOT, "tests", "golden", "c2_oracle_top50.json")
    if not os.path.exists(ref_path):
        return None
    from paper_2104_10785_amd import inputs
    ref_all = json.load(open(ref_path))
    ref = ref_all["check_every_10"] if check_every == 10 else (ref_all if check_every == 0 else None)
    if ref is None:
        return None
    want = np.array(ref["sigma"])
    err = np.abs(sigma - want)
    U = Ut.double().cpu().numpy().T
    V = Vt.double().cpu().numpy().T
    om_u = inputs.sketch_matrix(M, 32, 101, dtype=np.float64) / np.sqrt(32)
    om_v = inputs.sketch_matrix(N, 32, 102, dtype=np.float64) / np.sqrt(32)
    su, sv = om_u.T @ U, om_v.T @ V
    ru, rv = np.array(ref["U_sketch"]), np.array(ref["V_sketch"])
    sign = np.sign(np.sum(su * ru, axis=0) + np.sum(sv * rv, axis=0))
    sign[sign == 0] = 1.0
    du = np.linalg.norm(su - ru * sign[None, :], axis=0)
    dv = np.linalg.norm(sv - rv * sign[None, :], axis=0)
    return {"oracle_schedule": f"check_every={check_every}", "sigma_abs_err_max": float(err.max()),
            "sigma_rel_err_max": float(np.max(err / want)), "sigma_rel_err_median": float(np.median(err / want)),
            "sigma_rel_err_per_triplet": [float(x) for x in err / want],
            "u_dist_max_sketch": float(du.max()), "v_dist_max_sketch": float(dv.max()),
            "oracle_matvecs": ref["matvecs"], "oracle_checks": ref["checks"]}


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "cus": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2**30, 1), "hip": torch.version.hip}


def blas_threads():
    """Threads of the BLAS library numpy runs the oracle's products on."""
    try:
        from threadpoolctl import threadpool_info
        n = [d["num_threads"] for d in threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A32, q, warmup=2, reps=5, check_every=CHECK_EVERY):
    """Time the float64 oracle on the host, like for like with the GPU solve:
    full oracle.gk.partial_svd solves of the exact float64 upcast of the same
    matrix, with the same start vector, r, k, tol, restart limit, breakdown
    threshold and in-cycle test schedule; `warmup` untimed solves, then `reps`
    timed ones (mean and median wall time)."""
    from oracle import gk
    threads = blas_threads()
    t0 = time.time()
    A = A32.astype(np.float64)
    t_up = time.time() - t0

    def solve():
        return gk.partial_svd(A, R, K, TOL, RESTARTS, q, eps_break=1e-6, check_every=check_every)

    for _ in range(warmup):
        solve()
    times = []
    for _ in range(reps):
        t1 = time.perf_counter()
        ref = solve()
        times.append(time.perf_counter() - t1)
    del A
    mean_s, med_s = float(np.mean(times)), float(np.median(times))
    return {"value": ref["nconv"] / mean_s, "unit": "triplets/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(), "nproc": os.cpu_count(),
            "s_per_solve_mean": mean_s, "s_per_solve_median": med_s, "s_per_solve": times,
            "triplets_per_s_median": ref["nconv"] / med_s, "nconv": ref["nconv"], "matvecs": ref["matvecs"],
            "checks": ref["checks"], "status": ref["status"],
            "sample": f"{reps} full oracle solves (after {warmup} untimed) of the 50000x20000 workload on the "
                      f"exact float64 upcast of the same float32 matrix: top {R}, k {K}, tol {TOL}, in-cycle "
                      f"test every {check_every}, same start vector; numpy/BLAS on {threads} threads; the "
                      f"upcast ({t_up:.1f} s) is outside the timing"}


def bf16_leg(gkb, torch, Ad, qd, stream, steps, one_pass=True):
    """bfloat16 storage + float32 Rayleigh-Ritz refinement of the same matrix;
    one sweep of the bfloat16 A per step (and two, for comparison)."""
    A16 = gkb.gkb_cast_bf16(Ad)
    ws = torch.empty(max(gkb.gkb_workspace_size(A16, R, K, refine=Ad),
                         gkb.gkb_workspace_size(A16, R, K, refine=Ad, one_pass=True)),
                     dtype=torch.uint8, device=Ad.device)

    def run(one):
        return gkb.gkb_partial_svd(A16, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream,
                                   check_every=CHECK_EVERY, refine=Ad, one_pass=one)

    def timed(one):
        run(one)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = run(one)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / steps, res

    ms, (sig, _, _, status, st) = timed(one_pass)
    ms_other, (sig_o, _, _, _, st_o) = timed(not one_pass)
    un = gkb.gkb_partial_svd(A16, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream, check_every=CHECK_EVERY,
                             one_pass=one_pass)[0]
    out = {"step": "one_sweep" if one_pass else "two_product", "ms": ms,
           "triplets_per_s": st["nconv"] / (ms / 1000.0), "matvecs": st["matvecs"],
           "ms_refine": st["ms_refine"], "refined": st["refined"],
           ("two_product" if one_pass else "one_sweep"): {
               "ms": ms_other, "triplets_per_s": st_o["nconv"] / (ms_other / 1000.0), "matvecs": st_o["matvecs"]}}
    ref_path = os.path.join(ROOT, "tests", "golden", "c2_oracle_top50.json")
    if os.path.exists(ref_path):
        want = np.array(json.load(open(ref_path))["sigma"])
        e_ref = np.abs(sig - want) / want
        e_un = np.abs(un - want) / want
        e_o = np.abs(sig_o - want) / want
        out["sigma_rel_err_vs_f64_oracle"] = {
            "unrefined_max": float(e_un.max()), "unrefined_median": float(np.median(e_un)),
            "refined_max": float(e_ref.max()), "refined_median": float(np.median(e_ref)),
            "refined_max_other_step": float(e_o.max()),
            "refined_per_triplet": [float(x) for x in e_ref]}
    xn = torch.randn(N, dtype=torch.float32, device=Ad.device)
    xm = torch.randn(M, dtype=torch.float32, device=Ad.device)
    yn = torch.empty(M, dtype=torch.float64, device=Ad.device)
    ym = torch.empty(N, dtype=torch.float64, device=Ad.device)
    mws = torch.empty(gkb.gkb_matvec_workspace_size(A16), dtype=torch.uint8, device=Ad.device)
    ms_n = time_kernel(lambda: gkb.gkb_matvec(A16, xn, 0, y=yn, stream=stream), 20, stream)
    ms_t = time_kernel(lambda: gkb.gkb_matvec(A16, xm, 1, y=ym, workspace=mws, stream=stream), 20, stream)
    fp, fw, fy, fws = fused_operands(gkb, torch, A16, Ad.device)
    ms_f = time_kernel(lambda: gkb.gkb_matvec_fused(A16, fp, fw, fy, fws, stream=stream), 20, stream)
    out["gemv_n_bf16_GBps"] = (M * N * 2 + N * 4 + M * 8) / (ms_n * 1e-3) / 1e9
    out["gemv_t_bf16_GBps"] = (M * N * 2 + M * 4 + N * 8) / (ms_t * 1e-3) / 1e9
    out["gemv_fused_bf16_ms"] = ms_f
    out["gemv_fused_bf16_GBps"] = (M * N * 2 + N * 4 + M * 8 + N * 8) / (ms_f * 1e-3) / 1e9
    del A16, ws
    return out


def rank_leg(gkb, inputs, torch, dev, stream):
    """Numerical rank at the gap after index 200: the same construction with
    noise std 1e-10, threshold 1e-6 * sigma_1; one sweep of A per step, and
    two for comparison."""
    A32, s, _, _ = inputs.lowrank_noise(M, N, RANK, DECAY, 1e-10, seed=SEED, dtype=np.float32)
    Ad = torch.from_numpy(A32).to(dev)
    del A32
    q = torch.from_numpy(inputs.start_vector(M, seed=QSEED)).to(dev)
    ws = torch.empty(max(gkb.gkb_rank_workspace_size(Ad, 400), gkb.gkb_rank_workspace_size(Ad, 400, one_pass=True)),
                     dtype=torch.uint8, device=dev)
    out = {"workload": "low-rank(200, 0.95^i) + noise(1e-10) 50000x20000 f32, tau = 1e-6 sigma_1", "expected": 200}
    for one_pass in (True, False):
        gkb.gkb_numerical_rank(Ad, 1e-6, k_max=400, q1=q, workspace=ws, stream=stream, one_pass=one_pass)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rank, rank_s, sig, status, st = gkb.gkb_numerical_rank(Ad, 1e-6, k_max=400, q1=q, workspace=ws,
                                                               stream=stream, one_pass=one_pass)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0
        res = {"rank": rank, "rank_sturm": rank_s, "steps": len(sig), "matvecs": st["matvecs"], "ms": ms}
        if one_pass:
            res["recomputed_columns"] = st["refreshes"]
            out.update(res)
        else:
            out["two_product"] = res
    del Ad, ws
    return out


def batched_leg(gkb, inputs, torch, dev, stream):
    """512 uneven problems in one persistent, graph-captured launch."""
    specs = inputs.batch_problems(512, seed=2, materialize=False)
    As = [inputs.batch_matrix_torch(sp, dev) for sp in specs]
    rs = [sp["r"] for sp in specs]
    ks = [min(sp["n"], sp["m"], 2 * sp["r"] + 10) for sp in specs]
    torch.cuda.synchronize()
    plan = gkb.BatchPlan(As, rs, ks, 1e-6, 50, seed=5, check_every=5, tune=True, stream=stream)
    plan.run(stream)
    plan.info(stream)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    plan.run(stream)
    end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end)
    info = plan.info(stream)
    byts = sum(int(info[i, 3]) * sp["m"] * sp["n"] * 4 for i, sp in enumerate(specs))
    out = {"workload": "512 problems, m U[500,4000], n U[200,2000], rho U[0.8,0.99], r U[5,20], k=min(n,2r+10), "
                       "tol 1e-6, f32",
           "ms": ms, "problems_per_s": 512 / (ms / 1000.0),
           "triplets_per_s": int(info[:, 1].sum()) / (ms / 1000.0),
           "converged_problems": int((info[:, 0] == 0).sum()), "matvecs": int(info[:, 3].sum()),
           "A_bytes_GB": sum(sp["m"] * sp["n"] * 4 for sp in specs) / 1e9,
           "streamed_GBps": byts / (ms * 1e-3) / 1e9,
           "threads": plan.tuning["threads"], "workgroups": plan.tuning["workgroups"],
           "form": "out of line" if plan.tuning["form"] == 2 else "inline", "max_team": plan.tuning["max_team"],
           "autotune_ms": plan.tuning["times_ms"]}
    plan.close()
    del As
    return out


C1_M, C1_N, C1_R, C1_K, C1_TOL, C1_RESTARTS, C1_TAU, C1_RANK = 2000, 1000, 10, 30, 1e-10, 50, 10 ** -6.005, 601


def wall_times(fn, warmup, reps, torch=None):
    """warmup untimed calls, then reps timed ones (ms each; the stream is
    synchronised inside each timed call when torch is given)."""
    for _ in range(warmup):
        out = fn()
    if torch is not None:
        torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        if torch is not None:
            torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1000.0)
    return ms, out


def c1_leg(gkb, inputs, torch, dev, stream, warmup=2, reps=5, oracle=True):
    """The CPU-sized float64 workload: A = Q1 diag(10^(-i/100)) Q2^T, 2000 x 1000
    (16 MB, resident in the GPU's caches), top 10 triplets, Krylov dimension
    30, tol 1e-10, and the numerical rank at tau = 10^-6.005 relative to
    sigma_1, i.e. 10^-6.015 (rank 601: the log-midpoint between s_601 and
    s_602; the literal 1e-6 s_1 lands on s_601).  GPU solve and rank: warmup untimed, reps
    timed (mean and median), directly and through a solve plan (the
    stretches between host synchronisations replayed as HIP graphs).  The
    float64 oracle runs the same solve and rank on the host with the same
    inputs and schedule."""
    from oracle import gk
    from oracle import rank as orank
    s = inputs.decade_spectrum(1000)
    A, _, _ = inputs.svd_matrix(C1_M, C1_N, s, seed=0)
    q = inputs.start_vector(C1_M, seed=1)
    Ad = torch.from_numpy(A).to(dev)
    qd = torch.from_numpy(q).to(dev)
    ws = torch.empty(gkb.gkb_workspace_size(Ad, C1_R, C1_K), dtype=torch.uint8, device=dev)
    rws = torch.empty(gkb.gkb_rank_workspace_size(Ad, 0), dtype=torch.uint8, device=dev)
    solve = lambda: gkb.gkb_partial_svd(Ad, C1_R, C1_K, C1_TOL, C1_RESTARTS, q1=qd, workspace=ws, stream=stream)
    rank = lambda: gkb.gkb_numerical_rank(Ad, C1_TAU, q1=qd, workspace=rws, stream=stream)
    ms, (sig, _, _, status, st) = wall_times(solve, warmup, reps, torch)
    ph = gkb.gkb_partial_svd(Ad, C1_R, C1_K, C1_TOL, C1_RESTARTS, q1=qd, workspace=ws, stream=stream,
                             phase_timing=True)[4]
    plan = gkb.SvdPlan(Ad, C1_R, C1_K, C1_TOL, C1_RESTARTS, workspace=ws, q1=qd)
    ms_p, (sig_p, _, _, _, st_p) = wall_times(lambda: plan.run(stream=stream), warmup, reps, torch)
    plan.close()
    ms_r, (rk, rk_s, rsig, _, rst) = wall_times(rank, warmup, reps, torch)
    steps = (st["matvecs"] - 1) / 2
    out = {"workload": "Q1 diag(10^(-i/100)) Q2^T 2000x1000 f64; top 10, k 30, tol 1e-10; rank at tau 10^-6.005 sigma_1",
           "solve_ms_mean": float(np.mean(ms)), "solve_ms_median": float(np.median(ms)),
           "triplets_per_s": st["nconv"] / (np.mean(ms) / 1000.0), "status": status, "matvecs": st["matvecs"],
           "restarts": st["restarts"], "us_per_step": 1000.0 * float(np.mean(ms)) / steps,
           "sigma_rel_err_vs_spectrum_max": float(np.max(np.abs(sig - s[:C1_R]) / s[:C1_R])),
           "phases_ms": {k2: ph[k2] for k2 in ("ms_matvec", "ms_reorth", "ms_sync", "ms_ritz", "ms_other")},
           "ms_host_svd": st["ms_host"],
           "plan_solve_ms_mean": float(np.mean(ms_p)), "plan_solve_ms_median": float(np.median(ms_p)),
           "plan_triplets_per_s": st_p["nconv"] / (np.mean(ms_p) / 1000.0),
           "plan_same_sigma": bool(np.array_equal(sig_p, sig)),
           "rank": rk, "rank_sturm": rk_s, "rank_expected": C1_RANK, "rank_steps": int(rsig.size),
           "rank_ms_mean": float(np.mean(ms_r)), "rank_ms_median": float(np.median(ms_r)),
           "rank_us_per_step": 1000.0 * float(np.mean(ms_r)) / max(1, rsig.size),
           "warmup": warmup, "reps": reps}
    if oracle:
        ms_o, ref = wall_times(lambda: gk.partial_svd(A, C1_R, C1_K, C1_TOL, C1_RESTARTS, q), warmup, reps)
        ms_or, rref = wall_times(lambda: orank.numerical_rank(A, C1_TAU, q), 1, 2)
        out["oracle"] = {"solve_ms_mean": float(np.mean(ms_o)), "solve_ms_median": float(np.median(ms_o)),
                         "triplets_per_s": ref["nconv"] / (np.mean(ms_o) / 1000.0), "matvecs": ref["matvecs"],
                         "rank": rref["rank"], "rank_ms_mean": float(np.mean(ms_or)), "rank_reps": 2,
                         "cores": blas_threads(), "cpu": cpu_model()}
        out["sigma_rel_err_vs_oracle_max"] = float(np.max(np.abs(sig - ref["sigma"]) / ref["sigma"]))
    del Ad, ws, rws
    return out


def f64_leg(gkb, torch, Ad32, qd, stream, reps=3):
    """The 50000 x 20000 matrix in float64 (the exact upcast of the float32
    matrix, 8.0 GB): the two products' HBM rate and the float64 partial SVD
    (two-product step, float64 bases) against the stored float64 oracle run on
    the same matrix; beside it the one-sweep solve (team sweep on float64
    rows) and its largest singular-value difference from the two-product one."""
    Ad = Ad32.double()
    torch.cuda.synchronize()
    xn = torch.randn(N, dtype=torch.float64, device=Ad.device)
    xm = torch.randn(M, dtype=torch.float64, device=Ad.device)
    yn = torch.empty(M, dtype=torch.float64, device=Ad.device)
    ym = torch.empty(N, dtype=torch.float64, device=Ad.device)
    mws = torch.empty(gkb.gkb_matvec_workspace_size(Ad), dtype=torch.uint8, device=Ad.device)
    ms_n = time_kernel(lambda: gkb.gkb_matvec(Ad, xn, 0, y=yn, stream=stream), 20, stream)
    ms_t = time_kernel(lambda: gkb.gkb_matvec(Ad, xm, 1, y=ym, workspace=mws, stream=stream), 20, stream)
    b_n = M * N * 8 + N * 8 + M * 8
    b_t = M * N * 8 + M * 8 + N * 8
    ws = torch.empty(max(gkb.gkb_workspace_size(Ad, R, K), gkb.gkb_workspace_size(Ad, R, K, one_pass=True)),
                     dtype=torch.uint8, device=Ad.device)
    solve1 = lambda: gkb.gkb_partial_svd(Ad, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream,
                                         check_every=CHECK_EVERY, one_pass=True)
    ms1, (sig1, Ut1, Vt1, status1, st1) = wall_times(solve1, 1, reps, torch)
    del Ut1, Vt1
    solve = lambda: gkb.gkb_partial_svd(Ad, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream,
                                        check_every=CHECK_EVERY)
    ms, (sig, Ut, Vt, status, st) = wall_times(solve, 1, reps, torch)
    out = {"workload": "low-rank(200, 0.95^i)+noise(1e-6) 50000x20000 f64 (upcast of the f32 matrix); "
                       "top 50, k 120, tol 1e-6, checks every 10",
           "gemv_n_ms": ms_n, "gemv_n_GBps": b_n / (ms_n * 1e-3) / 1e9, "gemv_n_frac": b_n / (ms_n * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "gemv_t_ms": ms_t, "gemv_t_GBps": b_t / (ms_t * 1e-3) / 1e9, "gemv_t_frac": b_t / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "solve_ms_mean": float(np.mean(ms)), "solve_ms_median": float(np.median(ms)),
           "triplets_per_s": st["nconv"] / (np.mean(ms) / 1000.0), "status": status, "matvecs": st["matvecs"],
           "checks": st["checks"], "reps": reps,
           "one_sweep": {"solve_ms_mean": float(np.mean(ms1)), "solve_ms_median": float(np.median(ms1)),
                         "triplets_per_s": st1["nconv"] / (np.mean(ms1) / 1000.0), "status": status1,
                         "matvecs": st1["matvecs"], "refreshes": st1["refreshes"],
                         "one_pass_used": st1["one_pass_used"],
                         "sigma_rel_diff_vs_two_product_max": float(np.max(np.abs(sig1 - sig)) / sig[0])}}
    acc = headline_accuracy(sig, Ut, Vt, CHECK_EVERY)
    if acc:
        out["sigma_rel_err_vs_f64_oracle_max"] = acc["sigma_rel_err_max"]
        out["u_dist_max_sketch"] = acc["u_dist_max_sketch"]
        out["v_dist_max_sketch"] = acc["v_dist_max_sketch"]
        out["oracle_matvecs"] = acc["oracle_matvecs"]
    del Ad, ws, mws
    torch.cuda.empty_cache()
    return out


WIDE_M, WIDE_N, WIDE_SEED = 50000, 40000, 5


def wide_matrix(torch, dev):
    """The 50000 x 40000 float32 low-rank(200, 0.95^i) + noise(1e-6) matrix,
    formed on the device (U, V from QR of seeded Gaussian blocks); returns it
    and the generator (for the vectors drawn after it)."""
    g = torch.Generator(device=dev)
    g.manual_seed(WIDE_SEED)
    Uq, _ = torch.linalg.qr(torch.randn(WIDE_M, RANK, generator=g, device=dev, dtype=torch.float64))
    Vq, _ = torch.linalg.qr(torch.randn(WIDE_N, RANK, generator=g, device=dev, dtype=torch.float64))
    s = DECAY ** torch.arange(RANK, device=dev, dtype=torch.float64)
    Ad = ((Uq * s) @ Vq.T).float()
    del Uq, Vq
    Ad += NOISE * torch.randn(WIDE_M, WIDE_N, generator=g, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    return Ad, g


def wide_kernels_only(gkb, torch, dev, stream, reps):
    """The team sweep on the 50000 x 40000 float32 matrix alone (reps
    launches), the two products on it, and a plain 1 GiB device copy (3
    launches) whose counter readings calibrate the traffic figures."""
    Ad, g = wide_matrix(torch, dev)
    m, n = WIDE_M, WIDE_N
    p = torch.randn(n, generator=g, device=dev, dtype=torch.float32)
    xm = torch.randn(m, generator=g, device=dev, dtype=torch.float32)
    w = torch.empty(m, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    fws = torch.empty(gkb.lib().gkb_matvec_fused_workspace_size(gkb.C.byref(gkb.make_matrix(Ad))),
                      dtype=torch.uint8, device=dev)
    mws = torch.empty(gkb.gkb_matvec_workspace_size(Ad), dtype=torch.uint8, device=dev)
    ms_f = time_kernel(lambda: gkb.gkb_matvec_fused(Ad, p, w, y, workspace=fws, stream=stream), reps, stream)
    ms_n = time_kernel(lambda: gkb.gkb_matvec(Ad, p, 0, y=w, stream=stream), reps, stream)
    ms_t = time_kernel(lambda: gkb.gkb_matvec(Ad, xm, 1, y=y, workspace=mws, stream=stream), reps, stream)
    src = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    b_f = m * n * 4 + n * 4 + m * 8 + n * 8
    print(json.dumps({"kernels_only": True, "dtype": "f32", "shape": [m, n], "team_sweep_ms": ms_f,
                      "team_sweep_GBps": b_f / (ms_f * 1e-3) / 1e9, "gemv_n_ms": ms_n, "gemv_t_ms": ms_t,
                      "gemv_n_GBps": (m * n * 4 + n * 4 + m * 8) / (ms_n * 1e-3) / 1e9,
                      "gemv_t_GBps": (m * n * 4 + m * 4 + n * 8) / (ms_t * 1e-3) / 1e9, "reps": reps,
                      "copy_bytes": 2 ** 30}), flush=True)


def wide_leg(gkb, torch, qd, stream, reps=3):
    """A 50000 x 40000 float32 matrix (8.0 GB; rows longer than one workgroup
    of the sweep holds): low-rank(200, 0.95^i) + noise(1e-6), formed on the
    device from a seeded generator (U, V orthonormal from QR of Gaussian
    blocks), the headline's solve settings.  The one-sweep solve (team sweep)
    against the two-product solve of the same matrix: time, products, and the
    largest relative difference of their singular values; the team sweep's
    own rate."""
    dev = qd.device
    m, n = WIDE_M, WIDE_N
    Ad, g = wide_matrix(torch, dev)
    p = torch.randn(n, generator=g, device=dev, dtype=torch.float32)
    w = torch.empty(m, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    fws = torch.empty(gkb.lib().gkb_matvec_fused_workspace_size(gkb.C.byref(gkb.make_matrix(Ad))),
                      dtype=torch.uint8, device=dev)
    ms_sweep = time_kernel(lambda: gkb.gkb_matvec_fused(Ad, p, w, y, workspace=fws, stream=stream), 20, stream)
    b_sweep = m * n * 4 + n * 4 + m * 8 + n * 8
    ws = torch.empty(max(gkb.gkb_workspace_size(Ad, R, K), gkb.gkb_workspace_size(Ad, R, K, one_pass=True)),
                     dtype=torch.uint8, device=dev)
    out = {"workload": "low-rank(200, 0.95^i)+noise(1e-6) 50000x40000 f32 (device generator, seed 5); "
                       "top 50, k 120, tol 1e-6, checks every 10",
           "team_sweep_ms": ms_sweep, "team_sweep_GBps": b_sweep / (ms_sweep * 1e-3) / 1e9,
           "team_sweep_frac": b_sweep / (ms_sweep * 1e-3) / 1e9 / HBM_PEAK_GBS}
    q = torch.ones(m, dtype=torch.float64, device=dev) + 0.5 * torch.randn(m, generator=g, device=dev,
                                                                            dtype=torch.float64)
    sig = {}
    for name, one in (("one_sweep", True), ("two_product", False)):
        solve = lambda: gkb.gkb_partial_svd(Ad, R, K, TOL, RESTARTS, q1=q, workspace=ws, stream=stream,
                                            check_every=CHECK_EVERY, one_pass=one)
        ms, (sg, Ut, Vt, status, st) = wall_times(solve, 1, reps, torch)
        sig[name] = sg
        out[name] = {"solve_ms_mean": float(np.mean(ms)), "solve_ms_median": float(np.median(ms)),
                     "triplets_per_s": st["nconv"] / (np.mean(ms) / 1000.0), "status": status,
                     "matvecs": st["matvecs"], "one_pass_used": st["one_pass_used"], "restarts": st["restarts"]}
        del Ut, Vt
    out["sigma_rel_diff_one_vs_two_max"] = float(np.max(np.abs(sig["one_sweep"] - sig["two_product"]) /
                                                        sig["two_product"][0]))
    del Ad, ws, fws
    torch.cuda.empty_cache()
    return out


SPARSE_M, SPARSE_N, SPARSE_NNZ, SPARSE_SEED, SPARSE_QSEED = 1000000, 200000, 50000000, 7, 8
SPARSE_R, SPARSE_K, SPARSE_EVERY = 20, 60, 5


def sparse_leg(gkb, inputs, torch, dev, stream, steps):
    """Sparse A (CSR of A and of A^T, power-law degrees): the partial SVD through
    the column-panel products, and both products in the panel layout and in
    the binned CSR form, timed with HIP events on the launch stream."""
    S = inputs.sparse_powerlaw(SPARSE_M, SPARSE_N, SPARSE_NNZ, seed=SPARSE_SEED)
    t0 = time.perf_counter()
    plan = gkb.SparsePlan(SPARSE_M, SPARSE_N, S, device=dev, stream=stream)
    plan_s = time.perf_counter() - t0
    csr_plan = gkb.SparsePlan(SPARSE_M, SPARSE_N, S, device=dev, stream=stream, panels=False)
    del S
    q = torch.from_numpy(inputs.start_vector(SPARSE_M, seed=SPARSE_QSEED)).to(dev)
    ws = torch.empty(plan.workspace_size(SPARSE_R, SPARSE_K), dtype=torch.uint8, device=dev)
    run = lambda: plan.partial_svd(SPARSE_R, SPARSE_K, 1e-6, 50, workspace=ws, stream=stream, q1=q,
                                   check_every=SPARSE_EVERY)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sig, _, _, status, st = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    xn = torch.randn(SPARSE_N, dtype=torch.float32, device=dev)
    xm = torch.randn(SPARSE_M, dtype=torch.float32, device=dev)
    yn = torch.empty(SPARSE_M, dtype=torch.float64, device=dev)
    ym = torch.empty(SPARSE_N, dtype=torch.float64, device=dev)
    ms_n = time_kernel(lambda: plan.matvec(xn, 0, y=yn, stream=stream), 20, stream)
    ms_t = time_kernel(lambda: plan.matvec(xm, 1, y=ym, stream=stream), 20, stream)
    csr_n = time_kernel(lambda: csr_plan.matvec(xn, 0, y=yn, stream=stream), 20, stream)
    csr_t = time_kernel(lambda: csr_plan.matvec(xm, 1, y=ym, stream=stream), 20, stream)
    # algorithmic bytes: the caller's CSR once (index and value of every entry,
    # the offsets), the output (float64) and the input vector once
    b_n = SPARSE_NNZ * 8 + (SPARSE_M + 1) * 8 + SPARSE_M * 8 + SPARSE_N * 4
    b_t = SPARSE_NNZ * 8 + (SPARSE_N + 1) * 8 + SPARSE_N * 8 + SPARSE_M * 4
    # bytes the panel products move: 6 per entry, 4 per row and panel of offsets,
    # the per-panel row sums written and read back (4 + 4), the output and input
    pw = 28672
    npn, npt = -(-SPARSE_N // pw), -(-SPARSE_M // pw)
    p_n = SPARSE_NNZ * 6 + npn * (SPARSE_M + 1) * 4 + 8 * npn * SPARSE_M + SPARSE_M * 8 + SPARSE_N * 4
    p_t = SPARSE_NNZ * 6 + npt * (SPARSE_N + 1) * 4 + 8 * npt * SPARSE_N + SPARSE_N * 8 + SPARSE_M * 4
    out = {"workload": f"sparse power-law {SPARSE_M}x{SPARSE_N}, nnz {SPARSE_NNZ}, f32 CSR + CSR of A^T; "
                       f"top {SPARSE_R}, k {SPARSE_K}, tol 1e-6, checks every {SPARSE_EVERY}",
           "ms": ms, "triplets_per_s": st["nconv"] / (ms / 1000.0), "status": status, "matvecs": st["matvecs"],
           "restarts": st["restarts"], "layout": "column panels" if plan.panels == 3 else f"panels mask {plan.panels}",
           "plan_s": plan_s, "spmv_ms": ms_n, "spmv_GBps": b_n / (ms_n * 1e-3) / 1e9,
           "spmv_t_ms": ms_t, "spmv_t_GBps": b_t / (ms_t * 1e-3) / 1e9,
           "panel_bytes_GBps": [p_n / (ms_n * 1e-3) / 1e9, p_t / (ms_t * 1e-3) / 1e9],
           "csr_spmv_ms": csr_n, "csr_spmv_t_ms": csr_t, "csr_spmv_GBps": b_n / (csr_n * 1e-3) / 1e9,
           "csr_spmv_t_GBps": b_t / (csr_t * 1e-3) / 1e9, "sigma1": float(sig[0])}
    plan.close()
    csr_plan.close()
    return out


def sparse_kernels_only(gkb, inputs, torch, dev, stream, reps):
    """The sparse products alone on the 1000000 x 200000, 5e7-entry workload
    (reps launches each of A p and A^T q through the column panels and through
    the CSR kernels) and a plain 1 GiB device copy (3 launches) whose counter
    readings calibrate the traffic figures."""
    S = inputs.sparse_powerlaw(SPARSE_M, SPARSE_N, SPARSE_NNZ, seed=SPARSE_SEED)
    plan = gkb.SparsePlan(SPARSE_M, SPARSE_N, S, device=dev, stream=stream)
    csr_plan = gkb.SparsePlan(SPARSE_M, SPARSE_N, S, device=dev, stream=stream, panels=False)
    del S
    xn = torch.randn(SPARSE_N, dtype=torch.float32, device=dev)
    xm = torch.randn(SPARSE_M, dtype=torch.float32, device=dev)
    yn = torch.empty(SPARSE_M, dtype=torch.float64, device=dev)
    ym = torch.empty(SPARSE_N, dtype=torch.float64, device=dev)
    out = {"kernels_only": True, "sparse": True, "reps": reps, "panels": plan.panels}
    for name, p in (("panels", plan), ("csr", csr_plan)):
        out[name + "_n_ms"] = time_kernel(lambda: p.matvec(xn, 0, y=yn, stream=stream), reps, stream)
        out[name + "_t_ms"] = time_kernel(lambda: p.matvec(xm, 1, y=ym, stream=stream), reps, stream)
    src = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    plan.close()
    csr_plan.close()


RSGD_D1, RSGD_D2, RSGD_R, RSGD_B, RSGD_ETA, RSGD_LAM = 784, 256, 5, 64, 2.0, 1e-3


def rsgd_leg(gkb, inputs, torch, dev, stream):
    """Riemannian similarity learning (rank 5, 784 x 256, batches of 64): steps/s of
    the captured step (projection products + batched-solver retraction) for
    Krylov dimensions 20 and 35, held-out accuracy, and the float64 oracle's
    time per step on the host for context."""
    from oracle import rsgd
    steps = 300
    X, V, y, _, _ = inputs.similarity_pairs(steps * RSGD_B, RSGD_D1, RSGD_D2, seed=1)
    Xt, Vt, yt, _, _ = inputs.similarity_pairs(4000, RSGD_D1, RSGD_D2, seed=2)
    U0, s0, V0 = inputs.rank_r_point(RSGD_D1, RSGD_D2, RSGD_R, seed=3, scale=0.01)
    Xd = torch.from_numpy(X).to(dev)
    Vd = torch.from_numpy(V).to(dev)
    yd = torch.from_numpy(y).to(dev)
    out = {"workload": f"similarity learning, W {RSGD_D1}x{RSGD_D2} rank {RSGD_R}, batch {RSGD_B}, eta {RSGD_ETA}, "
                       f"lambda {RSGD_LAM}, synthetic two-domain pairs (10 classes)"}
    for k in (20, 35):
        plan = gkb.RsgdPlan(RSGD_D1, RSGD_D2, RSGD_R, k, RSGD_B, RSGD_ETA, RSGD_LAM, U0, s0, V0, device=dev,
                            stream=stream)
        plan.step(Xd[:RSGD_B], Vd[:RSGD_B], yd[:RSGD_B], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, steps):
            sl = slice(t * RSGD_B, (t + 1) * RSGD_B)
            plan.step(Xd[sl], Vd[sl], yd[sl], stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / (steps - 1)
        W = plan.weights(stream=stream).double().cpu().numpy()
        out[f"k{k}"] = {"ms_per_step": ms, "steps_per_s": 1000.0 / ms, "status": plan.info(stream)[0],
                        "heldout_accuracy": rsgd.accuracy(Xt, Vt, yt, W)}
        plan.close()
    t0 = time.perf_counter()
    U, s, Vf = U0, s0, V0
    for t in range(5):
        sl = slice(t * RSGD_B, (t + 1) * RSGD_B)
        U, s, Vf, _, _ = rsgd.step(X[sl], V[sl], y[sl], U, s, Vf, RSGD_ETA, RSGD_LAM)
    out["oracle_ms_per_step_host"] = (time.perf_counter() - t0) * 1000.0 / 5
    return out


def learned_leg(dev):
    """Learned start on the drifting 20000 x 5000 sequence (train on solves 1-100,
    evaluate on 101-200 against the random and the heuristic start)."""
    from paper_2104_10785_amd import learned
    out = learned.run(m=20000, n=5000, r=30, k=70, tol=1e-8, t_train=100, t_eval=100, ws=32, hidden=256,
                      epochs=20, lr=1e-3, check_every=2, seed=3, device=dev, log=log, init="heuristic")
    out.pop("per_t", None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-warmup", type=int, default=2, help="untimed oracle solves before the CPU timing")
    ap.add_argument("--cpu-reps", type=int, default=5, help="timed full oracle solves (CPU baseline)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--check-every", type=int, default=CHECK_EVERY)
    ap.add_argument("--two-pass", action="store_true",
                    help="time the two-product step (A read twice per step) instead of the one-sweep step")
    ap.add_argument("--legs", default="c1,f64,wide,bf16,rank,batched,learned,sparse,rsgd",
                    help="extra legs after the main timing (comma list; empty for none)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="time only the two matvec kernels and a 1 GiB copy (for counter runs)")
    ap.add_argument("--f64", action="store_true", help="with --kernels-only: the float64 upcast of the matrix")
    ap.add_argument("--bf16", action="store_true", help="with --kernels-only: the bfloat16 rounding of the matrix")
    ap.add_argument("--unaligned", action="store_true",
                    help="with --kernels-only: the float32 matrix in rows of n + 1 elements")
    ap.add_argument("--sparse", action="store_true",
                    help="with --kernels-only: the sparse products (column panels and CSR) instead")
    ap.add_argument("--wide", action="store_true",
                    help="with --kernels-only: the team sweep and the two products on the 50000 x 40000 matrix")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Golub-Kahan path runs on a single MI355X; "
              "sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_10785_amd import gkb, inputs

    dev = torch.device("cuda:0")
    if args.kernels_only and args.sparse:
        sparse_kernels_only(gkb, inputs, torch, dev, torch.cuda.current_stream(), args.kernel_reps)
        return
    if args.kernels_only and args.wide:
        wide_kernels_only(gkb, torch, dev, torch.cuda.current_stream(), args.kernel_reps)
        return
    log("generating 50000x20000 float32 low-rank-plus-noise matrix")
    t0 = time.time()
    A32, s, _, _ = inputs.lowrank_noise(M, N, RANK, DECAY, NOISE, seed=SEED, dtype=np.float32)
    q = inputs.start_vector(M, seed=QSEED)
    log(f"generated in {time.time() - t0:.1f} s; copying to device")
    Ad = torch.from_numpy(A32).to(dev)
    qd = torch.from_numpy(q).to(dev)
    one_pass = not args.two_pass
    ws = torch.empty(max(gkb.gkb_workspace_size(Ad, R, K), gkb.gkb_workspace_size(Ad, R, K, one_pass=True)),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    if args.kernels_only:
        kernels_only(gkb, torch, Ad, dev, stream, args.kernel_reps, f64=args.f64, bf16=args.bf16,
                     unaligned=args.unaligned)
        return

    def step(check_every=args.check_every, one_pass=one_pass):
        return gkb.gkb_partial_svd(Ad, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream,
                                   check_every=check_every, one_pass=one_pass)

    for i in range(args.warmup):
        out = step()
        log(f"warmup {i}: status={out[3]} stats={out[4]}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nconv = 0
    stats = None
    per_step = []
    for i in range(args.steps):
        ts = time.perf_counter()
        sigma, Ut, Vt, status, stats = step()   # returns after the stream has completed
        per_step.append((time.perf_counter() - ts) * 1000.0)
        nconv += stats["nconv"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1000.0 / args.steps
    value = nconv / dt
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, stats={stats}")

    # accuracy of the timed solve against the stored float64 oracle (same schedule)
    accuracy = headline_accuracy(sigma, Ut, Vt, args.check_every)

    # one more solve with HIP events at every phase boundary (not timed above)
    ph = gkb.gkb_partial_svd(Ad, R, K, TOL, RESTARTS, q1=qd, workspace=ws, stream=stream,
                             check_every=args.check_every, one_pass=one_pass, phase_timing=True)[4]
    phase_keys = ("ms_matvec", "ms_reorth", "ms_sync", "ms_ritz", "ms_other")
    phases = {k2: ph[k2] for k2 in phase_keys}
    phases["sum"] = sum(phases.values())
    phases["ms_total"] = ph["ms_total"]
    phases["bytes_A"] = ph["bytes_A"]
    phases["A_GBps_over_matvec_phase"] = ph["bytes_A"] / (ph["ms_matvec"] * 1e-3) / 1e9
    phases["per_step_us"] = {k2: 1000.0 * ph[k2] / max(1, ph["krylov_dim"]) for k2 in ("ms_matvec", "ms_reorth")}
    log(f"phases: {phases}")

    # the same solve with the test only at the end of the cycle (fixed k = 120)
    t1 = time.perf_counter()
    fixed = step(check_every=0)
    torch.cuda.synchronize()
    fixed_ms = (time.perf_counter() - t1) * 1000.0
    log(f"fixed-k solve: {fixed_ms:.2f} ms, stats={fixed[4]}")

    # the other step form at the same configuration, for comparison
    t1 = time.perf_counter()
    other = step(one_pass=not one_pass)
    torch.cuda.synchronize()
    other_ms = (time.perf_counter() - t1) * 1000.0
    log(f"{'two-product' if one_pass else 'one-sweep'} solve: {other_ms:.2f} ms, stats={other[4]}")

    # ---- dominant kernels: the two A-streaming matvecs, timed live with HIP events
    mws = torch.empty(gkb.gkb_matvec_workspace_size(Ad), dtype=torch.uint8, device=dev)
    xn, xm, yn, ym = matvec_operands(torch, Ad, dev)
    ms_n = time_kernel(lambda: gkb.gkb_matvec(Ad, xn, 0, y=yn, stream=stream), args.kernel_reps, stream)
    ms_t = time_kernel(lambda: gkb.gkb_matvec(Ad, xm, 1, y=ym, workspace=mws, stream=stream), args.kernel_reps,
                       stream)
    # algorithmic bytes per launch: every element of A once (4 B), the input
    # vector once, the float64 output once
    bytes_n = M * N * 4 + N * 4 + M * 8
    bytes_t = M * N * 4 + M * 4 + N * 8
    gbs_n = bytes_n / (ms_n * 1e-3) / 1e9
    gbs_t = bytes_t / (ms_t * 1e-3) / 1e9
    # the one-sweep pair: A once, p once, w and A^T w written once
    fp, fw, fy, fws = fused_operands(gkb, torch, Ad, dev)
    ms_f = time_kernel(lambda: gkb.gkb_matvec_fused(Ad, fp, fw, fy, fws, stream=stream), args.kernel_reps, stream)
    bytes_f = M * N * 4 + N * 4 + M * 8 + N * 8
    gbs_f = bytes_f / (ms_f * 1e-3) / 1e9
    if one_pass:
        dom_ms, dom_bytes, dom_name = ms_f, bytes_f, "gemv_fused"
    else:
        dom_ms, dom_bytes, dom_name = (ms_t, bytes_t, "gemv_t") if ms_t >= ms_n else (ms_n, bytes_n, "gemv_n")
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    log(f"gemv_n {ms_n:.4f} ms {gbs_n:.0f} GB/s; gemv_t {ms_t:.4f} ms {gbs_t:.0f} GB/s; "
        f"fused sweep {ms_f:.4f} ms {gbs_f:.0f} GB/s")
    ritz = ritz_gemms(gkb, torch, dev, stream, args.kernel_reps)
    log(f"Ritz GEMMs: {ritz}")

    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        log(f"leg {leg}")
        if leg == "bf16":
            legs["bf16_refined"] = bf16_leg(gkb, torch, Ad, qd, stream, args.steps, one_pass)
        elif leg == "rank":
            legs["rank_gapped"] = rank_leg(gkb, inputs, torch, dev, stream)
        elif leg == "batched":
            legs["batched"] = batched_leg(gkb, inputs, torch, dev, stream)
        elif leg == "learned":
            legs["learned_start"] = learned_leg(dev)
        elif leg == "sparse":
            legs["sparse"] = sparse_leg(gkb, inputs, torch, dev, stream, args.steps)
        elif leg == "rsgd":
            legs["rsgd"] = rsgd_leg(gkb, inputs, torch, dev, stream)
        elif leg == "c1":
            legs["c1_f64"] = c1_leg(gkb, inputs, torch, dev, stream, oracle=not args.no_cpu_baseline)
        elif leg == "f64":
            legs["f64_large"] = f64_leg(gkb, torch, Ad, qd, stream)
        elif leg == "wide":
            legs["wide_f32"] = wide_leg(gkb, torch, qd, stream)
        log(f"leg {leg} done: {json.dumps(legs)[-300:]}")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle: {args.cpu_warmup} + {args.cpu_reps} full solves")
        cpu = cpu_baseline(A32, q, args.cpu_warmup, args.cpu_reps, args.check_every)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "converged triplets/s (top-50 partial SVD, tol 1e-6) + matvec HBM GB/s",
        "value": value, "unit": "triplets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "ms_per_step_median": float(np.median(per_step)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gk_partial_svd low-rank(200, 0.95^i)+noise(1e-6) 50000x20000 f32",
                   "r": R, "k": K, "tol": TOL, "max_restarts": RESTARTS, "check_every": args.check_every,
                   "step": "one_sweep" if one_pass else "two_product", "parallelism": "single-gpu",
                   "seed": SEED, "start_seed": QSEED},
        "device": device_info(torch),
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom_name),
                     "algorithmic_bytes": dom_bytes, "kernel_ms": dom_ms},
        "matvec": {"gemv_n_ms": ms_n, "gemv_n_GBps": gbs_n, "gemv_t_ms": ms_t, "gemv_t_GBps": gbs_t,
                   "gemv_fused_ms": ms_f, "gemv_fused_GBps": gbs_f},
        "ritz_gemm": ritz,
        "solve": {"nconv": stats["nconv"], "matvecs": stats["matvecs"], "restarts": stats["restarts"],
                  "recomputed_columns": stats["refreshes"],
                  "krylov_dim": stats["krylov_dim"], "checks": stats["checks"],
                  "ms_host_svd": stats["ms_host"], "sigma1": float(sigma[0]), "sigma50": float(sigma[-1])},
        "phases": phases,
        "accuracy_vs_f64_oracle": accuracy,
        "fixed_k_solve": {"ms": fixed_ms, "triplets_per_s": fixed[4]["nconv"] / (fixed_ms / 1000.0),
                          "matvecs": fixed[4]["matvecs"]},
        ("two_product_solve" if one_pass else "one_sweep_solve"): {
            "ms": other_ms, "triplets_per_s": other[4]["nconv"] / (other_ms / 1000.0),
            "matvecs": other[4]["matvecs"], "sigma1": float(other[0][0]), "sigma50": float(other[0][-1])},
        "cpu_baseline": cpu,
    }
    line.update(legs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
