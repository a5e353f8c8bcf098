"""Benchmark: plane-wave EFIE solves per second on one MI355X.

Workload (default): PEC sphere of radius 1 m, 5120-triangle icosphere
(7680 RWG unknowns), k = 10 rad/m, one x-polarised plane wave arriving from
+z, complex FP64 matrix, unpreconditioned GMRES(50) to a relative residual of
1e-6 under the standard criterion.  One step is the whole path: mesh -> RWG
table and pair list -> FP64 fill (regular + singular pairs) -> excitation ->
GMRES with the criterion on the true residual.  value = solves per second of
such steps (1 right-hand side per step).

Also reported: the solve alone with the matrix resident, the FP32 fill, the
dense-product kernel against the HBM roofline (HIP events around every launch
in the timed region), and the CPU oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
METRIC = "GMRES solves/s to 1e-6 residual: batched mixed+learned vs plain FP64; GEMV GB/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--k", type=float, default=10.0)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-mixed", dest="mixed", action="store_false", help="skip the mixed-precision leg")
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    return ap.parse_args()


def product_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2606_13482_amd", "csrc", "blas.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(kernel_hash: str, N: int):
    """HBM bytes per launch of the product kernel from the committed counter summary,
    or None if absent or taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "gemv_c128_n7680_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash or int(kv.get("N", -1)) != N:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(level: int, k: float, restart: int, mvps_gpu: float):
    """The oracle (C fill with OpenMP + numpy GMRES) on a bounded sample of the workload:
    the full FP64 fill and one GMRES(restart) cycle; the solve is extrapolated
    to the number of products the GPU run needed."""
    from oracle import cfill, efie, krylov
    from oracle.mesh import rwg_table
    from paper_2606_13482_amd.inputs import icosphere, planewave_set
    V, T = icosphere(level)
    t0 = time.perf_counter()
    rwg = rwg_table(V, T)
    Z = cfill.fill(rwg, k)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    b = efie.rhs(rwg, k, d, e)[0]
    t_fill = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = krylov.gmres(Z, b, m=restart, tol=1e-30, max_mvp=restart)
    t_cycle = time.perf_counter() - t0
    t_mvp = t_cycle / max(1, st.mvps)
    t_step = t_fill + mvps_gpu * t_mvp
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / t_step, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"full oracle FP64 fill of the {rwg['N']}-unknown matrix ({t_fill:.2f} s) + one "
                       f"GMRES({restart}) cycle ({t_mvp * 1e3:.1f} ms per iteration); solve extrapolated "
                       f"to the GPU run's {mvps_gpu:.0f} products")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2606_13482_amd import bie
    from paper_2606_13482_amd.inputs import icosphere, planewave_set

    V, T = icosphere(args.level)
    k = args.k
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    opts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def step():
        op = bie.Operator(V, T, k)
        B = op.rhs(d, e)
        X, st = op.solve(B, opts)
        return op, B, X, st

    for _ in range(args.warmup):
        op, B, X, st = step()
        op.close()
    torch.cuda.synchronize()

    bie.prof_read()
    bie.prof_enable(True)
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        op, B, X, st = step()
        stats.append(st[0])
        if _ != args.steps - 1:
            op.close()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    launches, gemv_ms = bie.prof_read()
    bie.prof_enable(False)
    ms_per_step = 1e3 * t_steps / args.steps
    N = op.N

    # correctness of the last step: the true FP64 residual with the GPU matrix
    R = B - op.apply(X)
    relres = float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))

    # solve alone with the matrix resident
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X2, st2 = op.solve(B, opts)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    # fill alone (FP64 and FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op64 = bie.Operator(V, T, k)
    torch.cuda.synchronize()
    t_fill64 = time.perf_counter() - t0
    op64.close()
    t0 = time.perf_counter()
    op32 = bie.Operator(V, T, k, storage="c64")
    torch.cuda.synchronize()
    t_fill32 = time.perf_counter() - t0
    op32.close()
    op.close()

    # mixed precision with iterative refinement on the same workload: FP64 fill,
    # FP32 rounding, inner GMRES on the FP32 matrix, FP64 outer residual
    mixed = None
    if args.mixed:
        mopts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000, precision="mixed",
                          inner_tol=args.inner_tol)

        def mstep():
            opm = bie.Operator(V, T, k, storage="c64", keep_fp64=True)
            Bm = opm.rhs(d, e)
            Xm, stm = opm.solve(Bm, mopts)
            return opm, Bm, Xm, stm
        opm, Bm, Xm, stm = mstep()
        opm.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            opm, Bm, Xm, stm = mstep()
            if _ != args.steps - 1:
                opm.close()
        torch.cuda.synchronize()
        tm = (time.perf_counter() - t0) / args.steps
        Rm = Bm - opm.apply(Xm)    # FP64 matrix
        t0 = time.perf_counter()
        Xm2, stm2 = opm.solve(Bm, mopts)
        torch.cuda.synchronize()
        tms = time.perf_counter() - t0
        mixed = {"solves_per_s": round(1.0 / tm, 4), "ms_per_step": round(tm * 1e3, 3),
                 "solves_per_s_matrix_resident": round(1.0 / tms, 3), "iters": int(stm[0]["iters"]),
                 "mvps": int(stm[0]["mvps"]), "outer_checks": int(stm[0]["checks"]),
                 "relres_true_fp64": float(torch.linalg.vector_norm(Rm) / torch.linalg.vector_norm(Bm)),
                 "rel_diff_vs_plain": float(torch.linalg.vector_norm(Xm - X) / torch.linalg.vector_norm(X)),
                 "inner_tol": args.inner_tol, "speedup_vs_plain": round(ms_per_step / (tm * 1e3), 3)}
        opm.close()

    gemv_avg_ms = gemv_ms / max(1, launches)
    # the matrix is symmetric: a product reads each of the N(N+1)/2 distinct
    # entries once (complex128), plus x read and y written
    alg_bytes = N * (N + 1) // 2 * 16 + 2 * N * 16
    achieved = alg_bytes / (gemv_avg_ms * 1e-3) / 1e9
    khash = product_source_hash()
    traffic = traffic_from_profiles(khash, N)

    mvps = float(np.mean([s["mvps"] for s in stats]))
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"PEC sphere r=1 m, icosphere {T.shape[0]} triangles ({N} RWG), k={k:g}, "
                               f"1 plane wave (x-pol, from +z), FP64 fill + GMRES({args.restart}) to "
                               f"{args.tol:g} (SCC)", "N": N, "k": k, "restart": args.restart,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "packed symmetric complex128 product (tile pass + reduce)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": round(gemv_avg_ms * 1e3, 2),
                     "launches": launches},
        "solve": {"iters": int(stats[-1]["iters"]), "mvps": int(stats[-1]["mvps"]),
                  "relres_true_fp64": relres, "converged": bool(stats[-1]["converged"]),
                  "solve_only_s": round(t_solve, 4), "solves_per_s_matrix_resident": round(1.0 / t_solve, 3),
                  "fill_fp64_s": round(t_fill64, 4), "fill_fp32_s": round(t_fill32, 4),
                  "gemv_share_of_step": round(gemv_ms / (t_steps * 1e3), 3)},
        "mixed_fp32_ir": mixed,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.level, k, args.restart, mvps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
