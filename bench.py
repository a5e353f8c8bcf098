"""Benchmark: plane-wave EFIE solves per second on one MI355X.

Headline (value): batched mixed precision + learned warm start on the PEC
sphere of radius 1 m, 5120-triangle icosphere (7680 RWG unknowns), k = 10
rad/m.  One step serves a batch of 512 held-out plane waves (256 directions
uniform on the sphere x theta/phi polarisation) with the operator and the
warm start resident: RHS assembly, warm-start inference (POD basis + MLP, with
the zero fallback), and block GMRES(50) over groups of 32 right-hand sides (one
shared block Krylov space per group) with split-BF16 block products on the
matrix cores and FP64 iterative refinement, to a true FP64 relative residual of
1e-6 for every right-hand side (--method gmres: column GMRES as a continuous
batch of 256 slots instead).
value = right-hand sides per second over the timed steps.

Beside it, on the same GPU:
  - plain FP64 GMRES(50) from zero on a sample of the same right-hand sides
    (matrix resident) -> speedup of the headline over the plain method;
  - the same batch without the warm start (mixed precision + batching alone);
  - the plain FP64 whole-path step of one x-polarised plane wave from +z
    (mesh -> fill -> RHS -> GMRES), with the packed FP64 product against the
    HBM roofline (roofline_gemv);
  - training of the warm start (snapshot solves, POD, MLP epochs), timed once;
  - the CPU oracle on a bounded sample (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--c5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
FP64_VALU_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops (FMA) x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
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
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="inner tolerance of the refinement; default 1e-3 with the Calderon preconditioner, else 0.1")
    ap.add_argument("--inner-terms", type=int, default=None, choices=[2, 3],
                    help="terms of the inner split-BF16 products: 3 (hi/lo matrix x hi/lo vectors) or 2 (hi/lo "
                         "matrix x BF16 vectors); default 2 for unpreconditioned block GMRES, else 3")
    ap.add_argument("--basis", default="f16", choices=["f16", "c64"],
                    help="storage of the inner Krylov basis (FP16 pairs or complex64)")
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--method", default="bgmres", choices=["gmres", "bgmres"],
                    help="inner solver of the mixed-precision forms: column GMRES as a continuous batch, or "
                         "block GMRES over groups of --block right-hand sides")
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--no-calderon", dest="calderon", action="store_false",
                    help="headline without the multiplicative Calderon preconditioner (block GMRES only uses it)")
    ap.add_argument("--train-dirs", type=int, default=512)
    ap.add_argument("--test-dirs", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=1500)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--c5", action="store_true",
                    help="full learned warm-start configuration: 2048 training / 512 test directions, 3000 epochs")
    ap.add_argument("--c3", action="store_true",
                    help="large-sphere workload instead: 30720 unknowns, k=20, the 512 plane waves of a 16x16 "
                         "(theta, phi) grid x theta/phi, split-BF16 block GMRES with FP64 refinement")
    ap.add_argument("--no-batch", dest="batch", action="store_false",
                    help="skip the uneven batch of 64 surfaces (batched solves over many operators)")
    ap.add_argument("--no-star", dest="star", action="store_false",
                    help="skip the star-split operator leg (low-frequency mixed precision, product times)")
    ap.add_argument("--counters", action="store_true",
                    help="only launch the dense product kernels a few times at the bench sizes, and a 1 GiB "
                         "device copy as calibration, for hardware-counter runs")
    a = ap.parse_args()
    cal = a.calderon and a.method == "bgmres" and not a.c3
    if a.inner_terms is None:   # 2 terms only pay with long unpreconditioned inner solves
        a.inner_terms = 2 if (a.method == "bgmres" and not cal) else 3
    if a.inner_tol is None:   # the preconditioned inner solves are short: a tighter tolerance saves outer cycles
        a.inner_tol = 1e-3 if cal else 0.1
    if a.c5:
        a.train_dirs, a.test_dirs, a.epochs = 2048, 512, 3000
    return a


def source_hash(name: str) -> str:
    with open(os.path.join(ROOT, "paper_2606_13482_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(fname: str, kernel_src: str, N: int):
    """HBM bytes per launch of a kernel from a committed counter summary, or None
    if absent or taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != source_hash(kernel_src) or int(kv.get("N", -1)) != N:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def solver_text(args, restart, calderon=False):
    if args.method == "bgmres":
        pre = "Calderon-preconditioned (right, M = -G^-1 T_BC G^-T) " if calderon else ""
        return f"{pre}block GMRES({restart}) over groups of {args.block} right-hand sides"
    return (f"GMRES({restart}), {'FP16' if args.basis == 'f16' else 'complex64'} inner Krylov basis, continuous "
            f"batch of {args.slots} slots")


def mixed_opts(args, bie, restart, pc=None):
    """Options of the mixed-precision solves: column GMRES as a continuous batch
    (FP16 or complex64 basis), or block GMRES (complex64 basis, all right-hand
    sides at once; right-preconditioned by pc when given)."""
    if args.method == "bgmres":
        return bie.Solve(method="bgmres", block=args.block, restart=restart, tol=args.tol, max_mvp=20000,
                         precision="mixed", inner_tol=args.inner_tol, inner_terms=args.inner_terms, calderon=pc)
    return bie.Solve(restart=restart, tol=args.tol, max_mvp=20000, precision="mixed", inner_tol=args.inner_tol,
                     slots=args.slots, inner_terms=args.inner_terms, basis=args.basis)


def planewave_batch(bie, inc):
    from paper_2606_13482_amd.inputs import planewave_set
    d_t, e_t = planewave_set(inc, "theta")
    d_p, e_p = planewave_set(inc, "phi")
    dirs = np.concatenate([d_t, d_p])
    pols = np.concatenate([e_t, e_p])
    flags = np.concatenate([np.ones(len(inc)), -np.ones(len(inc))])
    return dirs, pols, bie.features(dirs, flags)


def plain_leg(args, bie, torch, V, T, k):
    """Plain FP64 whole path for one x-polarised plane wave from +z."""
    from paper_2606_13482_amd.inputs import planewave_set
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    opts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000)

    def step():
        op = bie.Operator(V, T, k)
        B = op.rhs(d, e)
        X, st = op.solve(B, opts)
        return op, B, X, st

    for _ in range(args.warmup):
        step()[0].close()
    torch.cuda.synchronize()
    bie.prof_read(0)
    bie.prof_read(3)
    bie.prof_enable(True)
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        op, B, X, st = step()
        stats.append(st[0])
        if i != args.steps - 1:
            op.close()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    launches, gemv_ms = bie.prof_read(0)      # tile pass (the dominant kernel)
    r_launches, red_ms = bie.prof_read(3)     # reduction of its partial sums
    bie.prof_enable(False)
    N = op.N
    relres = float(torch.linalg.vector_norm(B - op.apply(X)) / torch.linalg.vector_norm(B))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.solve(B, opts)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    op.close()
    t0 = time.perf_counter()
    bie.Operator(V, T, k).close()
    torch.cuda.synchronize()
    t_fill64 = time.perf_counter() - t0
    t0 = time.perf_counter()
    bie.Operator(V, T, k, storage="c64").close()
    torch.cuda.synchronize()
    t_fill32 = time.perf_counter() - t0

    avg_ms = gemv_ms / max(1, launches)
    red_avg_ms = red_ms / max(1, r_launches)
    # Z = Z^T: a product reads each of the N(N+1)/2 distinct complex128 entries
    # once, plus x read and y written
    alg_bytes = N * (N + 1) // 2 * 16 + 2 * N * 16
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles("gemv_c128_n7680_counters.txt", "blas.hip", N),
            "kernel": "packed symmetric complex128 product, tile pass (k_sym_tiles)",
            "alg_bytes_per_launch": alg_bytes, "avg_launch_us": round(avg_ms * 1e3, 2), "launches": launches,
            "reduce_avg_us": round(red_avg_ms * 1e3, 2),
            "product_frac_with_reduce": round(alg_bytes / ((avg_ms + red_avg_ms) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "dense_equivalent_bytes_per_launch": N * N * 16}
    ms_step = 1e3 * t_steps / args.steps
    out = {"workload": f"PEC sphere, {T.shape[0]} triangles ({N} RWG), k={k:g}, 1 plane wave (x-pol, from +z), "
                       f"FP64 fill + GMRES({args.restart}) to {args.tol:g} (SCC)",
           "solves_per_s": round(1e3 / ms_step, 4), "ms_per_step": round(ms_step, 3),
           "iters": int(stats[-1]["iters"]), "mvps": int(stats[-1]["mvps"]), "relres_true_fp64": relres,
           "converged": bool(stats[-1]["converged"]), "solve_only_s": round(t_solve, 4),
           "fill_fp64_s": round(t_fill64, 4), "fill_fp32_s": round(t_fill32, 4),
           "gemv_share_of_step": round((gemv_ms + red_ms) / (t_steps * 1e3), 3)}
    return out, roof


def headline_leg(args, bie, torch, V, T, k):
    from paper_2606_13482_amd.inputs import random_directions
    sync = torch.cuda.synchronize
    res = {}
    t0 = time.perf_counter()
    op = bie.Operator(V, T, k, storage="split_bf16")
    sync()
    res["setup_fill_split_s"] = round(time.perf_counter() - t0, 4)
    N = op.N
    pc = None
    if args.calderon and args.method == "bgmres":
        t0 = time.perf_counter()
        pc = bie.Calderon(op)
        sync()
        res["setup_calderon_s"] = round(time.perf_counter() - t0, 4)
        ci = pc.info()
        res["calderon"] = {"refined_unknowns": ci["Nb"], "bc_nonzeros": ci["nnz_bc"], "gram_nonzeros": ci["nnz_gram"],
                           "gram_cg_iters": ci["cg_iters"], "gram_cg_relres": max(ci["cg_relres"])}
    mopts = mixed_opts(args, bie, args.restart, pc)
    popts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000)

    # training: solutions the method computes, then POD + MLP on the GPU
    dtr, ptr, ftr = planewave_batch(bie, random_directions(args.train_dirs, 5))
    t0 = time.perf_counter()
    Btr = op.rhs(dtr, ptr)
    Xtr, sttr = op.solve(Btr, mopts)
    sync()
    t_snap = time.perf_counter() - t0
    K = min(256, Xtr.shape[0])
    t0 = time.perf_counter()
    ws = bie.WarmStart.train(op, ftr, Xtr, pod_rank=K, hidden=512, epochs=args.epochs, batch=256,
                             pols=ptr, pol_model=1)
    sync()
    t_train = time.perf_counter() - t0
    res["training"] = {"snapshots": int(Xtr.shape[0]), "snapshot_solve_s": round(t_snap, 3),
                       "snapshots_converged": float(np.mean([s["converged"] for s in sttr])),
                       "pod_rank": K, "hidden": 512, "epochs": args.epochs, "train_s": round(t_train, 3),
                       "final_loss": ws.final_loss, "model": "linear in the polarisation (inputs d; 3 x 2K outputs)"}
    del Xtr, Btr

    dte, pte, fte = planewave_batch(bie, random_directions(args.test_dirs, 55))
    R = dte.shape[0]

    def step():
        B = op.rhs(dte, pte)
        X0, _ = ws.predict(fte, None, pols=pte)
        X, st = op.solve(B, mopts, x0=X0, x0_fallback=True)   # the fallback uses the solver's first FP64 residual
        return B, X, X0, np.array([s["x0_kept"] for s in st], bool), st

    for _ in range(args.warmup):
        step()
    sync()
    for k in (0, 1, 2, 4, 5):
        bie.prof_read(k)
    bie.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B, X, X0, used, st = step()
    sync()
    t_steps = time.perf_counter() - t0
    g_launch, g_ms, g_cols = bie.prof_read(1, columns=True)
    f_launch, f_ms, f_cols = bie.prof_read(2, columns=True)
    p_launch, p_ms = bie.prof_read(0)
    orth = {k: bie.prof_read(k, columns=True) for k in (4, 5)}
    bie.prof_enable(False)
    ms_step = 1e3 * t_steps / args.steps
    conv = np.array([s["converged"] for s in st], bool)
    relres = np.array([s["relres_true"] for s in st])
    iters_w = np.array([s["iters"] for s in st])
    r0 = (torch.linalg.vector_norm(B - op.apply(X0), dim=1) / torch.linalg.vector_norm(B, dim=1)).cpu().numpy()
    # independent FP64 residual of the returned solutions
    rchk = (torch.linalg.vector_norm(B - op.apply(X), dim=1) / torch.linalg.vector_norm(B, dim=1)).cpu().numpy()

    # the same batch without the warm start
    sync()
    t0 = time.perf_counter()
    Xz, stz = op.solve(B, mopts)
    sync()
    t_zero = time.perf_counter() - t0
    iters_z = np.array([s["iters"] for s in stz])

    # plain FP64 GMRES from zero on a sample of the batch, one right-hand side at a time
    ns = min(args.plain_sample, R)
    idx = np.linspace(0, R - 1, ns).round().astype(int)
    Xp, itp = [], []
    sync()
    t0 = time.perf_counter()
    for i in idx:
        x, s = op.solve(B[i:i + 1], popts)
        Xp.append(x)
        itp.append((s[0]["iters"], s[0]["mvps"]))
    sync()
    t_plain = (time.perf_counter() - t0) / ns
    Xp = torch.cat(Xp)
    # the paper's preconditioned method in plain FP64 (column GMRES on T M u = b) on the same sample
    plain_cal = None
    if pc is not None:
        copts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000, calderon=pc)
        itc = []
        sync()
        t0 = time.perf_counter()
        for i in idx:
            _, s = op.solve(B[i:i + 1], copts)
            itc.append(s[0]["iters"])
        sync()
        t_cal = (time.perf_counter() - t0) / ns
        plain_cal = {"rhs": int(ns), "solves_per_s": round(1.0 / t_cal, 4), "iters_mean": float(np.mean(itc))}
    # a tight FP64 solution of the sample for the forward errors
    Xt, _ = op.solve(B[idx], bie.Solve(restart=args.restart, tol=1e-10, max_mvp=40000))
    nt = torch.linalg.vector_norm(Xt, dim=1)
    fwd = lambda Y: float((torch.linalg.vector_norm(Y - Xt, dim=1) / nt).max())

    value = R / (ms_step * 1e-3)
    plain_rate = 1.0 / t_plain
    res.update({
        "rhs_per_step": R,
        "solves_per_s": round(value, 3),
        "converged": float(conv.mean()),
        "relres_true_fp64_max": float(relres.max()),
        "relres_recomputed_fp64_max": float(rchk.max()),
        "iters_mean": float(iters_w.mean()), "iters_max": int(iters_w.max()),
        "warm_start": {"kept": float(used.mean()), "initial_relres_median": float(np.median(r0)),
                       "initial_relres_max": float(r0.max())},
        "no_warm_start": {"solves_per_s": round(R / t_zero, 3), "iters_mean": float(iters_z.mean()),
                          "iters_max": int(iters_z.max())},
        "plain_fp64_sample": {"rhs": int(ns), "solves_per_s": round(plain_rate, 4),
                              "iters_mean": float(np.mean([a for a, _ in itp]))},
        "speedup_vs_plain_fp64": round(value / plain_rate, 2),
        "plain_fp64_calderon_sample": plain_cal,
        "speedup_vs_plain_fp64_calderon": None if plain_cal is None else round(value / plain_cal["solves_per_s"], 2),
        "speedup_no_warm_start_vs_plain_fp64": round((R / t_zero) / plain_rate, 2),
        "forward_error_vs_tight_fp64": {"plain_fp64": fwd(Xp), "mixed_learned": fwd(X[idx]),
                                        "mixed_zero": fwd(Xz[idx]), "reference": "FP64 GMRES to 1e-10 on the sample"},
        "packed_fp64_share_of_step": round(p_ms / (t_steps * 1e3), 3),
    })
    avg = g_ms / max(1, g_launch)
    alg_flops = 8.0 * N * N * g_cols / max(1, g_launch)   # per launch: complex product, 8 real flops per entry and column
    achieved = alg_flops / (avg * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
            "traffic": traffic_from_profiles("gemm_split_bf16_n7680_r512_counters.txt", "gemm.hip", N),
            "traffic_note": "HBM bytes per launch at 512 columns (counters), null if the kernel changed since",
            "kernel": "split-BF16 complex block product (k_gemm_split, v_mfma_f32_32x32x16_bf16)",
            "alg_flops_per_launch": alg_flops, "issued_tflops": round(3 * achieved, 1),
            "avg_columns_per_launch": round(g_cols / max(1, g_launch), 1),
            "avg_launch_us": round(avg * 1e3, 2), "launches": g_launch,
            "gemm_share_of_step": round(g_ms / (t_steps * 1e3), 3)}
    # block GMRES orthogonalisation (first pass): dots V^H W and update W -= V C
    # on the complex64 basis of the refinement's inner solves, FP32 matrix cores;
    # 8 real flops per row for every basis vector x column pair
    cands = [(g_ms, roof)]
    # the refinement's FP64 residuals B - T X (FP64 matrix cores, 8 N^2 flops per column)
    if f_launch:
        avg_f = f_ms / f_launch
        alg_f = 8.0 * N * N * f_cols / f_launch
        ach_f = alg_f / (avg_f * 1e-3) / 1e12
        cands.append((f_ms, {"bound": "mfma", "achieved": round(ach_f, 1), "peak": FP64_MFMA_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(ach_f / FP64_MFMA_PEAK_TFLOPS, 4),
                             "traffic": traffic_from_profiles("gemm64_fp64_n7680_r512_counters.txt", "gemm.hip", N),
                             "traffic_note": "HBM bytes per launch at 512 columns (counters), null if the kernel "
                                             "changed since",
                             "kernel": "FP64 complex block product of the refinement residuals (k_gemm64, "
                                       "v_mfma_f64_16x16x4f64)",
                             "alg_flops_per_launch": alg_f, "avg_columns_per_launch": round(f_cols / f_launch, 1),
                             "avg_launch_us": round(avg_f * 1e3, 2), "launches": f_launch,
                             "share_of_step": round(f_ms / (t_steps * 1e3), 3)}))
    names = {4: "block GMRES basis dots V^H W (k_bdots_mf + k_bdots_fin, v_mfma_f32_32x32x2f32)",
             5: "block GMRES basis update W -= V C (k_bcomb_mf, v_mfma_f32_32x32x2f32)"}
    for k, (n_l, ms, pairs) in orth.items():
        if n_l == 0:
            continue
        avg_o = ms / n_l
        alg_o = 8.0 * N * pairs / n_l
        ach_o = alg_o / (avg_o * 1e-3) / 1e12
        cands.append((ms, {"bound": "mfma", "achieved": round(ach_o, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(ach_o / FP32_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                           "traffic_note": "no counter summary for this kernel",
                           "kernel": names[k], "alg_flops_per_launch": alg_o,
                           "avg_launch_us": round(avg_o * 1e3, 2), "launches": n_l,
                           "share_of_step": round(ms / (t_steps * 1e3), 3)}))
    cands.sort(key=lambda c: -c[0])
    res["kernel_rooflines"] = [c[1] for c in cands]
    if pc is not None:
        pc.close()
    op.close()
    return res, cands[0][1], ms_step, float(np.mean([b for _, b in itp])), int(ns)


def c3_run(args, bie, torch):
    """Large sphere: 20480-triangle icosphere (30720 RWG), k = 20, 512 plane waves
    (16 x 16 (theta, phi) grid x theta/phi) per step, operator resident; GMRES(30)
    with split-BF16 block products and FP64 refinement (block GMRES over groups of
    --block right-hand sides, or column GMRES as a continuous batch of --slots) to
    FP64 SCC 1e-6; plain FP64 GMRES(30) on a sample of the same waves."""
    from paper_2606_13482_amd.inputs import grid_planewaves, icosphere
    sync = torch.cuda.synchronize
    V, T = icosphere(5)
    k = 20.0
    t0 = time.perf_counter()
    op = bie.Operator(V, T, k, storage="split_bf16")
    sync()
    t_fill = time.perf_counter() - t0
    N = op.N
    dirs, pols = grid_planewaves(16, 16)
    R = dirs.shape[0]
    mopts = mixed_opts(args, bie, 30)

    def step():
        B = op.rhs(dirs, pols)
        X, st = op.solve(B, mopts)
        return B, X, st

    for _ in range(args.warmup):
        step()
    sync()
    bie.prof_read(1)
    bie.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B, X, st = step()
    sync()
    t_steps = time.perf_counter() - t0
    g_launch, g_ms, g_cols = bie.prof_read(1, columns=True)
    bie.prof_enable(False)
    ms_step = 1e3 * t_steps / args.steps
    its = np.array([s["iters"] for s in st])
    conv = np.array([s["converged"] for s in st], bool)
    ns = 2
    idx = np.linspace(0, R - 1, ns).round().astype(int)
    popts = bie.Solve(restart=30, tol=args.tol, max_mvp=20000)
    sync()
    t0 = time.perf_counter()
    itp = []
    for i in idx:
        _, s = op.solve(B[i:i + 1], popts)
        itp.append(s[0]["iters"])
    sync()
    t_plain = (time.perf_counter() - t0) / ns
    avg = g_ms / max(1, g_launch)
    alg = 8.0 * N * N * g_cols / max(1, g_launch)
    ach = alg / (avg * 1e-3) / 1e12
    value = R / (ms_step * 1e-3)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "split-bf16 products (f32 accumulate) + f64 refinement", "data": "synthetic",
        "config": {"workload": (f"PEC sphere r=1 m, icosphere {T.shape[0]} triangles ({N} RWG), k={k:g}; {R} plane "
                                f"waves (16x16 theta/phi grid x theta/phi) per step, operator resident; "
                                f"{solver_text(args, 30)} on split-BF16 MFMA products with FP64 refinement to "
                                f"{args.tol:g} (FP64 SCC)"),
                   "N": N, "k": k, "restart": 30, "inner_tol": args.inner_tol, "method": args.method,
                   "block": args.block if args.method == "bgmres" else None,
                   "slots": args.slots if args.method == "gmres" else None,
                   "rhs_per_step": R, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(ach, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / BF16_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "split-BF16 complex block product (k_gemm_split)", "alg_flops_per_launch": alg,
                     "issued_tflops": round(3 * ach, 1), "avg_columns_per_launch": round(g_cols / max(1, g_launch), 1),
                     "avg_launch_us": round(avg * 1e3, 2), "launches": g_launch,
                     "gemm_share_of_step": round(g_ms / (t_steps * 1e3), 3)},
        "c3": {"fill_and_split_s": round(t_fill, 3), "converged": float(conv.mean()),
               "relres_true_fp64_max": float(max(s["relres_true"] for s in st)), "iters_mean": float(its.mean()),
               "iters_max": int(its.max()), "plain_fp64_sample": {"rhs": ns, "solves_per_s": round(1.0 / t_plain, 4),
                                                                  "iters": itp},
               "speedup_vs_plain_fp64": round(value * t_plain, 2)},
    }
    op.close()
    return out


def star_leg(args, bie, torch, V, T):
    """Star-split operator (Sec. VI-A: T = jk T_A + Sigma V Sigma^T / (jk)) against
    the assembled one on the bench sphere: (1) mixed precision with FP32 storage at
    low frequency (k = 0.1), 16 plane waves to FP64 SCC 1e-6; (2) the FP64 product
    time of both forms at the bench wavenumber."""
    from paper_2606_13482_amd.inputs import random_directions, planewave_set
    sync = torch.cuda.synchronize
    d, e = planewave_set(random_directions(8, 66), "theta")
    d2, e2 = planewave_set(random_directions(8, 66), "phi")
    dirs, pols = np.concatenate([d, d2]), np.concatenate([e, e2])
    out = {"workload": f"PEC sphere, {T.shape[0]} triangles, k = 0.1 (low frequency), {dirs.shape[0]} plane waves, "
                       f"FP32 storage, GMRES({args.restart}) inner solves (tolerance 1e-3) with FP64 refinement "
                       f"to {args.tol:g}"}
    opts = bie.Solve(restart=args.restart, tol=args.tol, precision="mixed", inner_tol=1e-3, max_mvp=20000)
    for star in (False, True):
        op = bie.Operator(V, T, 0.1, storage="c64", keep_fp64=True, star=star)
        B = op.rhs(dirs, pols)
        op.solve(B[:1], opts)
        sync()
        t0 = time.perf_counter()
        X, st = op.solve(B, opts)
        sync()
        t = time.perf_counter() - t0
        out["star" if star else "assembled"] = {
            "solves_per_s": round(B.shape[0] / t, 2), "iters_mean": float(np.mean([s["iters"] for s in st])),
            "converged": float(np.mean([s["converged"] for s in st])),
            "relres_true_fp64_max": float(max(s["relres_true"] for s in st))}
        op.close()
    out["speedup_star_vs_assembled"] = round(out["star"]["solves_per_s"] / out["assembled"]["solves_per_s"], 2)
    # FP64 product times at the bench wavenumber
    from paper_2606_13482_amd.inputs import complex_gaussian
    prod = {}
    for star in (False, True):
        op = bie.Operator(V, T, args.k, star=star)
        x = torch.from_numpy(complex_gaussian(op.N, 7)).cuda().reshape(1, -1)
        y = op.apply(x)
        sync()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(20):
            op.apply(x, out=y)
        ev1.record()
        sync()
        us = ev0.elapsed_time(ev1) / 20 * 1e3
        N, F = op.N, T.shape[0]
        nbytes = N * (N + 1) // 2 * 16 + (F * (F + 1) // 2 * 16 if star else 0)
        prod["star" if star else "assembled"] = {"us_per_product": round(us, 1), "packed_bytes": nbytes,
                                                  "GB_per_s": round(nbytes / us / 1e3, 1)}
        op.close()
    out["fp64_product"] = prod
    return out


def uneven_batch_leg(args, bie, torch):
    """64 closed surfaces (spheres, ellipsoids, rounded cubes; 648..5832 unknowns,
    10 edges per wavelength), 1..32 plane waves each, FP32 matrices: the batched
    solve (grouped products, graph-replayed cycles, autotuned work units) against
    the same operators solved one after another."""
    from paper_2606_13482_amd.inputs import uneven_batch
    sync = torch.cuda.synchronize
    probs = uneven_batch()
    sync()
    t0 = time.perf_counter()
    ops = [bie.Operator(p["V"], p["T"], p["k"], storage="c64") for p in probs]
    Bs = [op.rhs(p["dirs"], p["pols"]) for op, p in zip(ops, probs)]
    sync()
    t_fill = time.perf_counter() - t0
    Ns = [op.N for op in ops]
    Rs = [b.shape[0] for b in Bs]
    opts = bie.Solve(restart=50, tol=args.tol)
    bie.batch_config(0, True)
    t0 = time.perf_counter()
    bie.batch_solve(ops, Bs, opts)          # first call: autotuner
    sync()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xs, sts = bie.batch_solve(ops, Bs, opts)
    sync()
    t_batch = time.perf_counter() - t0
    its = np.array([s["iters"] for st in sts for s in st])
    conv = np.array([s["converged"] for st in sts for s in st], bool)
    t0 = time.perf_counter()
    for op, B in zip(ops, Bs):
        op.solve(B, opts)
    sync()
    t_seq = time.perf_counter() - t0
    nrhs = int(sum(Rs))
    out = {"workload": (f"{len(ops)} surfaces, N {min(Ns)}..{max(Ns)}, {nrhs} plane waves, FP32 matrices, "
                        f"GMRES(50) to {args.tol:g} (SCC), max 10000 products per right-hand side"),
           "solves_per_s": round(int(conv.sum()) / t_batch, 2), "batch_s": round(t_batch, 3),
           "first_call_s_with_autotune": round(t_first, 3), "fill_s": round(t_fill, 3),
           "tiles_per_unit": bie.batch_tuned(ops, Rs), "converged": float(conv.mean()),
           "iters_mean": float(its.mean()), "iters_max": int(its.max()),
           "relres_max_converged": float(max(s["relres_true"] for st in sts for s in st if s["converged"])),
           "sequential_s": round(t_seq, 3), "speedup_vs_sequential": round(t_seq / t_batch, 3),
           "packed_fp32_bytes_per_product": int(sum(4 * n * (n + 1) for n in Ns))}
    if args.calderon:
        # the same operators with the Calderon preconditioner, one after another:
        # setup per surface, then GMRES(50) on T M u = b (FP32 T, FP64 M)
        sync()
        t0 = time.perf_counter()
        pcs = [bie.Calderon(op) for op in ops]
        sync()
        t_pc = time.perf_counter() - t0
        stc = []
        t0 = time.perf_counter()
        for op, B, pc in zip(ops, Bs, pcs):
            stc.append(op.solve(B, bie.Solve(restart=50, tol=args.tol, calderon=pc))[1])
        sync()
        t_cal = time.perf_counter() - t0
        convc = np.array([s["converged"] for st in stc for s in st], bool)
        itsc = np.array([s["iters"] for st in stc for s in st])
        out["calderon_sequential"] = {
            "setup_s": round(t_pc, 3), "solve_s": round(t_cal, 3),
            "solves_per_s": round(int(convc.sum()) / t_cal, 2),
            "solves_per_s_with_setup": round(int(convc.sum()) / (t_cal + t_pc), 2),
            "converged": float(convc.mean()), "iters_mean": float(itsc.mean()), "iters_max": int(itsc.max()),
            "relres_max": float(max(s["relres_true"] for st in stc for s in st))}
        for pc in pcs:
            pc.close()
    for op in ops:
        op.close()
    return out


def counters_probe(args, bie, torch):
    """Kernels for the HBM traffic counters: 5 launches each of the packed FP64
    product (one column), the split-BF16 block product and the FP64 block product
    (512 columns, the headline's 16 groups of 32) on the bench operator, and 3
    plain copies of 1 GiB (FETCH_SIZE / WRITE_SIZE calibration)."""
    from paper_2606_13482_amd.inputs import icosphere, complex_gaussian
    V, T = icosphere(args.level)
    op = bie.Operator(V, T, args.k, storage="split_bf16")
    x = torch.from_numpy(complex_gaussian(op.N, 7)).cuda().reshape(1, -1)
    Xb = torch.from_numpy(complex_gaussian(op.N, 7, cols=512)).cuda()
    for _ in range(5):
        op.apply(x)
    for _ in range(5):
        op.apply(Xb, block=True)
    for _ in range(5):
        op.apply(Xb, block="fp64")
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_probe": {"N": op.N, "packed_fp64_launches": 5, "block_launches": 5,
                                         "block_columns": 512, "copy_bytes": a.numel() * 4, "copies": 3}}),
          flush=True)
    op.close()


def cpu_baseline(level: int, k: float, restart: int, plain_mvps: float):
    """The oracle (C fill with OpenMP + numpy GMRES) on a bounded sample: the full
    FP64 fill and one GMRES(restart) cycle; a solve with the matrix resident is
    extrapolated to the mean number of products plain FP64 GMRES needed on the GPU."""
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
    t_solve = plain_mvps * t_mvp
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(1.0 / t_solve, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"full oracle FP64 fill of the {rwg['N']}-unknown matrix ({t_fill:.2f} s) and one "
                       f"GMRES({restart}) cycle ({t_mvp * 1e3:.1f} ms per iteration); a matrix-resident solve "
                       f"extrapolated to the {plain_mvps:.0f} products plain FP64 GMRES took on the GPU sample"),
            "fill_s": round(t_fill, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2606_13482_amd import bie
    from paper_2606_13482_amd.inputs import icosphere

    torch.cuda.set_device(torch.device("cuda:0"))
    if args.counters:
        counters_probe(args, bie, torch)
        return
    if args.c3:
        print(json.dumps(c3_run(args, bie, torch)), flush=True)
        return
    V, T = icosphere(args.level)
    k = args.k
    plain, roof_gemv = plain_leg(args, bie, torch, V, T, k)
    head, roof, ms_step, plain_mvps, ns = headline_leg(args, bie, torch, V, T, k)
    N = 3 * T.shape[0] // 2
    out = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "split-bf16 products (f32 accumulate) + f64 refinement",
        "data": "synthetic",
        "config": {"workload": (f"PEC sphere r=1 m, icosphere {T.shape[0]} triangles ({N} RWG), k={k:g}; batches of "
                                f"{2 * args.test_dirs} held-out plane waves ({args.test_dirs} directions x theta/phi), "
                                f"operator and warm start resident; learned warm start (POD {min(256, 2 * args.train_dirs)}, "
                                f"MLP 4-512-512, trained on {2 * args.train_dirs} solves); "
                                f"{solver_text(args, args.restart, args.calderon)} on split-BF16 MFMA products with "
                                f"FP64 refinement to {args.tol:g} (FP64 SCC)"),
                   "N": N, "k": k, "restart": args.restart, "inner_tol": args.inner_tol, "method": args.method,
                   "block": args.block if args.method == "bgmres" else None,
                   "slots": args.slots if args.method == "gmres" else None,
                   "inner_terms": args.inner_terms, "basis": args.basis if args.method == "gmres" else "c64",
                   "calderon": bool(args.calderon and args.method == "bgmres"),
                   "rhs_per_step": 2 * args.test_dirs, "train_directions": args.train_dirs,
                   "test_directions": args.test_dirs, "parallelism": "single GPU"},
        "roofline": roof,
        "roofline_gemv": roof_gemv,
        "headline": head,
        "plain_fp64_step": plain,
    }
    if args.star:
        out["star_split"] = star_leg(args, bie, torch, V, T)
    if args.batch:
        out["uneven_batch"] = uneven_batch_leg(args, bie, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.level, k, args.restart, plain_mvps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
