"""Benchmark: plane-wave EFIE solves per second on one MI355X.

Headline (value): the learned warm-start workload on the PEC sphere of radius
1 m, 5120-triangle icosphere (7680 RWG unknowns), k = 10 rad/m.  Training: the
method solves 2048 directions uniform on the sphere x theta/phi polarisation
(4096 right-hand sides); a 256-mode POD basis of those solutions and a
4 -> 512 -> 512 -> 512 network (Re/Im of 256 coefficients) trained 3000 epochs
on the GPU.  One timed step serves the 1024 held-out right-hand sides (512
directions x theta/phi) with the operator and the warm start resident: RHS
assembly, network inference with the zero fallback, and block GMRES(50) over
groups of 32 right-hand sides (one shared block Krylov space per group) with
2-term split-BF16 block products on the matrix cores, an FP16-pair inner basis
and FP64 iterative refinement (inner tolerance 1e-2), to a true FP64 relative
residual of 1e-6.
value = right-hand sides meeting that criterion per second, summed over the
timed steps.

Beside it, on the same GPU and right-hand sides:
  - plain FP64 GMRES(50) from zero, one right-hand side at a time (matrix
    resident), on a sample -> speedup of the headline over the plain method;
  - the same batch from zero (mixed precision + batching alone), from the
    linear-in-polarisation network, and from the POD projection of the
    solutions (the best any K-mode prediction can do);
  - forward errors against a direct LU solve of the FP64 matrix, and its
    1-norm condition number;
  - the Calderon-preconditioned form of the same batch (own key, setup timed);
  - the plain FP64 whole path of one x-polarised plane wave from +z, with the
    packed FP64 product against the HBM roofline (roofline_gemv);
  - the 30720-unknown sphere at k = 20 with the 512 plane waves of a 16 x 16
    (theta, phi) grid (key c3; 1 warm-up and 2 timed steps);
  - the B-spline far field (single level and multilevel) and the fast operator
    (sparse near entries + multilevel far field, no dense matrix) on the
    30720-unknown sphere against the dense operator and on a 491520-unknown
    sphere no dense matrix fits;
  - the star-split operator at low frequency, the uneven batch of 64 surfaces;
  - the CPU oracle on a bounded sample (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-c3]
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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
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
    ap.add_argument("--inner-tol", type=float, default=0.01, help="inner tolerance of the refinement")
    ap.add_argument("--inner-terms", type=int, default=2, choices=[2, 3],
                    help="terms of the inner split-BF16 products: 3 (hi/lo matrix x hi/lo vectors) or 2 (hi/lo "
                         "matrix x BF16 vectors)")
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--basis", default="f16", choices=["c64", "f16"],
                    help="inner Krylov basis of the unpreconditioned mixed block solves (FP16 pairs or complex64)")
    ap.add_argument("--train-dirs", type=int, default=2048)
    ap.add_argument("--test-dirs", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--pod-rank", type=int, default=256)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-calderon", dest="calderon", action="store_false",
                    help="skip the Calderon-preconditioned legs")
    ap.add_argument("--no-c3", dest="c3", action="store_false", help="skip the 30720-unknown sphere leg")
    ap.add_argument("--no-batch", dest="batch", action="store_false",
                    help="skip the uneven batch of 64 surfaces (batched solves over many operators)")
    ap.add_argument("--no-star", dest="star", action="store_false",
                    help="skip the star-split operator leg (low-frequency mixed precision, product times)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the uneven batch of 64 surfaces (its JSON object on one line)")
    ap.add_argument("--counters", action="store_true",
                    help="only launch the dense product kernels a few times at the bench sizes, and a 1 GiB "
                         "device copy as calibration, for hardware-counter runs")
    return ap.parse_args()


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


def mixed_opts(args, bie, restart, pc=None, inner_tol=None, terms=None, basis=None):
    """Block GMRES over groups of --block right-hand sides on split-BF16 products
    with FP64 refinement (right-preconditioned by pc when given), inner basis
    --basis unless given."""
    return bie.Solve(method="bgmres", block=args.block, restart=restart, tol=args.tol, max_mvp=20000,
                     precision="mixed", inner_tol=args.inner_tol if inner_tol is None else inner_tol,
                     inner_terms=args.inner_terms if terms is None else terms, calderon=pc,
                     basis=args.basis if basis is None else basis)


def planewave_batch(bie, inc):
    from paper_2606_13482_amd.inputs import planewave_set
    d_t, e_t = planewave_set(inc, "theta")
    d_p, e_p = planewave_set(inc, "phi")
    dirs = np.concatenate([d_t, d_p])
    pols = np.concatenate([e_t, e_p])
    flags = np.concatenate([np.ones(len(inc)), -np.ones(len(inc))])
    return dirs, pols, bie.features(dirs, flags)


def stats_of(st):
    conv = np.array([s["converged"] for s in st], bool)
    its = np.array([s["iters"] for s in st])
    rel = np.array([s["relres_true"] for s in st])
    return conv, its, rel


def relres(torch, op, B, X):
    """FP64 relative residuals ||b - T x|| / ||b|| (packed FP64 product)."""
    return (torch.linalg.vector_norm(B - op.apply(X), dim=1) / torch.linalg.vector_norm(B, dim=1)).cpu().numpy()


def plain_leg(args, bie, torch, V, T, k):
    """Plain FP64 whole path for one x-polarised plane wave from +z."""
    from paper_2606_13482_amd.inputs import planewave_set
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    opts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000)
    steps = max(1, min(args.steps, 10))

    def step():
        op = bie.Operator(V, T, k)
        B = op.rhs(d, e)
        X, st = op.solve(B, opts)
        return op, B, X, st

    for _ in range(min(args.warmup, 2)):
        step()[0].close()
    torch.cuda.synchronize()
    bie.prof_read(0)
    bie.prof_read(3)
    bie.prof_enable(True)
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        op, B, X, st = step()
        stats.append(st[0])
        if i != steps - 1:
            op.close()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    launches, gemv_ms = bie.prof_read(0)      # tile pass (the dominant kernel)
    r_launches, red_ms = bie.prof_read(3)     # reduction of its partial sums
    bie.prof_enable(False)
    N = op.N
    rr = float(relres(torch, op, B, X)[0])
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
    ms_step = 1e3 * t_steps / steps
    out = {"workload": f"PEC sphere, {T.shape[0]} triangles ({N} RWG), k={k:g}, 1 plane wave (x-pol, from +z), "
                       f"FP64 fill + GMRES({args.restart}) to {args.tol:g} (SCC)",
           "solves_per_s": round(1e3 / ms_step, 4), "ms_per_step": round(ms_step, 3), "steps": steps,
           "iters": int(stats[-1]["iters"]), "mvps": int(stats[-1]["mvps"]), "relres_true_fp64": rr,
           "converged": bool(stats[-1]["converged"]), "fill_fp64_s": round(t_fill64, 4),
           "fill_fp32_s": round(t_fill32, 4), "gemv_share_of_step": round((gemv_ms + red_ms) / (t_steps * 1e3), 3)}
    return out, roof


def block_rooflines(bie, N, terms, t_ms, g, f, orth, basis_bytes):
    """Rooflines of the block-solver kernels from the live HIP-event records:
    the split-BF16 product (BF16 peak, algorithmic flops), the FP64 product of
    the refinement residuals (FP64 matrix peak) and the two block-GMRES
    orthogonalisation kernels (HBM: the basis they read, basis_bytes per entry;
    their 3-term BF16 matrix-core rate beside it); sorted by total time."""
    cands = []
    g_launch, g_ms, g_cols = g
    if g_launch:
        avg = g_ms / g_launch
        alg = 8.0 * N * N * g_cols / g_launch   # complex product: 8 real flops per entry and column
        ach = alg / (avg * 1e-3) / 1e12
        cands.append((g_ms, {"bound": "mfma", "achieved": round(ach, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(ach / BF16_PEAK_TFLOPS, 4),
                             "traffic": traffic_from_profiles("gemm_split_bf16_n7680_r512_counters.txt", "gemm.hip",
                                                              N),
                             "traffic_note": "HBM bytes per launch at 512 columns (counters), null if the kernel "
                                             "changed since or another size",
                             "kernel": "split-BF16 complex block product (k_gemm_split, v_mfma_f32_32x32x16_bf16)",
                             "alg_flops_per_launch": alg, "terms": terms, "issued_tflops": round(terms * ach, 1),
                             "issued_frac": round(terms * ach / BF16_PEAK_TFLOPS, 4),
                             "avg_columns_per_launch": round(g_cols / g_launch, 1),
                             "avg_launch_us": round(avg * 1e3, 2), "launches": g_launch,
                             "share_of_step": round(g_ms / t_ms, 3)}))
    f_launch, f_ms, f_cols = f
    if f_launch:
        avg = f_ms / f_launch
        alg = 8.0 * N * N * f_cols / f_launch
        ach = alg / (avg * 1e-3) / 1e12
        cands.append((f_ms, {"bound": "mfma", "achieved": round(ach, 1), "peak": FP64_MFMA_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(ach / FP64_MFMA_PEAK_TFLOPS, 4),
                             "traffic": traffic_from_profiles("gemm64_fp64_n7680_r512_counters.txt", "gemm.hip", N),
                             "traffic_note": "HBM bytes per launch at 512 columns (counters), null if the kernel "
                                             "changed since or another size",
                             "kernel": "FP64 complex block product of the refinement residuals (k_gemm64, "
                                       "v_mfma_f64_16x16x4f64)",
                             "alg_flops_per_launch": alg, "avg_columns_per_launch": round(f_cols / f_launch, 1),
                             "avg_launch_us": round(avg * 1e3, 2), "launches": f_launch,
                             "share_of_step": round(f_ms / t_ms, 3)}))
    names = {4: "block GMRES basis dots V^H W (k_bdots_bd + k_bdots_fin, v_mfma_f32_32x32x16_bf16, 3-term splits)",
             5: "block GMRES basis update W -= V C (k_bcomb_bd, v_mfma_f32_32x32x16_bf16, 3-term splits)"}
    n4, _, pairs = orth.get(4, (0, 0.0, 0))
    n5, _, vecs = orth.get(5, (0, 0.0, 0))
    if n4 and n5:
        # both kernels of a step read the same basis vectors: sum of K over the groups
        bytes_l = float(vecs) / n5 * N * basis_bytes
        flops_l = 8.0 * N * pairs / n4
        for kk in (4, 5):
            n_l, ms, _ = orth[kk]
            avg = ms / n_l
            ach = bytes_l / (avg * 1e-3) / 1e9
            fr = flops_l / (avg * 1e-3) / 1e12
            cands.append((ms, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                               "traffic_note": "no counter summary for this kernel",
                               "kernel": names[kk], "alg_bytes_per_launch": round(bytes_l),
                               "alg_bytes_note": "the basis entries read (sum of K N entries); the columns W add "
                                                 "16 B per row and column",
                               "alg_flops_per_launch": flops_l, "alg_tflops": round(fr, 2),
                               "issued_frac_bf16": round(3 * fr / BF16_PEAK_TFLOPS, 4),
                               "avg_launch_us": round(avg * 1e3, 2), "launches": n_l,
                               "share_of_step": round(ms / t_ms, 3)}))
    cands.sort(key=lambda c: -c[0])
    return [c[1] for c in cands]


def prof_reset(bie):
    for kk in (0, 1, 2, 3, 4, 5):
        bie.prof_read(kk)


def headline_leg(args, bie, torch, V, T, k):
    """The learned warm-start workload (see the module docstring)."""
    from paper_2606_13482_amd.inputs import random_directions
    sync = torch.cuda.synchronize
    res = {}
    t0 = time.perf_counter()
    op = bie.Operator(V, T, k, storage="split_bf16")
    sync()
    res["setup_fill_split_s"] = round(time.perf_counter() - t0, 4)
    N = op.N
    mopts = mixed_opts(args, bie, args.restart)
    popts = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000)

    # training: solutions the method computes, then POD + network on the GPU
    dtr, ptr, ftr = planewave_batch(bie, random_directions(args.train_dirs, 5))
    t0 = time.perf_counter()
    Btr = op.rhs(dtr, ptr)
    Xtr, sttr = op.solve(Btr, mopts)
    sync()
    t_snap = time.perf_counter() - t0
    K = min(args.pod_rank, Xtr.shape[0])
    train = {"snapshots": int(Xtr.shape[0]), "snapshot_solve_s": round(t_snap, 3),
             "snapshots_converged": float(np.mean([s["converged"] for s in sttr])), "pod_rank": K,
             "hidden": args.hidden, "epochs": args.epochs, "batch": 256}
    wss = {}
    for pm, name in ((0, "network"), (1, "linear_pol")):
        t0 = time.perf_counter()
        wss[pm] = bie.WarmStart.train(op, ftr, Xtr, pod_rank=K, hidden=args.hidden, epochs=args.epochs, batch=256,
                                      pols=ptr if pm else None, pol_model=pm)
        sync()
        train[name] = {"train_s": round(time.perf_counter() - t0, 3), "final_loss": wss[pm].final_loss,
                       "outputs": wss[pm].outputs,
                       "model": ("inputs (d, s), 4 -> %d -> %d -> %d: Re/Im of %d coefficients" %
                                 (args.hidden, args.hidden, 2 * K, K)) if pm == 0 else
                                ("linear in the polarisation: input d, 4 -> %d -> %d -> %d (three coefficient "
                                 "sets combined with e)" % (args.hidden, args.hidden, 6 * K))}
    res["training"] = train
    del Btr
    sigma = wss[0].sigma()
    snap_norm2 = float(torch.sum(torch.abs(Xtr) ** 2))
    res["training"]["pod_captured_energy"] = float(np.sum(sigma ** 2) / snap_norm2)
    del Xtr
    ws = wss[0]

    dte, pte, fte = planewave_batch(bie, random_directions(args.test_dirs, 55))
    R = dte.shape[0]

    def step():
        B = op.rhs(dte, pte)
        X0, _ = ws.predict(fte)
        X, st = op.solve(B, mopts, x0=X0, x0_fallback=True)   # the fallback uses the solver's first residual
        return B, X, X0, st

    for _ in range(args.warmup):
        step()
    sync()
    prof_reset(bie)
    bie.prof_enable(True)
    n_conv, n_rhs, iters_all, kept_all = 0, 0, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B, X, X0, st = step()
        conv, its, _ = stats_of(st)
        n_conv += int(conv.sum())
        n_rhs += len(st)
        iters_all.append(its)
        kept_all.append([s["x0_kept"] for s in st])
    sync()
    t_steps = time.perf_counter() - t0
    g = bie.prof_read(1, columns=True)
    f = bie.prof_read(2, columns=True)
    orth = {kk: bie.prof_read(kk, columns=True) for kk in (4, 5)}
    bie.prof_enable(False)
    ms_step = 1e3 * t_steps / args.steps
    value = n_conv / t_steps
    its_w = np.concatenate(iters_all)
    rchk = relres(torch, op, B, X)            # independent FP64 residual of the last step's solutions
    r0 = relres(torch, op, B, X0)
    _, _, rel_last = stats_of(st)

    def timed_solve(x0=None, fallback=True):
        sync()
        t0 = time.perf_counter()
        Xs, sts = op.solve(B, mopts, x0=x0, x0_fallback=fallback)
        sync()
        dt = time.perf_counter() - t0
        cv, it, _ = stats_of(sts)
        return Xs, {"solves_per_s": round(int(cv.sum()) / dt, 3), "converged": float(cv.mean()),
                    "iters_mean": float(it.mean()), "iters_max": int(it.max())}

    # the same batch from zero, from the linear-in-polarisation network, and from
    # the POD projection of the solutions (the best a K-mode prediction can do)
    Xz, zero = timed_solve()
    X1, _ = wss[1].predict(fte, pols=pte)
    r1 = relres(torch, op, B, X1)
    _, lin = timed_solve(X1)
    lin["initial_relres_median"] = float(np.median(r1))
    wss[1].close()
    U = ws.basis()                                        # K x N
    Xp = (X @ U.conj().T) @ U                              # rows: U U^H x*
    proj_err = (torch.linalg.vector_norm(X - Xp, dim=1) / torch.linalg.vector_norm(X, dim=1)).cpu().numpy()
    rp = relres(torch, op, B, Xp)
    _, proj = timed_solve(Xp)
    proj.update({"projection_error_median": float(np.median(proj_err)), "initial_relres_median": float(np.median(rp))})
    del U, Xp, X1

    # plain FP64 GMRES from zero on a sample of the batch, one right-hand side at a time
    ns = min(args.plain_sample, R)
    idx = np.linspace(0, R - 1, ns).round().astype(int)
    Xpl, itp = [], []
    sync()
    t0 = time.perf_counter()
    for i in idx:
        x, s = op.solve(B[i:i + 1], popts)
        Xpl.append(x)
        itp.append((s[0]["iters"], s[0]["mvps"], s[0]["converged"]))
    sync()
    t_plain = (time.perf_counter() - t0) / ns
    Xpl = torch.cat(Xpl)
    plain_rate = sum(c for _, _, c in itp) / (t_plain * ns)

    # forward errors against a direct LU solve of the FP64 matrix; its 1-norm condition number
    Zd = op.matrix()
    Xlu = torch.linalg.solve(Zd, B[idx].T).T.contiguous()
    kappa1 = float(torch.linalg.matrix_norm(Zd, ord=1) * torch.linalg.matrix_norm(torch.linalg.inv(Zd), ord=1))
    del Zd
    nlu = torch.linalg.vector_norm(Xlu, dim=1)
    fwd = lambda Y: float((torch.linalg.vector_norm(Y - Xlu, dim=1) / nlu).max())

    res.update({
        "rhs_per_step": R,
        "solves_per_s": round(value, 3),
        "converged": n_conv / max(1, n_rhs),
        "relres_true_fp64_max": float(rel_last.max()),
        "relres_recomputed_fp64_max": float(rchk.max()),
        "iters_mean": float(its_w.mean()), "iters_max": int(its_w.max()),
        "warm_start": {"kept": float(np.mean(np.concatenate(kept_all))), "initial_relres_median": float(np.median(r0)),
                       "initial_relres_max": float(r0.max())},
        "no_warm_start": zero,
        "linear_pol_warm_start": lin,
        "pod_projection_start": proj,
        "plain_fp64_sample": {"rhs": int(ns), "solves_per_s": round(plain_rate, 4),
                              "iters_mean": float(np.mean([a for a, _, _ in itp]))},
        "speedup_vs_plain_fp64": round(value / plain_rate, 2),
        "speedup_no_warm_start_vs_plain_fp64": round(zero["solves_per_s"] / plain_rate, 2),
        "forward_error_vs_lu": {"plain_fp64": fwd(Xpl), "mixed_learned": fwd(X[idx]), "mixed_zero": fwd(Xz[idx]),
                                "reference": "direct LU (torch.linalg.solve, FP64) of the operator's FP64 matrix on "
                                             "the sample", "kappa1": kappa1},
    })
    kr = block_rooflines(bie, N, args.inner_terms, t_steps * 1e3, g, f, orth, 4 if args.basis == "f16" else 8)
    res["kernel_rooflines"] = kr
    plain_mvps = float(np.mean([b for _, b, _ in itp]))
    return op, ws, res, kr[0], ms_step, plain_mvps, (B, fte, idx, popts)


def calderon_leg(args, bie, torch, op, ws, batch):
    """The same held-out batch with the multiplicative Calderon preconditioner:
    right-preconditioned mixed block GMRES (T M products split to BF16, 3 terms,
    inner tolerance 1e-3, FP64 refinement) from the network's prediction; setup
    timed; the preconditioned plain FP64 column GMRES on the sample."""
    B, fte, idx, popts = batch
    sync = torch.cuda.synchronize
    R = B.shape[0]
    t0 = time.perf_counter()
    pc = bie.Calderon(op)
    sync()
    t_setup = time.perf_counter() - t0
    ci = pc.info()
    copts = mixed_opts(args, bie, args.restart, pc=pc, inner_tol=1e-3, terms=3, basis="c64")
    X0, _ = ws.predict(fte)
    op.solve(B, copts, x0=X0, x0_fallback=True)
    reps = 3
    n_conv, its = 0, []
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        X0, _ = ws.predict(fte)
        X, st = op.solve(B, copts, x0=X0, x0_fallback=True)
        conv, it, _ = stats_of(st)
        n_conv += int(conv.sum())
        its.append(it)
    sync()
    t_solve = (time.perf_counter() - t0) / reps
    rr = relres(torch, op, B, X)
    itc = []
    cpl = bie.Solve(restart=args.restart, tol=args.tol, max_mvp=20000, calderon=pc)
    sync()
    t0 = time.perf_counter()
    for i in idx:
        _, s = op.solve(B[i:i + 1], cpl)
        itc.append(s[0]["iters"])
    sync()
    t_cal = (time.perf_counter() - t0) / len(idx)
    pc.close()
    its = np.concatenate(its)
    rate = n_conv / reps / t_solve
    return {"workload": f"the headline's {R} held-out right-hand sides, right-preconditioned by "
                        "M = -G^-1 T_BC G^-T (Buffa-Christiansen functions on the barycentric refinement)",
            "setup_s": round(t_setup, 3), "refined_unknowns": ci["Nb"], "gram_iters": ci["cg_iters"],
            "gram_relres": max(ci["cg_relres"]), "solves_per_s": round(rate, 2),
            "solves_per_s_with_setup": round(n_conv / reps / (t_solve + t_setup), 2),
            "converged": n_conv / reps / R, "relres_recomputed_fp64_max": float(rr.max()),
            "iters_mean": float(its.mean()), "iters_max": int(its.max()),
            "plain_fp64_calderon_sample": {"rhs": len(idx), "solves_per_s": round(1.0 / t_cal, 3),
                                           "iters_mean": float(np.mean(itc))}}


def c3_leg(args, bie, torch):
    """Large sphere: 20480-triangle icosphere (30720 RWG), k = 20, the 512 plane
    waves of a 16 x 16 (theta, phi) grid x theta/phi per step, operator resident;
    block GMRES(30) over groups of 32 with 2-term split-BF16 block products and
    FP64 refinement to FP64 SCC 1e-6; 1 warm-up and 2 timed steps; plain FP64
    GMRES(30) on 2 of the waves."""
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
    mopts = mixed_opts(args, bie, 30, terms=2)

    def step():
        B = op.rhs(dirs, pols)
        X, st = op.solve(B, mopts)
        return B, X, st

    step()
    sync()
    prof_reset(bie)
    bie.prof_enable(True)
    steps, n_conv, its = 2, 0, []
    t0 = time.perf_counter()
    for _ in range(steps):
        B, X, st = step()
        conv, it, _ = stats_of(st)
        n_conv += int(conv.sum())
        its.append(it)
    sync()
    t_steps = time.perf_counter() - t0
    g = bie.prof_read(1, columns=True)
    f = bie.prof_read(2, columns=True)
    orth = {kk: bie.prof_read(kk, columns=True) for kk in (4, 5)}
    bie.prof_enable(False)
    rr = relres(torch, op, B, X)
    popts = bie.Solve(restart=30, tol=args.tol, max_mvp=20000)
    ns = 2
    idx = np.linspace(0, R - 1, ns).round().astype(int)
    sync()
    t0 = time.perf_counter()
    itp = []
    for i in idx:
        _, s = op.solve(B[i:i + 1], popts)
        itp.append(s[0]["iters"])
    sync()
    t_plain = (time.perf_counter() - t0) / ns
    op.close()
    its = np.concatenate(its)
    value = n_conv / t_steps
    kr = block_rooflines(bie, N, 2, t_steps * 1e3, g, f, orth, 4 if args.basis == "f16" else 8)
    return {"workload": (f"PEC sphere r=1 m, icosphere {T.shape[0]} triangles ({N} RWG), k={k:g}; {R} plane waves "
                         f"(16x16 theta/phi grid x theta/phi) per step, operator resident; block GMRES(30) over groups "
                         f"of {args.block} on 2-term split-BF16 MFMA products, "
                         f"{'FP16-pair' if args.basis == 'f16' else 'complex64'} inner basis, FP64 refinement to {args.tol:g} "
                         f"(FP64 SCC)"),
            "steps": steps, "warmup": 1, "ms_per_step": round(1e3 * t_steps / steps, 3),
            "solves_per_s": round(value, 3), "fill_and_split_s": round(t_fill, 3), "converged": n_conv / (steps * R),
            "relres_recomputed_fp64_max": float(rr.max()), "iters_mean": float(its.mean()),
            "iters_max": int(its.max()),
            "plain_fp64_sample": {"rhs": ns, "solves_per_s": round(1.0 / t_plain, 4), "iters": itp},
            "speedup_vs_plain_fp64": round(value * t_plain, 2), "kernel_rooflines": kr}


def counters_from_profiles(fname: str, kernel_src: str):
    """key = value lines of a committed counter summary taken on the current kernel
    source, else None."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != source_hash(kernel_src):
        return None
    return kv


def fill_leg(args, bie, torch):
    """The fill kernels at full size (HIP events around each launch): regular
    triangle pairs (49 point pairs each, Radon 7 x 7) in FP64 and FP32, the flagged
    pairs (always FP64), the assembly into packed tiles; at 7680 and 30720 unknowns."""
    from paper_2606_13482_amd.inputs import icosphere
    sync = torch.cuda.synchronize
    out = {}
    for level, k in ((4, 10.0), (5, 20.0)):
        V, T = icosphere(level)
        row = {}
        for storage, rec in (("c128", 6), ("c64", 9)):
            bie.Operator(V, T, k, storage=storage).close()      # warm-up (code objects, tables)
            sync()
            for kk in (6, 7, 8, 9):
                bie.prof_read(kk)
            bie.prof_enable(True)
            t0 = time.perf_counter()
            op = bie.Operator(V, T, k, storage=storage)
            sync()
            t_create = time.perf_counter() - t0
            bie.prof_enable(False)
            n_r, ms_r, pairs = bie.prof_read(rec, columns=True)
            n_s, ms_s, npairs = bie.prof_read(7, columns=True)
            n_a, ms_a = bie.prof_read(8)
            N = op.N
            op.close()
            row[storage] = {"regular_pairs_ms": round(ms_r, 3), "triangle_pairs": pairs,
                            "point_pairs_per_s": round(49 * pairs / (ms_r * 1e-3), 1),
                            "flagged_pairs_ms": round(ms_s, 3), "flagged_pairs": npairs,
                            "assembly_ms": round(ms_a, 3), "operator_create_s": round(t_create, 4)}
        out[f"N{N}"] = row
    kv = counters_from_profiles("fill_pairs_regular_n7680_counters.txt", "fill.hip")
    if kv:
        out["counters_n7680"] = {k: kv[k] for k in kv if k.startswith(("valu", "lds", "fp64", "fp32"))}
    return out


def far_leg(args, bie, torch, V, T, k):
    """The single-level B-spline far field (Sec. III) on the bench sphere: cubes of
    0.4 m, cubic splines, s = 8; setup (moments, table of g) and the far product
    of one vector (HIP events on the current stream), against the dense packed
    product of the same operator."""
    sync = torch.cuda.synchronize
    from paper_2606_13482_amd.inputs import complex_gaussian
    op = bie.Operator(V, T, k)
    t0 = time.perf_counter()
    far = bie.FarField(op, 0.4, 8, 3)
    sync()
    t_setup = time.perf_counter() - t0
    info = far.info()
    x = torch.from_numpy(complex_gaussian(op.N, 7)).cuda().reshape(1, -1)
    y = far.apply(x)
    yd = op.apply(x)
    sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        far.apply(x, out=y)
    ev1.record()
    sync()
    ms = ev0.elapsed_time(ev1) / reps
    ev0.record()
    for _ in range(reps):
        op.apply(x, out=yd)
    ev1.record()
    sync()
    ms_dense = ev0.elapsed_time(ev1) / reps
    n3 = info["points_per_axis"] ** 3
    pairs = info["far_pairs"] * n3 * n3
    # translation: 4 complex multiply-adds (32 flops) per pair of interpolation points
    tf = 32.0 * pairs / (ms * 1e-3) / 1e12
    far.close()
    op.close()
    return {"workload": f"PEC sphere, {T.shape[0]} triangles, k={k:g}: cubes 0.4 m, p = 3, s = 8 (single level)",
            "setup_s": round(t_setup, 3), "cubes": info["boxes"], "far_cube_pairs": info["far_pairs"],
            "points_per_cube": n3, "buffer_knots": info["buffer_knots"], "ms_per_far_product": round(ms, 3),
            "point_pairs_per_s": round(pairs / (ms * 1e-3), 1), "translation_tflops": round(tf, 2),
            "translation_frac_fp64_vector_peak": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
            "ms_per_dense_packed_product": round(ms_dense, 4),
            "multilevel": far_ml_leg(bie, torch, V, T, k)}


def far_ml_leg(bie, torch, V, T, k, box=0.2, levels=2, s=8, p=3):
    """The multilevel far field (Sec. IV) on the bench sphere: leaf cubes of 0.2 m,
    two levels, cubic splines, s = 8 (the parent level doubles s: its cubes exceed
    half a wavelength); time per far product (HIP events), per-level data, the
    error against the operator's dense FP64 matrix masked to the far leaf cubes
    (cube indices from the library), and the single-level far field on the same
    leaf cubes (one product) for comparison."""
    from paper_2606_13482_amd.inputs import complex_gaussian
    sync = torch.cuda.synchronize
    op = bie.Operator(V, T, k)
    t0 = time.perf_counter()
    fm = bie.FarFieldML(op, box, levels, s, p)
    sync()
    t_setup = time.perf_counter() - t0
    lv = [fm.level_info(l) for l in range(levels)]
    x = torch.from_numpy(complex_gaussian(op.N, 8, cols=1)).cuda()
    y = fm.apply(x)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    sync()
    ev0.record()
    for _ in range(reps):
        fm.apply(x, out=y)
    ev1.record()
    sync()
    ms = ev0.elapsed_time(ev1) / reps
    f1 = bie.FarField(op, box, s, p)
    y1 = f1.apply(x)
    sync()
    ev0.record()
    f1.apply(x, out=y1)
    ev1.record()
    sync()
    ms1 = ev0.elapsed_time(ev1)
    cubes = f1.boxes()
    _, inv = np.unique(cubes, axis=0, return_inverse=True)
    uc = np.unique(cubes, axis=0)
    far = (np.max(np.abs(uc[:, None, :] - uc[None, :, :]), axis=2) > 1)[inv.ravel()][:, inv.ravel()]
    Z = op.matrix()
    yd = x @ (Z * torch.from_numpy(far).cuda()).T
    err = float(torch.linalg.norm(y - yd) / torch.linalg.norm(yd))
    err1 = float(torch.linalg.norm(y1 - yd) / torch.linalg.norm(yd))
    del Z
    f1.close()
    fm.close()
    op.close()
    return {"workload": f"leaf cubes {box:g} m, {levels} levels, p = {p}, s = {s} on the leaves",
            "setup_s": round(t_setup, 3), "ms_per_far_product": round(ms, 3),
            "levels": [{"cubes": l["boxes"], "pairs": l["far_pairs"], "splines": l["splines"],
                        "points_per_axis": l["points_per_axis"], "buffer_knots": l["buffer_knots"]} for l in lv],
            "relerr_vs_dense_far": err, "far_fraction_of_entries": float(far.mean()),
            "single_level_same_cubes": {"ms_per_far_product": round(ms1, 3), "relerr_vs_dense_far": err1}}


def fast_leg(args, bie, torch):
    """The fast operator (near entries stored sparse + multilevel B-spline far
    field, no dense matrix): (1) on the 30720-unknown sphere at k = 20 (leaf
    cubes 0.2 m, two levels) against the dense FP64 operator: product error and
    times, and one plane-wave GMRES(50) solve to 1e-6 with each; (2) on the
    491520-unknown sphere (icosphere level 7) at k = 4 (leaf cubes 0.05 m, four
    levels), where the packed FP64 matrix alone would take 1.9 TB: setup, memory
    and time per product (HIP events)."""
    from paper_2606_13482_amd.inputs import icosphere, complex_gaussian, planewave_set
    sync = torch.cuda.synchronize

    def ev_ms(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        sync()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        sync()
        return e0.elapsed_time(e1) / reps

    out = {}
    V, T = icosphere(5)
    k = 20.0
    sync()
    t0 = time.perf_counter()
    op = bie.FastOperator(V, T, k, 0.2, 2, 8, 3)
    sync()
    t_setup = time.perf_counter() - t0
    od = bie.Operator(V, T, k)
    x = torch.from_numpy(complex_gaussian(op.N, 5, cols=1)).cuda()
    y, yd = op.apply(x), od.apply(x)
    err = float(torch.linalg.norm(y - yd) / torch.linalg.norm(yd))
    ms_fast = ev_ms(lambda: op.apply(x, out=y), 5)
    ms_dense = ev_ms(lambda: od.apply(x, out=yd), 10)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    B = op.rhs(d, e)
    opts = bie.Solve(restart=50, tol=args.tol, max_mvp=20000)
    sync()
    t0 = time.perf_counter()
    X, st = op.solve(B, opts)
    sync()
    t_fast = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xd, std = od.solve(B, opts)
    sync()
    t_dense = time.perf_counter() - t0
    out["sphere30720_k20"] = {
        "workload": "PEC sphere, 20480 triangles (30720 RWG), k = 20; leaf cubes 0.2 m, 2 levels, s = 8, p = 3",
        "fast": op.fast_info(), "setup_s": round(t_setup, 3), "ms_per_product": round(ms_fast, 3),
        "ms_per_dense_fp64_product": round(ms_dense, 3), "product_relerr_vs_dense": err,
        "solve": {"fast_s": round(t_fast, 3), "fast_iters": st[0]["iters"], "fast_converged": bool(st[0]["converged"]),
                  "dense_s": round(t_dense, 3), "dense_iters": std[0]["iters"],
                  "solution_relerr_vs_dense": float(torch.linalg.norm(X - Xd) / torch.linalg.norm(Xd))}}
    od.close()
    op.close()
    V, T = icosphere(7)
    free0 = torch.cuda.mem_get_info()[0]
    sync()
    t0 = time.perf_counter()
    op = bie.FastOperator(V, T, 4.0, 0.05, 4, 8, 3)
    sync()
    t_setup = time.perf_counter() - t0
    used = (free0 - torch.cuda.mem_get_info()[0]) / 2 ** 30
    x = torch.from_numpy(complex_gaussian(op.N, 6, cols=1)).cuda()
    y = op.apply(x)
    ms = ev_ms(lambda: op.apply(x, out=y), 3)
    N = op.N
    out["sphere491520_k4"] = {
        "workload": "PEC sphere, 327680 triangles (491520 RWG), k = 4; leaf cubes 0.05 m, 4 levels, s = 8, p = 3",
        "fast": op.fast_info(), "setup_s": round(t_setup, 3), "gib_on_device": round(used, 2),
        "ms_per_product": round(ms, 3), "packed_fp64_matrix_gib": round(8.0 * N * (N + 64) / 2 ** 30, 1)}
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
        conv, its, rel = stats_of(st)
        out["star" if star else "assembled"] = {
            "solves_per_s": round(int(conv.sum()) / t, 2), "iters_mean": float(its.mean()),
            "converged": float(conv.mean()), "relres_true_fp64_max": float(rel.max())}
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
    10 edges per wavelength), 1..32 plane waves each, FP32 matrices with FP64
    copies: the batched solve certified in FP64 (cycles on the FP32 tiles, every
    residual on the FP64 tiles), right-preconditioned per surface with its
    Calderon preconditioner, against the same solves one surface after another
    (the same method, one operator per call) and against the batch without the
    preconditioner."""
    from paper_2606_13482_amd.inputs import uneven_batch
    sync = torch.cuda.synchronize
    probs = uneven_batch()
    sync()
    t0 = time.perf_counter()
    ops = [bie.Operator(p["V"], p["T"], p["k"], storage="c64", keep_fp64=True) for p in probs]
    Bs = [op.rhs(p["dirs"], p["pols"]) for op, p in zip(ops, probs)]
    sync()
    t_fill = time.perf_counter() - t0
    Ns = [op.N for op in ops]
    Rs = [b.shape[0] for b in Bs]
    nrhs = int(sum(Rs))
    opts = bie.Solve(restart=50, tol=args.tol, precision="mixed")
    # the combined criterion: 512 sampled FP64 rows gate each check, the full FP64 residual confirms
    opts_ccc = bie.Solve(restart=50, tol=args.tol, precision="mixed", crit="ccc", rscc_rows=512)

    def summary(sts, t):
        conv = np.array([s["converged"] for st in sts for s in st], bool)
        its = np.array([s["iters"] for st in sts for s in st])
        rel = [s["relres_true"] for st in sts for s in st]
        return {"solves_per_s": round(int(conv.sum()) / t, 2), "s": round(t, 3), "converged": float(conv.mean()),
                "iters_mean": float(its.mean()), "iters_max": int(its.max()),
                "relres_true_fp64_max": float(max(rel))}

    sync()
    t0 = time.perf_counter()
    pcs = [bie.Calderon(op) for op in ops]
    sync()
    t_pc = time.perf_counter() - t0
    bie.batch_config(0, True)
    t0 = time.perf_counter()
    bie.batch_solve(ops, Bs, opts, pcs=pcs)          # first call: autotuner, FP32 copies of M
    sync()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xs, sts = bie.batch_solve(ops, Bs, opts, pcs=pcs)
    sync()
    t_batch = time.perf_counter() - t0
    main = summary(sts, t_batch)
    # FP64 residuals recomputed from the returned solutions (FP64 tiles)
    rec = 0.0
    for op, B, X in zip(ops, Bs, Xs):
        rr = torch.linalg.vector_norm(B - op.apply(X), dim=1) / torch.linalg.vector_norm(B, dim=1)
        rec = max(rec, float(rr.max()))
    # one surface after another, the same method (a batch of one per call, fixed units)
    bie.batch_config(8, True)
    try:
        stq = []
        sync()
        t0 = time.perf_counter()
        for op, B, pc in zip(ops, Bs, pcs):
            stq.append(bie.batch_solve([op], [B], opts, pcs=[pc])[1][0])
        sync()
        t_seq = time.perf_counter() - t0
    finally:
        bie.batch_config(0, True)
    seq = summary(stq, t_seq)
    # the same batch to the combined criterion (one untimed call, then the timed one)
    bie.batch_solve(ops, Bs, opts_ccc, pcs=pcs)
    sync()
    t0 = time.perf_counter()
    _, stc = bie.batch_solve(ops, Bs, opts_ccc, pcs=pcs)
    sync()
    ccc = summary(stc, time.perf_counter() - t0)
    out = {"workload": (f"{len(ops)} surfaces, N {min(Ns)}..{max(Ns)}, {nrhs} plane waves; GMRES(50) on the FP32 "
                        f"matrices (grouped products on the FP32 matrix cores) right-preconditioned per surface "
                        f"(Calderon, FP32 copy of M), every residual on the FP64 matrices (FP64 matrix cores), to "
                        f"{args.tol:g} (FP64 SCC; "
                        f"key ccc: 512 sampled FP64 rows gate, the FP64 SCC confirms), max 10000 products per "
                        f"right-hand side"),
           **{k: v for k, v in main.items() if k != "s"}, "batch_s": main["s"], "relres_recomputed_fp64_max": rec,
           "first_call_s_with_autotune": round(t_first, 3), "fill_s": round(t_fill, 3),
           "calderon_setup_s": round(t_pc, 3),
           "solves_per_s_with_setup": round(main["solves_per_s"] * t_batch / (t_batch + t_pc), 2),
           "tiles_per_unit": bie.batch_tuned(ops, Rs),
           "ccc": ccc, "sequential": seq, "speedup_vs_sequential": round(t_seq / t_batch, 3),
           "packed_fp32_bytes_per_product": int(sum(4 * n * (n + 1) for n in Ns))}
    for pc in pcs:
        pc.close()
    if args.calderon:
        # the batch without the preconditioner (one call, autotuning included)
        sync()
        t0 = time.perf_counter()
        _, st0 = bie.batch_solve(ops, Bs, opts)
        sync()
        out["no_preconditioner"] = summary(st0, time.perf_counter() - t0)
    for op in ops:
        op.close()
    return out


def counters_probe(args, bie, torch):
    """Kernels for the hardware counters: 5 launches each of the packed FP64
    product (one column), the split-BF16 block product and the FP64 block product
    (512 columns, the headline's 16 groups of 32) on the bench operator; the
    fill of that operator in FP64 and in FP32; the grouped products of the uneven
    batch (FP32 and FP64 matrices, all 1069 columns, the autotuned layouts: the
    candidates' timing launches, then one restart cycle of 1 step on the FP32
    tiles and its residuals on the FP64 tiles, once with the vector-unit pass and
    once with the matrix-core pass); one solve of the headline's batch from zero (1024
    right-hand sides of 512 directions, the headline's mixed block GMRES: 2-term
    products, FP16-pair basis; the kernels at the shapes the bench times); and 3
    plain copies of 1 GiB (FETCH_SIZE / WRITE_SIZE
    calibration)."""
    from paper_2606_13482_amd.inputs import icosphere, complex_gaussian, uneven_batch, random_directions
    V, T = icosphere(args.level)
    for storage in ("c128", "c64"):
        bie.Operator(V, T, args.k, storage=storage).close()
    op = bie.Operator(V, T, args.k, storage="split_bf16")
    x = torch.from_numpy(complex_gaussian(op.N, 7)).cuda().reshape(1, -1)
    Xb = torch.from_numpy(complex_gaussian(op.N, 7, cols=512)).cuda()
    for _ in range(5):
        op.apply(x)
    for _ in range(5):
        op.apply(Xb, block=True)
    for _ in range(5):
        op.apply(Xb, block="fp64")
    dte, pte, _ = planewave_batch(bie, random_directions(args.test_dirs, 55))
    Bh = op.rhs(dte, pte)
    torch.cuda.synchronize()
    bie.prof_enable(True)
    prof_reset(bie)
    _, sth = op.solve(Bh, mixed_opts(args, bie, args.restart))
    torch.cuda.synchronize()
    orth = {kk: bie.prof_read(kk, columns=True) for kk in (4, 5)}   # launches, ms, basis pairs / vectors
    bie.prof_enable(False)
    del Bh
    probs = uneven_batch()
    ops = [bie.Operator(p["V"], p["T"], p["k"], storage="c64", keep_fp64=True) for p in probs]
    Bs = [o.rhs(p["dirs"], p["pols"]) for o, p in zip(ops, probs)]
    one = bie.Solve(restart=1, tol=1e-6, max_mvp=2, precision="mixed")
    try:
        for mfma in (False, True):      # the autotuned layout, cycles launched one by one
            bie.batch_config(0, False, matrix_cores=mfma)
            bie.batch_solve(ops, Bs, one)
    finally:
        bie.batch_config(0, True)
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_probe": {"N": op.N, "packed_fp64_launches": 5, "block_launches": 5,
                                         "block_columns": 512, "copy_bytes": a.numel() * 4, "copies": 3,
                                         "headline_solve_rhs": len(sth),
                                         "headline_solve_converged": float(np.mean([s["converged"] for s in sth])),
                                         "headline_solve_basis_dots": {"launches": orth[4][0],
                                                                       "basis_vector_column_pairs": orth[4][2]},
                                         "headline_solve_basis_update": {"launches": orth[5][0],
                                                                         "basis_vectors_read": orth[5][2],
                                                                         "basis_bytes_per_entry": 4},
                                         "batch_packed_fp32_bytes": int(sum(4 * o.N * (o.N + 1) for o in ops)),
                                         "batch_columns": int(sum(b.shape[0] for b in Bs))}}),
          flush=True)
    for o in ops:
        o.close()
    op.close()


def autotune_summary(rep: dict) -> dict:
    """The autotuner's choices by kind: packed-product units per size, the
    block products' (wave tile, K slices) and K slices counted over the shapes
    met, and the batch layouts (tiles per unit, columns per item)."""
    out = {"entries": len(rep)}
    for kind in ("sym", "gemm_split", "gemm64", "batch"):
        sel = {k: v for k, v in rep.items() if k.split(":")[0] == kind}
        if not sel:
            continue
        if kind in ("sym", "batch"):
            out[kind] = sel
        else:
            counts = {}
            for v in sel.values():
                counts[str(v)] = counts.get(str(v), 0) + 1
            out[kind] = {"shapes": len(sel), "choices": counts}
    return out


def cpu_baseline(level: int, k: float, restart: int, plain_mvps: float):
    """The oracle (C fill with OpenMP + numpy GMRES) on a bounded sample: the full
    FP64 fill and one GMRES(restart) cycle with all host threads, and one cycle
    with a single thread; a solve with the matrix resident is extrapolated to the
    mean number of products plain FP64 GMRES needed on the GPU sample."""
    from threadpoolctl import threadpool_info, threadpool_limits
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
    pools = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in pools] + [1])

    def cycle():
        t0 = time.perf_counter()
        _, st = krylov.gmres(Z, b, m=restart, tol=1e-30, max_mvp=restart)
        return (time.perf_counter() - t0) / max(1, st.mvps)

    t_mvp = cycle()
    with threadpool_limits(limits=1):
        t_mvp1 = cycle()
    return {"value": round(1.0 / (plain_mvps * t_mvp), 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"full oracle FP64 fill of the {rwg['N']}-unknown matrix ({t_fill:.2f} s, {threads} threads) "
                       f"and one GMRES({restart}) cycle ({t_mvp * 1e3:.1f} ms per iteration); a matrix-resident "
                       f"solve extrapolated to the {plain_mvps:.0f} products plain FP64 GMRES took on the GPU sample"),
            "fill_s": round(t_fill, 3),
            "single_thread": {"value": round(1.0 / (plain_mvps * t_mvp1), 5), "cores": 1,
                              "sample": f"one GMRES({restart}) cycle on one thread ({t_mvp1 * 1e3:.1f} ms per "
                                        f"iteration), extrapolated the same way"}}


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
    if args.batch_only:
        print(json.dumps({"uneven_batch": uneven_batch_leg(args, bie, torch)}), flush=True)
        return
    V, T = icosphere(args.level)
    k = args.k
    N = 3 * T.shape[0] // 2
    plain, roof_gemv = plain_leg(args, bie, torch, V, T, k)
    print(json.dumps({"progress": "plain leg done", "solves_per_s": plain["solves_per_s"]}), file=sys.stderr,
          flush=True)
    op, ws, head, roof, ms_step, plain_mvps, batch = headline_leg(args, bie, torch, V, T, k)
    print(json.dumps({"progress": "headline done", "solves_per_s": head["solves_per_s"]}), file=sys.stderr, flush=True)
    K = head["training"]["pod_rank"]
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
        "config": {"workload": (f"learned warm start on the PEC sphere r=1 m, icosphere {T.shape[0]} triangles ({N} "
                                f"RWG), k={k:g}: trained on {2 * args.train_dirs} solves ({args.train_dirs} directions "
                                f"x theta/phi), POD {K} modes, MLP 4-{args.hidden}-{args.hidden}-{2 * K} "
                                f"({args.epochs} epochs); each step serves {2 * args.test_dirs} held-out plane waves "
                                f"({args.test_dirs} directions x theta/phi) with operator and warm start resident: "
                                f"block GMRES({args.restart}) over groups of {args.block} on {args.inner_terms}-term "
                                f"split-BF16 MFMA products, {'FP16-pair' if args.basis == 'f16' else 'complex64'} "
                                f"inner basis, FP64 refinement to {args.tol:g} (FP64 SCC), unpreconditioned"),
                   "N": N, "k": k, "restart": args.restart, "inner_tol": args.inner_tol, "method": "bgmres",
                   "block": args.block, "inner_terms": args.inner_terms, "inner_basis": args.basis, "calderon": False,
                   "rhs_per_step": 2 * args.test_dirs, "train_directions": args.train_dirs,
                   "test_directions": args.test_dirs, "pod_rank": K, "hidden": args.hidden, "epochs": args.epochs,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "roofline_gemv": roof_gemv,
        "headline": head,
        "plain_fp64_step": plain,
    }
    if args.calderon:
        out["calderon"] = calderon_leg(args, bie, torch, op, ws, batch)
    ws.close()
    op.close()
    del batch
    torch.cuda.empty_cache()
    if args.c3:
        out["c3"] = c3_leg(args, bie, torch)
        print(json.dumps({"progress": "c3 done", "solves_per_s": out["c3"]["solves_per_s"]}), file=sys.stderr,
              flush=True)
    out["fill"] = fill_leg(args, bie, torch)
    out["far_field"] = far_leg(args, bie, torch, V, T, k)
    if args.star:
        out["star_split"] = star_leg(args, bie, torch, V, T)
    out["fast_operator"] = fast_leg(args, bie, torch)
    print(json.dumps({"progress": "fast operator done"}), file=sys.stderr, flush=True)
    if args.batch:
        out["uneven_batch"] = uneven_batch_leg(args, bie, torch)
        print(json.dumps({"progress": "uneven batch done"}), file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.level, k, args.restart, plain_mvps)
    # launch shapes the autotuner chose in this run (packed product units per
    # size; block products' wave tiles and K slices per shape; batch units)
    out["autotune"] = autotune_summary(bie.autotune_report())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
