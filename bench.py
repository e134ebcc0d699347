#!/usr/bin/env python3
"""AFN-PCG benchmark on one MI355X.

Default workload (the mixed-precision head-to-head): n = 200000 points
~ N(0, I) in R^8, Gaussian kernel l = 2, mu = 1e-2, k = 4000 FPS landmarks, one
right-hand side b ~ N(0, 1), relative residual 1e-6.  One step = one complete
solve of (K + mu I) a = b through the C-ABI: landmark selection by FPS
(Algorithm 6), the preconditioner (Algorithm 5's Nystrom branch at k = 4000:
chol(K11 + nu I), W = L^{-1} K[S, :], chol(W W^T + mu I)) and PCG, in mixed
precision (FP32 operator and preconditioner inside FP64 iterative
refinement); the FP64 path solves the same input beside it, and the AFN
branch (Algorithm 2's factorization) is reported by --c3-branch afn.
Inputs are resident in HBM before the timed region.

Prints ONE JSON line: value = mixed-precision solves/s; roofline of the
dominant kernel (the FP32 kernel-matvec tile kernel of the inner solves, timed
live with HIP events around each of its launches inside the timed solves);
cpu_baseline = the FP64 oracle on a bounded sample of the same workload,
extrapolated to one solve.  --workload c2|c4|highd|batch and --serving select the
other workloads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAK_FP64_TFLOPS = 78.6          # MI355X FP64 vector (FMA = 2 flops)
PEAK_FP32_TFLOPS = 157.3         # MI355X FP32 (vector, and dense MFMA)
# FP64 VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_F64_LANE_OPS = 256 * 4 * 16 * 2.4e9
# VALU instructions per unique kernel evaluation in the tile-pair loop of
# kmv_sym_mf<0, 3, double, double> (AMD assembly of the compiled kernel, per lane and
# tile pair, i.e. per 16 pairs, besides 4 MFMAs that also add the squared
# norms): 245 where the software FP64 2^-t runs (13 instructions per
# table-driven exponential plus one LDS read, 2 FMAs for the row and column
# products; tile pairs whose boxes bound t), 80 on tile pairs whose values are
# all below 2^-46 (FP32 exponential), and 26 for the column sums across lane
# groups and the loop itself.
VALU_F64_OPS_PER_PAIR_D3 = (245 + 26) / 16
VALU_F64_OPS_PER_FAR_PAIR_D3 = (80 + 26) / 16


def kmv_flops(n: int, d: int, nrhs: int = 1) -> float:
    """Algorithmic flops of one (K + mu I) v: E = n(n-1)/2 unique kernel
    evaluations at (3d + 1) flops each (difference, square and sum per
    coordinate, the exponential counted as one flop), 2 n^2 R flops for the
    products with v and 2 n R for mu v."""
    E = n * (n - 1) / 2
    return E * (3 * d + 1) + 2.0 * n * n * nrhs + 2.0 * n * nrhs


def source_hash(path: pathlib.Path) -> str:
    """sha256[:16] of a tile-kernel source together with the kernel-function
    header and the tile-kernel body it includes."""
    h = hashlib.sha256(path.read_bytes())
    h.update((path.parent / "kfun.h").read_bytes())
    body = path.parent / "kmv_sym_mf_body.inc"
    if body.exists():
        h.update(body.read_bytes())
    return h.hexdigest()[:16]


def counters_from_profile(kernel_src: pathlib.Path, name: str = "kmv_f64_sym_c2_counters.txt") -> dict:
    """HBM bytes per launch, clock and VALU issue fraction of the tile kernel
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source (else an empty dict)."""
    f = ROOT / "profiles" / name
    if not f.exists():
        return {}
    vals = {}
    for line in f.read_text().splitlines():
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != source_hash(kernel_src):
        return {}
    out = {}
    for key in ("hbm_bytes_per_launch", "clock_ghz", "valu_issue_frac"):
        try:
            out[key] = float(vals[key])
        except (KeyError, ValueError):
            pass
    return out


def cpu_baseline(X, b, l, mu, k, w, iters, n_rows=2000, n_knn=500, n_fsai=6):
    """The oracle on a bounded sample, extrapolated to one full solve:
    FPS and chol(K11 + mu I) in full; kernel-matvec rows, kNN rows and FSAI
    rows (each with its own L^{-1} K12 columns) on uniform samples scaled by
    the row count; one full Algorithm 3 apply.  t = setup + iters (matvec +
    apply), with iters the GPU's iteration count."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(7)
    n = X.shape[0]
    nr = n - k
    t = {}
    t0 = time.perf_counter()
    idx, _ = oracle.fps(X, k)
    t["fps"] = time.perf_counter() - t0
    perm = oracle.permutation(n, idx)
    Xp = X[perm]
    t0 = time.perf_counter()
    L = oracle.landmark_cholesky(Xp, k, l, mu)
    t["chol"] = time.perf_counter() - t0
    rows = rng.integers(0, nr, n_knn)
    t0 = time.perf_counter()
    oracle.knn_rows(Xp[k:], w, rows)
    t["knn"] = (time.perf_counter() - t0) * nr / n_knn
    rows = rng.integers(w, nr, n_fsai)
    t0 = time.perf_counter()
    oracle.fsai_rows(X, l, mu, perm, L, w, rows)
    per_row = (time.perf_counter() - t0) / n_fsai
    # each sampled row forms its w columns of L^{-1} K12; the full build forms
    # every column once, so V + FSAI ~ nr * per_row / w (a lower bound: the
    # Gram work per row is counted w times too few)
    t["v_fsai"] = nr * per_row / w
    rows = rng.integers(0, n, n_rows)
    t0 = time.perf_counter()
    oracle.kernel_matvec_rows(X, l, mu, b, rows)
    t_mv = (time.perf_counter() - t0) * n / n_rows
    # Algorithm 3 in the oracle recomputes K12 twice (2 k nr kernel
    # evaluations), which dominates its cost: timed as kernel rows of the
    # landmark block
    t0 = time.perf_counter()
    lm_rows = np.arange(min(k, 200))
    oracle.kernel_matvec_rows(Xp[: k + nr], l, 0.0, np.ones(n), lm_rows)
    t_apply = (time.perf_counter() - t0) * k / len(lm_rows) * 2
    t_total = sum(t.values()) + iters * (t_mv + t_apply)
    hc = host_cpu()
    return {
        **hc,
        "value": 1.0 / t_total,
        "unit": "solves/s",
        "cores": hc["omp_num_threads"],
        "kind": "oracle",
        "sample": (f"FPS and chol(K11+mu I) in full; {n_rows} kernel-matvec rows, {n_knn} kNN "
                   f"rows, {n_fsai} FSAI rows (with their L^-1 K12 columns) and {len(lm_rows)} "
                   f"landmark kernel rows, scaled to n={n}, k={k}; {iters} PCG iterations; "
                   f"extrapolated seconds per solve {t_total:.1f} "
                   f"(setup {sum(t.values()):.1f}, matvec {t_mv:.2f}/it, apply {t_apply:.2f}/it)"),
    }


def _line(metric, value, unit, steps, warmup, ms, dtype, config, **extra):
    out = {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out))


def tune_decisions(args) -> dict:
    """The autotuner's decisions of this run (taken in the warm-up): how many
    shape classes it timed, and those where a candidate other than the
    built-in heuristic's won, with the ms of each candidate."""
    from paper_2304_05460_amd import afn
    out = {"mode": args.tune, "shape_classes": 0, "kmv_tile": {}, "not_heuristic": {}}
    for line in afn.tune_report().splitlines():
        f = line.split()
        if len(f) < 2:
            continue
        out["shape_classes"] += 1
        key = f[0].rsplit("|", 1)[0]
        val = [int(f[1])] + [round(float(t), 4) for t in f[2:]]
        if key.startswith("kmv_tile"):
            out["kmv_tile"][key] = val
        elif val[0] != 0:
            out["not_heuristic"][key] = val
    return out


def host_cpu() -> dict:
    """The host the oracle ran on: CPU model (lscpu), logical CPUs (nproc) and
    the OpenMP thread count it used."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:  # noqa: BLE001
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"cpu_model": model, "nproc": os.cpu_count(), "omp_num_threads": threads}


def cpu_baseline_nystrom(X, l, mu, k, iters, n_rows=1000, n_mv=2000, seed=7):
    """The oracle's Nystrom-branch solve (FPS, Y = K[:, S], chol(K_SS + nu I),
    B = Y C^{-T}, thin SVD, then PCG with the Woodbury apply) on a bounded
    sample, extrapolated to one full solve: FPS in full; the kernel columns,
    the triangular solve and the SVD on n_rows-row slices scaled by the row
    count (each is linear in n for n >> k); kernel-matvec rows on n_mv rows;
    the apply's two products with U on an n_rows-row slice; iters PCG
    iterations (the GPU's FP64 count)."""
    import numpy as np
    import scipy.linalg
    import oracle
    from oracle import nystrom as ny
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    t = {}
    t0 = time.perf_counter()
    idx, _ = oracle.fps(X, k)
    t["fps"] = time.perf_counter() - t0
    rows = rng.choice(n, n_rows, replace=False)
    Xs = np.vstack([X[rows], X[idx]])
    t0 = time.perf_counter()
    Y = ny.kernel_columns(Xs, l, np.arange(n_rows, n_rows + k))     # K[rows and S, S]
    t["kernel_columns"] = (time.perf_counter() - t0) * n / (n_rows + k)
    Ys, Kss = Y[:n_rows], Y[n_rows:]
    t0 = time.perf_counter()
    C = np.linalg.cholesky(Kss + 1e-12 * np.eye(k))
    t["chol"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Bs = scipy.linalg.solve_triangular(C, Ys.T, lower=True).T
    t["trsm"] = (time.perf_counter() - t0) * n / n_rows
    t0 = time.perf_counter()
    Bs2 = np.vstack([Bs] * max(1, (2 * k) // n_rows + 1))     # at least 2k rows: the thin-SVD regime
    np.linalg.svd(Bs2, full_matrices=False)
    t["svd"] = (time.perf_counter() - t0) * n / Bs2.shape[0]
    v = rng.standard_normal(n)
    mv_rows = rng.integers(0, n, n_mv)
    t0 = time.perf_counter()
    oracle.kernel_matvec_rows(X, l, mu, v, mv_rows)
    t_mv = (time.perf_counter() - t0) * n / n_mv
    U = np.linalg.qr(Bs)[0]
    r = rng.standard_normal(n_rows)
    t0 = time.perf_counter()
    for _ in range(3):
        tt = U.T @ r
        _ = U @ tt + r
    t_apply = (time.perf_counter() - t0) / 3 * n / n_rows
    setup = sum(t.values())
    total = setup + iters * (t_mv + t_apply)
    hc = host_cpu()
    return dict({"value": 1.0 / total, "unit": "solves/s", "cores": hc["omp_num_threads"], "kind": "oracle",
                 "sample": (f"FPS (k={k}) in full; kernel columns, triangular solve and SVD on {n_rows}-row "
                            f"slices, {n_mv} kernel-matvec rows and the apply on a {n_rows}-row slice, "
                            f"scaled to n={n}; {iters} PCG iterations; extrapolated seconds per solve "
                            f"{total:.1f} (setup {setup:.1f}: " +
                            ", ".join(f"{k_} {v_:.1f}" for k_, v_ in t.items()) +
                            f"; matvec {t_mv:.2f}/it, apply {t_apply:.3f}/it)")}, **hc)


def c3_bench(args):
    """n = 2e5 standard normal points in R^8, l = 2, mu = 1e-2, k = 4000 FPS
    landmarks, tol 1e-6: the mixed-precision solve (value, args.steps timed
    solves after args.warmup) against the FP64 solve of the same input
    (min(steps, 2) timed solves), both through the C-ABI."""
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    p = W.C3
    X_np, b_np = W.make(p)
    X = torch.tensor(X_np, device="cuda")
    b = torch.tensor(b_np, device="cuda")
    afn.lib()
    method = afn.AFN_METHOD_AFN if args.c3_branch == "afn" else afn.AFN_METHOD_NYSTROM
    maxit = args.maxit if args.maxit else (8000 if args.c3_branch == "afn" else p.maxit)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def step(prec):
        h = afn.afn_setup(X, p.l, p.mu, k=p.k, w=p.w, precision=prec, method=method, nrhs_max=0)
        x, info = afn.afn_pcg_solve(h, b, tol=p.tol, maxit=maxit)
        si = h.info()
        h.close()
        return x, info, si

    def timed(prec, label, steps, warmup):
        log(f"c3 {label}: {args.c3_branch} branch; warmup {warmup}, timed {steps}")
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        for i in range(steps):
            out.append(step(prec))
            log(f"c3 {label}: step {i + 1}/{steps}: {afn.status_name(out[-1][1]['status'])}, "
                f"{out[-1][1]['iterations']} its")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return out, el

    res32, el32 = timed(afn.AFN_FP32, "mixed", args.steps, args.warmup)
    if args.mixed_only:      # profiling runs: the timed mixed solves alone
        i32 = res32[-1][1]
        print(json.dumps({"workload": p.name, "mixed_only": True, "solves_per_s": args.steps / el32,
                          "status": afn.status_name(i32["status"]), "iterations_inner": i32["iterations"],
                          "kmv_f32_avg_launch_ms": i32["ms_matvec"] / max(i32["matvec_launches"], 1)}))
        return
    steps64 = min(args.steps, 2)
    res64, el64 = timed(afn.AFN_FP64, "fp64", steps64, min(args.warmup, 1))
    res16, el16 = timed(afn.AFN_BF16, "mixed-bf16", steps64, min(args.warmup, 1))
    x32, i32, s32 = res32[-1]
    x64, i64, s64 = res64[-1]
    rel = float(torch.linalg.vector_norm(x32 - x64) / torch.linalg.vector_norm(x64))
    launches = sum(r[1]["matvec_launches"] for r in res32)
    kmv_ms = sum(r[1]["ms_matvec"] for r in res32) / max(launches, 1)
    F = kmv_flops(p.n, p.d)
    achieved = F * s32.kmv_kept_f32 / (kmv_ms * 1e-3) / 1e12
    ctrs = counters_from_profile(ROOT / "paper_2304_05460_amd" / "csrc" / "kmv.hip", "kmv_d8_c3_counters.txt")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": ctrs.get("hbm_bytes_per_launch"),
                "kernel": "kmv_sym_mf<0, 8, float, float> (inner solves)",
                "avg_launch_ms": round(kmv_ms, 4), "launches": launches,
                "flops_per_launch": F * s32.kmv_kept_f32, "tile_pairs_evaluated": round(s32.kmv_kept_f32, 4)}
    if "valu_issue_frac" in ctrs:
        roofline["valu_issue_frac_counters"] = ctrs["valu_issue_frac"]
        roofline["clock_ghz_counters"] = ctrs.get("clock_ghz")
    ms64 = sum(r[1]["ms_matvec"] for r in res64) / max(sum(r[1]["matvec_launches"] for r in res64), 1)
    value = args.steps / el32
    fp64_value = steps64 / el64
    out = {
        "metric": "AFN-PCG solves/s at rel-res 1e-6, mixed precision (FP64 path on the same input beside it)",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el32 / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "d": p.d, "points": "normal", "l": p.l, "mu": p.mu,
                   "k": p.k, "landmarks": "fps", "tol": p.tol, "maxit": maxit, "nrhs": 1,
                   "preconditioner": args.c3_branch,
                   "branch_note": ("Algorithm 5's Nystrom branch at k = 4000; Algorithm 2's AFN "
                                   "factorization (--c3-branch afn) needs thousands of iterations on "
                                   "this distribution") if args.c3_branch == "nystrom" else
                                  "Algorithm 2's AFN factorization, w = 64"},
        "mixed": {"status": afn.status_name(i32["status"]), "iterations_inner": i32["iterations"],
                  "outer_iterations": i32["outer_iterations"], "fp64_fallback_iterations": i32["fp64_iterations"],
                  "relres_true_fp64": i32["relres_true"], "rel_diff_vs_fp64_solution": rel,
                  "setup_ms": round(s32.ms["total"], 1), "solve_ms": round(i32["ms_solve"], 1),
                  "kmv_f32_avg_launch_ms": round(kmv_ms, 4)},
        "fp64": {"value": round(fp64_value, 4), "unit": "solves/s", "steps": steps64,
                 "ms_per_step": round(el64 / steps64 * 1e3, 2), "status": afn.status_name(i64["status"]),
                 "iterations": i64["iterations"], "relres_true": i64["relres_true"],
                 "setup_ms": round(s64.ms["total"], 1), "solve_ms": round(i64["ms_solve"], 1),
                 "kmv_f64_avg_launch_ms": round(ms64, 4),
                 "kmv_f64_tflops": round(F * s64.kmv_kept_f64 / (ms64 * 1e-3) / 1e12, 3)},
        "mixed_bf16": {"value": round(steps64 / el16, 4), "unit": "solves/s", "steps": steps64,
                       "status": afn.status_name(res16[-1][1]["status"]),
                       "iterations_inner": res16[-1][1]["iterations"],
                       "outer_iterations": res16[-1][1]["outer_iterations"],
                       "relres_true_fp64": res16[-1][1]["relres_true"],
                       "rel_diff_vs_fp64_solution": float(torch.linalg.vector_norm(res16[-1][0] - x64)
                                                          / torch.linalg.vector_norm(x64)),
                       "setup_ms": round(res16[-1][2].ms["total"], 1),
                       "solve_ms": round(res16[-1][1]["ms_solve"], 1)},
        "speedup_mixed_vs_fp64": round(value / fp64_value, 3),
        "roofline": roofline,
    }
    out["autotune"] = tune_decisions(args)
    if not args.no_serving:
        # the latency side of the metric: a short request stream (48 requests,
        # n log-uniform in [2e3, 2e4], d in {3, 8}, Algorithm 5's method each)
        log("serving leg: 48 requests, burst then Poisson")
        sb, sp, rate, pois, ns = run_serving(48, 2e3, 2e4, 8, 2, log)
        out["serving"] = {"workload": "serving_48_requests_n2e3_2e4_d3_8", "slots": 8,
                          "poisson_rate_per_s": round(rate, 3), "burst_solves_per_s": round(sb["solves_per_s"], 3),
                          "poisson": _fmt({k: sp[k] for k in ("completed", "failed", "solves_per_s", "p50_s",
                                                              "p99_s", "max_relres_true", "grouped_frac")})}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline_nystrom(X_np, p.l, p.mu, p.k, i64["iterations"])
    print(json.dumps(out))


def highd_bench(args):
    """n = 49990 uniform points in [0,1]^22, l = 1, mu = n 1e-6, adaptive k <= 2000:
    Algorithm 2 takes uniform landmarks above d = 10; FP64 (the packed tile
    kernels cover d <= 8, so the generic FP64 tile kernel runs)."""
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    p = W.HIGHD
    X_np, b_np = W.make(p)
    X = torch.tensor(X_np, device="cuda")
    b = torch.tensor(b_np, device="cuda")
    afn.lib()

    def step():
        h = afn.afn_setup(X, p.l, p.mu, k=p.k, w=p.w, k_max=p.k_max)
        x, info = afn.afn_pcg_solve(h, b, tol=p.tol, maxit=p.maxit)
        si = h.info()
        h.close()
        return info, si

    print(f"[bench] highd warmup", file=sys.stderr, flush=True)
    info, si = step()
    print(f"[bench] highd warmup done: {afn.status_name(info['status'])} {info['iterations']} its, "
          f"setup {si.ms['total']:.0f} ms, solve {info['ms_solve']:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for st in range(args.steps):
        infos.append(step())
        print(f"[bench] highd step {st + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info, si = infos[-1]
    _line("AFN-PCG solves/s at rel-res 1e-6 (FP64, d = 22, uniform landmarks)", args.steps / el,
          "solves/s", args.steps, 1, el / args.steps * 1e3, "f64",
          {"workload": p.name, "n": p.n, "d": p.d, "l": p.l, "mu": p.mu, "k": si.k, "w": p.w,
           "tol": p.tol},
          highd={"status": afn.status_name(info["status"]), "iterations": info["iterations"],
                 "relres_true": info["relres_true"], "landmarks": ["auto", "fps", "uniform"][si.landmarks],
                 "rank": {"r": si.rank_r, "k_est": si.rank_k_est}, "setup_ms": round(si.ms["total"], 1),
                 "setup_phases_ms": {k: round(v, 1) for k, v in si.ms.items()},
                 "solve_ms": round(info["ms_solve"], 1),
                 "kmv_avg_launch_ms": round(info["ms_matvec"] / max(info["matvec_launches"], 1), 3)})


def c4_bench(args):
    """n = 1.5e5 uniform in [0,1]^3, l = 0.05, mu = 1e-4, k = 3000, w = 64, 64
    right-hand sides: FP32 setup + graph-captured block PCG with per-column FP64
    refinement to rel-res 1e-6.  value = right-hand sides solved per second."""
    import numpy as np
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    p = W.C4
    X_np, B_np = W.make(p)
    X = torch.tensor(X_np, device="cuda")
    B = torch.tensor(np.ascontiguousarray(B_np.T), device="cuda").t()
    afn.lib()
    print("[bench] c4 kernel matvec, 64 columns", file=sys.stderr, flush=True)
    mv = {}
    for name, prec in (("f32", afn.AFN_FP32), ("f64", afn.AFN_FP64)):
        afn.kernel_matvec(X, p.l, p.mu, B, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        afn.kernel_matvec(X, p.l, p.mu, B, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        mv[name + "_ms"] = round(e0.elapsed_time(e1), 3)
    print(f"[bench] c4 setup + block solve", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = afn.afn_setup(X, p.l, p.mu, k=p.k, w=p.w, precision=afn.AFN_FP32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, info = afn.afn_pcg_solve(h, B, tol=p.tol, maxit=p.maxit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    si = h.info()
    h.close()
    R = B.shape[1]
    n = p.n
    F = (n * (n - 1) / 2) * (3 * p.d + 1) + 2.0 * n * n * R + 2.0 * n * R
    _line("right-hand sides solved per second (64 per block, setup included)", R / (t2 - t0),
          "rhs-solves/s", 1, 0, (t2 - t0) * 1e3, "f32+f64",
          {"workload": p.name, "n": n, "d": p.d, "l": p.l, "mu": p.mu, "k": p.k, "w": p.w,
           "tol": p.tol, "nrhs": R},
          c4={"setup_ms": round((t1 - t0) * 1e3, 1), "solve_ms": round((t2 - t1) * 1e3, 1),
              "status": afn.status_name(info["status"]), "inner_iterations": info["iterations"],
              "outer_iterations": info["outer_iterations"], "relres_true_max": info["relres_true"],
              "setup_phases_ms": {k: round(v, 1) for k, v in si.ms.items()},
              "kmv_64rhs": dict(mv, tile_pairs_evaluated_f32=round(si.kmv_kept_f32, 4),
                                 tile_pairs_evaluated_f64=round(si.kmv_kept_f64, 4),
                                 evaluated_tflops_f32=round(F * si.kmv_kept_f32 / (mv["f32_ms"] * 1e-3) / 1e12, 2),
                                 evaluated_tflops_f64=round(F * si.kmv_kept_f64 / (mv["f64_ms"] * 1e-3) / 1e12, 2))},
          roofline=_c4_roofline(F * si.kmv_kept_f32 / (mv["f32_ms"] * 1e-3) / 1e12))


def _c4_roofline(evaluated_tflops: float) -> dict:
    """The 64-column FP32 tile kernel is bound by the matrix cores: 2 R flops
    per evaluated pair on MFMA against one kernel value on the VALU.
    achieved = the algorithmic flops of the tile pairs it evaluates over the
    time of the whole 64-column kernel_matvec call (its ordering, packing and
    gathers included, so a lower bound for the kernel itself)."""
    return {"bound": "mfma", "achieved": round(evaluated_tflops, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(evaluated_tflops / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": "kmv_mrhs_pipe<0, 3, 4>"}


def batch_bench(args):
    """Continuous batching of like small solves: 16 mixed-precision AFN solves
    (n = 3000 .. 3555, d = 3 uniform, l = 0.3, mu = 1e-3, k = 150, w = 32, one
    right-hand side each), set up first, then advanced together by
    afn_pcg_step_many to rel-res 1e-6; the iteration phase timed with grouped
    launches (one ragged launch per kernel over all like solves) and with
    every solve's kernels launched on their own.  The solutions of the two
    modes must agree bit for bit."""
    import numpy as np
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    afn.lib()
    G = 16
    hs, bs = [], []
    for i in range(G):
        n = 3000 + 37 * i
        X = torch.tensor(W.points("uniform", n, 3, 900 + i), device="cuda")
        hs.append(afn.afn_setup(X, 0.3, 1e-3, k=150, w=32, precision=afn.AFN_FP32, nrhs_max=0))
        bs.append(torch.tensor(np.random.default_rng(950 + i).standard_normal(n), device="cuda"))

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        states = [afn.afn_pcg_begin(h, b, tol=1e-6, maxit=400) for h, b in zip(hs, bs)]
        while not all(s.query()[0] for s in states):
            afn.afn_pcg_step_many(states, iters=8)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        infos = [s.query()[1] for s in states]
        xs = [s.x.clone() for s in states]
        for s in states:
            s.end()
        return t, infos, xs

    res = {}
    for mode in (False, True):
        afn.group_config(mode)
        for _ in range(max(1, args.warmup)):
            run()
        best = None
        for _ in range(max(1, args.steps)):
            t, infos, xs = run()
            if best is None or t < best[0]:
                best = (t, infos, xs)
        res[mode] = best
    afn.group_config(True)
    same = all(torch.equal(a, b) for a, b in zip(res[False][2], res[True][2]))
    its = sum(i["iterations"] for i in res[True][1])
    grp = sum(i["grouped_units"] for i in res[True][1])
    tg, tn = res[True][0], res[False][0]
    print(json.dumps({
        "metric": "batched small solves/s (iteration phase, 16 like mixed-precision solves)",
        "value": round(G / tg, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tg * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch16_uniform3d_n3000_3555", "solves": G, "tol": 1e-6},
        "ungrouped": {"value": round(G / tn, 3), "ms": round(tn * 1e3, 3)},
        "speedup": round(tn / tg, 3),
        "us_per_iteration": {"grouped": round(tg / its * 1e6, 2), "ungrouped": round(tn / its * 1e6, 2)},
        "iterations": its, "grouped_frac": round(grp / max(1, its), 4), "bitwise_equal": same,
    }))
    for h in hs:
        h.close()


def setups_bench(args):
    """Setups of small requests: the first 16 requests of the serving mix
    with n log-uniform in [2e3, 2e4] (workloads.serving_requests, seed 5:
    d in {3, 8}, l log-uniform in [0.01, 2], mu in {1e-4, 1e-2}), Algorithm 5
    choosing the branch, FP32 precision, one after another on one stream;
    per request the setup time (inputs resident) and afn_setup's phase times,
    the best of --steps timed runs after --warmup."""
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    afn.lib()
    probs = W.serving_requests(48, n_lo=2e3, n_hi=2e4)[:16]
    data = [torch.tensor(W.make(q)[0], device="cuda") for q in probs]

    def once():
        rows = []
        for q, X in zip(probs, data):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = afn.afn_setup(X, q.l, q.mu, k=q.k, w=q.w, k_max=q.k_max, precision=afn.AFN_FP32,
                              method=afn.AFN_METHOD_AUTO, nrhs_max=0)
            si = h.info()
            torch.cuda.synchronize()
            rows.append((time.perf_counter() - t0, q, si))
            h.close()
        return rows

    for _ in range(max(0, args.warmup)):
        once()
    best = None
    for _ in range(max(1, args.steps)):
        rows = once()
        if best is None or sum(r[0] for r in rows) < sum(r[0] for r in best):
            best = rows
    total = sum(r[0] for r in best)
    print(json.dumps({
        "metric": "small-request setups/s (16 requests of the serving mix, one after another)",
        "value": round(len(best) / total, 3), "unit": "setups/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "setups16_serving_mix_n2e3_2e4", "requests": len(best)},
        "requests": [{"n": q.n, "d": q.d, "k": si.k, "method": "nystrom" if si.method else "afn",
                      "setup_ms": round(t * 1e3, 2), "phases_ms": {k: round(v, 2) for k, v in si.ms.items()}}
                     for t, q, si in best],
        "phases_ms_total": {k: round(sum(si.ms[k] for _, _, si in best), 1) for k in best[0][2].ms},
    }))


def run_serving(count, n_lo, n_hi, slots, setup_workers, log=None):
    """A mixed-size request stream (workloads.serving_requests): a burst run
    (every request at t = 0) gives the saturated throughput; a Poisson stream
    at 0.7 x that rate gives the latency percentiles.  Mixed precision (FP32
    inner PCG, FP64 refinement to rel-res 1e-6), one right-hand side per
    request.  Returns (burst summary, Poisson summary, rate, Poisson results,
    request sizes)."""
    import numpy as np
    from paper_2304_05460_amd import afn, serving, workloads as W

    afn.lib()
    probs = W.serving_requests(count, n_lo=n_lo, n_hi=n_hi)
    data = [W.make(q) for q in probs]

    def reqs(arrivals):
        return [serving.Request(i, X, b, q.l, q.mu, arrival=float(arrivals[i]), k=q.k, w=q.w,
                                k_max=q.k_max, tol=q.tol, maxit=q.maxit, method=afn.AFN_METHOD_AUTO)
                for i, (q, (X, b)) in enumerate(zip(probs, data))]

    def progress(label):
        done = [0]
        lock = __import__("threading").Lock()

        def cb(res):
            with lock:
                done[0] += 1
                if log and (done[0] % 16 == 0 or done[0] == len(probs)):
                    log(f"{label}: {done[0]}/{len(probs)} done")
        return cb

    def server():
        return serving.Server(slots=slots, precision=afn.AFN_FP32, setup_workers=setup_workers)

    # warm-up: one small request (library load, first allocations)
    small = int(np.argmin([q.n for q in probs]))
    server().run([reqs(np.zeros(len(probs)))[small]])
    t0 = time.perf_counter()
    burst = server().run(reqs(np.zeros(len(probs))), on_done=progress("burst"))
    t_burst = time.perf_counter() - t0
    sb = serving.summarize(burst)
    rate = 0.7 * sb["completed"] / t_burst
    if log:
        log(f"burst: {sb}; Poisson run at {rate:.3f} requests/s")
    t0 = time.perf_counter()
    pois = server().run(reqs(W.poisson_arrivals(len(probs), rate, seed=5)), on_done=progress("poisson"))
    t_pois = time.perf_counter() - t0
    sp = serving.summarize(pois)
    sp["wall_s"] = t_pois
    return sb, sp, rate, pois, np.array([q.n for q in probs])


def _fmt(d):
    return {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in d.items()}


def serving_bench(args):
    """The request stream of run_serving at its full size (--serving-count
    requests, sizes --serving-n)."""
    import numpy as np
    from paper_2304_05460_amd import afn

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    n_lo, n_hi = (float(v) for v in args.serving_n.split(","))
    log(f"{args.serving_count} requests; burst run, then Poisson")
    sb, sp, rate, pois, ns = run_serving(args.serving_count, n_lo, n_hi, args.slots, args.setup_workers, log)
    out = {
        "metric": "serving solves/s under a Poisson stream (p50/p99 latency beside it)",
        "value": round(sp["completed"] / sp["wall_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(ns),
        "warmup": 1,
        "ms_per_step": round(sp["wall_s"] / len(ns) * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"serving_{len(ns)}_requests_n{n_lo:.0e}_{n_hi:.0e}_d3_8".replace("+0", ""),
                   "grouped_launches": os.environ.get("AFN_NO_GROUP") != "1",
                   "slots": args.slots, "setup_workers": args.setup_workers,
                   "poisson_rate_per_s": round(rate, 4),
                   "n_median": int(np.median(ns)), "n_max": int(ns.max())},
        "poisson": _fmt(sp),
        "burst": _fmt(sb),
        "statuses": {str(s): int(c) for s, c in
                     zip(*np.unique([r.status for r in pois], return_counts=True))},
        "methods": {["afn", "nystrom"][m]: int(c) for m, c in
                    zip(*np.unique([r.method for r in pois if r.method >= 0], return_counts=True))},
        "fp64_fallbacks": int(sum(1 for r in pois if r.fp64_iterations > 0)),
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--l", type=float, default=0.1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="default (C3) line: skip the short serving leg that reports p50/p99")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision and Algorithm 5 runs on the same input")
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "highd", "batch", "setups"],
                    help="c3 (default): mixed vs FP64 at n=2e5, d=8; c2: FP64 at n=1e5, d=3 "
                         "(--l 0.01 / 0.1 / 1); c4: 64 right-hand sides at n=1.5e5; highd: n=49990, "
                         "d=22 (uniform landmarks); batch: 16 like small solves, grouped against "
                         "ungrouped; setups: the setups of 16 small serving requests")
    ap.add_argument("--c3-branch", default="nystrom", choices=["nystrom", "afn"],
                    help="preconditioner of the c3 solves (Algorithm 5's branches)")
    ap.add_argument("--maxit", type=int, default=0, help="PCG iteration cap (0: the workload's)")
    ap.add_argument("--tune", default="on", choices=["on", "off"],
                    help="autotuner of launch shapes (decisions taken during the warm-up and reported)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="c3: time the mixed-precision solves only (for counter runs; no JSON contract line)")
    ap.add_argument("--serving", action="store_true",
                    help="run the mixed-size request stream instead (p50/p99 latency, solves/s)")
    ap.add_argument("--serving-count", type=int, default=256)
    ap.add_argument("--setup-workers", type=int, default=2,
                    help="serving: host threads running afn_setup for admitted requests")
    ap.add_argument("--serving-n", default="5e3,2e5",
                    help="request sizes: n log-uniform between these two values")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(sharding rows over several GPUs is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_05460_amd import afn as _afn

    _afn.lib()
    _afn.tune_config(_afn.AFN_TUNE_ON if args.tune == "on" else _afn.AFN_TUNE_OFF)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}))
        return

    if args.serving:
        serving_bench(args)
        return
    if args.workload == "c3":
        c3_bench(args)
        return
    if args.workload == "c4":
        c4_bench(args)
        return
    if args.workload == "highd":
        highd_bench(args)
        return
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "setups":
        setups_bench(args)
        return

    c2_bench(args)


def c2_bench(args):
    """n = 1e5 points of a 5-centre mixture in [0,1]^3, adaptive k <= 2000,
    w = 64, FP64 (value), with the mixed path and Algorithm 5's choice on the
    same input beside it."""
    import numpy as np  # noqa: F401
    import torch
    from paper_2304_05460_amd import afn, workloads as W

    p = W.c2(args.l, tol=args.tol)
    X_np, b_np = W.make(p)
    X = torch.tensor(X_np, device="cuda")
    b = torch.tensor(b_np, device="cuda")
    afn.lib()

    def step(precision=afn.AFN_FP64, method=afn.AFN_METHOD_AFN):
        h = afn.afn_setup(X, p.l, p.mu, k=p.k, w=p.w, k_max=p.k_max, precision=precision, method=method,
                          nrhs_max=0)
        x, info = afn.afn_pcg_solve(h, b, tol=p.tol, maxit=p.maxit)
        sinfo = h.info()
        h.close()
        return x, info, sinfo

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def timed(precision, label, method=afn.AFN_METHOD_AFN):
        log(f"{label}: workload {p.name}; warmup {args.warmup} step(s)")
        for _ in range(args.warmup):
            step(precision, method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            x, info, sinfo = step(precision, method)
            infos.append((info, sinfo))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        log(f"{label}: timed {args.steps} step(s) in {elapsed:.3f} s")
        return x, infos, elapsed

    def mixed_block(x64, value, precision=afn.AFN_FP32, label="mixed"):
        x32, infos32, elapsed32 = timed(precision, label)
        i32, s32 = infos32[-1]
        rel = float(torch.linalg.vector_norm(x32 - x64) / torch.linalg.vector_norm(x64))
        return {"value": round(args.steps / elapsed32, 4), "unit": "solves/s",
                "ms_per_step": round(elapsed32 / args.steps * 1e3, 2),
                "speedup_vs_fp64": round((args.steps / elapsed32) / value, 3),
                "inner_iterations": i32["iterations"], "outer_iterations": i32["outer_iterations"],
                "relres_true_fp64": i32["relres_true"], "rel_diff_vs_fp64_solution": rel,
                "setup_ms": round(s32.ms["total"], 2), "solve_ms": round(i32["ms_solve"], 2),
                "kmv_f32_avg_launch_ms": round(i32["ms_matvec"] / max(i32["matvec_launches"], 1), 4)}

    x64, infos, elapsed = timed(afn.AFN_FP64, "fp64")
    ms_per_step = elapsed / args.steps * 1e3
    value = args.steps / elapsed

    info, sinfo = infos[-1]
    launches = sum(i["matvec_launches"] for i, _ in infos)
    kmv_ms = sum(i["ms_matvec"] for i, _ in infos) / max(launches, 1)
    F = kmv_flops(p.n, p.d)
    achieved = F / (kmv_ms * 1e-3) / 1e12
    kern_src = ROOT / "paper_2304_05460_amd" / "csrc" / "kmv.hip"
    ctrs = counters_from_profile(kern_src)
    traffic = ctrs.get("hbm_bytes_per_launch")
    E = p.n * (p.n - 1) / 2
    # the pruned kernel evaluates only the tile pairs whose kernel values can
    # exceed 2^-64, those below 2^-46 with the FP32 exponential; the
    # instruction floor is for the pairs it evaluates
    kept, far = sinfo.kmv_kept_f64, sinfo.kmv_far_f64
    valu_floor_ms = E * ((kept - far) * VALU_F64_OPS_PER_PAIR_D3
                         + far * VALU_F64_OPS_PER_FAR_PAIR_D3) / VALU_F64_LANE_OPS * 1e3
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": traffic, "kernel": "kmv_sym_mf<0, 3, double, double>",
                "avg_launch_ms": round(kmv_ms, 4), "launches": launches,
                "flops_per_launch": F,
                "kernel_evals_per_s": round(E / (kmv_ms * 1e-3), 1),
                "tile_pairs_evaluated": round(kept, 4),
                "tile_pairs_fp32_exp": round(far, 4),
                "valu_instr_floor_ms": round(valu_floor_ms, 4),
                "valu_instr_frac": round(valu_floor_ms / kmv_ms, 4)}
    if "valu_issue_frac" in ctrs:
        # measured by counters on this kernel source: VALU instructions issued
        # per SIMD-cycle against one every 4 cycles, at the measured clock
        roofline["valu_issue_frac_counters"] = ctrs["valu_issue_frac"]
        roofline["clock_ghz_counters"] = ctrs.get("clock_ghz")

    # the same input through the mixed-precision path (FP32 inner PCG inside
    # FP64 iterative refinement)
    mixed = mixed_bf16 = None
    if not args.no_mixed:
        mixed = mixed_block(x64, value)
        mixed_bf16 = mixed_block(x64, value, afn.AFN_BF16, "mixed-bf16")
    # Algorithm 5 on the same input: Nystrom below the rank switch, AFN above
    alg5 = None
    if not args.no_mixed:
        x5, infos5, el5 = timed(afn.AFN_FP64, "alg5", afn.AFN_METHOD_AUTO)
        i5, s5 = infos5[-1]
        alg5 = {"value": round(args.steps / el5, 4), "unit": "solves/s",
                "method": ["afn", "nystrom"][s5.method], "k": s5.k, "iterations": i5["iterations"],
                "relres_true": i5["relres_true"], "setup_ms": round(s5.ms["total"], 2),
                "solve_ms": round(i5["ms_solve"], 2)}

    out = {
        "metric": "AFN-PCG solves/s at rel-res 1e-6 (FP64; mixed precision on the same input beside it)",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "d": p.d, "l": p.l, "mu": p.mu,
                   "k": sinfo.k, "w": p.w, "tol": p.tol, "nrhs": 1},
        "solve": {"iterations": info["iterations"], "relres_true": info["relres_true"],
                  "setup_ms": round(sinfo.ms["total"], 2), "solve_ms": round(info["ms_solve"], 2),
                  "setup_phases_ms": {k: round(v, 2) for k, v in sinfo.ms.items()},
                  "rank": {"r": sinfo.rank_r, "k_est": sinfo.rank_k_est,
                           "eig_branch": sinfo.rank_eig_branch}},
        "mixed": mixed,
        "mixed_bf16": mixed_bf16,
        "alg5": alg5,
        "roofline": roofline,
    }
    out["autotune"] = tune_decisions(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(X_np, b_np, p.l, p.mu, sinfo.k, p.w,
                                           info["iterations"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
