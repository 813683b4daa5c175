#!/usr/bin/env python3
"""Throughput of the NysADMM hot path on one MI355X.

Workload: lasso, A 100000 x 4000 FP32 with singular values j^-0.8 (random
orthogonal factors), x* 2% sparse, b = A x* + 0.01 noise,
gamma = 0.01 ||A^T b||_inf, rho = 1e-4, adaptive Nystrom rank 50 -> 800 with
Tol = 2, subproblem tolerance 1e-6 (relative residual, FP64-accumulated true
residual checked), PCG warm-started at the previous x.

One step = one pass of the whole hot path: the adaptive sketch and its FP64
core (Algorithm AdaptiveRandNysAppx) followed by --admm-iters iterations of
Algorithm NysADMM (right-hand side, Nystrom PCG subproblem solve, soft
threshold, dual update).  value = subproblem solves per second over the timed
steps, the sketch cost included (amortised over the step's solves).

Also reported: the same steps with the BF16-MFMA sketch ("mixed"), the
matvec-pair kernel's achieved HBM bandwidth measured with HIP events around
every launch in the timed region (with the HBM bytes from the committed
rocprofv3 counter record when it was taken on the current kernel source), the
whole-solve roofline fraction, and the FP64 CPU oracle timed on a bounded
sample on this host (cpu_baseline).

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "ADMM subproblem solves/s at 1e-6 rel. residual; GEMV HBM GB/s; vs plain FP32"
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--admm-iters", type=int, default=30)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--d", type=int, default=4000)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--true-res-every", type=int, default=1,
                    help="check the FP64 true residual of every k-th subproblem (and the last "
                         "of a run); the others stop PCG on its recursive residual (the "
                         "headline checks every solve; a 1-in-10 variant is reported beside it)")
    ap.add_argument("--workload",
                    choices=["lasso", "logistic", "path", "learned", "cg", "svm", "sparse",
                             "precision_path", "sketch"],
                    default="lasso",
                    help="lasso: 100000x4000 adaptive rank (default line); logistic: 200000x2000 "
                         "l1-logistic; path: 64 uneven lasso instances x 16 gammas, batched; "
                         "learned: warm-start network trained on 20000 recorded solves, "
                         "100000x4000 at rank 128, arms compared on held-out right-hand sides")
    ap.add_argument("--ranks", type=str, default="50,100,200",
                    help="sketch workload: the fixed ranks, comma-separated")
    ap.add_argument("--precs", type=str, default="fp32,bf16",
                    help="sketch workload: the sketch precisions, comma-separated")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--gammas", type=int, default=16)
    ap.add_argument("--copy-reference", action="store_true",
                    help="also run one 1.6 GB device copy (reference for HBM byte counters)")
    ap.add_argument("--host-data", action="store_true",
                    help="draw the lasso matrix on the host and copy it over (same recipe, "
                         "another random stream; for runs under a counter-collecting profiler)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs of this bench (FETCH_SIZE, then "
                         "WRITE_SIZE, with --copy-reference) into profiles/gram_traffic.json")
    return ap.parse_args()


# lasso weight gamma = LASSO_GAMMA_FRAC * ||A^T b||_inf on the 100000 x 4000
# problem: at this value a 30-iteration step from x = z = u = 0 reaches a
# 437-sparse z with KKT residual ~5e-5 (at 0.1 the optimum has 2-4 nonzeros and
# z stays 0 for the first ~200 iterations)
LASSO_GAMMA_FRAC = 0.01


def traffic_record(n, d):
    """HBM bytes per matvec-pair launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "gram_traffic.json")
    try:
        rec = json.load(open(path))
        if rec.get("kernel_source_sha256") != kernel_source_sha() or rec.get("n") != n or \
                rec.get("d") != d:
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def failed_solves(N, info):
    """Subproblems of an ADMM run that did not reach the PCG tolerance (stopped
    at max_iter), plus one if the run itself ended on another error."""
    return int(info.maxiter_solves) + int(info.status not in (N.NYS_OK, N.NYS_ERR_MAXITER))


def kernel_source_sha():
    csrc = os.path.join(ROOT, "paper_2202_11599_amd", "csrc")
    h = hashlib.sha256()
    for f in ("gemv.hip", "gram_device.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def _pmc_rows(d, counter):
    """(kernel name, counter value) per dispatch from a rocprofv3 --pmc csv run."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"]),
                                 int(r.get("Dispatch_Id", 0))))
    if not rows:
        raise SystemExit(f"no {counter} rows under {d}")
    return rows


def pmc_summary(fetch_dir, write_dir, n, d, commands):
    """HBM bytes per full matvec-pair launch from FETCH_SIZE / WRITE_SIZE (KiB
    per dispatch), each scaled by what the same counter reads for the
    1.6e9-byte device copy of the same run.  Full passes are the dispatches of
    the most frequent k_gram instantiation that read at least half of the
    largest; launches queued past PCG convergence return at once and read
    almost nothing."""
    import statistics
    out = {}
    for key, dd, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _pmc_rows(dd, counter)
        gram = [r for r in rows if "k_gram" in r[0]]
        names = {}
        for r in gram:
            names[r[0]] = names.get(r[0], 0) + 1
        kname = max(names, key=names.get)
        vals = [v for nm, v, _ in gram if nm == kname]
        top = max(vals)
        full = [v for v in vals if v >= 0.5 * top] if key == "fetch" else None
        out[key] = dict(kernel=kname, values=vals, full=full,
                        copy=max(v for nm, v, _ in rows if "k_gram" not in nm))
    # a write-counter dispatch is a full pass when its fetch twin is (same order)
    f, w = out["fetch"], out["write"]
    fvals, wvals = f["values"], w["values"]
    m = min(len(fvals), len(wvals))
    wfull = [wvals[i] for i in range(m) if fvals[i] >= 0.5 * max(fvals)]
    fetch_kib = statistics.mean(f["full"])
    write_kib = statistics.mean(wfull)
    copy_bytes = 1.6e9
    ff = copy_bytes / (f["copy"] * 1024)
    wf = copy_bytes / (w["copy"] * 1024)
    rec = {
        "kernel": f["kernel"],
        "kernel_source_sha256": kernel_source_sha(),
        "kernel_source": ["paper_2202_11599_amd/csrc/gemv.hip",
                          "paper_2202_11599_amd/csrc/gram_device.h"],
        "n": n, "d": d,
        "full_passes": len(f["full"]),
        "fetch_kib_per_dispatch": round(fetch_kib, 1),
        "write_kib_per_dispatch": round(write_kib, 1),
        "copy_reference": {"bytes": int(copy_bytes), "fetch_kib": round(f["copy"], 1),
                           "write_kib": round(w["copy"], 1)},
        "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
        "bytes_per_launch": int(round(fetch_kib * 1024 * ff + write_kib * 1024 * wf)),
        "algorithmic_bytes_per_launch": float(n) * d * 4,
        "commands": commands,
        "note": ("per dispatch: mean over the full passes of the matvec-pair kernel in the bench "
                 "run (launches queued past PCG convergence excluded); factors scale the counters "
                 "so that the 1.6e9-byte device copy of the same run reads 1.6e9 fetched and "
                 "1.6e9 written bytes"),
    }
    return rec


def run_steps(N, ctx, A, prob, omega, p, prec, steps, admm_iters, tr_every, profile=False,
              pcg_timing=False):
    import torch
    if steps <= 0:
        return None
    infos = []
    ranks = []
    step_rates = []
    sketch_s = 0.0
    bad = 0
    tr_max = -1.0
    if profile:
        ctx.profile_start()
    if pcg_timing:
        ctx.profile_pcg_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        F = N.nys_sketch_adaptive(ctx, A, omega, 50, 800, p.rho, 2.0, prec=prec)
        torch.cuda.synchronize()
        sketch_s += time.perf_counter() - ts
        ranks.append(F.info()["rank"])
        # admm_iters NysADMM iterations with the factor just built (no early stop)
        opts = N.admm_opts(p.rho, ranks[-1], omega, sketch_prec=prec, max_iter=admm_iters,
                           pcg=N.pcg_opts(tol=p.pcg_tol, max_iter=1000), factor=F,
                           true_res_every=tr_every)
        st = N.State(p.d, "cuda")
        info = N.admm_solve(ctx, [prob], [opts], [st], allow=(N.NYS_OK, N.NYS_ERR_MAXITER))[0]
        infos.append((info.pcg_iters, info.iters, info.pcg_max, info.eta))
        tr_max = max(tr_max, info.true_res_max)
        bad += failed_solves(N, info)
        F.close()
        torch.cuda.synchronize()
        step_rates.append(info.iters / (time.perf_counter() - ts))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_stop() if profile else None
    pcg = None
    if pcg_timing:
        pcg = ctx.profile_pcg()
        ctx.profile_pcg_enable(False)
    solves = sum(n for _, n, _, _ in infos)
    return dict(wall=wall, sketch_s=sketch_s, ranks=ranks, pcg=pcg,
                pcg_mean=sum(i for i, _, _, _ in infos) / max(solves, 1),
                pcg_max=max(m for _, _, m, _ in infos), solves=solves, unconverged=bad, prof=prof,
                eta=infos[-1][3], true_res_max=tr_max, step_rates=step_rates)


def solve_roofline(run, launches, n, d):
    r = run["ranks"][-1]
    b_it = 4.0 * n * d + 2 * 4.0 * d * r + 12 * 8.0 * d
    passes = launches / max(run["solves"], 1)
    bound = PEAK_HBM_GBS * 1e9 / (passes * b_it)
    meas = run["solves"] / (run["wall"] - run["sketch_s"])
    return {"bytes_per_pcg_iteration": b_it, "pair_passes_per_solve": round(passes, 3),
            "solves_per_s_bound": round(bound, 1), "solves_per_s_excl_sketch": round(meas, 3),
            "frac": round(meas / bound, 4)}


def host_description():
    """Model, sockets, cores and threads of the host (lscpu), and nproc."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                     "CPU(s)", "NUMA node(s)"):
                info[k] = v
    except Exception:
        pass
    return info


def cpu_baseline(A, b, omega, p, admm_iters, cpu_iters):
    """The FP64 oracle as it stands, on this host: its adaptive sketch once and
    `cpu_iters` NysADMM iterations; scaled to the step definition."""
    import numpy as np
    from oracle import nystrom as ny
    from oracle import admm as ad
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    A64 = A.double().cpu().numpy()
    b64 = b.cpu().numpy()
    om = omega.cpu().numpy().T
    t0 = time.perf_counter()
    f, hist = ny.adaptive_rand_nys_appx(A64, None, 0.0, om, p.rho, 50, 800, 2.0)
    t_sketch = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = ad.admm_lasso(A64, b64, p.gamma, p.rho, factor=f, iters=cpu_iters, pcg_tol=p.pcg_tol)
    t_iter = (time.perf_counter() - t0) / cpu_iters
    step = t_sketch + admm_iters * t_iter
    # the oracle's matvec pair A^T (A p) on the FP64 A (two passes over it):
    # its memory rate beside the GPU's
    pv = np.random.default_rng(0).standard_normal((A64.shape[1], 1))
    ny.hessian_apply(A64, None, 0.0, pv)
    t0 = time.perf_counter()
    for _ in range(3):
        ny.hessian_apply(A64, None, 0.0, pv)
    t_pair = (time.perf_counter() - t0) / 3
    pair_bytes = 2.0 * A64.shape[0] * A64.shape[1] * 8
    # the same oracle iteration on one thread (the sketch is not repeated)
    t1 = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            ad.admm_lasso(A64, b64, p.gamma, p.rho, factor=f, iters=1, pcg_tol=p.pcg_tol)
            t1 = time.perf_counter() - t0
    except Exception:
        t1 = None
    return {
        "value": admm_iters / step, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "host": host_description(),
        "gemv_pair": {"ms": round(1e3 * t_pair, 2), "gbs": round(pair_bytes / t_pair / 1e9, 1),
                      "note": "oracle A^T (A p) on the FP64 A, 2 n d 8 bytes per pair"},
        "single_thread": None if t1 is None else {
            "solves_per_s_excl_sketch": round(1.0 / t1, 4), "seconds_per_iteration": round(t1, 3),
            "note": "one NysADMM iteration of the oracle with BLAS limited to one thread"},
        "sample": (f"FP64 NumPy oracle on this host: adaptive sketch (rank {f.rank}, "
                   f"{t_sketch:.1f} s) and {cpu_iters} NysADMM iterations "
                   f"({t_iter:.2f} s each, {np.mean(r.pcg_iters):.1f} PCG iterations) on the same "
                   f"A upcast to FP64; value = {admm_iters} solves / (sketch + {admm_iters} x "
                   f"mean iteration), the GPU step definition"),
    }


def base_record(metric_value, steps, warmup, wall, dtype, config):
    return {
        "metric": METRIC, "value": round(metric_value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(1e3 * wall / max(steps, 1), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": config,
    }


def roofline(prof, alg_bytes, n, d):
    launches, kms = prof
    avg_s = kms / 1e3 / max(launches, 1)
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_record(n, d),
        "kernel": "k_gram (fused A^T D A p, FP32 A, FP64 products and sums)",
        "alg_bytes_per_launch": alg_bytes, "launches": launches,
        "avg_launch_us": round(avg_s * 1e6, 2),
    }


def bench_logistic(args, N, synth, torch):
    """l1 logistic regression 200000 x 2000 FP32: step = 30 linearised NysADMM
    iterations, the factor (rank 200) rebuilt every 10 with the current weights."""
    n, d, its = 200000, 2000, args.admm_iters
    p = synth.logistic_decay(n, d, seed=0, device="cuda", dtype=torch.float32, rho=200.0,
                             rank=200, pcg_tol=1e-6)
    ctx = N.Context()
    A, b, omega = p.A, p.b.contiguous(), p.omega.contiguous()
    prob = N.problem(A, b, p.gamma, loss=N.NYS_LOSS_LOGISTIC)

    def steps(k, profile=False):
        tot, bad, pcg, trm = 0, 0, 0, -1.0
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            # `its` iterations from a cold start, the factor built at the first
            # and rebuilt every 10th with the current weights
            opts = N.admm_opts(p.rho, 200, omega, resketch_every=10, sketch_prec=N.NYS_F32,
                               pcg=N.pcg_opts(tol=1e-6), max_iter=its,
                               true_res_every=args.true_res_every)
            st = N.State(d, "cuda")
            info = N.admm_solve(ctx, [prob], [opts], [st], allow=(N.NYS_OK, N.NYS_ERR_MAXITER))[0]
            tot += info.iters
            pcg += info.pcg_iters
            bad += failed_solves(N, info)
            trm = max(trm, info.true_res_max)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, tot, bad, pcg, trm, (ctx.profile_stop() if profile else None)

    steps(args.warmup)
    wall, tot, bad, pcg, trm, prof = steps(args.steps, profile=True)
    out = base_record(tot / wall, args.steps, args.warmup, wall, "f32", {
        "workload": f"l1-logistic-{n}x{d}-fp32-Sigma_j=1/j-rank200-resketch10",
        "n": n, "d": d, "rho": p.rho, "gamma": p.gamma, "pcg_tol": 1e-6,
        "admm_iters_per_step": its, "true_res_every": args.true_res_every})
    # the pair launches include the logistic right-hand-side passes (same bytes)
    out["roofline"] = roofline(prof, float(n) * d * 4, n, d)
    out["pcg_iters_mean"] = round(pcg / max(tot, 1), 3)
    out["unconverged_solves"] = bad
    out["true_rel_res_max"] = trm
    return out


def bench_cg(args, N, synth, torch):
    """NysADMM against inexact ADMM with plain CG (Table t-ComplexityComparison)
    on the 100000 x 4000 lasso over a path of subproblem tolerances: for each
    tolerance, `its` ADMM iterations from a cold start with each method (NysADMM
    including its adaptive sketch).  value = NysADMM solves/s at 1e-6."""
    its = 10
    p = synth.lasso_decay(args.n, args.d, 0.8, seed=0, device="cuda", dtype=torch.float32,
                          frac=0.02, noise=0.01, gamma_frac=LASSO_GAMMA_FRAC, rho=1e-4, rank=50, s_max=800,
                          pcg_tol=1e-6)
    torch.cuda.synchronize()
    A, b, omega = p.A, p.b.contiguous(), p.omega.contiguous()
    ctx = N.Context()
    prob = N.problem(A, b, p.gamma)

    def run(tol, cg, profile=False):
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = None
        if not cg:
            F = N.nys_sketch_adaptive(ctx, A, omega, 50, 800, p.rho, 2.0, prec=N.NYS_F32)
        rank = 0 if cg else F.info()["rank"]
        o = N.admm_opts(p.rho, rank, None if cg else omega, sketch_prec=N.NYS_F32, max_iter=its,
                        pcg=N.pcg_opts(tol=tol, max_iter=20000), factor=F,
                        true_res_every=args.true_res_every)
        st = N.State(p.d, "cuda")
        info = N.admm_solve(ctx, [prob], [o], [st], allow=(N.NYS_OK, N.NYS_ERR_MAXITER))[0]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if F is not None:
            F.close()
        prof = ctx.profile_stop() if profile else None
        return wall, info, rank, prof

    run(1e-6, False)
    run(1e-2, True)
    rows, value, prof = [], None, None
    for tol in (1e-2, 1e-4, 1e-6, 1e-8):
        wn, inn, rank, _ = run(tol, False)
        wc, inc, _, pr = run(tol, True, profile=(tol == 1e-6))
        prof = pr or prof
        row = {"tol": tol,
               "nysadmm": {"solves_per_s": round(inn.iters / wn, 3),
                           "iters_per_solve": round(inn.pcg_iters / inn.iters, 2),
                           "rank": rank, "eta": inn.eta},
               "cg_admm": {"solves_per_s": round(inc.iters / wc, 3),
                           "iters_per_solve": round(inc.pcg_iters / inc.iters, 2),
                           "eta": inc.eta},
               "speedup": round(wc / wn, 2)}
        rows.append(row)
        print(f"[bench] tol {tol:g}: NysADMM {row['nysadmm']} CG {row['cg_admm']}",
              file=sys.stderr, flush=True)
        if tol == 1e-6:
            value = inn.iters / wn
    out = base_record(value, 1, 1, its / value, "f32", {
        "workload": f"lasso-{args.n}x{args.d}-fp32-sigma_j=j^-0.8-nysadmm-vs-cg-admm-"
                    f"tol-path-{its}iters-cold",
        "n": args.n, "d": args.d, "rho": p.rho, "gamma": p.gamma,
        "admm_iters_per_point": its, "true_res_every": args.true_res_every})
    out["roofline"] = roofline(prof, float(args.n) * args.d * 4, args.n, args.d)
    out["roofline"]["note"] = "pair launches of the CG run at 1e-6"
    out["tol_path"] = rows
    return out


def bench_svm(args, N, synth, torch):
    """Kernel SVM dual (eq. 8) by NysADMM: n = 20000 two-class points in 16
    dimensions, RBF kernel (gamma = 1/16), C = 1, rho = 10, rank 800, PCG tol
    1e-6, stopped at a relative duality gap of 1e-4 (the paper's SVM stop,
    checked every 10 iterations).  H = diag(b) K diag(b) is formed once (FP32,
    1.6 GB, timed apart); a step = the factor built (Y = H Omega with FP32
    products, FP64 core) plus one solve to the gap
    from a cold start.  value = subproblem solves/s over the steps."""
    n, p, r, rho = 20000, 16, 800, 10.0
    X, b = synth.svm_points(n, p, seed=0, sep=1.5, device="cuda")
    ctx = N.Context()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = N.kernel_rbf(ctx, X, 1.0 / p, b)
    torch.cuda.synchronize()
    kernel_s = time.perf_counter() - t0
    omega = synth.omega_raw(n, r, seed=1, device="cuda").contiguous()

    def steps(k, profile=False):
        tot, pcg, bad, trm, sk, last = 0, 0, 0, -1.0, 0.0, None
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            ts = time.perf_counter()
            F = N.nys_sketch_sym(ctx, H, omega, prec=N.NYS_F32)
            torch.cuda.synchronize()
            sk += time.perf_counter() - ts
            o = N.svm_opts(rho, r, pcg=N.pcg_opts(tol=1e-6), max_iter=1000, factor=F,
                           gap_tol=1e-4, gap_every=10, true_res_every=args.true_res_every)
            st = N.State(n, "cuda")
            info = N.svm_solve(ctx, H, b, 1.0, o, st, allow=(N.NYS_OK, N.NYS_ERR_MAXITER))
            tot += info.iters
            pcg += info.pcg_iters
            bad += failed_solves(N, info) + (info.converged != 1)
            trm = max(trm, info.true_res_max)
            last = info
            F.close()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        return wall, tot, pcg, bad, trm, sk, last, (ctx.profile_stop() if profile else None)

    steps(args.warmup)
    wall, tot, pcg, bad, trm, sk, last, prof = steps(args.steps, profile=True)
    out = base_record(tot / wall, args.steps, args.warmup, wall, "f32", {
        "workload": f"kernel-svm-dual-rbf-n{n}-p{p}-C1-rho{rho:g}-rank{r}-to-gap-1e-4",
        "n": n, "p": p, "gamma": 1.0 / p, "C": 1.0, "rho": rho, "rank": r, "pcg_tol": 1e-6,
        "gap_tol": 1e-4, "true_res_every": args.true_res_every, "sketch": "fp32 products, fp64 core"})
    out["roofline"] = roofline(prof, float(n) * n * 4, n, n)
    out["roofline"]["kernel"] = "k_rowdot (y = H p by column blocks, FP32 H, FP64 sums)"
    out["admm_iters_per_solve_to_gap"] = round(tot / args.steps, 1)
    out["time_to_gap_s"] = round(wall / args.steps, 4)
    out["pcg_iters_mean"] = round(pcg / max(tot, 1), 3)
    out["unconverged"] = bad
    out["true_rel_res_max"] = trm
    out["sketch_ms"] = round(1e3 * sk / args.steps, 2)
    out["kernel_matrix_ms"] = round(1e3 * kernel_s, 2)
    out["at_stop"] = {"gap_rel": last.gap_rel, "primal": last.primal, "dual": last.dual,
                      "bias": last.bias}
    # precision path (the experiment that sweeps the target precision from 1 to
    # 1e-3, here to 1e-4): time from a cold start to each relative duality gap,
    # the factor built once and its time added to every point
    torch.cuda.synchronize()
    ts = time.perf_counter()
    F = N.nys_sketch_sym(ctx, H, omega, prec=N.NYS_F32)
    torch.cuda.synchronize()
    sk_s = time.perf_counter() - ts
    path = []
    for tol in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        o = N.svm_opts(rho, r, pcg=N.pcg_opts(tol=1e-6), max_iter=1000, factor=F,
                       gap_tol=tol, gap_every=10, true_res_every=args.true_res_every)
        st = N.State(n, "cuda")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        info = N.svm_solve(ctx, H, b, 1.0, o, st, allow=(N.NYS_OK, N.NYS_ERR_MAXITER))
        torch.cuda.synchronize()
        path.append({"gap_tol": tol, "admm_iters": info.iters, "gap_rel": info.gap_rel,
                     "time_s": round(sk_s + time.perf_counter() - ts, 4),
                     "converged": bool(info.converged)})
    F.close()
    out["precision_path"] = path
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = svm_cpu_baseline(H, b, omega, rho, tot / args.steps, args.cpu_iters)
    return out


def svm_cpu_baseline(H, b, omega, rho, iters_per_solve, cpu_iters):
    """The FP64 SVM oracle on this host: its sketch of the same H (upcast) and
    `cpu_iters` ADMM iterations, scaled to the GPU step (sketch + the GPU's
    iteration count to the gap)."""
    import numpy as np
    from oracle import svm as osvm
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    Hd = H.double().cpu().numpy()
    bd = b.cpu().numpy()
    Kd = Hd * bd[:, None] * bd[None, :]
    om = omega.cpu().numpy().T
    t0 = time.perf_counter()
    f = osvm.nys_factor_of(Hd, om)
    t_sketch = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = osvm.admm_svm(Kd, bd, 1.0, rho, iters=cpu_iters, pcg_tol=1e-6, factor=f)
    t_iter = (time.perf_counter() - t0) / cpu_iters
    step = t_sketch + iters_per_solve * t_iter
    return {
        "value": iters_per_solve / step, "unit": "solves/s", "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 NumPy SVM oracle on this host: sketch of the same H upcast to FP64 "
                   f"(rank {om.shape[1]}, {t_sketch:.1f} s) and {cpu_iters} NysADMM iterations "
                   f"({t_iter:.2f} s each, {np.mean(r.pcg_iters):.1f} PCG iterations); value = "
                   f"{iters_per_solve:.0f} solves / (sketch + {iters_per_solve:.0f} x mean "
                   f"iteration), the GPU step definition"),
    }


def bench_sketch(args, N, synth, torch):
    """The sketch alone on the 100000 x 4000 FP32 lasso matrix: one fixed-rank
    Algorithm RandNysAppx per rank r in {50, 100, 200} and sketch precision
    (FP32 MFMA, BF16 MFMA), each timed over --steps calls after a warm-up
    call (the FP64 core included).  The MFMA kernels' own durations and
    utilisation come from rocprofv3 runs of this workload: T = A Omega and
    Y = A^T T each do 2 n d r flops and read A once (n d 4 bytes), so their
    bound is min(MFMA peak, (r / 2 flop per byte) x 8 TB/s).
    value = sketches/s at r = 200, FP32 (else the first rank and precision run)."""
    n, d = args.n, args.d
    p = synth.lasso_decay(n, d, 0.8, seed=0, device="cpu" if args.host_data else "cuda",
                          dtype=torch.float32, frac=0.02, noise=0.01, gamma_frac=LASSO_GAMMA_FRAC,
                          rho=1e-4, rank=50, s_max=800, pcg_tol=1e-6)
    A, omega = p.A.cuda(), p.omega.cuda().contiguous()
    ctx = N.Context()
    rows = []
    value = None
    ranks = [int(x) for x in args.ranks.split(",")]
    precs = [x for x in args.precs.split(",")]
    for pname in precs:
        prec = {"fp32": N.NYS_F32, "bf16": N.NYS_BF16, "fp64": N.NYS_F64}[pname]
        for r in ranks:
            om = omega[:r].contiguous()
            N.nys_sketch(ctx, A, om, prec=prec).close()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                F = N.nys_sketch(ctx, A, om, prec=prec)
                F.close()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            flops = 4.0 * n * d * r
            rows.append({"prec": pname, "rank": r, "ms_per_sketch": round(ms, 3),
                         "gemm_flops": flops,
                         "mfma_peak_tflops": 157.3 if pname == "fp32" else 2500.0,
                         "hbm_bound_tflops": round(r / 2.0 * 8.0, 1)})
            print(f"[bench] sketch {pname} r={r}: {ms:.2f} ms", file=sys.stderr, flush=True)
            if value is None or (pname == "fp32" and r == 200):
                value = 1e3 / ms
    out = base_record(value, args.steps, 1, 1e3 / value, "f32", {
        "workload": (f"sketch-{n}x{d}-fp32-sigma_j=j^-0.8-fixed-rank-"
                     f"{'-'.join(map(str, ranks))}-{'-'.join(precs)}"),
        "n": n, "d": d})
    out["unit"] = "sketches/s"
    out["metric"] = "Nystrom sketches/s (fixed rank) on the lasso matrix"
    out["sketch"] = rows
    return out


def bench_precision_path(args, N, synth, torch):
    """Lasso precision path on an STL-10-shaped matrix (Section 5, Figure
    precisionpath; Table dataset: 13000 x 27648, dense): time from a cold start
    until the relative KKT residual eq. (31) falls below eps, for eps from 1 to
    1e-3, NysADMM (rank 50, the paper's sketch size, FP32 sketch) against
    inexact ADMM with plain CG, both with the paper's subproblem tolerance
    eps^{k+1} = sqrt(r_p r_d) and gamma = 1.  The data set is not available:
    A = 100 Q1 diag(j^-0.5) Q2^T (Haar factors, FP32), x* 2% sparse,
    b = A x* + N(0, 1) noise; rho = 10.  The matrix is wider than one
    workgroup's row, so every pair takes the two-pass wide form (A read
    twice).  eta is checked every 5 iterations (one more pair each, timed).
    value = NysADMM subproblem solves/s over its run to eps = 1e-2."""
    n, d, r, rho, gamma = 13000, 27648, 50, 10.0, 1.0
    t0 = time.perf_counter()
    a64 = synth.decay_matrix(n, d, 0.5, seed=0, device="cuda")
    A = (100.0 * a64).to(torch.float32).contiguous()
    del a64
    x = synth.sparse_truth(d, 0.02, 0, "cuda")
    b = (A.double() @ x + synth.gaussian((n,), 0, "noise", "cuda")).contiguous()
    omega = synth.omega_raw(d, r, seed=0, device="cuda").contiguous()
    torch.cuda.synchronize()
    print(f"[bench] generated {n}x{d} in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    ctx = N.Context()
    prob = N.problem(A, b, gamma)

    def run(eps, cg, profile=False):
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o = N.admm_opts(rho, 0 if cg else r, None if cg else omega, sketch_prec=N.NYS_F32,
                        pcg=N.pcg_opts(tol=1e-6, max_iter=20000), tol_schedule=True,
                        max_iter=5000, kkt_tol=eps, kkt_every=5,
                        true_res_every=args.true_res_every)
        st = N.State(d, "cuda")
        info = N.admm_solve(ctx, [prob], [o], [st], allow=(N.NYS_OK, N.NYS_ERR_MAXITER))[0]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        prof = ctx.profile_stop() if profile else None
        return wall, info, prof

    run(1e-1, False)
    run(1e-1, True)
    rows, value, prof = [], None, None
    for eps in (1.0, 1e-1, 1e-2, 1e-3):
        wn, inn, pr = run(eps, False, profile=(eps == 1e-2))
        prof = pr or prof
        wc, inc, _ = run(eps, True)
        row = {"eps": eps,
               "nysadmm": {"seconds": round(wn, 4), "admm_iters": inn.iters,
                           "pcg_iters": inn.pcg_iters, "eta": inn.eta,
                           "converged": inn.converged, "unconverged_solves": failed_solves(N, inn)},
               "cg_admm": {"seconds": round(wc, 4), "admm_iters": inc.iters,
                           "pcg_iters": inc.pcg_iters, "eta": inc.eta,
                           "converged": inc.converged, "unconverged_solves": failed_solves(N, inc)},
               "speedup": round(wc / wn, 2)}
        rows.append(row)
        print(f"[bench] eps {eps:g}: NysADMM {row['nysadmm']} CG {row['cg_admm']}",
              file=sys.stderr, flush=True)
        if eps == 1e-2:
            value = inn.iters / wn
    out = base_record(value, 1, 1, 0.0, "f32", {
        "workload": f"lasso-precision-path-stl10-shape-{n}x{d}-fp32-sigma_j=100j^-0.5-"
                    f"gamma=1-rho=10-rank{r}-nysadmm-vs-cg-admm",
        "n": n, "d": d, "rho": rho, "gamma": gamma, "rank": r, "kkt_every": 5,
        "tol_schedule": "sqrt(r_p r_d)"})
    out["ms_per_step"] = None
    out["roofline"] = roofline(prof, 2.0 * n * d * 4, n, d)
    out["roofline"]["kernel"] = ("wide pair: row dots per column block + epilogue + A^T pass "
                                 "(A read twice)")
    out["roofline"]["traffic"] = None
    out["roofline"]["note"] = "pair launches of the NysADMM run to eps = 1e-2; 2 n d 4 bytes each"
    out["precision_path"] = rows
    out["paper_context"] = ("paper, Tables lassolowres/lassohighres, STL-10 on 128 CPU cores: "
                            "NysADMM 165 s at eps 1e-1, 406 s at 1e-2 (real data, not comparable)")
    return out


def copy_reference(torch):
    """A plain 1.6e9-byte device copy (400M floats): the reference a counter
    run scales FETCH_SIZE / WRITE_SIZE by."""
    xs = torch.empty(400_000_000, dtype=torch.float32, device="cuda")
    ys = torch.empty_like(xs)
    ys.copy_(xs)
    torch.cuda.synchronize()
    del xs, ys


def bench_sparse(args, N, synth, torch):
    """Sparse lasso shaped like E2006.train (16087 x 150348, 0.8% nonzero):
    bag-of-words rows with Zipf column popularity, unit-norm rows; gamma =
    0.01 ||A^T b||_inf, rho = 1e-3, rank 50 (FP64 sketch products and core,
    the preconditioner applying an FP32 copy of U), PCG tol 1e-6; a step =
    factor built + `admm_iters` iterations from a cold start."""
    n, d, dens, r, rho, its = 16087, 150348, 0.008, 50, 1e-3, args.admm_iters
    rp, col, val, b, gamma, _ = synth.sparse_lasso(n, d, dens, seed=0, device="cuda")
    torch.cuda.synchronize()
    ctx = N.Context()
    S = N.SparseMatrix(ctx, rp, col, val, (n, d))
    omega = synth.omega_raw(d, r, seed=1, device="cuda").contiguous()
    prob = N.problem(S, b.contiguous(), gamma)
    if args.copy_reference:
        copy_reference(torch)

    def steps(k, profile=False):
        tot, pcg, bad, trm, sk, eta = 0, 0, 0, -1.0, 0.0, None
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            ts = time.perf_counter()
            F = N.nys_sketch(ctx, S, omega, prec=N.NYS_F32)
            torch.cuda.synchronize()
            sk += time.perf_counter() - ts
            o = N.admm_opts(rho, r, omega, sketch_prec=N.NYS_F32, max_iter=its,
                            pcg=N.pcg_opts(tol=1e-6, max_iter=2000), factor=F,
                            true_res_every=args.true_res_every)
            st = N.State(d, "cuda")
            info = N.admm_solve(ctx, [prob], [o], [st], allow=(N.NYS_OK, N.NYS_ERR_MAXITER))[0]
            tot += info.iters
            pcg += info.pcg_iters
            bad += failed_solves(N, info)
            trm = max(trm, info.true_res_max)
            eta = info.eta
            F.close()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        return wall, tot, pcg, bad, trm, sk, eta, (ctx.profile_stop() if profile else None)

    steps(args.warmup)
    wall, tot, pcg, bad, trm, sk, eta, prof = steps(args.steps, profile=True)
    nnz = S.nnz
    out = base_record(tot / wall, args.steps, args.warmup, wall, "f32", {
        "workload": f"sparse-lasso-E2006-shape-{n}x{d}-nnz{nnz}-rank{r}-{its}iters",
        "n": n, "d": d, "nnz": nnz, "rho": rho, "gamma": gamma, "rank": r, "pcg_tol": 1e-6,
        "preconditioner_U": "fp32 copy of the FP64 factor",
        "admm_iters_per_step": its, "true_res_every": args.true_res_every})
    # CSR pass: rowptr, colidx, val, p, s; CSC pass: colptr, rows, values, s, y
    alg = 16.0 * nnz + 4.0 * (n + 1) + 4.0 * (d + 1) + 16.0 * n + 16.0 * d
    out["roofline"] = roofline(prof, alg, n, d)
    out["roofline"]["kernel"] = "k_csr_pass + k_csc_pass (sparse A^T D A p, FP32 values, FP64 sums)"
    out["pcg_iters_mean"] = round(pcg / max(tot, 1), 3)
    out["unconverged_solves"] = bad
    out["true_rel_res_max"] = trm
    out["sketch_ms"] = round(1e3 * sk / args.steps, 2)
    out["kkt_eta_after_step"] = eta
    S.close()
    return out


def bench_path(args, N, synth, torch):
    """Regularisation path: `instances` uneven lasso problems (n in [5000,
    50000], d in [500, 3000], sigma_j = j^-0.7, rank 100, rho 1e-3), each
    solved on a 16-point gamma grid largest first, warm-started, 50 NysADMM
    iterations per gamma, all instances in lockstep (batched admm_solve).
    One step = the whole path with the factors built once."""
    probs = synth.batched_instances(args.instances, seed=0, device="cuda", dtype=torch.float32,
                                    gamma_points=args.gammas)
    torch.cuda.synchronize()
    ctx = N.Context()
    total_bytes = float(sum(p.n * p.d * 4 for p in probs))

    def one_path(profile=False, gammas=None):
        gammas = gammas or args.gammas
        if profile:
            ctx.profile_start()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fs = [N.nys_sketch(ctx, p.A, p.omega, prec=N.NYS_F32) for p in probs]
        states = [N.State(p.d, "cuda") for p in probs]
        solves, pcg, bad, trm = 0, 0, 0, -1.0
        for g in range(gammas):
            P = [N.problem(p.A, p.b, p.meta["gammas"][g]) for p in probs]
            O = [N.admm_opts(p.rho, 100, p.omega, max_iter=50, factor=Fs[k], sketch_prec=N.NYS_F32,
                             pcg=N.pcg_opts(tol=1e-6), true_res_every=args.true_res_every)
                 for k, p in enumerate(probs)]
            infos = N.admm_solve(ctx, P, O, states)
            trm = max([trm] + [i.true_res_max for i in infos])
            solves += sum(i.iters for i in infos)
            pcg += sum(i.pcg_iters for i in infos)
            bad += sum(failed_solves(N, i) for i in infos)
        for F in Fs:
            F.close()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, solves, pcg, bad, trm, (ctx.profile_stop() if profile else None)

    one_path(gammas=1)
    wall, solves, pcg, bad, trm, prof = one_path(profile=True)
    out = base_record(solves / wall, 1, 1, wall, "f32", {
        "workload": f"lasso-path-{len(probs)}-instances-n5000..50000-d500..3000-fp32-"
                    f"sigma_j=j^-0.7-rank100-{args.gammas}gammas-50iters",
        "instances": len(probs), "gammas": args.gammas, "rho": 1e-3, "pcg_tol": 1e-6,
        "total_A_bytes": total_bytes, "true_res_every": args.true_res_every})
    out["pcg_iters_mean"] = round(pcg / max(solves, 1), 3)
    out["unconverged_solves"] = bad
    out["true_rel_res_max"] = trm
    # the timed passes are the true-residual passes of every ADMM step, outside
    # the captured PCG graphs: one batched pair launch per row-width bucket
    # over all instances (all stay active through the fixed 50 iterations)
    out["roofline"] = roofline(prof, total_bytes, None, None)
    out["roofline"]["kernel"] = ("k_bgram (batched fused pair, one launch per row-width bucket; "
                                 "timed over the true-residual passes)")
    out["roofline"]["traffic"] = None
    out["roofline"]["alg_bytes_per_launch_note"] = "sum over instances of n_i d_i 4 bytes"
    return out


def bench_learned(args, N, synth, torch):
    """Learned warm start on the 100000 x 4000 generator at rank 128: record
    20000 subproblem solves (200 right-hand sides x 4 (gamma, rho) pairs x 25
    ADMM steps), train the 130-256-256-128 network on the GPU, then solve
    held-out right-hand sides (20 x 2 pairs) with each start rule at
    tolerance 1e-6."""
    from paper_2202_11599_amd import warmstart as W
    n, d, r, its = 100000, 4000, 128, 25
    t0 = time.perf_counter()
    p = synth.lasso_decay(n, d, 0.8, seed=0, device="cuda", dtype=torch.float32, rank=r, s_max=r)
    A, omega = p.A, p.omega.contiguous()
    ctx = N.Context()
    F = N.nys_sketch(ctx, A, omega, prec=N.NYS_F32)
    lam = F.info()["lam"]
    train = synth.warmstart_draws(A, 200, 4, seed=1)
    test = synth.warmstart_draws(A, 20, 2, seed=2)
    torch.cuda.synchronize()
    print(f"[bench] learned: data in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    parts = []
    for k in range(0, len(train), 100):
        parts.append(W.record(ctx, A, F, omega, train[k:k + 100], its))
        print(f"[bench] learned: recorded {(k + 100) * its} solves, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    X = torch.cat([q[0] for q in parts])
    T = torch.cat([q[1] for q in parts])
    del parts
    rec_s = time.perf_counter() - t0
    Xt, Tt = W.record(ctx, A, F, omega, test, its)
    print(f"[bench] learned: recorded {X.shape[0]} solves in {rec_s:.1f} s", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    model, hist = W.fit(ctx, X, T, lam, hidden=256, steps=3000, batch=256, lr=1e-3, seed=3,
                        log_every=500)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    print(f"[bench] learned: trained in {train_s:.1f} s, loss {hist[0][1]:.3e} -> "
          f"{hist[-1][1]:.3e}", file=sys.stderr, flush=True)
    errs = {"analytic": W.energy_error(W.analytic(Xt, lam), Xt, Tt, lam),
            "network": W.energy_error(W.proposals(model, Xt, lam), Xt, Tt, lam),
            "network_train": W.energy_error(W.proposals(model, X, lam), X, T, lam)}
    idx0 = torch.arange(0, Xt.shape[0], its, device=Xt.device)   # first step of each run
    X0, T0 = Xt[idx0].contiguous(), Tt[idx0].contiguous()
    errs["network_cold"] = W.energy_error(W.proposals(model, X0, lam), X0, T0, lam)
    errs["analytic_cold"] = W.energy_error(W.analytic(X0, lam), X0, T0, lam)
    W.run_arm(ctx, A, F, omega, test[:2], its, "mlp", model=model)   # warm the paths
    arms = {}
    for arm in ("prev", "mlp", "analytic", "mlp_every_step"):
        tot, _ = W.run_arm(ctx, A, F, omega, test, its, arm.replace("_every_step", ""),
                           model=model, every_step=arm.endswith("every_step"))
        arms[arm] = {"solves_per_s": round(tot["solves"] / tot["seconds"], 3),
                     "pcg_iters_mean": round(tot["pcg_iters"] / tot["solves"], 3),
                     "cold_start_pcg_iters_mean": round(tot["first_iters"] / len(test), 3),
                     "candidate_used": tot["ws_used"], "solves": tot["solves"]}
        print(f"[bench] learned arm {arm}: {arms[arm]}", file=sys.stderr, flush=True)
    wall = sum(a["solves"] / a["solves_per_s"] for a in arms.values() if a["solves_per_s"] > 0)
    out = base_record(arms["mlp"]["solves_per_s"], 1, 1, wall, "f32", {
        "workload": "lasso-100000x4000-fp32-sigma_j=j^-0.8-rank128-learned-warm-start",
        "n": n, "d": d, "rank": r, "pcg_tol": 1e-6, "train_solves": int(X.shape[0]),
        "test_solves_per_arm": len(test) * its, "network": "130-256-256-128 GELU, analytic skip"})
    out["arms"] = arms
    out["mlp_vs_prev"] = round(arms["mlp"]["solves_per_s"] / arms["prev"]["solves_per_s"], 4)
    out["heldout_energy_error"] = {k: float(f"{v:.4e}") for k, v in errs.items()}
    out["record_s"] = round(rec_s, 2)
    out["train_s"] = round(train_s, 2)
    out["loss_first_last"] = [hist[0][1], hist[-1][1]]
    model.close()
    F.close()
    return out


def main():
    args = parse()
    if args.pmc_summary:
        # R = the repository root
        cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 400 rocprofv3 --pmc {c} "
               "--kernel-include-regex 'k_gram|elementwise|copy' -d $R/{d} -o run "
               "--output-format csv -- python $R/bench.py --steps 1 --warmup 0 --admm-iters 5 "
               "--no-mixed --no-cpu-baseline --copy-reference --host-data")
        rec = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.n, args.d,
                          [cmd.format(c="FETCH_SIZE", d="gpurun_out/pmc_fetch"),
                           cmd.format(c="WRITE_SIZE", d="gpurun_out/pmc_write"),
                           "cd $R && python bench.py --pmc-summary gpurun_out/pmc_fetch "
                           "gpurun_out/pmc_write"])
        path = os.path.join(ROOT, "profiles", "gram_traffic.json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=2)
            fh.write("\n")
        print(json.dumps(rec, indent=2))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, ROOT)
    import torch
    if args.workload != "lasso":
        from paper_2202_11599_amd import nysadmm as N
        from paper_2202_11599_amd import synth
        torch.cuda.set_device(0)
        fn = {"logistic": bench_logistic, "path": bench_path,
              "learned": bench_learned, "cg": bench_cg, "svm": bench_svm,
              "sparse": bench_sparse, "precision_path": bench_precision_path,
              "sketch": bench_sketch}[args.workload]
        print(json.dumps(fn(args, N, synth, torch)), flush=True)
        return
    from paper_2202_11599_amd import nysadmm as N
    from paper_2202_11599_amd import synth

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    p = synth.lasso_decay(args.n, args.d, 0.8, seed=0, device="cpu" if args.host_data else "cuda",
                          dtype=torch.float32, frac=0.02, noise=0.01, gamma_frac=LASSO_GAMMA_FRAC,
                          rho=1e-4, rank=50, s_max=800, pcg_tol=1e-6)
    if args.host_data:
        p.A, p.b, p.omega = p.A.cuda(), p.b.cuda(), p.omega.cuda()
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {args.n}x{args.d} in {gen_s:.1f} s", file=sys.stderr, flush=True)
    A, b = p.A, p.b.contiguous()
    ctx = N.Context()
    # the adaptive sketch's d x 800 Gaussian test matrix, drawn by the library
    # on the device (Philox4x32-10 + Box-Muller, seed 1)
    omega = N.gaussian_omega(ctx, args.d, 800, seed=1)
    prob = N.problem(A, b, p.gamma)
    if args.copy_reference:
        copy_reference(torch)

    tre = args.true_res_every
    run_steps(N, ctx, A, prob, omega, p, N.NYS_F32, args.warmup, args.admm_iters, tre)
    print("[bench] warmup done", file=sys.stderr, flush=True)
    plain = run_steps(N, ctx, A, prob, omega, p, N.NYS_F32, args.steps, args.admm_iters, tre,
                      profile=True)
    print(f"[bench] plain fp32: {plain['solves'] / plain['wall']:.1f} solves/s", file=sys.stderr,
          flush=True)
    # rate (i), PCG alone: the same steps again with HIP events around each
    # subproblem's PCG solve (kept out of the headline run)
    pcgrun = run_steps(N, ctx, A, prob, omega, p, N.NYS_F32, args.steps, args.admm_iters, tre,
                       pcg_timing=True)
    # the same steps with the FP64 true residual formed at every 10th solve only
    # (the others stop on the recursive residual and carry H_rho x = rhs - w)
    carried = run_steps(N, ctx, A, prob, omega, p, N.NYS_F32, args.steps, args.admm_iters, 10)
    print(f"[bench] true residual every 10th solve: "
          f"{carried['solves'] / carried['wall']:.1f} solves/s", file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        run_steps(N, ctx, A, prob, omega, p, N.NYS_BF16, 1, args.admm_iters, tre)
        mixed = run_steps(N, ctx, A, prob, omega, p, N.NYS_BF16, args.steps, args.admm_iters, tre)
        print(f"[bench] mixed bf16: {mixed['solves'] / mixed['wall']:.1f} solves/s",
              file=sys.stderr, flush=True)

    launches, kms = plain["prof"]
    avg_s = kms / 1e3 / max(launches, 1)
    alg_bytes = float(args.n) * args.d * 4
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = traffic_record(args.n, args.d)
    value = plain["solves"] / plain["wall"]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * plain["wall"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"lasso-{args.n}x{args.d}-fp32-sigma_j=j^-0.8-adaptive-rank-50..800-"
                        f"gamma={LASSO_GAMMA_FRAC}||A^Tb||inf",
            "n": args.n, "d": args.d, "rho": p.rho, "gamma": p.gamma, "pcg_tol": p.pcg_tol,
            "admm_iters_per_step": args.admm_iters, "ada_tol": 2.0,
            "rank_final": plain["ranks"][-1], "true_res_every": tre,
            "test_matrix": "nys_gaussian seed 1 (device Philox4x32-10, Box-Muller)",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "k_gram (fused A^T D A p, FP32 A, FP64 products and sums)",
            "alg_bytes_per_launch": alg_bytes, "launches": launches,
            "avg_launch_us": round(avg_s * 1e6, 2),
        },
        "plain_fp32": {
            "solves_per_s": round(value, 3),
            "solves_per_s_excl_sketch": round(plain["solves"] / (plain["wall"] - plain["sketch_s"]), 3),
            "sketch_ms": round(1e3 * plain["sketch_s"] / args.steps, 2),
            "pcg_iters_mean": round(plain["pcg_mean"], 3), "pcg_iters_max": plain["pcg_max"],
            "unconverged_solves": plain["unconverged"], "kkt_eta_after_step": plain["eta"],
            "true_rel_res_max": plain["true_res_max"],
            "per_step_solves_per_s": {"min": round(min(plain["step_rates"]), 3),
                                      "max": round(max(plain["step_rates"]), 3)},
        },
        # whole-solve roofline (sketch excluded): per PCG iteration the method
        # must move A once (fused pair), U twice (FP32) and about 12 FP64
        # d-vectors; the pair passes per solve are those the event timing saw
        "solve_roofline": solve_roofline(plain, launches, args.n, args.d),
        # rate (i): the subproblems' PCG solves alone (right-hand sides, prox
        # and dual updates, and the sketch excluded)
        "pcg_only": {"solves": pcgrun["pcg"][0], "pcg_ms_total": round(pcgrun["pcg"][1], 3),
                     "solves_per_s": round(pcgrun["pcg"][0] / (pcgrun["pcg"][1] / 1e3), 3)
                     if pcgrun["pcg"][1] > 0 else None,
                     "note": "same steps, separate run, events around every PCG solve"},
        "gemv_hbm_gbs": round(achieved, 1),
        "true_residual_every_10th_solve": {
            "solves_per_s": round(carried["solves"] / carried["wall"], 3),
            "pcg_iters_mean": round(carried["pcg_mean"], 3),
            "unconverged_solves": carried["unconverged"],
            "true_rel_res_max": carried["true_res_max"],
        },
    }
    if mixed is not None:
        out["mixed_bf16_sketch"] = {
            "solves_per_s": round(mixed["solves"] / mixed["wall"], 3),
            "solves_per_s_excl_sketch": round(mixed["solves"] / (mixed["wall"] - mixed["sketch_s"]), 3),
            "sketch_ms": round(1e3 * mixed["sketch_s"] / args.steps, 2),
            "pcg_iters_mean": round(mixed["pcg_mean"], 3), "rank_final": mixed["ranks"][-1],
            "unconverged_solves": mixed["unconverged"], "kkt_eta_after_step": mixed["eta"],
            "true_rel_res_max": mixed["true_res_max"],
            "vs_plain_fp32": round((mixed["solves"] / mixed["wall"]) / value, 4),
        }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A, b, omega, p, args.admm_iters, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
