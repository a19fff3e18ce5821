#!/usr/bin/env python3
"""Benchmark: interpolated (piCholesky) vs exact per-lambda Cholesky k-fold
cross-validation on one MI355X, FP64.

One step is one pass of the whole path over the benchmark workload (random
Fourier features, n=60000, d=4096, c=10, k=5, g=6, r=2, q=64, lambda range
[1e-6, 1] * trace(X^T X / n)/d):
    fold Gram matrices -> piCholesky CV (g sample factorizations per fold,
    fit, fused evaluation + solves at q values, hold-out errors)
    -> exact CV (q factorizations per fold, solves, hold-out errors).
The headline value is interpolated lambda-solves per second, k*q / (time of
the piCholesky stage), with the Gram matrices resident (they are shared by
both methods and timed separately).  A lambda-solve is one (fold, lambda)
pair: its c-column ridge solution and its hold-out error.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("interpolated λ-solves/sec vs exact per-λ Cholesky CV "
          "(d=4096,k=5,q=64); err gap")
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0
NB = 128


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def update_flops(d: int, nfac: int) -> float:
    """Algorithmic flops of all trailing updates of a blocked factorization
    of nfac matrices of order d: after each 128-wide panel the remaining
    m x m lower triangle receives a rank-128 update, 128 * m * (m + 1) flops
    (m = d - 128 (kk + 1)).  However the updates are grouped into launches,
    their total is this sum."""
    nt = (d + NB - 1) // NB
    tot = 0.0
    for kk in range(nt - 1):
        m = max(0, d - (kk + 1) * NB)
        tot += float(nfac) * NB * m * (m + 1)
    return tot


def measured_traffic(stage: str, lookahead: int, group: int):
    """HBM bytes per launch of k_potrf_update in one stage ("interp" or
    "exact") from the committed rocprofv3 counter record
    (profiles/k_potrf_update_traffic.json), or None when the kernel's sources
    changed since the counters were taken or this run's launch mix
    (look-ahead, panel group) differs from the profiled one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_potrf_update_traffic.json")
    if not os.path.exists(path) or lookahead != 0:
        return None
    rec = json.load(open(path))
    st = rec.get("stages", {}).get(stage)
    if st is None or rec.get("panel_group") != group:
        return None
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return st["read_bytes_per_launch"] + st["write_bytes_per_launch"]


def gaps(cp, ce, lam):
    tp = int(np.argmin(np.where(np.isfinite(cp), cp, np.inf)))
    te = int(np.argmin(np.where(np.isfinite(ce), ce, np.inf)))
    return {
        "curve_gap_max_rel": float(np.max(np.abs(cp - ce) / np.abs(ce))),
        "min_err_interp": float(cp.min()), "min_err_exact": float(ce.min()),
        "min_gap_rel": float((cp.min() - ce.min()) / ce.min()),
        "regret": float(ce[tp] - ce.min()),
        "sel_lambda_interp": float(lam[tp]), "sel_lambda_exact": float(lam[te]),
        "sel_err_log10": float(abs(np.log10(lam[tp] / lam[te]))),
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, gpu_err_fold0, gpu_err_exact_fold0=None):
    """CPU baselines on bounded samples of the workload's fold 0, from its
    Gram matrices (formed with numpy outside the timed regions):
      value      the oracle's interpolated fold (g sample factorizations,
                 fit, q evaluations + solves + hold-out errors) on all the
                 oracle's threads;
      one_thread the same fold's rate on one thread, extrapolated from parts
                 timed on one thread (one factorization, one fit, two units);
      exact      the oracle's exact method at 8 of the q grid values, on all
                 threads, extrapolated to the whole job;
      lapack     numpy/LAPACK (multi-threaded BLAS) running both methods on
                 fold 0, the analogue of a multi-threaded CPU library setting."""
    import oracle
    nv = len(np.array_split(np.arange(prob.n), prob.k)[0])
    Xv, Yv = prob.X[:nv], prob.Y[:nv]
    Xt, Yt = prob.X[nv:], prob.Y[nv:]
    log("cpu baseline: forming fold-0 Gram matrices with numpy (untimed)")
    H = Xt.T @ Xt / Xt.shape[0]
    Bm = Xt.T @ Yt / Xt.shape[0]
    oracle.build()
    nthr = oracle.num_threads()
    k, q, g, r, d = prob.k, prob.q, prob.g, prob.r, prob.d
    log(f"cpu baseline: oracle fold 0 on {nthr} threads")
    t0 = time.perf_counter()
    out = oracle.fold_interp(H, Bm, Xv, Yv, prob.lam_s, prob.lam_grid, r)
    dt = time.perf_counter() - t0
    rel = np.abs(np.asarray(gpu_err_fold0) - out["mse"]) / np.abs(out["mse"])
    log(f"cpu baseline: {dt:.1f} s, max rel diff vs GPU fold-0 errors {rel.max():.2e}")

    # one thread: the fold's parts, each timed once
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        L0, _ = oracle.cholesky(H, float(prob.lam_s[-1]))
        t_chol = time.perf_counter() - t0
        T = np.tile(oracle.pack_lower(L0), (g, 1))
        t0 = time.perf_counter()
        Th = oracle.fit(T, prob.lam_s, r, prob.lam_ref)
        t_fit = time.perf_counter() - t0
        del T
        t0 = time.perf_counter()
        for lam in prob.lam_grid[[0, q - 1]]:
            Lh = oracle.unpack_lower(oracle.evaluate(Th, float(lam), prob.lam_ref), d)
            W, _ = oracle.solve(Lh, Bm)
            oracle.holdout_sse(Xv, Yv, W)
        t_unit = (time.perf_counter() - t0) / 2
    finally:
        oracle.set_num_threads(nthr)
    t_one = g * t_chol + t_fit + q * t_unit
    log(f"cpu baseline, 1 thread: factorization {t_chol:.1f} s, fit {t_fit:.1f} s, "
        f"unit {t_unit:.2f} s -> fold {t_one:.0f} s (extrapolated)")

    # the exact method at 8 grid values
    idx = np.linspace(0, q - 1, 8).round().astype(int)
    t0 = time.perf_counter()
    ex = oracle.fold_exact(H, Bm, Xv, Yv, prob.lam_grid[idx])
    t_ex = time.perf_counter() - t0
    exact = {"value": len(idx) / t_ex, "unit": "λ-solves/s", "cores": nthr,
             "kind": "oracle", "seconds": t_ex,
             "sample": f"fold 0, exact factorization + solves + hold-out at {len(idx)} "
                       f"of the {q} grid values (indices {idx.tolist()})",
             "whole_job_seconds_extrapolated": k * q * t_ex / len(idx)}
    if gpu_err_exact_fold0 is not None:
        exact["max_rel_diff_vs_gpu"] = float(np.max(
            np.abs(np.asarray(gpu_err_exact_fold0)[idx] - ex["mse"]) / ex["mse"]))
    log(f"cpu baseline, exact oracle: {len(idx)} grid values in {t_ex:.1f} s")

    return {
        "value": q / dt, "unit": "λ-solves/s",
        "cores": nthr, "kind": "oracle",
        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
        "sample": (f"fold 0 of {k} at n={prob.n}, d={d}, c={prob.c}: "
                   f"g={g} sample factorizations, fit, q={q} "
                   "evaluations + solves + hold-out errors, from numpy-formed "
                   "Gram matrices"),
        "seconds": dt,
        "whole_job_seconds_extrapolated": k * dt,
        "fold0_err_max_rel_diff_vs_gpu": float(rel.max()),
        "one_thread": {
            "value": q / t_one, "unit": "λ-solves/s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": "fold 0 on one thread from parts timed once: one sample "
                      "factorization, one fit of g packed factors, two "
                      "evaluate + solve + hold-out units; g*fact + fit + q*unit",
            "factorization_s": t_chol, "fit_s": t_fit, "unit_s": t_unit,
        },
        "exact": exact,
        "lapack": lapack_baseline(prob, H, Bm, Xv, Yv),
        "conditioning": conditioning(prob, H, float(rel.max())),
    }


def conditioning(prob, H, achieved):
    """The conditioning behind the parity bar at full size (untimed):
    kappa(H_0 + lambda I) of fold 0 from its eigenvalues at the grid's ends
    and the samples' ends, and cond(V) of the fit's basis in tau =
    lambda/lam_ref (the library's and the oracle's) and in raw lambda,
    beside the relative difference between the GPU's and the oracle's
    fold-0 hold-out errors.  Two backward-stable FP64 solvers agree to
    about kappa * eps * (a low power of d)."""
    ev = np.linalg.eigvalsh(H)
    eps = float(np.finfo(np.float64).eps)

    def kappa(lam):
        return float((ev[-1] + lam) / (ev[0] + lam))

    r = prob.r
    tau = prob.lam_s / prob.lam_ref
    out = {
        "eig_min": float(ev[0]), "eig_max": float(ev[-1]),
        "kappa_at_lambda_min": kappa(float(prob.lam_grid.min())),
        "kappa_at_lambda_max": kappa(float(prob.lam_grid.max())),
        "kappa_at_sample_min": kappa(float(prob.lam_s.min())),
        "cond_V_tau": float(np.linalg.cond(np.vander(tau, r + 1, increasing=True))),
        "cond_V_raw_lambda": float(np.linalg.cond(
            np.vander(prob.lam_s, r + 1, increasing=True))),
        "fold0_err_max_rel_diff_vs_oracle": achieved,
    }
    out["kappa_eps_at_lambda_min"] = out["kappa_at_lambda_min"] * eps
    log(f"conditioning: kappa(H_0 + lambda_min I) = {out['kappa_at_lambda_min']:.3g}, "
        f"cond(V) = {out['cond_V_tau']:.3g} in tau, "
        f"{out['cond_V_raw_lambda']:.3g} in raw lambda; achieved {achieved:.2e}")
    return out


def lapack_baseline(prob, H, Bm, Xv, Yv):
    """Both methods on fold 0 with numpy/scipy LAPACK and the host's
    multi-threaded BLAS (not the oracle): exact Cholesky at 8 grid values,
    and piCholesky (6 factorizations, least-squares fit by one product with
    the pseudo-inverse, evaluation, solves and residuals at all q values)."""
    import scipy.linalg
    k, q, g, r, d = prob.k, prob.q, prob.g, prob.r, prob.d
    I = np.eye(d)

    def unit(L):
        z = scipy.linalg.solve_triangular(L, Bm, lower=True, check_finite=False)
        w = scipy.linalg.solve_triangular(L, z, lower=True, trans="T",
                                          check_finite=False)
        res = Yv - Xv @ w
        return float(np.sum(res * res)) / Yv.size

    idx = np.linspace(0, q - 1, 8).round().astype(int)
    t0 = time.perf_counter()
    for lam in prob.lam_grid[idx]:
        unit(np.linalg.cholesky(H + lam * I))
    t_ex = time.perf_counter() - t0
    t0 = time.perf_counter()
    tri = np.tril_indices(d)
    T = np.stack([np.linalg.cholesky(H + lam * I)[tri] for lam in prob.lam_s])
    V = np.vander(prob.lam_s / prob.lam_ref, r + 1, increasing=True)
    Th = np.linalg.pinv(V) @ T
    del T
    mse = []
    L = np.zeros((d, d))
    for lam in prob.lam_grid:
        L[tri] = np.vander([lam / prob.lam_ref], r + 1, increasing=True)[0] @ Th
        mse.append(unit(L))
    t_int = time.perf_counter() - t0
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = ", ".join(sorted({f"{i.get('internal_api')} {i.get('num_threads')} threads"
                                 for i in info if i.get("user_api") == "blas"}))
    except Exception:
        blas = "unknown"
    log(f"lapack baseline: exact {len(idx)} values {t_ex:.1f} s, "
        f"interpolated fold {t_int:.1f} s ({blas})")
    return {
        "kind": "numpy/LAPACK", "blas": blas,
        "interp": {"value": q / t_int, "unit": "λ-solves/s", "seconds": t_int,
                   "sample": f"fold 0, all {q} grid values"},
        "exact": {"value": len(idx) / t_ex, "unit": "λ-solves/s", "seconds": t_ex,
                  "sample": f"fold 0, {len(idx)} of the {q} grid values"},
    }


def variant_leg(args, B, p, ws, nbytes, prob, ei64, ee64, stream, precision,
                refine, W64, basis=0):
    """Time the piCholesky (and exact) stages with another precision and/or
    refinement count on the resident Gram matrices, and compare the hold-out
    errors with the FP64 run of the same step (FP64 interpolated and FP64
    exact)."""
    import torch
    k, q, g = prob.k, prob.q, prob.g
    pm = B.make_problem(p.n, p.d, p.c, k, g, p.r, q, True, precision=precision,
                        refine=refine, basis=basis)
    dev = torch.device("cuda:0")
    err_i = torch.empty(k * q, dtype=torch.float64, device=dev)
    err_e = torch.empty(k * q, dtype=torch.float64, device=dev)
    info_i = torch.empty(k * g, dtype=torch.int32, device=dev)
    info_e = torch.empty(k * q, dtype=torch.int32, device=dev)
    flags_i = torch.empty(k * q, dtype=torch.int32, device=dev)
    flags_e = torch.empty(k * q, dtype=torch.int32, device=dev)
    exact = ee64 is not None

    def run(ev):
        ev[0].record(stream)
        B.pichol_cv_interp(pm, prob.lam_s, prob.lam_grid, prob.lam_ref, ws, nbytes,
                           err_i, None, info_i, flags_i)
        ev[1].record(stream)
        if exact:
            B.pichol_cv_exact(pm, prob.lam_grid, ws, nbytes, err_e, None, info_e,
                              flags_e)
        ev[2].record(stream)

    name = (("mixed" if precision else "fp64") + f", refine={refine}"
            + (", log-lambda basis" if basis else ""))
    log(f"leg {name}")
    for _ in range(args.warmup):
        run([torch.cuda.Event(enable_timing=True) for _ in range(3)])
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
           for _ in range(args.steps)]
    for e in evs:
        run(e)
    torch.cuda.synchronize()
    t_int = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_ex = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ei = err_i.cpu().numpy().reshape(k, q)
    # relative weight error against the FP64 runs (one more, untimed call)
    Wv = torch.empty_like(W64["interp"])
    B.pichol_cv_interp(pm, prob.lam_s, prob.lam_grid, prob.lam_ref, ws, nbytes,
                       err_i, Wv, info_i, flags_i)
    wscale_i = float(W64["interp"].abs().max())
    w_rel_i = float((Wv - W64["interp"]).abs().max()) / wscale_i
    w_rel_ie = None
    w_rel_e = None
    if exact:
        wscale_e = float(W64["exact"].abs().max())
        w_rel_ie = float((Wv - W64["exact"]).abs().max()) / wscale_e
        B.pichol_cv_exact(pm, prob.lam_grid, ws, nbytes, err_e, Wv, info_e, flags_e)
        w_rel_e = float((Wv - W64["exact"]).abs().max()) / wscale_e
    del Wv
    out = {
        "precision": ("FP32-MFMA trailing updates, FP64 elsewhere" if precision
                      else "FP64"),
        "refine": refine, "basis": "log(lambda/lam_ref)" if basis else "lambda/lam_ref",
        "interp_ms": t_int, "value": k * q / (t_int * 1e-3),
        "interp_ok": bool((info_i.cpu().numpy() == 0).all()
                          and (flags_i.cpu().numpy() == 0).all()),
        "interp_max_rel_err_vs_fp64_interp": float(np.max(np.abs(ei - ei64) / ei64)),
        "interp_weight_rel_err_vs_fp64_interp": w_rel_i,
    }
    msg = (f"{name}: interp {t_int:.2f} ms -> {out['value']:.1f} lambda-solves/s, "
           f"max rel diff vs FP64 interp {out['interp_max_rel_err_vs_fp64_interp']:.2e}")
    if exact:
        ee = err_e.cpu().numpy().reshape(k, q)
        out.update({
            "interp_max_rel_err_vs_fp64_exact": float(np.max(np.abs(ei - ee64) / ee64)),
            "exact_ms": t_ex, "exact_value": k * q / (t_ex * 1e-3),
            "exact_ok": bool((info_e.cpu().numpy() == 0).all()
                             and (flags_e.cpu().numpy() == 0).all()),
            "exact_max_rel_err_vs_fp64_exact": float(np.max(np.abs(ee - ee64) / ee64)),
            "interp_weight_rel_err_vs_fp64_exact": w_rel_ie,
            "exact_weight_rel_err_vs_fp64_exact": w_rel_e,
            "interp_speedup_vs_fp64_exact": None,
            "err_gap_vs_fp64_exact": gaps(ei.mean(0), ee64.mean(0), prob.lam_grid),
        })
        msg += (f"; vs FP64 exact {out['interp_max_rel_err_vs_fp64_exact']:.2e}; "
                f"exact {t_ex:.2f} ms, max rel diff vs FP64 exact "
                f"{out['exact_max_rel_err_vs_fp64_exact']:.2e}")
    log(msg)
    return out


def batching_leg(args, B, stream):
    """The many-problem workload (48 ridge problems of uneven d, k=5, g=5,
    r=2, q=32, FP64): every problem, fold and lambda through pichol_cv_batch
    (Gram included), eager and as one replayed HIP graph with an autotuned
    schedule, against the same problems run one after another through the
    single-problem pipeline, and against the batched exact method."""
    import torch
    import workloads
    from paper_1404_0466_amd import autotune

    t0 = time.perf_counter()
    probs = workloads.batch_problems()
    log(f"many-problem workload: {len(probs)} problems "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    dev = torch.device("cuda:0")
    ents_i, ents_e, keep = [], [], []
    for pb in probs:
        k, q, g = pb.k, pb.q, pb.g
        X = torch.from_numpy(pb.X).to(dev)
        Y = torch.from_numpy(pb.Y).to(dev)
        bi = dict(err=torch.empty(k * q, dtype=torch.float64, device=dev),
                  info=torch.empty(k * g, dtype=torch.int32, device=dev),
                  flags=torch.empty(k * q, dtype=torch.int32, device=dev))
        be = dict(err=torch.empty(k * q, dtype=torch.float64, device=dev),
                  info=torch.empty(k * q, dtype=torch.int32, device=dev),
                  flags=torch.empty(k * q, dtype=torch.int32, device=dev))
        keep.append((X, Y, bi, be))
        prob = B.make_problem(pb.n, pb.d, pb.c, k, g, pb.r, q, True)
        ents_i.append(dict(p=prob, X=X, Y=Y, lam_s=pb.lam_s, lam_grid=pb.lam_grid,
                           lam_ref=pb.lam_ref, W=None, **bi))
        ents_e.append(dict(p=prob, X=X, Y=Y, lam_s=None, lam_grid=pb.lam_grid,
                           lam_ref=pb.lam_ref, W=None, **be))
    bat_i, bat_e = B.Batch(ents_i), B.Batch(ents_e)
    nb_i = B.pichol_batch_workspace_size(bat_i, B.PICHOL_METHOD_INTERP)
    nb_e = B.pichol_batch_workspace_size(bat_e, B.PICHOL_METHOD_EXACT)
    nbytes = max(nb_i, nb_e)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    nsolves = sum(pb.k * pb.q for pb in probs)

    def timed(fn, reps):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    reps = args.steps
    tune_i, times_i = autotune.tune(bat_i, B.PICHOL_METHOD_INTERP, ws, nbytes, cache=None)
    log(f"autotuned: {tune_i}; schedules "
        + ", ".join(f"{k_}={v:.2f} ms" for k_, v in times_i["schedule"].items())
        + "; panel groups per nt "
        + "; ".join(f"{nt}: " + ", ".join(f"{g_}={v:.2f}" for g_, v in tv.items())
                    for nt, tv in times_i["panel_group"].items())
        + "; solve forms per nt "
        + "; ".join(f"{nt}: " + ", ".join(f"{f_}={v:.2f}" for f_, v in tv.items())
                    for nt, tv in times_i["solve_form"].items()))
    t_eager = timed(lambda: B.pichol_cv_batch(bat_i, B.PICHOL_METHOD_INTERP, tune_i,
                                              ws, nbytes), reps)
    gi = B.pichol_cv_batch_graph(bat_i, B.PICHOL_METHOD_INTERP, tune_i, ws, nbytes)
    t_graph = timed(lambda: B.pichol_graph_launch(gi), reps)
    B.pichol_graph_destroy(gi)
    # the same batch without its problems of d <= 768 (the buckets whose
    # factorizations and solves have at most six tile columns): how much of
    # the batch's time those buckets account for at all
    big = [e for e in ents_i if e["p"].d > 768]
    bat_big = B.Batch(big)
    gb = B.pichol_cv_batch_graph(bat_big, B.PICHOL_METHOD_INTERP, tune_i, ws, nbytes)
    t_big = timed(lambda: B.pichol_graph_launch(gb), reps)
    B.pichol_graph_destroy(gb)
    del bat_big
    ei = [b[2]["err"].cpu().numpy().reshape(pb.k, pb.q) for b, pb in zip(keep, probs)]
    ok_i = all(bool((b[2]["info"] == 0).all()) and bool((b[2]["flags"] == 0).all())
               for b in keep)
    # the same problems one after another through the single-problem pipeline
    err1 = torch.empty(max(pb.k * pb.q for pb in probs), dtype=torch.float64, device=dev)
    inf1 = torch.empty(max(pb.k * pb.g for pb in probs), dtype=torch.int32, device=dev)
    fl1 = torch.empty(max(pb.k * pb.q for pb in probs), dtype=torch.int32, device=dev)

    def sequential():
        for (X, Y, _, _), e in zip(keep, ents_i):
            B.pichol_cv(e["p"], X, Y, e["lam_s"], e["lam_grid"], e["lam_ref"], ws,
                        nbytes, err1, None, inf1, fl1)
    t_seq = timed(sequential, max(1, reps // 2))
    # the exact method, batched
    tune_e, _ = autotune.tune(bat_e, B.PICHOL_METHOD_EXACT, ws, nbytes, cache=None, reps=2)
    ge = B.pichol_cv_batch_graph(bat_e, B.PICHOL_METHOD_EXACT, tune_e, ws, nbytes)
    t_exact = timed(lambda: B.pichol_graph_launch(ge), reps)
    B.pichol_graph_destroy(ge)
    ee = [b[3]["err"].cpu().numpy().reshape(pb.k, pb.q) for b, pb in zip(keep, probs)]
    ok_e = all(bool((b[3]["info"] == 0).all()) and bool((b[3]["flags"] == 0).all())
               for b in keep)
    gap = [float(np.max(np.abs(a.mean(0) - b.mean(0)) / b.mean(0))) for a, b in zip(ei, ee)]
    same_sel = sum(int(np.argmin(a.mean(0)) == np.argmin(b.mean(0))) for a, b in zip(ei, ee))
    # the same batch with polynomials in log(lambda) (one untimed call)
    ents_l = []
    for e in ents_i:
        pl = B.make_problem(e["p"].n, e["p"].d, e["p"].c, e["p"].k, e["p"].g, e["p"].r,
                            e["p"].q, True, basis=1)
        ents_l.append(dict(e, p=pl))
    bat_l = B.Batch(ents_l)
    B.pichol_cv_batch(bat_l, B.PICHOL_METHOD_INTERP, tune_i, ws, nbytes)
    torch.cuda.synchronize()
    el = [b[2]["err"].cpu().numpy().reshape(pb.k, pb.q) for b, pb in zip(keep, probs)]
    gap_l = [float(np.max(np.abs(a.mean(0) - b.mean(0)) / b.mean(0))) for a, b in zip(el, ee)]
    same_l = sum(int(np.argmin(a.mean(0)) == np.argmin(b.mean(0))) for a, b in zip(el, ee))
    out = {
        "workload": "48 power-law Gaussian problems, d in {256..2048}, n=8d, c in {1,10}, "
                    "k=5, g=5, r=2, q=32, lambda in [1e-4,1e1]*s",
        "lambda_solves": nsolves, "buckets": B.pichol_batch_buckets(bat_i, B.PICHOL_METHOD_INTERP),
        "tuning": tune_i, "tuning_times_ms": times_i,
        "graph_ms": t_graph, "value": nsolves / (t_graph * 1e-3),
        "graph_ms_without_d_le_768": t_big,
        "problems_d_le_768": len(ents_i) - len(big),
        "eager_ms": t_eager, "sequential_single_ms": t_seq,
        "speedup_vs_sequential": t_seq / t_graph,
        "exact_graph_ms": t_exact, "exact_value": nsolves / (t_exact * 1e-3),
        "speedup_vs_exact": t_exact / t_graph,
        "interp_ok": ok_i, "exact_ok": ok_e,
        "curve_gap_max_rel": max(gap), "curve_gap_median_rel": float(np.median(gap)),
        "same_selection": f"{same_sel}/{len(probs)}",
        "log_basis_curve_gap_max_rel": max(gap_l),
        "log_basis_curve_gap_median_rel": float(np.median(gap_l)),
        "log_basis_same_selection": f"{same_l}/{len(probs)}",
        "note": "times include the Gram step of every problem",
    }
    log(f"many problems: without the {len(ents_i) - len(big)} problems of d <= 768 "
        f"the graph takes {t_big:.2f} ms")
    log(f"many problems: graph {t_graph:.2f} ms ({out['value']:.0f} lambda-solves/s), "
        f"eager {t_eager:.2f} ms, one by one {t_seq:.2f} ms, exact {t_exact:.2f} ms; "
        f"gap max {max(gap):.2e}, same selection {same_sel}/{len(probs)}")
    del ws
    return out


def differentiation_leg(args, B, stream):
    """d(hold-out error)/d(log lambda) at 64 grid values on the d = 2048
    random-Fourier-feature workload (n = 20000, k = 5, g = 6, r = 2):
    the forward piCholesky stage alone, forward + adjoint, the exact
    method's gradient, a central-difference check of the adjoint and its gap
    to the exact gradient."""
    import torch
    import workloads

    t0 = time.perf_counter()
    pb = workloads.named("rff_n20000_d2048")
    log(f"differentiation workload {pb.name} ({time.perf_counter() - t0:.1f} s)")
    dev = torch.device("cuda:0")
    n, d, c, k, g, r, q = pb.n, pb.d, pb.c, pb.k, pb.g, pb.r, pb.q
    p = B.make_problem(n, d, c, k, g, r, q, True)
    nbytes = B.pichol_workspace_size(
        p, B.PICHOL_METHOD_INTERP | B.PICHOL_METHOD_EXACT | B.PICHOL_METHOD_GRAD)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    X = torch.from_numpy(pb.X).to(dev)
    Y = torch.from_numpy(pb.Y).to(dev)
    err = torch.empty(k * q, dtype=torch.float64, device=dev)
    dlog = torch.empty(k * q, dtype=torch.float64, device=dev)
    err_e = torch.empty(k * q, dtype=torch.float64, device=dev)
    dlog_e = torch.empty(k * q, dtype=torch.float64, device=dev)
    info = torch.empty(k * q, dtype=torch.int32, device=dev)
    flags = torch.empty(k * q, dtype=torch.int32, device=dev)
    B.pichol_cv_gram(p, X, Y, ws, nbytes)

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            fn()
        s1.record(stream)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / args.steps

    fwd = lambda lam: B.pichol_cv_interp(p, pb.lam_s, lam, pb.lam_ref, ws, nbytes, err,
                                         None, info, flags)
    t_fwd = timed(lambda: fwd(pb.lam_grid))
    t_grad = timed(lambda: B.pichol_cv_interp_grad(p, pb.lam_s, pb.lam_grid, pb.lam_ref,
                                                   ws, nbytes, err, dlog, None, info,
                                                   flags))
    ok = bool((info[:k * g] == 0).all()) and bool((flags == 0).all())
    gi = dlog.cpu().numpy().reshape(k, q)
    mi = err.cpu().numpy().reshape(k, q)
    t_ex = timed(lambda: B.pichol_cv_exact_grad(p, pb.lam_grid, ws, nbytes, err_e, dlog_e,
                                                None, info, flags))
    ge = dlog_e.cpu().numpy().reshape(k, q)
    h = 1e-4
    fwd(pb.lam_grid * np.exp(h))
    up = err.cpu().numpy().reshape(k, q)
    fwd(pb.lam_grid * np.exp(-h))
    dn = err.cpu().numpy().reshape(k, q)
    fd = (up - dn) / (2 * h)
    fd_err = float(np.abs(fd - gi).max() / np.abs(gi).max())
    cm_i, cm_e = gi.mean(0), ge.mean(0)

    def zero_cross(v):
        idx = np.nonzero((v[:-1] < 0) & (v[1:] >= 0))[0]
        return float(pb.lam_grid[idx[0]]) if idx.size else None

    out = {
        "workload": f"{pb.name}: random Fourier features n={n}, d={d}, c={c}, k={k}, "
                    f"g={g}, r={r}, q={q}",
        "forward_ms": t_fwd, "forward_plus_grad_ms": t_grad,
        "grad_overhead": t_grad / t_fwd - 1.0,
        "exact_grad_ms": t_ex,
        "value": k * q / (t_grad * 1e-3), "unit": "λ-solves with d err/d log λ per s",
        "ok": ok, "dtype": "f64",
        "fd_check_max_rel": fd_err,
        "grad_gap_vs_exact_max_rel": float(np.abs(cm_i - cm_e).max() / np.abs(cm_e).max()),
        "stationary_lambda_interp": zero_cross(cm_i),
        "stationary_lambda_exact": zero_cross(cm_e),
        "mse_gap_vs_exact_max_rel": float(np.max(np.abs(mi.mean(0) - err_e.cpu().numpy()
                                                        .reshape(k, q).mean(0))
                                                 / err_e.cpu().numpy().reshape(k, q).mean(0))),
    }
    log(f"differentiation: forward {t_fwd:.2f} ms, forward+grad {t_grad:.2f} ms, exact grad "
        f"{t_ex:.2f} ms; FD check {fd_err:.2e}; gap to exact gradient "
        f"{out['grad_gap_vs_exact_max_rel']:.2e}")
    del ws
    return out


def potrf_flops(d: int) -> float:
    """Flops of one Cholesky factorization of order d, the usual count
    d^3/3 + d^2/2 + d/6 (multiplies and adds; the d square roots are not
    counted)."""
    return d ** 3 / 3.0 + d ** 2 / 2.0 + d / 6.0


def factorization_leg(args, B, prob, X, Y, stream):
    """The whole blocked factorization stage alone (every kernel of it:
    diagonal tiles, panels, column and trailing updates), timed with events
    around pichol_potrf_shifted_batched at both of the workload's shapes:
    k*g sample factorizations (the interpolated method) and k*q grid
    factorizations (the exact method), against the FP64 MFMA peak."""
    import torch
    n, d, c, k, g, r, q = prob.n, prob.d, prob.c, prob.k, prob.g, prob.r, prob.q
    dev = X.device
    f64 = dict(dtype=torch.float64, device=dev)
    p = B.make_problem(n, d, c, k, g, r, q, True)
    dp, S = B.pichol_padded_order(d), B.pichol_packed_elems(d)
    G = torch.empty(k * dp * dp, **f64)
    Cb, yy = torch.empty(k * dp * c, **f64), torch.empty(k, **f64)
    H, Bf = torch.empty(k * S, **f64), torch.empty(k * dp * c, **f64)
    B.pichol_gram(p, X, Y, G, Cb, yy, H, Bf)
    del G, Cb, yy, Bf
    L = torch.empty(k * q * S, **f64)
    info = torch.empty(k * q, dtype=torch.int32, device=dev)
    nb = B.pichol_potrf_workspace(k, q)
    wsp = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = {"what": "pichol_potrf_shifted_batched alone, all of its kernels, "
                   "event-timed; flops d^3/3 + d^2/2 + d/6 per factor",
           "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    for name, ns, lam in (("sample_factors", g, prob.lam_s),
                          ("grid_factors", q, prob.lam_grid)):
        def run():
            B.pichol_potrf_shifted_batched(d, k, H, ns, lam, L, info, wsp, nb)
        run()
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ok = bool((info.cpu().numpy()[:k * ns] == 0).all())
        tf = k * ns * potrf_flops(d) / (ms * 1e-3) / 1e12
        out[name] = {"factors": k * ns, "ms": ms, "achieved": tf,
                     "frac": tf / PEAK_FP64_TFLOPS, "info_ok": ok}
        log(f"factorization: {k * ns} factors of order {d} in {ms:.2f} ms, "
            f"{tf:.2f} TFLOP/s ({100 * tf / PEAK_FP64_TFLOPS:.1f}% of FP64 peak)")
        if not args.no_profile:
            # the trailing-update kernel alone, on a GPU it does not share
            # (in the piCholesky stage the second stream runs beside the
            # last columns' launches)
            B.pichol_profile_start(4000 * reps)
            for _ in range(reps):
                run()
            torch.cuda.synchronize()
            B.pichol_profile_stop()
            upd = merged(B.pichol_profile_summary(), "k_potrf_update")
            B.pichol_profile_reset()
            if upd:
                nl, tot = upd
                ut = update_flops(d, k * ns) * reps / nl / (tot / nl * 1e-3) / 1e12
                out[name]["k_potrf_update"] = {
                    "achieved": ut, "frac": ut / PEAK_FP64_TFLOPS,
                    "avg_launch_ms": tot / nl, "launches": nl / reps}
                log(f"factorization: k_potrf_update alone {ut:.2f} TFLOP/s "
                    f"({100 * ut / PEAK_FP64_TFLOPS:.1f}% of FP64 peak)")
    del L, H, wsp
    torch.cuda.empty_cache()
    return out


def library_leg(prob, X, stream, ours_ms=None):
    """GPU library context, not the product path: the ROCm build of torch's
    batched dense Cholesky (torch.linalg.cholesky_ex) on the same k*g shifted
    fold matrices H_f + lambda_s I that the piCholesky stage factors, in FP64,
    event-timed like the factorization leg."""
    import torch
    n, d, k, g = prob.n, prob.d, prob.k, prob.g
    dev = X.device
    sizes = [len(a) for a in np.array_split(np.arange(n), k)]
    starts = np.cumsum([0] + sizes)
    Gb = [X[starts[b]:starts[b + 1]].T @ X[starts[b]:starts[b + 1]] for b in range(k)]
    Gs = sum(Gb)
    eye = torch.eye(d, dtype=torch.float64, device=dev)
    A = torch.empty(k * g, d, d, dtype=torch.float64, device=dev)
    for f in range(k):
        Hf = (Gs - Gb[f]) / (n - sizes[f])
        for s_, lam in enumerate(prob.lam_s):
            A[f * g + s_] = Hf + float(lam) * eye
    del Gb, Gs, Hf
    L, info = torch.linalg.cholesky_ex(A)
    torch.cuda.synchronize()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        L, info = torch.linalg.cholesky_ex(A)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool((info == 0).all().item())
    tf = k * g * potrf_flops(d) / (ms * 1e-3) / 1e12
    log(f"library context: torch.linalg.cholesky_ex on {k * g} matrices of order {d}: "
        f"{ms:.2f} ms, {tf:.2f} TFLOP/s")
    del A, L, info
    torch.cuda.empty_cache()
    out = {"what": "torch.linalg.cholesky_ex (ROCm build), dense FP64, the k*g "
                   "sample matrices H_f + lambda_s I; context only",
           "torch": torch.__version__, "factors": k * g, "ms": ms, "achieved": tf,
           "frac": tf / PEAK_FP64_TFLOPS, "info_ok": ok}
    if ours_ms:
        out["pichol_potrf_shifted_batched_ms"] = ours_ms
        out["speedup_of_pichol"] = ms / ours_ms
    return out


def accuracy_leg(args, B, prob, X, Y, stream):
    """Interpolation accuracy on fold 0 of the headline workload (untimed):
    the NRMSE of every interpolated factor at the q grid values against the
    exact factor there (pichol_eval vs pichol_potrf_shifted_batched, then
    pichol_factor_nrmse), the measure of the paper's NRMSE section."""
    import torch
    n, d, c, k, g, r, q = prob.n, prob.d, prob.c, prob.k, prob.g, prob.r, prob.q
    dev = X.device
    log("accuracy: fold-0 factors at every grid value")
    f64 = dict(dtype=torch.float64, device=dev)
    p = B.make_problem(n, d, c, k, g, r, q, True)
    dp, S = B.pichol_padded_order(d), B.pichol_packed_elems(d)
    G = torch.empty(k * dp * dp, **f64)
    Cb, yy = torch.empty(k * dp * c, **f64), torch.empty(k, **f64)
    H, Bf = torch.empty(k * S, **f64), torch.empty(k * dp * c, **f64)
    B.pichol_gram(p, X, Y, G, Cb, yy, H, Bf)
    del G, Cb, yy, Bf
    H0 = H[:S]
    Ls = torch.empty(g * S, **f64)
    info = torch.empty(max(g, q), dtype=torch.int32, device=dev)
    nb = B.pichol_potrf_workspace(1, max(g, q))
    wsp = torch.empty(nb, dtype=torch.uint8, device=dev)
    B.pichol_potrf_shifted_batched(d, 1, H0, g, prob.lam_s, Ls, info, wsp, nb)
    th, tht = torch.empty((r + 1) * S, **f64), torch.empty((r + 1) * S, **f64)
    B.pichol_fit(d, 1, g, r, prob.lam_s, prob.lam_ref, Ls, th, tht)
    del Ls, tht
    Lhat = torch.empty(q * S, **f64)
    nbe = B.pichol_lambda_workspace(q)
    B.pichol_eval(d, 1, r, th, q, prob.lam_grid, prob.lam_ref, Lhat,
                  torch.empty(nbe, dtype=torch.uint8, device=dev), nbe)
    Lex = torch.empty(q * S, **f64)
    B.pichol_potrf_shifted_batched(d, 1, H0, q, prob.lam_grid, Lex, info, wsp, nb)
    out = torch.empty(q, **f64)
    nbn = B.pichol_factor_nrmse_workspace(d, q)
    B.pichol_factor_nrmse(d, q, Lhat, Lex, out,
                          torch.empty(nbn, dtype=torch.uint8, device=dev), nbn)
    torch.cuda.synchronize()
    nr = out.cpu().numpy()
    ok = bool((info.cpu().numpy()[:q] == 0).all())
    del Lhat, Lex, H, th
    torch.cuda.empty_cache()
    t = int(np.argmax(nr))
    log(f"accuracy: factor NRMSE max {nr.max():.3e} at lambda/s={prob.lam_grid[t] / prob.scale:.3g}, "
        f"median {np.median(nr):.3e}")
    return {
        "what": "NRMSE of the interpolated factor against the exact factor, "
                "fold 0, every grid value (paper's NRMSE section)",
        "factor_nrmse_max": float(nr.max()),
        "factor_nrmse_median": float(np.median(nr)),
        "factor_nrmse_at_samples_max": float(max(nr[int(np.argmin(np.abs(prob.lam_grid - ls)))]
                                                 for ls in prob.lam_s)),
        "lambda_over_s_at_max": float(prob.lam_grid[t] / prob.scale),
        "exact_factors_ok": ok,
        "paper_context": "max 0.0457 reported on MNIST (other data, other d)",
    }


def layout_leg(args, B, stream):
    """Table-1-style comparison of factor vectorisations (Sec. 5) on the GPU:
    for one fold with g = 4 sample factors, r = 2 and q = 31 grid values,
    the time to vectorise the factors (Vec), fit the polynomials (Fit) and
    evaluate them at the grid (Interp), for the row-wise, full-matrix and
    recursive (threshold 128) layouts and the tile-packed layout the
    factorization writes directly (no Vec step).  Factor values are random:
    the three steps are data movement and streaming arithmetic."""
    import torch
    dev = torch.device("cuda:0")
    g, r, q, h0 = 4, 2, 31, 128
    lam_s = np.logspace(-3, 0, g)
    lam = np.logspace(-3, 0, q)
    lam_ref = float(lam_s.max())
    nbw = B.pichol_lambda_workspace(q)
    wsl = torch.empty(nbw, dtype=torch.uint8, device=dev)
    names = {B.PICHOL_LAYOUT_ROWWISE: "row-wise", B.PICHOL_LAYOUT_FULL: "full-matrix",
             B.PICHOL_LAYOUT_RECURSIVE: "recursive", B.PICHOL_LAYOUT_TILE: "tile-packed"}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(reps):
            fn()
        s1.record(stream)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / reps

    rows = []
    for d in (1024, 2048, 4096):
        S = B.pichol_packed_elems(d)
        L = torch.randn(g * S, dtype=torch.float64, device=dev)
        for layout in (B.PICHOL_LAYOUT_ROWWISE, B.PICHOL_LAYOUT_FULL,
                       B.PICHOL_LAYOUT_RECURSIVE, B.PICHOL_LAYOUT_TILE):
            N = B.pichol_vector_length(d, layout)
            if layout == B.PICHOL_LAYOUT_TILE:
                T, t_vec = L, 0.0
            else:
                T = torch.zeros(g * N, dtype=torch.float64, device=dev)
                t_vec = timed(lambda: B.pichol_vectorize(d, g, L, layout, h0, T))
            th = torch.empty((r + 1) * N, dtype=torch.float64, device=dev)
            out = torch.empty(q * N, dtype=torch.float64, device=dev)
            t_fit = timed(lambda: B.pichol_fit_vec(N, 1, g, r, lam_s, lam_ref, T, th))
            t_int = timed(lambda: B.pichol_eval_vec(N, 1, r, th, q, lam, lam_ref, out, wsl,
                                                    nbw))
            rows.append({
                "d": d, "layout": names[layout], "vector_length": N,
                "vec_ms": t_vec, "fit_ms": t_fit, "interp_ms": t_int,
                "total_ms": t_vec + t_fit + t_int,
                "fit_GBps": (g + r + 1) * N * 8 / (t_fit * 1e-3) / 1e9,
                "interp_GBps": (r + 1 + q) * N * 8 / (t_int * 1e-3) / 1e9,
            })
            del T, th, out
        del L
    for rw in rows:
        log(f"layouts d={rw['d']:5d} {rw['layout']:12s} vec {rw['vec_ms']:7.3f} fit "
            f"{rw['fit_ms']:7.3f} interp {rw['interp_ms']:7.3f} total {rw['total_ms']:7.3f} ms "
            f"(fit {rw['fit_GBps']:.0f} GB/s, interp {rw['interp_GBps']:.0f} GB/s)")
    return {"setting": "one fold, g=4, r=2, q=31, recursive threshold 128", "rows": rows}


def merged(summ, base):
    """(launches, total ms) of every instantiation of a kernel."""
    parts = [v for nm, v in summ.items()
             if nm.strip("()") == base or nm.strip("()").startswith(base + "<")]
    if not parts:
        return None
    return sum(x[0] for x in parts), sum(x[1] for x in parts)


def solve_tiles(d: int) -> int:
    """Off-diagonal tile products of one blocked forward (or back)
    substitution: sum over the steps of the tile rows left to update."""
    nt = (d + NB - 1) // NB
    return nt * (nt - 1) // 2


def stage_rooflines(summ, prob, steps, stage, lookahead, B):
    """Roofline entries of one stage's main kernels, from the event pass:
    algorithmic work per launch (the per-unit counts written out below, times
    the units of one launch) over the mean launch duration."""
    d, k, g, q, c, r = prob.d, prob.k, prob.g, prob.q, prob.c, prob.r
    nfac = k * (g if stage == "interp" else q)
    out = {}
    upd = merged(summ, "k_potrf_update")
    if upd:
        nl, tot = upd
        flops = update_flops(d, nfac) * steps / nl
        ms = tot / nl
        tf = flops / (ms * 1e-3) / 1e12
        out["k_potrf_update"] = {
            "kernel": "k_potrf_update", "bound": "mfma", "achieved": tf,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(stage, lookahead,
                                        B.pichol_get_option(B.PICHOL_OPT_PANEL_GROUP)),
            "flops_per_launch": flops, "avg_launch_ms": ms,
            "launches_per_step": nl / steps, "factorizations": nfac,
        }
    ldz = ((q * c + NB - 1) // NB) * NB
    dp = ((d + NB - 1) // NB) * NB
    ui = merged(summ, "k_update_interp")
    if ui and stage == "interp":
        nl, tot = ui
        stacked = 2 * k * solve_tiles(d) * 2.0 * NB * NB * (r + 1) * ldz * steps / nl
        method = k * q * 2.0 * c * d * d * steps / nl
        ms = tot / nl
        tf = stacked / (ms * 1e-3) / 1e12
        out["k_update_interp"] = {
            "kernel": "k_update_interp", "bound": "mfma", "achieved": tf,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
            "flops_per_launch": stacked, "avg_launch_ms": ms,
            "method_flops_per_launch": method,
            "method_frac": method / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "launches_per_step": nl / steps,
        }
    si = merged(summ, "k_step_interp")
    if si and stage == "interp":
        nl, tot = si
        # per-lambda form: every off-diagonal tile of Lhat_t times that
        # lambda's c columns, once per direction (the method's products);
        # the MFMA products run on columns padded to a multiple of 16, and
        # the coefficient planes are read once per fold, the slab rows read
        # and written once per step
        tiles = 2 * k * solve_tiles(d) * steps / nl
        method = q * tiles * 2.0 * NB * NB * c
        mfma = q * tiles * 2.0 * NB * NB * 16 * ((c + 15) // 16)
        byts = tiles * ((r + 1) * NB * NB * 8 + 2 * NB * ldz * 8)
        ms = tot / nl
        tf = method / (ms * 1e-3) / 1e12
        out["k_step_interp"] = {
            "kernel": "k_step_interp", "bound": "mfma", "achieved": tf,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
            "flops_per_launch": method, "mfma_flops_per_launch": mfma,
            "mfma_frac": mfma / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "bytes_per_launch": byts,
            "hbm_frac": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "avg_launch_ms": ms, "launches_per_step": nl / steps,
        }
    uf = merged(summ, "k_update_factors")
    if uf and stage == "exact":
        nl, tot = uf
        # every off-diagonal factor tile read once per (fold, lambda) and
        # direction, and the c-column slab rows it updates read and written
        byts = 2 * k * q * solve_tiles(d) * (NB * NB * 8 + 2 * NB * c * 8) * steps / nl
        ms = tot / nl
        gbs = byts / (ms * 1e-3) / 1e9
        out["k_update_factors"] = {
            "kernel": "k_update_factors", "bound": "hbm", "achieved": gbs,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "bytes_per_launch": byts, "avg_launch_ms": ms, "launches_per_step": nl / steps,
        }
    hp = merged(summ, "k_holdout_partial")
    if hp:
        nl, tot = hp
        nt = dp // NB
        flops = k * nt * (nt + 1) / 2 * 2.0 * NB * NB * ldz * steps / nl
        ms = tot / nl
        tf = flops / (ms * 1e-3) / 1e12
        out["k_holdout_partial"] = {
            "kernel": "k_holdout_partial", "bound": "mfma", "achieved": tf,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
            "flops_per_launch": flops, "avg_launch_ms": ms, "launches_per_step": nl / steps,
        }
    return out


def main():
    import workloads

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rff_n60000_d4096",
                    choices=workloads.WORKLOADS,
                    help="named workload (default: the d=4096 one)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact baseline stage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-kernel event pass (no roofline)")
    ap.add_argument("--lookahead", type=int, default=0, choices=[0, 1],
                    help="side-stream look-ahead in the factorizations")
    ap.add_argument("--panel-group", type=int, default=0,
                    help="panel group G of the factorizations, 1..8 (0: the "
                         "library's default)")
    ap.add_argument("--solve-form", type=int, default=0, choices=[0, 1, 2],
                    help="interpolated solves: automatic (0), stacked over the "
                         "planes (1) or per lambda with fused diagonal blocks (2)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the precision-form legs timed after the FP64 "
                         "headline (FP32-MFMA trailing updates, iterative "
                         "refinement)")
    ap.add_argument("--no-layouts", action="store_true",
                    help="skip the vectorisation-layout comparison")
    ap.add_argument("--no-factorization", action="store_true",
                    help="skip the stand-alone factorization timing")
    ap.add_argument("--no-library", action="store_true",
                    help="skip the torch.linalg.cholesky_ex context timing")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the fold-0 factor-accuracy diagnostic (NRMSE)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the differentiation-form leg (d=2048 workload)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the many-problem (batching form) leg")
    ap.add_argument("--refine", type=int, default=2,
                    help="refinement steps of the refined legs")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="finish with one plain device copy of this many MiB "
                         "(reference dispatch for hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1404_0466_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    B.load()
    B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, args.lookahead)
    B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, args.solve_form)
    if args.panel_group:
        B.pichol_set_option(B.PICHOL_OPT_PANEL_GROUP, args.panel_group)
    dev = torch.device("cuda:0")

    log(f"generating workload {args.workload}")
    t0 = time.perf_counter()
    prob = workloads.named(args.workload)
    log(f"workload {prob.name}: n={prob.n} d={prob.d} c={prob.c} k={prob.k} "
        f"g={prob.g} r={prob.r} q={prob.q} ({time.perf_counter() - t0:.1f} s)")
    n, d, c, k, g, r, q = prob.n, prob.d, prob.c, prob.k, prob.g, prob.r, prob.q

    X = torch.from_numpy(prob.X).to(dev)
    Y = torch.from_numpy(prob.Y).to(dev)
    p = B.make_problem(n, d, c, k, g, r, q, True)
    methods = B.PICHOL_METHOD_INTERP | (0 if args.no_exact else B.PICHOL_METHOD_EXACT)
    # sized for the refined legs too (their scratch is appended at the end)
    p_ws = B.make_problem(n, d, c, k, g, r, q, True,
                          refine=0 if args.no_variants else args.refine)
    nbytes = B.pichol_workspace_size(p_ws, methods)
    log(f"workspace {nbytes / 2**30:.2f} GiB")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    err_i = torch.empty(k * q, dtype=torch.float64, device=dev)
    err_e = torch.empty(k * q, dtype=torch.float64, device=dev)
    info_i = torch.empty(k * g, dtype=torch.int32, device=dev)
    info_e = torch.empty(k * q, dtype=torch.int32, device=dev)
    flags_i = torch.empty(k * q, dtype=torch.int32, device=dev)
    flags_e = torch.empty(k * q, dtype=torch.int32, device=dev)
    lam_s, lam_grid, lam_ref = prob.lam_s, prob.lam_grid, prob.lam_ref
    stream = torch.cuda.current_stream()

    def step(ev):
        ev[0].record(stream)
        B.pichol_cv_gram(p, X, Y, ws, nbytes)
        ev[1].record(stream)
        B.pichol_cv_interp(p, lam_s, lam_grid, lam_ref, ws, nbytes, err_i, None,
                           info_i, flags_i)
        ev[2].record(stream)
        if not args.no_exact:
            B.pichol_cv_exact(p, lam_grid, ws, nbytes, err_e, None, info_e, flags_e)
        ev[3].record(stream)

    def new_events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step(new_events())
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    evs = [new_events() for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(args.steps):
        step(evs[i])
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    t_gram = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    t_int = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    t_ex = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    ms_per_step = total_ms / args.steps
    value = k * q / (t_int * 1e-3)
    log(f"step {ms_per_step:.2f} ms: gram {t_gram:.2f} ms, interp {t_int:.2f} ms, "
        f"exact {t_ex:.2f} ms -> {value:.1f} interpolated lambda-solves/s")

    ei = err_i.cpu().numpy().reshape(k, q)
    ok_i = bool((info_i.cpu().numpy() == 0).all() and (flags_i.cpu().numpy() == 0).all())
    result_extra = {
        "interp_ms": t_int, "gram_ms": t_gram,
        "value_with_gram": k * q / ((t_int + t_gram) * 1e-3),
        "interp_ok": ok_i,
    }
    if not args.no_exact:
        ee = err_e.cpu().numpy().reshape(k, q)
        ok_e = bool((info_e.cpu().numpy() == 0).all() and (flags_e.cpu().numpy() == 0).all())
        result_extra.update({
            "exact_ms": t_ex, "exact_value": k * q / (t_ex * 1e-3),
            "speedup_vs_exact": t_ex / t_int, "exact_ok": ok_e,
            "err_gap": gaps(ei.mean(0), ee.mean(0), lam_grid),
        })
        # the same curves as hold-out NRMSE (1 = predicting the fold's
        # column means), computed on the GPU from the hold-out MSEs
        nr_i = torch.empty(k * q, dtype=torch.float64, device=dev)
        nr_e = torch.empty(k * q, dtype=torch.float64, device=dev)
        B.pichol_holdout_nrmse(p, Y, err_i, nr_i)
        B.pichol_holdout_nrmse(p, Y, err_e, nr_e)
        torch.cuda.synchronize()
        ni = nr_i.cpu().numpy().reshape(k, q).mean(0)
        ne = nr_e.cpu().numpy().reshape(k, q).mean(0)
        result_extra["holdout_nrmse"] = {
            "min_interp": float(ni.min()), "min_exact": float(ne.min()),
            "curve_gap_max_rel": float(np.max(np.abs(ni - ne) / ne)),
        }

    variants = None
    if not args.no_variants:
        ee64 = None if args.no_exact else ee
        # FP64 weights of both methods (untimed), the reference of the
        # variants' relative weight errors
        W64 = {"interp": torch.empty(k * q * d * c, dtype=torch.float64, device=dev),
               "exact": None}
        B.pichol_cv_interp(p, lam_s, lam_grid, lam_ref, ws, nbytes, err_i, W64["interp"],
                           info_i, flags_i)
        if not args.no_exact:
            W64["exact"] = torch.empty_like(W64["interp"])
            B.pichol_cv_exact(p, lam_grid, ws, nbytes, err_e, W64["exact"], info_e,
                              flags_e)
        torch.cuda.synchronize()
        variants = {
            "mixed": variant_leg(args, B, p, ws, nbytes, prob, ei, ee64, stream,
                                 B.PICHOL_PREC_MIXED, 0, W64),
            f"mixed_refine{args.refine}": variant_leg(
                args, B, p, ws, nbytes, prob, ei, ee64, stream,
                B.PICHOL_PREC_MIXED, args.refine, W64),
            f"fp64_refine{args.refine}": variant_leg(
                args, B, p, ws, nbytes, prob, ei, ee64, stream,
                B.PICHOL_PREC_FP64, args.refine, W64),
            "fp64_log_basis": variant_leg(
                args, B, p, ws, nbytes, prob, ei, ee64, stream,
                B.PICHOL_PREC_FP64, 0, W64, basis=1),
        }
        if not args.no_exact:
            for v in variants.values():
                v["interp_speedup_vs_fp64_exact"] = t_ex / v["interp_ms"]
        del W64

    batching = None
    if not args.no_batch:
        batching = batching_leg(args, B, stream)

    factorization = None
    if not args.no_factorization:
        factorization = factorization_leg(args, B, prob, X, Y, stream)

    library = None
    if not args.no_library:
        library = library_leg(prob, X, stream,
                              factorization["sample_factors"]["ms"] if factorization else None)

    accuracy = None
    if not args.no_accuracy:
        accuracy = accuracy_leg(args, B, prob, X, Y, stream)

    layouts = None
    if not args.no_layouts:
        layouts = layout_leg(args, B, stream)

    differentiation = None
    if not args.no_grad:
        differentiation = differentiation_leg(args, B, stream)

    roofline = None
    rooflines = None
    kernels = None
    if not args.no_profile:
        def profile(fn, what):
            log(f"per-kernel event pass: {what}")
            B.pichol_profile_start(4000 * max(1, args.steps))
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            B.pichol_profile_stop()
            summ = B.pichol_profile_summary()
            B.pichol_profile_reset()
            return summ

        summ_i = profile(lambda: B.pichol_cv_interp(p, lam_s, lam_grid, lam_ref, ws, nbytes,
                                                    err_i, None, info_i, flags_i),
                         "interpolated stage")
        summ_e = None
        if not args.no_exact:
            summ_e = profile(lambda: B.pichol_cv_exact(p, lam_grid, ws, nbytes, err_e, None,
                                                       info_e, flags_e), "exact stage")

        def table(summ):
            return {name: {"launches_per_step": nl / args.steps, "avg_ms": tot / nl,
                           "total_ms_per_step": tot / args.steps}
                    for name, (nl, tot) in sorted(summ.items(), key=lambda kv: -kv[1][1])}

        kernels = {"interp": table(summ_i), "exact": table(summ_e) if summ_e else None}
        mix = "interp" if args.no_exact else "both"
        rooflines = {"interp": stage_rooflines(summ_i, prob, args.steps, "interp",
                                               args.lookahead, B),
                     "exact": (stage_rooflines(summ_e, prob, args.steps, "exact",
                                               args.lookahead, B) if summ_e else None)}
        roofline = rooflines["interp"].get("k_potrf_update")
        if roofline is not None:
            roofline = dict(roofline)
            roofline["stage"] = "pichol_cv_interp (the headline stage)"
        log("interpolated stage: " + ", ".join(
            f"{nm} {v['total_ms_per_step']:.2f} ms" for nm, v in list(kernels["interp"].items())[:6]))
        del mix

    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy_mib} MiB read + written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, ei[0], None if args.no_exact else ee[0])

    out = {
        "metric": METRIC, "value": value, "unit": "λ-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": prob.name, "n": n, "d": d, "c": c, "k": k, "g": g,
                   "r": r, "q": q, "lam_range": list(prob.meta.get("lam_range", [])),
                   "kind": prob.meta.get("kind"), "lookahead": args.lookahead,
                   "solve_form": args.solve_form,
                   "panel_group": B.pichol_get_option(B.PICHOL_OPT_PANEL_GROUP)},
        **result_extra,
        "precision_forms": variants,
        "batching_form": batching,
        "differentiation_form": differentiation,
        "layout_comparison": layouts,
        "accuracy": accuracy,
        "factorization": factorization,
        "library_context": library,
        "roofline": roofline,
        "rooflines": rooflines,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
