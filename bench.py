"""Benchmark: LOS projection + C_l on one MI355X.

One step = los_project (Eq. 2-3) + cl_integrate (Eq. 1) for one model of the
benchmark workload (default C2, FP64: T/E/lensing sources, l = 2..2500, 4000
log-k on [1e-4, 0.5], 3000 tau on [0, 14000]; outputs TT, EE, TE, phi-phi),
with all inputs resident in HBM.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--config C2] [--prec fp64|fp32|bf16x3]
                  [--no-cpu-baseline]

--config C3 --prec bf16x3 (or fp32) runs the mixed-precision workload (l up to
5000, 8000 k, 4000 tau; S and Delta in FP32, j_l in FP64, C_l sum in FP64).

--interp gives the sources on a coarse k grid (1000 knots for C2, 2000 for C3)
and adds the source preparation to every step: los_spline_sources +
los_interp_sources (natural cubic spline in k onto the workload's k grid),
then the projection and C_l as above.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "C_ℓ spectra/s and Δ_ℓ(k) GFMA/s vs FP64 plain path at ≤1e-4 rel err"
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
GOLDEN = {"C2": os.path.join(ROOT, "tests", "golden", "c2_cl_oracle.txt"),
          "C3": os.path.join(ROOT, "tests", "golden", "c3_cl_oracle.txt"),
          "T2": os.path.join(ROOT, "tests", "golden", "t2_cl_oracle.txt")}
PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def progress(msg):
    """One progress line on stderr (the JSON result is the only stdout line)."""
    print("bench.py: " + msg, file=sys.stderr, flush=True)


def tp_and_band_counts(wl, ls=None):
    """Per-launch work counts over all (k, tau) pairs (host-side counting only).
    TP: l in [lmin, lmax] with x = k (tau0 - tau) >= l + 1/2 (the oscillatory, threshold-free set).
    band: l up to the kernel's cut x + 14.2 x^(1/3) + 9.5.  With a sorted multipole list `ls`,
    also the TP entries whose l is in it."""
    chi = wl.tau0 - wl.tau
    tp = 0
    band = 0
    tps = 0
    for i in range(0, wl.nk, 256):
        x = wl.k[i:i + 256, None] * chi[None, :]
        top = np.minimum(np.floor(x - 0.5), wl.lmax)
        tp += int(np.sum(np.maximum(top - wl.lmin + 1, 0)))
        cut = np.minimum(np.floor(x + 14.2 * np.cbrt(x) + 9.5), wl.lmax)
        band += int(np.sum(np.maximum(cut - wl.lmin + 1, 0)))
        if ls is not None:
            tps += int(np.sum(np.searchsorted(ls, top, side="right")))
    return (tp, band, tps) if ls is not None else (tp, band)


def fp64_kernel():
    """(kernel name, source file) of the FP64 projection los_project launches."""
    if os.environ.get("LOS_PROJ_SCHEME", "1").strip() == "0":
        return "project_fp64_kernel", "project_fp64.hip"
    return "project_fp64_desc_kernel", "project_fp64_desc_kernel.hpp"


def traffic_for(prec, wl):
    """HBM bytes per projection launch from the committed counter profile of the same kernel
    source and workload (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    plain device copy of known size); None when there is none or the source has changed."""
    import hashlib
    if prec != 0:
        return None
    name, fname = fp64_kernel()
    path = os.path.join(ROOT, "profiles", "%s_%s.txt" % (name.replace("_kernel", ""), wl.name))
    src = os.path.join(ROOT, "paper_2509_25110_amd", "csrc", fname)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            key, val = line.split(":", 1)
            fields[key.strip()] = val.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(wl, stride):
    import oracle
    rows = np.arange(0, wl.nk, stride)
    S = np.ascontiguousarray(wl.S[:, rows, :])
    t0 = time.perf_counter()
    proj = oracle.project_tensor if wl.name == "T2" else oracle.project
    d = proj(wl.lmin, wl.lmax, wl.k[rows], wl.tau, wl.tau0, wl.w_tau, S)
    oracle.cl(d, wl.w_lnk[rows], wl.Pk[rows], wl.pairs)
    dt = time.perf_counter() - t0
    per_spectrum = dt * wl.nk / rows.size
    return {"value": 1.0 / per_spectrum, "unit": "spectra/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d of %d k rows (stride %d), all l and tau, %.1f s; scaled by nk/rows"
                      % (rows.size, wl.nk, stride, dt)}


def golden_error(c, wl):
    path = GOLDEN.get(wl.name)
    if path is None or not os.path.exists(path):
        return None
    g = np.loadtxt(path)
    ls = g[:, 0].astype(int) - wl.lmin
    worst = 0.0
    for p, (a, b) in enumerate(wl.pairs):
        ref = g[:, 1 + p]
        if a == b:
            rel = np.abs(c[p, ls] / ref - 1)
        else:
            rel = np.abs(c[p, ls] - ref) / np.sqrt(g[:, 1 + wl.pairs.index((a, a))] *
                                                   g[:, 1 + wl.pairs.index((b, b))])
        worst = max(worst, float(np.max(rel)))
    return worst


PEAK = {"fp32_mfma": 157.3, "bf16x3_mfma": 2516.6 / 3.0}
GOLDEN_C4 = os.path.join(ROOT, "tests", "golden", "c4_cl_oracle.txt")


def batch_tp_counts(b):
    """Sum over models of their TP entries (l <= lmax_m with x = k chi >= l + 1/2) and of their
    dense entries nk_m * ntau * (lmax_m - 1): host-side counting only."""
    chi = b.tau0 - b.tau                       # decreasing in n
    tp = 0
    rows = np.unique(b.k_index)
    t = np.floor(b.k_master[rows, None] * chi[None, :] - 0.5)      # [rows, ntau], non-increasing
    cum = np.concatenate([np.zeros((rows.size, 1)), np.cumsum(np.maximum(t - 1, 0), axis=1)], 1)
    pos = np.searchsorted(rows, b.k_index)
    for m in range(b.nmodels):
        lo, hi = b.koff[m], b.koff[m + 1]
        L = float(b.lmax[m])
        r = pos[lo:hi]
        c = np.sum(t[r] > L, axis=1)            # nodes above the l_max cap
        tp += int(np.sum((L - 1) * c + cum[r, -1] - cum[r, c]))
    dense = int(np.sum((b.koff[1:] - b.koff[:-1]) * b.ntau * (b.lmax.astype(np.int64) - 1)))
    return tp, dense


def golden_error_c4(cl, b):
    if not os.path.exists(GOLDEN_C4):
        return None
    g = np.loadtxt(GOLDEN_C4)
    worst = 0.0
    for m in np.unique(g[:, 0]).astype(int):
        gm = g[g[:, 0] == m]
        ls = gm[:, 1].astype(int) - 2
        ref = gm[:, 2:].T
        got = cl[m][:, ls]
        for p, (a, c) in enumerate(b.pairs):
            if a == c:
                rel = np.abs(got[p] / ref[p] - 1)
            else:
                rel = np.abs(got[p] - ref[p]) / np.sqrt(ref[b.pairs.index((a, a))] *
                                                        ref[b.pairs.index((c, c))])
            worst = max(worst, float(np.max(rel)))
    return worst


def batch_traffic(kernel, workload, launches, prec_name):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter profile of the
    same kernel source, precision and number of launches per step (FETCH_SIZE and WRITE_SIZE,
    each scaled by what the counter reads for a plain device copy of known size); None when
    there is none or any of those has changed."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s.txt" % (kernel.replace("_kernel", ""), workload))
    src = os.path.join(ROOT, "paper_2509_25110_amd", "csrc", "project_fused.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            key, val = line.split(":", 1)
            fields[key.strip()] = val.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if (fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in fields
            or fields.get("launches_per_step") != str(launches)
            or fields.get("precision") != prec_name):
        return None
    return float(fields["traffic_bytes_per_launch"])


def batch_run_prec(plan, b, S, dv, prec_name, steps, warmup, torch):
    """Time one precision of the C4 batch: K graph replays bracketed by HIP events (the step
    time and `value`), then instrumented eager solves for the per-kernel device times."""
    km, tau, w, wk, Pk = dv(b.k_master), dv(b.tau), dv(b.w_tau), dv(b.w_lnk), dv(b.Pk)
    cl = torch.empty((b.nmodels, 4, int(b.lmax.max()) - 1), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        plan.los_batch_solve(b.tau0, km, tau, w, S, wk, Pk, cl=cl)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(max(warmup - 1, 0)):
        step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = start.elapsed_time(end) / steps
    cl_host = cl.cpu().numpy()
    # per-kernel device times: instrumented solves (eager, events around every launch)
    nt = max(2, min(steps, 5))
    tot = {"bessel_ms": 0.0, "product_ms": 0.0, "cl_ms": 0.0}
    launches = 0
    for _ in range(nt):
        t = plan.los_batch_solve_timed(b.tau0, km, tau, w, S, wk, Pk, cl)
        for key in tot:
            tot[key] += t[key] / nt
        launches = t["launches"]
    info = plan.los_batch_info()
    return {"ms": ms, "first_ms": first_ms, "wall": wall, "cl": cl_host, "kernels": tot,
            "launches": launches, "info": info, "prec": prec_name}


def run_batch(args):
    """C4: 256 drawn models on the shared 8000-point master k grid, one graph launch per step,
    FP32 MFMA projection (the configured precision); split-BF16x3 on the same inputs as extra
    keys; the FP64 plain path on a sample of the models; the CPU oracle on a bounded sample."""
    import torch
    from paper_2509_25110_amd import inputs, los
    torch.cuda.set_device(0)
    prec_name = args.prec or "fp32"
    if prec_name == "fp64":
        print("bench.py: C4 runs the MFMA precisions (fp32, bf16x3); the FP64 plain path is "
              "reported beside them", file=sys.stderr)
        sys.exit(2)
    b = inputs.batch_inputs(inputs.draw_models(256))
    ctx = los.Context()
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    plan = ctx.los_batch_create(b.lmax, b.koff, b.k_index, b.k_master.size, b.ntau, b.pairs,
                                prec=PRECS[prec_name])
    col, ncols = plan.los_batch_columns()
    S = torch.empty((ncols, b.ntau), dtype=torch.float32, device="cuda")
    inputs.batch_sources_device(b, col, S, torch)
    progress("C4 plan and sources ready (%d packed columns)" % ncols)
    tp, dense = batch_tp_counts(b)
    flops = 2.0 * 3 * tp                     # useful flops: 2 per FMA, 3 sources per TP entry
    K = args.steps

    def summary(r, peak_key):
        peak = PEAK[peak_key]
        pk = r["kernels"]["product_ms"]
        achieved = flops / (pk * 1e-3) / 1e12
        return {"value": b.nmodels / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                "first_call_ms": r["first_ms"],
                "kernel_ms": r["kernels"], "launches_per_step": r["launches"],
                "max_rel_err_vs_oracle": golden_error_c4(r["cl"], b),
                "tuned_shape": r["info"]["fused_shape"] if r["info"]["fused"] else
                [r["info"]["tile_mb"], r["info"]["tile_nc"]],
                "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                             "unit": "TFLOP/s", "frac": achieved / peak,
                             "kernel": "fused_gemm_kernel" if r["info"]["fused"] else
                             "mfma_gemm_kernel",
                             "kernel_ms_per_step": pk,
                             "whole_step_frac": flops / (r["ms"] * 1e-3) / 1e12 / peak}}

    main = batch_run_prec(plan, b, S, dv, prec_name, K, args.warmup, torch)
    progress("C4 %s timed: %.2f ms per step" % (prec_name, main["ms"]))
    info = main["info"]
    plan.close()
    msum = summary(main, "bf16x3_mfma" if prec_name == "bf16x3" else "fp32_mfma")
    roof = dict(msum["roofline"])
    roof["traffic"] = batch_traffic(roof["kernel"], "C4", main["launches"], prec_name)
    roof["work"] = ("2 x 3 sources x %d TP entries (useful FP32-equivalent flops) per step, "
                    "over %d launches" % (tp, main["launches"]))
    roof["peak_note"] = ("bf16x3: 2516.6 TF dense bf16 / 3" if prec_name == "bf16x3" else
                         "dense FP32 MFMA")
    out = {
        "metric": METRIC,
        "value": msum["value"],
        "unit": "spectra/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": main["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f64 j_l, f32 product", "bf16x3": "f64 j_l, bf16x3 product"}[prec_name],
        "data": "synthetic",
        "config": {"workload": "C4: %s, shared master k grid, %s MFMA projection, Bessel tiles "
                               "regenerated in LDS, one graph launch per step"
                               % (inputs.DESCRIPTIONS["C4"], prec_name),
                   "models": b.nmodels, "packed_columns": ncols, "master_rows": info["rows"],
                   "ntau": b.ntau, "parallelism": "single GPU"},
        "roofline": roof,
        "gfma_per_s": 3 * tp / (main["ms"] * 1e-3) / 1e9,
        "tp_entries": tp, "dense_entries": dense,
        "first_call_ms": main["first_ms"], "wall_s_timed": main["wall"],
        "kernel_ms_per_step": main["kernels"], "chunks": info["chunks"],
        "tuned_shape": msum["tuned_shape"],
        "max_rel_err_vs_oracle": msum["max_rel_err_vs_oracle"],
        "oracle_models": "8 seeded models of the 256, every l (tests/golden/c4_cl_oracle.txt)",
    }
    if not args.no_other_prec:
        other = "bf16x3" if prec_name == "fp32" else "fp32"
        plan2 = ctx.los_batch_create(b.lmax, b.koff, b.k_index, b.k_master.size, b.ntau, b.pairs,
                                     prec=PRECS[other])
        r2 = batch_run_prec(plan2, b, S, dv, other, K, args.warmup, torch)
        progress("C4 %s timed: %.2f ms per step" % (other, r2["ms"]))
        plan2.close()
        o = summary(r2, "bf16x3_mfma" if other == "bf16x3" else "fp32_mfma")
        o["roofline"]["traffic"] = None
        out[other] = o
    if not args.no_fp64_compare:
        # the FP64 plain path on models of the batch solved one by one, scaled by TP work
        sample = [0, 3, 100, 200]
        tsum = 0.0
        for i in sample:
            wlm = inputs.model_workload(b.draws[i])
            a64 = [dv(wlm.k), dv(wlm.tau), wlm.tau0, dv(wlm.w_tau), dv(wlm.S)]
            wk, Pk = dv(wlm.w_lnk), dv(wlm.Pk)
            dd = ctx.los_project(wlm.lmin, wlm.lmax, *a64)
            ctx.cl_integrate(dd, wk, Pk, wlm.pairs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.los_project(wlm.lmin, wlm.lmax, *a64, delta=dd)
            ctx.cl_integrate(dd, wk, Pk, wlm.pairs)
            torch.cuda.synchronize()
            tsum += time.perf_counter() - t0
            del dd
        tp_sub, _ = batch_tp_counts(inputs.batch_inputs([b.draws[i] for i in sample]))
        fp64 = b.nmodels / (tsum * tp / tp_sub)
        progress("C4 FP64 plain path on models %s: %.3f s" % (sample, tsum))
        out["fp64_plain_path"] = {"value": fp64, "unit": "spectra/s",
                                  "sample": "models %s solved one by one with the FP64 path "
                                            "(%.3f s), scaled to the batch by TP work"
                                            % (sample, tsum)}
        out["speedup_vs_fp64_plain_path"] = out["value"] / fp64
        if "bf16x3" in out:
            out["bf16x3"]["speedup_vs_fp64_plain_path"] = out["bf16x3"]["value"] / fp64
    if not args.no_cpu_baseline:
        import oracle
        m = 3
        d = b.draws[m]
        wlm = inputs.model_workload(d)
        stride = args.cpu_stride or 1                   # all rows of the model: about 10 s
        rows = np.arange(0, wlm.nk, stride)
        Sm = np.ascontiguousarray(wlm.S[:, rows, :])
        t0 = time.perf_counter()
        oracle.project(wlm.lmin, wlm.lmax, wlm.k[rows], wlm.tau, wlm.tau0, wlm.w_tau, Sm)
        dt = time.perf_counter() - t0
        rate = rows.size * wlm.ntau * (wlm.lmax - 1) / dt      # dense entries per second
        total = dense / rate
        out["cpu_baseline"] = {"value": b.nmodels / total, "unit": "spectra/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "model %d, %d of its %d k rows (stride %d), all l and "
                                         "tau: %.1f s; scaled by the batch's dense (k, tau, l) "
                                         "count" % (m, rows.size, wlm.nk, stride, dt)}
    del S
    ctx.close()
    print(json.dumps(out), flush=True)


EMU_LO = np.array([260.0, 15.0, 0.0, 0.92, 2.9])     # tau*, width, ISW amp, n_s, ln(1e10 A_s)
EMU_HI = np.array([300.0, 25.0, 0.2, 1.0, 3.2])


def solve_models(ctx, draws, prec, torch, chunk=256, timed=None, tt_only=False):
    """Batched solve of drawn models (all on the full master grid, l_max 5000) in plans of
    `chunk` models; returns (params [n, 5], cl [n, 4, 4999] on the device, seconds), or with
    tt_only the temperature source alone and cl [n, 1, 4999] (TT).  The sources of each plan
    are generated on the device before its timed part; `timed` lists what the seconds include:
    "solve" (the solve call) or "plan+solve" (plan creation too)."""
    from paper_2509_25110_amd import inputs
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    out, secs = [], 0.0
    with_plan = timed == "plan+solve"
    for c0 in range(0, len(draws), chunk):
        b = inputs.batch_inputs(draws[c0:c0 + chunk])
        srcs = (0,) if tt_only else (0, 1, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = ctx.los_batch_create(b.lmax, b.koff, b.k_index, b.k_master.size, b.ntau,
                                    [(0, 0)] if tt_only else b.pairs, prec=prec, nsrc=len(srcs))
        col, ncols = plan.los_batch_columns()
        t_plan = time.perf_counter() - t0
        S = torch.empty((ncols, b.ntau), dtype=torch.float32, device="cuda")
        inputs.batch_sources_device(b, col, S, torch, sources=srcs)
        args = (b.tau0, dv(b.k_master), dv(b.tau), dv(b.w_tau), S, dv(b.w_lnk), dv(b.Pk))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cl = plan.los_batch_solve(*args)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0 + (t_plan if with_plan else 0.0)
        out.append(cl)
        del S
        plan.close()
        progress("solved %d / %d models" % (min(c0 + chunk, len(draws)), len(draws)))
    params = np.array([[d.tau_star, d.width, d.a_isw, d.n_s, d.ln1e10As] for d in draws])
    return params, torch.cat(out), secs


def fp64_solve(ctx, draws, torch):
    """The FP64 plain path (los_project + cl_integrate) on each drawn model alone, sources built
    on the device; returns (cl [n, 4, nl] host, seconds of projection + C_l)."""
    from paper_2509_25110_amd import inputs
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    out, secs = [], 0.0
    for d in draws:
        w = inputs.model_grid(d)
        S = inputs.model_sources_device(w, torch)
        a64 = (dv(w.k), dv(w.tau), w.tau0, dv(w.w_tau), S)
        wk, Pk = dv(w.w_lnk), dv(w.Pk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dd = ctx.los_project(w.lmin, w.lmax, *a64)
        c = ctx.cl_integrate(dd, wk, Pk, w.pairs)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        out.append(c.cpu().numpy())
        del dd, S
    return np.stack(out), secs


def run_emulator(args):
    """C5: emulator trained on batch-solver spectra (l = 2..5000, 8000 master k, 3000 tau);
    held-out error judged by the FP64 plain path, which also calibrates the ensemble's error
    estimate per spectrum; inference on a batch of 4096 new parameter sets with the fallback
    spectrum by spectrum: the spectra whose calibrated estimate is above 1e-3 are re-solved by
    the batched solver (the temperature source alone when TT is the only one) and merged, and
    the line's value is that end to end."""
    import tempfile
    import torch
    from paper_2509_25110_amd import inputs, los
    torch.cuda.set_device(0)
    cache = os.path.join(tempfile.mkdtemp(prefix="los_tune_"), "tune.txt")
    ctx = los.Context(tune_cache=cache)
    pin = dict(lmax_range=(5000, 5000), nk_range=(8000, 8000))
    tr = inputs.draw_models(args.emu_train, seed=1, **pin)
    ptr, ctr, gen_s = solve_models(ctx, tr, 2, torch)
    nl = ctr.shape[2]
    emu = los.Emulator(ctx, 5, nl, ncomp=96, width=512, depth=4, members=4, seed=7)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = emu.emu_train(dv(ptr), EMU_LO, EMU_HI, ctr, epochs=args.emu_epochs, batch=256,
                         lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del ctr
    progress("trained on %d spectra in %.1f s" % (len(tr), train_s))
    thr = 1e-3
    # held-out accuracy, judged by the FP64 plain path
    te = inputs.draw_models(args.emu_heldout, seed=2, **pin)
    ref, t64 = fp64_solve(ctx, te, torch)
    pte = np.array([[d.tau_star, d.width, d.a_isw, d.n_s, d.ln1e10As] for d in te])
    c, err, flag = emu.emu_infer(dv(pte), threshold=thr)
    c, err, flag = c.cpu().numpy(), err.cpu().numpy(), flag.cpu().numpy()
    scale = np.abs(ref).copy()
    scale[:, 2] = np.sqrt(ref[:, 0] * ref[:, 1])
    rel = np.abs(c - ref) / scale
    true_err = np.max(rel, axis=(1, 2))
    per_spec = {nm: float(np.median(np.max(rel[:, i], axis=1)))
                for i, nm in enumerate(("TT", "EE", "TE", "PP"))}
    progress("held-out (%d, FP64 judge): median error %.2e" % (len(te), np.median(true_err)))
    # calibration of the ensemble spread, spectrum by spectrum: the largest ratio of true error
    # (FP64 judge) to spread over the held-out models, with a 1.5 margin; the fallback below
    # flags a spectrum when spread x calibration > 1e-3
    _, e4h, _ = emu.emu_infer_spectra(dv(pte), threshold=thr)
    e4h = e4h.cpu().numpy().astype(np.float64)
    true4 = np.max(rel, axis=2)                                   # [held-out, 4]
    calib = 1.5 * np.max(true4 / np.maximum(e4h, 1e-30), axis=0)
    # end to end on 4096 new parameter sets: emulate, re-solve the flagged ones, merge
    n = 4096
    new = inputs.draw_models(n, seed=3, **pin)
    P = dv(np.array([[d.tau_star, d.width, d.a_isw, d.n_s, d.ln1e10As] for d in new]))
    cl_buf = torch.empty((n, 4, nl), dtype=torch.float64, device="cuda")
    emu.emu_infer(P, cl=cl_buf, threshold=thr)
    torch.cuda.synchronize()
    K = args.steps
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(K):
        emu.emu_infer(P, cl=cl_buf, threshold=thr)
    end.record()
    torch.cuda.synchronize()
    infer_ms = start.elapsed_time(end) / K
    # fallback spectrum by spectrum: a model whose EE, TE or PP misses the threshold is
    # re-solved in full; one whose TT alone misses it, for the temperature source only
    t0 = time.perf_counter()
    cl, err4, flag4 = emu.emu_infer_spectra(P, cl=cl_buf, threshold=thr)
    f4 = err4.cpu().numpy().astype(np.float64) * calib[None, :] > thr
    full = np.nonzero(f4[:, 1:].any(axis=1))[0]
    tt = np.setdiff1d(np.nonzero(f4[:, 0])[0], full)
    t_emu = time.perf_counter() - t0
    t_fb = 0.0
    # the tuner's choice for these shapes is in the context's cache after the first plan
    if full.size:
        _, cfb, dt = solve_models(ctx, [new[i] for i in full], 2, torch, timed="plan+solve")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        emu.emu_merge(full, cfb, cl)
        torch.cuda.synchronize()
        t_fb += dt + time.perf_counter() - t1
        del cfb
    if tt.size:
        _, ctt, dt = solve_models(ctx, [new[i] for i in tt], 2, torch, timed="plan+solve",
                                  tt_only=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        emu.emu_merge_spectrum(0, tt, ctt.reshape(tt.size, nl).contiguous(), cl, err4=err4,
                               flag4=flag4)
        torch.cuda.synchronize()
        t_fb += dt + time.perf_counter() - t1
        del ctt
    resolved = np.zeros_like(f4)
    resolved[full] = True
    resolved[tt, 0] = True
    assert np.all(resolved >= f4)
    effective = n / (t_emu + t_fb)
    # the same 4096 models solved by the batched solver alone (plan + solve): the time the
    # emulator competes with, and the reference for the spectra it kept
    _, call, t_all = solve_models(ctx, new, 2, torch, timed="plan+solve")
    got, want = cl.cpu().numpy(), call.cpu().numpy()
    del call
    kept_err = None
    if (~resolved).any():
        sc = np.abs(want).copy()
        sc[:, 2] = np.sqrt(want[:, 0] * want[:, 1])
        rel = np.max(np.abs(got - want) / sc, axis=2)       # [n, 4]
        kept_err = {name: rel[~resolved[:, i], i] for i, name in enumerate(("TT", "EE", "TE", "PP"))
                    if (~resolved[:, i]).any()}
    emu_rate = n / (infer_ms * 1e-3)
    fp64_rate = len(te) / t64
    flops = n * 2.0 * (emu.nparams + 4 * 96 * nl) * emu.members
    peak = PEAK["fp32_mfma"]
    out = {
        "metric": METRIC,
        "value": effective, "unit": "spectra/s", "n_gpus": 1, "steps": K, "warmup": 1,
        "ms_per_step": (t_emu + t_fb) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 MLP and reconstruction, f64 C_l; fallback bf16x3 batched solve",
        "data": "synthetic",
        "config": {"workload": "C5: emulator of TT/EE/TE/PP over l=2..5000 (8000 master k, 3000 "
                               "tau), 4 x MLP 5-512x4-384 GELU, PCA 96 per spectrum, %d training "
                               "spectra from the bf16x3 batched solver; one step = 4096 new "
                               "parameter sets emulated, every spectrum whose estimate is above "
                               "1e-3 re-solved by the batched solver (the temperature source "
                               "alone when TT is the only one; plan + solve, sources resident) "
                               "and merged" % len(tr),
                   "train_spectra": len(tr), "heldout_spectra": len(te), "epochs": args.emu_epochs,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": flops / (infer_ms * 1e-3) / 1e12, "peak": peak,
                     "unit": "TFLOP/s", "frac": flops / (infer_ms * 1e-3) / 1e12 / peak,
                     "traffic": None, "kernel": "emu_infer (4 members: MLP + reconstruction)",
                     "kernel_ms": infer_ms,
                     "work": "4096 x 4 members x 2 x (MLP params + 4 x 96 x %d)" % nl},
        "fallback_threshold": thr,
        "estimate_calibration": {nm: float(calib[i])
                                 for i, nm in enumerate(("TT", "EE", "TE", "PP"))},
        "fallback_models": int(resolved.any(axis=1).sum()),
        "fallback_fraction": float(resolved.any(axis=1).mean()),
        "fallback_full_models": int(full.size), "fallback_tt_only_models": int(tt.size),
        "fallback_spectra_fraction": float(resolved.mean()),
        "fallback_s": t_fb, "emulate_s": t_emu,
        "batched_solver_alone_spectra_per_s": n / t_all,
        "gain_vs_batched_solver": t_all / (t_emu + t_fb),
        "kept_spectra_err_vs_batched_solver": None if kept_err is None else {
            k: {"count": int(v.size), "median": float(np.median(v)), "max": float(np.max(v)),
                "above_threshold": int(np.sum(v > thr))} for k, v in kept_err.items()},
        "emulator_only_spectra_per_s": emu_rate,
        "fp64_plain_path_spectra_per_s": fp64_rate,
        "speedup_vs_fp64_plain_path": effective / fp64_rate,
        "heldout_judge": "FP64 plain path, each model alone",
        "heldout_err_median": float(np.median(true_err)),
        "heldout_err_p90": float(np.quantile(true_err, 0.9)),
        "heldout_err_max": float(true_err.max()),
        "heldout_err_median_per_spectrum": per_spec,
        "heldout_flagged_fraction": float(np.mean(flag)),
        "estimate_over_true_median": float(np.median(err / true_err)),
        "training_data_solve_s": gen_s, "train_s": train_s,
        "final_loss": [float(x) for x in hist[:, -1]],
    }
    if args.emu_save:
        emu.emu_save(args.emu_save)
        out["saved_to"] = args.emu_save
    emu.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C4",
                    help="C4 (default: the 256-model batch), C5 (emulator), C1/C2/C3 (one model), "
                         "T2 (tensor modes, FP64)")
    ap.add_argument("--prec", default=None, choices=list(PRECS),
                    help="default fp32 for C4, fp64 for C1-C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle sample: every n-th k row (default 1 for C2, T2 and the C4 model, "
                         "4 for C3)")
    ap.add_argument("--emu-train", type=int, default=100000, help="C5: training spectra")
    ap.add_argument("--emu-epochs", type=int, default=100, help="C5: training epochs")
    ap.add_argument("--emu-heldout", type=int, default=32,
                    help="C5: held-out models judged by the FP64 plain path")
    ap.add_argument("--emu-save", default="", help="C5: write the trained emulator to this file")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="C4: skip timing the FP64 plain path on a sample of the batch's models")
    ap.add_argument("--no-other-prec", action="store_true",
                    help="C4: skip the second MFMA precision (bf16x3 beside fp32)")
    ap.add_argument("--lsample", type=float, default=0.0,
                    help="C2/C3 FP64: compute the multipoles of inputs.l_samples(boost) only and "
                         "interpolate C_l (los_project_lsample + cl_integrate + los_cl_interp)")
    ap.add_argument("--interp", action="store_true",
                    help="C1-C3: sources on the coarse k grid, splined onto the LOS grid each step")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mib > 0:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py: only one GPU is measured (the projection would shard over k, with one "
              "all-reduce of the partial C_l); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.config in ("C4", "C5") and (args.lsample > 0 or args.interp):
        print("bench.py: --lsample and --interp apply to the one-model workloads C1-C3 "
              "(e.g. --config C2 --lsample 1)", file=sys.stderr)
        sys.exit(2)
    if args.config == "C4":
        return run_batch(args)
    if args.config == "C5":
        return run_emulator(args)

    import torch
    from paper_2509_25110_amd import inputs, los

    torch.cuda.set_device(0)
    tensor = args.config == "T2"
    wl = inputs.tensor_workload() if tensor else inputs.config(args.config)
    prec = PRECS[args.prec or "fp64"]
    if tensor and (prec != 0 or args.lsample > 0 or args.interp):
        print("bench.py: the tensor workload runs the FP64 path only", file=sys.stderr)
        sys.exit(2)
    sdt = np.float64 if prec == 0 else np.float32
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    k, tau, w, S = dv(wl.k), dv(wl.tau), dv(wl.w_tau), dv(wl.S.astype(sdt))
    wk, Pk = dv(wl.w_lnk), dv(wl.Pk)
    delta = torch.empty((wl.nk, wl.nl, 3 if tensor else wl.nsrc), dtype=S.dtype, device="cuda")
    cl = torch.empty((len(wl.pairs), wl.nl), dtype=torch.float64, device="cuda")
    ctx = los.Context()
    stream = torch.cuda.current_stream()

    if args.interp:
        cs = inputs.coarse_sources(wl, inputs.COARSE_NK[wl.name])
        q, Sc = dv(cs.q), dv(cs.Sc)
        M = torch.empty_like(Sc)

    def prepare():
        if args.interp:
            ctx.los_spline_sources(q, Sc, M=M)
            ctx.los_interp_sources(q, Sc, M, k, out_prec=0 if prec == 0 else 1, S=S)

    ls = None
    if args.lsample > 0:
        if prec != 0:
            print("bench.py: --lsample runs the FP64 path only", file=sys.stderr)
            sys.exit(2)
        ls = inputs.l_samples(wl.lmin, wl.lmax, args.lsample)
        delta = torch.empty((wl.nk, ls.size, wl.nsrc), dtype=torch.float64, device="cuda")
        cls = torch.empty((len(wl.pairs), ls.size), dtype=torch.float64, device="cuda")

    def project():
        if tensor:
            ctx.los_project_tensor(wl.lmin, wl.lmax, k, tau, wl.tau0, w, S, delta=delta)
        elif ls is None:
            ctx.los_project(wl.lmin, wl.lmax, k, tau, wl.tau0, w, S, prec=prec, delta=delta)
        else:
            ctx.los_project_lsample(wl.lmin, wl.lmax, ls, k, tau, wl.tau0, w, S, delta=delta)

    def spectra():
        if ls is None:
            ctx.cl_integrate(delta, wk, Pk, wl.pairs, cl=cl)
        else:
            ctx.cl_integrate(delta, wk, Pk, wl.pairs, cl=cls)
            ctx.los_cl_interp(ls, cls, wl.lmin, wl.lmax, cl=cl)

    def step():
        prepare()
        project()
        spectra()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(max(args.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    evi = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for i in range(K):
        evi[i].record(stream)
        prepare()
        ev[i][0].record(stream)
        project()
        ev[i][1].record(stream)
        spectra()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    proj_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    prep_ms = float(np.mean([a.elapsed_time(b[0]) for a, b in zip(evi, ev)]))
    ms_per_step = total_ms / K

    ncol = 4 if tensor else wl.nsrc  # the tensor sweep accumulates 4 columns
    if ls is None:
        tp, band = tp_and_band_counts(wl)
        flops = tp * (3.0 + 2.0 * ncol)  # recurrence FMA + coefficient add, ncol FMAs, per TP entry
    else:  # the recurrence at every TP entry, the accumulation at the sampled ones
        tp, band, tps = tp_and_band_counts(wl, ls)
        flops = tp * 3.0 + tps * 2.0 * wl.nsrc
    achieved = flops / (proj_ms * 1e-3) / 1e12
    gfma = ncol * tp / (ms_per_step * 1e-3) / 1e9
    err = golden_error(cl.cpu().numpy(), wl)
    lsample = None
    if ls is not None:
        lsample = {"boost": args.lsample, "nls": int(ls.size),
                   "cl_rel_dev_vs_all_l": err,
                   "within_1e-4_of_all_l": bool(err is not None and err <= 1e-4),
                   "note": "the C_l between the samples are interpolated in l; on these "
                           "workloads that moves them by more than the 1e-4 of the metric",
                   "tp_sampled_entries": tps}
        err = None  # the interpolated C_l differ from the all-l ones by the interpolation
    interp = None
    if args.interp:
        nkc = cs.q.size
        # algorithmic bytes: the spline reads Sc and writes M; the evaluation reads Sc and M
        # once and writes S
        byts = 8.0 * wl.nsrc * wl.ntau * (2 * nkc + 2 * nkc) + S.element_size() * S.numel()
        interp = {"nkc": int(nkc), "ms": prep_ms, "bytes": byts,
                  "GB_per_s": byts / (prep_ms * 1e-3) / 1e9,
                  "frac_hbm": byts / (prep_ms * 1e-3) / 8e12,
                  "cl_rel_dev_vs_direct_sources": err}
        err = None  # the golden C_l are for sources given on the LOS grid itself

    path = {0: "FP64 plain path", 1: "FP32 MFMA path", 2: "split-BF16x3 MFMA path"}[prec]
    if tensor:
        path = "FP64 tensor-mode path (sweep of S_P, S_P/x, S_P/x^2, S_T/x^2, row combination)"
    kernel = fp64_kernel()[0] if prec == 0 else "jseed_kernel + fused_gemm_kernel"
    out = {
        "metric": METRIC,
        "value": K / (total_ms * 1e-3),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f64", 1: "f64 j_l, f32 product", 2: "f64 j_l, bf16x3 product"}[prec],
        "data": "synthetic",
        "config": {"workload": "%s: %s, %s%s" % (wl.name, inputs.DESCRIPTIONS[wl.name], path,
                                                 ", sources splined from %d coarse k each step"
                                                 % inputs.COARSE_NK[wl.name] if args.interp else ""),
                   "nk": wl.nk, "ntau": wl.ntau, "lmax": wl.lmax, "nsrc": wl.nsrc,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic_for(prec, wl) if ls is None else None,
                     "kernel": kernel, "kernel_ms": proj_ms,
                     "work": ("%d TP (l,k,tau) entries x %d FP64 flops" % (tp, 3 + 2 * ncol)
                              if ls is None else
                              "%d TP entries x 3 + %d sampled TP entries x %d FP64 flops"
                              % (tp, tps, 2 * wl.nsrc))},
        "gfma_per_s": gfma,
        "tp_entries": tp,
        "band_entries": band,
        "first_call_ms": first_ms,
        "cl_ms": ms_per_step - proj_ms - prep_ms,
        "wall_s_timed": wall,
        "max_rel_err_vs_oracle": err,
    }
    if interp is not None:
        out["interp"] = interp
    if lsample is not None:
        out["lsample"] = lsample
        out["config"]["workload"] += ", multipoles of l_samples(boost=%g) (%d), C_l interpolated" % (
            args.lsample, ls.size)
    if not args.no_cpu_baseline and rank == 0 and not args.interp and ls is None:
        stride = args.cpu_stride or {"C3": 4}.get(wl.name, 1)
        out["cpu_baseline"] = cpu_baseline(wl, stride)
    ctx.close()
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
