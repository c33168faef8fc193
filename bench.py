#!/usr/bin/env python3
"""Benchmark: unknowns/s of full multigrid solves to a 1e-10 relative
residual on one MI355X.

Default workload (--config c3, the headline line): 3D Poisson, 7-point
stencil on the unit cube, 511 x 511 x 511 interior grid (133,432,831
unknowns), rhs i.i.d. N(0,1) (seed 3), red-black Gauss-Seidel V(2,2), full
weighting / trilinear transfers, 3^3 FP64 direct coarsest solve, plain FP64.
One "step" is one complete solve from u = 0 to ||f - A u||_2 / ||f||_2 <=
1e-10 (every level operation of every cycle, the stop test included), inputs
resident in HBM.  The same problem is then solved by FP32 V(2,2) cycles
inside FP64 iterative refinement, and by the same with the cycle's iterate
stored as bfloat16 (the mixed forms): their unknowns/s to the same FP64
residual, checked by the oracle, and their speedup over plain FP64 are
reported beside the headline ("forms", "speedup_vs_f64").

Other configurations (--config): c2 (2D Poisson 4095^2, FP64), c3-f32 /
c3-bf16 (the mixed 3D forms alone, with per-kernel timings), c4 / c4-f64
(256 uneven 2D diffusion systems, FP32 cycles in FP64 refinement / plain
FP64), c1 (1D Poisson n = 1023), c5 (2D diffusion 1023^2 with log-normal
coefficients: the learned smoother, trained here on pairs from the plain
solver's own cycles, against plain red-black Gauss-Seidel, both with FP32
cycles in FP64 refinement), jacobi (the paper's own fixed-iteration Jacobi
benchmark: 7168 x 7168, four iterations of the five-point average; metric:
interior point updates/s).

Prints ONE JSON line (rank 0 only; the solver runs on one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "unknowns/s solved to 1e-10 rel. residual; mixed/learned vs plain FP64"

CONFIGS = {
    "c2": dict(dim=2, n=4095, precision="f64", seed=2, form="plain FP64"),
    "c3": dict(dim=3, n=511, precision="f64", seed=3, form="plain FP64"),
    "c3-f32": dict(dim=3, n=511, precision="f32", seed=3, form="FP32 V(2,2) in FP64 iterative refinement"),
    "c3-bf16": dict(dim=3, n=511, precision="bf16", seed=3,
                    form="FP32 V(2,2) with bf16-stored iterate in FP64 iterative refinement"),
    "c1": dict(dim=1, n=1023, precision="f64", seed=1, form="plain FP64 (RB-GS on the GPU)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measured_traffic(kernel, record="traffic.json",
                     sources=("k_march2d.inc", "k_march2d_f64.hip", "dev_common.h", "mg_internal.h")):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", record)))
        csrc = os.path.join(ROOT, "paper_1210_7774_amd", "csrc")
        h = hashlib.sha256()
        for fn in sources:
            h.update(open(os.path.join(csrc, fn), "rb").read())
        if h.hexdigest()[:16] != rec["source_hash"] or kernel not in rec["kernels"]:
            return None
        k = rec["kernels"][kernel]
        return k["read_bytes"] + k["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def oracle_baseline(n, dim, seed, cycles, sample_n):
    """The oracle (plain C, one thread, as it stands) on a bounded sample of
    the same workload: one V(2,2) cycle plus one FP64 residual norm on the
    sample_n^dim grid of the same problem class, after a warm-up on a small
    grid, timed three times (mean, with min and max; the paper's performance
    study reports the mean of three runs).  The full solve is taken as
    `cycles` such units on the full grid, the time per unit scaling with the
    number of points."""
    import numpy as np

    import oracle as O
    from paper_1210_7774_amd import inputs as I

    def gen(m):
        return I.sine_plus_noise_1d(m, seed) if dim == 1 else I.normal_rhs(m, dim, seed)

    opts = O.Opts(ncoarse=1 if dim == 1 else 3)
    fw = gen(15 if dim == 3 else 63)
    O.vcycle(np.zeros_like(fw), fw, opts=opts)
    fs = gen(sample_n)
    times = []
    for _ in range(3):
        u = np.zeros_like(fs)
        t0 = time.perf_counter()
        O.vcycle(u, fs, opts=opts)
        r = O.residual(u, fs)
        _ = float(np.sqrt((r * r).sum()))
        times.append(time.perf_counter() - t0)
    t = sum(times) / 3
    per_point = t / sample_n ** dim
    per_solve = per_point * n ** dim * cycles
    return {"value": n ** dim / per_solve, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": "1 V(2,2) cycle + 1 FP64 residual norm on the %s grid of the same problem (rhs seed %d), "
                      "mean of 3 runs after a warm-up: %.2f s (min %.2f, max %.2f) on one core of %s; "
                      "the full solve is %d such cycles on %s points, time scaled by the point count"
                      % ("x".join([str(sample_n)] * dim), seed, t, min(times), max(times), cpu_model(), cycles,
                         "x".join([str(n)] * dim))}


def oracle_c1(f_np, rtol):
    """C1's CPU reference: the oracle's whole 1D solve with lexicographic
    Gauss-Seidel V(2,2) (and, for comparison, red-black), one warm-up, then
    the mean of three runs on one host core."""
    import oracle as O
    n = f_np.shape[0]
    res = {}
    for name, sm in (("lex", O.LEX), ("rb", O.RBGS)):
        opts = O.Opts(smoother=sm, ncoarse=1)
        O.solve(f_np, opts=opts, tol=rtol)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            r = O.solve(f_np, opts=opts, tol=rtol)
            ts.append(time.perf_counter() - t0)
        res[name] = (sum(ts) / 3, min(ts), max(ts), r.cycles)
    t, lo, hi, cyc = res["lex"]
    return {"value": n / t, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": "the whole solve with lexicographic Gauss-Seidel V(2,2) to %g: %d cycles, %.3f ms (mean of 3 "
                      "after a warm-up, min %.3f, max %.3f) on one core of %s; red-black: %d cycles, %.3f ms"
                      % (rtol, cyc, t * 1e3, lo * 1e3, hi * 1e3, cpu_model(), res["rb"][3], res["rb"][0] * 1e3)}


def kernel_table(timings):
    rows = sorted(timings.items(), key=lambda kv: -kv[1][0] * kv[1][1])
    tot = sum(v[0] * v[1] for v in timings.values()) or 1.0
    log("%-24s %8s %10s %10s %9s %7s" % ("kernel", "launches", "avg_us", "MB/launch", "GB/s", "share"))
    for name, (cnt, avg, b) in rows:
        gbs = b / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        log("%-24s %8d %10.2f %10.2f %9.1f %6.1f%%" % (name, cnt, avg * 1e3, b / 1e6, gbs, 100 * cnt * avg / tot))
    return rows


LEARNED_FLOP_PER_PX = 2 * 9 * (16 + 16 * 16 + 16 * 16 + 16)  # 9792: the network's multiply-adds x 2
MFMA_BF16_PEAK_TFLOPS = 2500.0


# committed counter records (profiles/) per kernel family, with the sources
# whose hash they were taken on
TRAFFIC_2D = ("traffic.json", ("k_march2d.inc", "k_march2d_f64.hip", "dev_common.h", "mg_internal.h"))
TRAFFIC_3D = ("traffic_c3.json", ("k_march3d.hip", "k_march3dw.hip", "mg_m3.h", "dev_common.h", "mg_internal.h"))
M3_CLASSES = ("pre_rr", "pre_sweep", "post_corr", "post_norm", "post_sweep", "post_acc", "pre_zero_rr",
              "pre_zero_sweep")


def traffic_of(name):
    cls = name.split(" ")[0]
    rec = TRAFFIC_3D if cls in M3_CLASSES or (cls[:1] == "w" and cls[2:] in M3_CLASSES) else TRAFFIC_2D
    return measured_traffic(name, rec[0], rec[1])


def roofline_of(rows, learned_px_per_launch=0):
    """Roofline of the dominant kernel that moves data (by total time).  The
    fused learned step is priced against the bf16 MFMA peak: its algorithmic
    work is the network's 9,792 flop per pixel and step."""
    for name, (cnt, avg, b) in rows:
        if name.startswith("learned_step") and avg > 0 and learned_px_per_launch:
            flops = LEARNED_FLOP_PER_PX * learned_px_per_launch
            achieved = flops / (avg * 1e-3) / 1e12
            return {"bound": "mfma", "achieved": round(achieved, 2), "peak": MFMA_BF16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 5), "traffic": None,
                    "kernel": name, "flop_per_launch": flops, "avg_ms": round(avg, 5), "launches": cnt}
        if b > 0 and avg > 0:
            achieved = b / (avg * 1e-3) / 1e9
            return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_of(name), "kernel": name,
                    "bytes_per_launch": b, "avg_ms": round(avg, 5), "launches": cnt}
    return None


PROFILE_ALL = False  # --profile-all: events around every launch (slower; diagnostics)


def timed(solve_once, K, W, solver, profile):
    import torch
    log("warmup %d" % W)
    for _ in range(W):
        solve_once(-1)
    torch.cuda.synchronize()
    if profile:
        # events bracket the finest level's launches only (the dominant
        # kernels), so the timed region pays for a handful of events per cycle
        solver.profile(True, finest_only=not PROFILE_ALL)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # (no full collection of the interpreter's start-up objects inside the
    # timed region: collect them now and move them out of the generations)
    import gc
    gc.collect()
    gc.freeze()
    torch.cuda.synchronize()
    e0.record()
    results = [solve_once(k) for k in range(K)]
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    timings = solver.kernel_timings() if profile else {}
    solver.profile(False)
    return ms, results, timings


def autotune(args, solver, us, fs, default):
    """Pick the fused 2D kernels' launch shapes by timing them (outside the
    timed region); returns the choices, or None when not tuned."""
    import torch
    on = default if args.autotune == "auto" else args.autotune == "on"
    if not on:
        return None
    t0 = time.time()
    if len(us) == 1 and not hasattr(solver, "ns"):
        choice = solver.autotune(us[0], fs[0], reps=5)
    else:
        choice = solver.autotune(us, fs, reps=5)
    torch.cuda.synchronize()
    log("autotune (%.2f s): %s" % (time.time() - t0, " ".join(
        "n=%d:%s" % (n, "tile" if t else "hb%d" % hb) for n, (hb, t) in sorted(choice.items()))))
    return {"seconds": round(time.time() - t0, 2),
            "choices": {str(n): ("tile32" if t else "march hb=%d" % hb) for n, (hb, t) in sorted(choice.items())}}


def run_single(args, cfg):
    import numpy as np
    import torch

    import paper_1210_7774_amd as M
    from paper_1210_7774_amd import inputs as I

    dim, n = cfg["dim"], (args.n or cfg["n"])
    if dim == 1:
        f_np = I.sine_plus_noise_1d(n, cfg["seed"])
    else:
        f_np = I.normal_rhs(n, dim, cfg["seed"])
    f = torch.from_numpy(f_np).to("cuda")
    # every solve starts from u = 0 (zero_start: the solver does not read the
    # u passed in, so one buffer serves every solve without zeroing it)
    solver = M.Solver(n, dim, precision=cfg["precision"], use_graph=args.graph, zero_start=True)
    K, W = args.steps, args.warmup
    nbuf = 1
    us = [torch.zeros((n,) * dim, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    scratch = torch.zeros((n,) * dim, dtype=torch.float64, device="cuda")
    tune = autotune(args, solver, [scratch], [f], default=True) if dim == 2 else None

    def solve_once(k):
        u = scratch if k < 0 else us[k % nbuf]
        rc, st = solver.solve(u, f, rtol=args.rtol)
        return rc, st.cycles, st.rel_res

    ms, results, timings = timed(solve_once, K, W, solver, not args.no_profile)
    for rc, c, r in results:
        if rc not in (0, 2) or not (r <= args.rtol):
            raise SystemExit("solve failed: status %d cycles %d rel %.3e" % (rc, c, r))
    cycles = results[0][1]
    unknowns = n ** dim
    out = dict(value=unknowns * K / (ms * 1e-3), ms=ms, cycles=cycles, unknowns=unknowns)
    if not args.no_verify:
        import oracle as O
        got = us[-1].cpu().numpy()
        r = O.residual(got, f_np)
        relres = float(np.linalg.norm(r) / np.linalg.norm(f_np))
        log("oracle residual of the returned solution: %.3e" % relres)
        if not relres <= args.rtol * 1.01:
            raise SystemExit("verification failed: oracle residual %.3e" % relres)
    rows = kernel_table(timings) if timings else []
    out["roofline"] = roofline_of(rows) if rows else None
    out["cpu_baseline"] = None
    if tune is not None:
        out["autotune"] = tune
    if not args.no_cpu_baseline and args.config in ("c2", "c3"):
        log("oracle CPU baseline (bounded sample)")
        out["cpu_baseline"] = oracle_baseline(n, dim, cfg["seed"], cycles, 1023 if dim == 2 else 255)
    if not args.no_cpu_baseline and args.config == "c1":
        out["cpu_baseline"] = oracle_c1(f_np, args.rtol)
    if dim == 3 and args.config == "c3" and not args.no_forms:
        out["forms"], out["speedup_vs_f64"] = mixed_forms(args, n, f, f_np, us[-1], ms / K)
    out["workload"] = ("%dD Poisson %d-point, %s interior (%d unknowns), RB-GS V(2,2), full weighting / %s, "
                       "%s FP64 coarsest solve, %s, u0 = 0, rtol %g"
                       % (dim, 2 * dim + 1, "x".join([str(n)] * dim), unknowns,
                          {1: "linear", 2: "bilinear", 3: "trilinear"}[dim], "1-point" if dim == 1 else "3^d",
                          cfg["form"], args.rtol))
    out["dtype"] = {"f64": "f64", "f32": "f32 (FP64 outer)", "bf16": "f32 math, bf16 state (FP64 outer)"}[
        cfg["precision"]]
    out["data"] = "synthetic: %s, seed %d" % ("pi^2 sin(pi x) + U(-1e-3,1e-3)" if dim == 1 else "f ~ N(0,1) i.i.d.",
                                            cfg["seed"])
    return out


def mixed_forms(args, n, f, f_np, u64, ms64):
    """The same 3D problem solved by FP32 V(2,2) cycles inside FP64 iterative
    refinement, and by the same with the cycle's iterate stored as bfloat16:
    unknowns/s to the same FP64 relative residual (checked by the oracle's
    own residual routine), the difference to the FP64 solution, and the
    speedup over the plain FP64 solve timed above."""
    import numpy as np
    import torch

    import paper_1210_7774_amd as M
    forms, speed = {}, {}
    ref = u64.cpu().numpy() if not args.no_verify else None
    K = max(1, min(args.steps, 5))
    forms["f64"] = {"ms": round(ms64, 3), "unknowns_per_s": n ** 3 / (ms64 * 1e-3)}
    for name, prec in (("f32_ir", "f32"), ("bf16_ir", "bf16")):
        solver = M.Solver(n, 3, precision=prec, zero_start=True)
        u = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")

        def solve_once(k):
            rc, st = solver.solve(u, f, rtol=args.rtol)
            return rc, st.cycles, st.rel_res, st.fell_back

        ms, results, _ = timed(solve_once, K, 1, solver, False)
        rc, cyc, rel, fb = results[-1]
        if rc not in (0, 2) or not (rel <= args.rtol):
            raise SystemExit("%s solve failed: status %d cycles %d rel %.3e" % (name, rc, cyc, rel))
        rec = {"ms": round(ms / K, 3), "unknowns_per_s": n ** 3 * K / (ms * 1e-3), "outer_steps": cyc,
               "fell_back": fb, "solver_rel_res": rel}
        if ref is not None:
            import oracle as O
            got = u.cpu().numpy()
            rr = float(np.linalg.norm(O.residual(got, f_np)) / np.linalg.norm(f_np))
            if not rr <= args.rtol * 1.01:
                raise SystemExit("%s verification failed: oracle residual %.3e" % (name, rr))
            rec["oracle_rel_res"] = rr
            rec["rel_diff_vs_f64_solution"] = float(np.abs(got - ref).max() / np.abs(ref).max())
        forms[name] = rec
        speed[name] = round(ms64 / rec["ms"], 3)
        log("%-8s %.3f ms/solve, %d outer steps, %.3f G unknowns/s, speedup %.2fx"
            % (name, rec["ms"], cyc, rec["unknowns_per_s"] / 1e9, speed[name]))
        solver.close()
        del u
    return forms, speed


def run_batch(args):
    import torch

    import paper_1210_7774_amd as M
    from paper_1210_7774_amd import inputs as I

    count = 256
    ns = [int(x) for x in I.batch_sizes(count, 40)]
    log("generating %d coefficient fields" % count)
    coefs = [torch.from_numpy(I.lognormal_coef_2d(n, 4000 + s)).to("cuda") for s, n in enumerate(ns)]
    fs = [torch.from_numpy(I.normal_rhs(n, 2, 4500 + s)).to("cuda") for s, n in enumerate(ns)]
    prec = "f64" if args.config == "c4-f64" else "f32"
    solver = M.BatchSolver(ns, coefs=coefs, precision=prec, use_graph=args.graph)
    K, W = args.steps, args.warmup
    us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for n in ns]
    tune = autotune(args, solver, us, fs, default=True)

    def solve_once(k):
        for u in us:
            u.zero_()
        rc, st = solver.solve(us, fs, rtol=args.rtol)
        return rc, max(s.cycles for s in st), max(s.rel_res for s in st)

    ms, results, timings = timed(solve_once, K, W, solver, not args.no_profile)
    for rc, c, r in results:
        if rc not in (0, 2) or not (r <= args.rtol):
            raise SystemExit("batch solve failed: status %d cycles %d rel %.3e" % (rc, c, r))
    unknowns = sum(n * n for n in ns)
    out = dict(value=unknowns * K / (ms * 1e-3), ms=ms, cycles=results[0][1], unknowns=unknowns)
    if not args.no_verify:
        import numpy as np

        import oracle as O
        worst = 0.0
        for s, n in enumerate(ns):
            f_np = fs[s].cpu().numpy()
            r = O.residual(us[s].cpu().numpy(), f_np, a=coefs[s].cpu().numpy())
            worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(f_np)))
        log("oracle residual of the returned solutions: worst %.3e over %d systems" % (worst, len(ns)))
        if not worst <= args.rtol * 1.01:
            raise SystemExit("batch verification failed: oracle residual %.3e" % worst)
        out["oracle_worst_rel_res"] = worst
    rows = kernel_table(timings) if timings else []
    out["roofline"] = roofline_of(rows) if rows else None
    out["cpu_baseline"] = None
    out["autotune"] = tune
    out["workload"] = ("batch of 256 2D diffusion systems, n from {127,255,511,1023} (seed 40; %d unknowns), "
                       "a = exp(g), g Gaussian field sigma 1, correlation length 1/16; RB-GS V(2,2), %s; "
                       "u zeroed inside the timed region" % (unknowns, "plain FP64" if prec == "f64" else
                                                             "FP32 cycles in FP64 refinement"))
    out["dtype"] = "f64" if prec == "f64" else "f32 (FP64 outer)"
    out["data"] = "synthetic: f ~ N(0,1) seeds 4500+s, coefficients seeds 4000+s"
    return out


def run_jacobi(args):
    """The paper's own fixed-iteration Jacobi benchmark: a 7168 x 7168 FP64
    array, four iterations of the five-point average with a fixed boundary
    (one temporally blocked launch per step); values U(0,1), seed 8."""
    import numpy as np
    import torch

    import paper_1210_7774_amd as M
    from paper_1210_7774_amd import inputs as I

    n = args.n or 7168
    iters = 4
    x = I.uniform_field((n, n), 8)
    inp = torch.from_numpy(x).to("cuda")
    out = torch.empty_like(inp)
    K, W = args.steps, args.warmup
    for _ in range(W):
        M.jacobi5(inp, iters=iters, out=out)
    torch.cuda.synchronize()
    # one launch per step on torch's current stream: events on that stream
    # bracket exactly the kernels
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        M.jacobi5(inp, iters=iters, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    updates = (n - 2) * (n - 2) * iters
    res = dict(value=updates * K / (ms * 1e-3), ms=ms, cycles=iters, unknowns=n * n,
               metric="interior point updates/s of the fixed-iteration Jacobi benchmark", unit="point updates/s")
    avg = ms / K
    b = 16.0 * n * n  # read the array once, write it once
    achieved = b / (avg * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic("jacobi5 n=%d" % n, "traffic_jacobi5.json",
                                                                  ("k_jacobi5.hip", "dev_common.h")),
                       "kernel": "k_jacobi5", "bytes_per_launch": b, "avg_ms": round(avg, 5), "launches": K}
    res["cpu_baseline"] = None
    want = None
    if not args.no_cpu_baseline or not args.no_verify:
        from oracle.jacobi5 import jacobi5 as oracle_jacobi5
        t0 = time.perf_counter()
        want = oracle_jacobi5(x, iters)
        t = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = {"value": updates / t, "unit": "point updates/s", "cores": 1, "kind": "oracle",
                                   "sample": "the whole job (%dx%d, %d iterations) in %.2f s, numpy on one core (%s)"
                                             % (n, n, iters, t, cpu_model())}
    if not args.no_verify:
        if not np.array_equal(out.cpu().numpy(), want):
            raise SystemExit("jacobi5 verification failed: the result differs from the oracle")
        log("jacobi5 result equals the oracle's bit for bit")
    res["workload"] = ("the paper's Jacobi benchmark: %dx%d FP64 array, %d iterations of "
                       "0.2*(centre+up+down+left+right) on the interior, fixed boundary ring" % (n, n, iters))
    res["dtype"] = "f64"
    res["data"] = "synthetic: U(0,1) i.i.d., seed 8"
    res["paper"] = {"seconds_numpy": 3.98, "seconds_score_engine": 2.8, "machine": "Intel i5-2510M (the paper's)",
                    "seconds_here": round(avg * 1e-3, 6)}
    return res


def run_vector(args):
    """The paper's own method on the GPU: a NumPy-style program recorded as
    vector bytecode through the bridge and run by the engine (kernels formed
    by the blockable rule, generated and compiled at run time).
    vjacobi: the paper's Jacobi benchmark, 7168 x 7168 FP64, 4 iterations of
             the five-view loop (work = centre + up + down + left + right,
             times 0.2, copied back: two kernels per iteration), U(0,1) seed 8;
    stencil: the synthetic stencil, 10240 x 1024 FP64, 10 steps of the 3 x 3
             mean into the other of two arrays (one kernel per step), U(0,1)
             seed 9."""
    import numpy as np
    import torch

    import paper_1210_7774_amd.vector as X
    from paper_1210_7774_amd import inputs as I

    jac = args.config == "vjacobi"
    if jac:
        R = C = args.n or 7168
        steps, seed = 4, 8
    else:
        R, C = (args.n or 10240), 1024
        steps, seed = 10, 9
    x = I.uniform_field((R, C), seed)
    t0 = torch.from_numpy(x).to("cuda")
    ta, tb = t0.clone(), t0.clone()
    eng = X.Engine()
    A, B = eng.asarray(ta), eng.asarray(tb)
    nb = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]

    def job():
        nonlocal A, B
        if jac:
            center, up, down = A[1:-1, 1:-1], A[:-2, 1:-1], A[2:, 1:-1]
            left, right = A[1:-1, :-2], A[1:-1, 2:]
            for _ in range(steps):
                work = (((center + up) + down) + left) + right
                work *= 0.2
                center[...] = work
                del work
        else:
            for _ in range(steps):
                views = [A[1 + di:R - 1 + di, 1 + dj:C - 1 + dj] for di, dj in nb]
                acc = views[0] + views[1]
                for v in views[2:]:
                    acc = acc + v
                B[1:-1, 1:-1] = acc / 9.0
                del acc, views
                A, B = B, A
        eng.flush()

    def reset():
        ta.copy_(t0)
        tb.copy_(t0)

    K, W = args.steps, args.warmup
    for _ in range(max(W, 1)):          # the first job compiles the kernels
        reset()
        job()
    torch.cuda.synchronize()
    st0 = eng.stats()
    # the timed region: K whole jobs from the initial array (the reset copy
    # is timed separately and subtracted).  A full collection of the
    # interpreter's start-up objects (torch's modules: tens of ms) would land
    # in it at a random job; collect them now and move them out of the
    # collector's generations (the jobs' own garbage is collected as usual)
    import gc
    gc.collect()
    gc.freeze()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(K):
        reset()
    ev[1].record()
    eng.profile(True)
    ev[2].record()
    for _ in range(K):
        reset()
        job()
    ev[3].record()
    torch.cuda.synchronize()
    prof = eng.profile_read()
    eng.profile(False)
    ms = ev[2].elapsed_time(ev[3]) - ev[0].elapsed_time(ev[1])
    st = eng.stats()
    updates = (R - 2) * (C - 2) * steps
    res = dict(value=updates * K / (ms * 1e-3), ms=ms, cycles=steps, unknowns=R * C, unit="point updates/s",
               metric=("interior point updates/s of the fixed-iteration Jacobi benchmark" if jac else
                       "interior point updates/s of the synthetic stencil"))
    # the dominant generated kernel (events around every launch in the timed region)
    prof.sort(key=lambda r: -r[1] * r[2])
    name, cnt, avg, b = prof[0]
    achieved = b / (avg * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "generated " + name,
                       "bytes_per_launch": b, "avg_ms": round(avg, 5), "launches": cnt}
    res["engine"] = {"kernels_per_job": (st["kernels"] - st0["kernels"]) // K, "compiled": st["compiled"],
                     "stores_elided_per_job": (st["stores_elided"] - st0["stores_elided"]) // K,
                     "compile_ms": round(st["compile_ms"], 1),
                     "kernels": [{"name": n_, "launches": c_, "avg_ms": round(a_, 5), "bytes_per_launch": b_}
                                 for n_, c_, a_, b_ in prof]}
    eng.close()
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline or not args.no_verify:
        if jac:
            from oracle.jacobi5 import jacobi5 as ref
            t_ = time.perf_counter()
            want = ref(x, steps)
        else:
            from oracle.stencil import stencil9 as ref
            t_ = time.perf_counter()
            want = ref(x, steps)
        sec = time.perf_counter() - t_
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = {"value": updates / sec, "unit": "point updates/s", "cores": 1, "kind": "oracle",
                                   "sample": "the whole job (%dx%d, %d steps) in %.2f s, numpy on one core (%s)"
                                             % (R, C, steps, sec, cpu_model())}
        if not args.no_verify:
            got = (ta if jac or steps % 2 == 0 else tb).cpu().numpy()
            if not np.array_equal(got, want):
                raise SystemExit("vector engine verification failed: the result differs from the oracle")
            log("vector engine result equals the oracle's bit for bit")
    if jac:
        import paper_1210_7774_amd as M
        out = torch.empty_like(t0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        M.jacobi5(t0, iters=steps, out=out)
        e0.record()
        for _ in range(K):
            M.jacobi5(t0, iters=steps, out=out)
        e1.record()
        torch.cuda.synchronize()
        hand = updates * K / (e0.elapsed_time(e1) * 1e-3)
        res["comparison"] = {"hand_written_k_jacobi5_updates_per_s": hand,
                             "engine_vs_hand_written": round(res["value"] / hand, 3)}
        res["workload"] = ("the paper's Jacobi benchmark through the vector-bytecode engine: %dx%d FP64, %d "
                           "iterations of the five-view loop (0.2*(centre+up+down+left+right), copied back)"
                           % (R, C, steps))
        res["paper"] = {"seconds_numpy": 3.98, "seconds_score_engine": 2.8,
                        "machine": "Intel i5-2510M (the paper's)", "seconds_here": round(ms / K * 1e-3, 6)}
    else:
        res["workload"] = ("the synthetic stencil through the vector-bytecode engine: %dx%d FP64, %d steps of the "
                           "3x3 mean (nine shifted views) into the other of two arrays" % (R, C, steps))
        res["paper"] = {"seconds_numpy": 6.60, "seconds_score_engine": 4.09, "seconds_mcore_engine": 2.17,
                        "machine": "the paper's CPU", "seconds_here": round(ms / K * 1e-3, 6)}
    res["dtype"] = "f64"
    res["data"] = "synthetic: U(0,1) i.i.d., seed %d" % seed
    return res


def run_lstep(args):
    """The solver's fused learned step alone (mg_learned_step) at 1023^2 with
    He-normal weights (seed 7000), log-normal coefficients (seed 5000), N(0,1)
    rhs (seed 5001), FP32 state (bf16 state with --precision-bf16); priced
    against the dense bf16 MFMA peak."""
    import ctypes

    import numpy as np
    import torch

    from paper_1210_7774_amd import _abi
    from paper_1210_7774_amd import inputs as I

    L = _abi.lib()
    n = args.n or 1023
    st = args.lstep_state
    a = torch.from_numpy(I.lognormal_coef_2d(n, 5000).astype(np.float32)).to("cuda")
    f = torch.from_numpy(I.normal_rhs(n, 2, 5001).astype(np.float32)).to("cuda")
    w = torch.from_numpy(I.he_normal_weights(7000)).to("cuda")
    dt = torch.float32 if st == "f32" else torch.bfloat16
    e = [torch.zeros(n, n, dtype=dt, device="cuda") for _ in range(2)]
    nb = L.mg_learned_scratch_bytes(1, 3)
    scratch = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    prec = _abi.MG_P_F32_IR if st == "f32" else _abi.MG_P_F32_BF16_IR
    P = lambda t: ctypes.c_void_p(t.data_ptr())

    # every step from the same iterate (a random one of the size of a smoothed
    # error), so each launch sees the same values
    e[0].copy_(torch.from_numpy(1e-3 * I.normal_rhs(n, 2, 5002)).to(dt))

    def step(k):
        rc = L.mg_learned_step(P(e[0]), P(e[1]), P(f), P(a), n, prec, P(w), P(scratch), nb, sp)
        if rc != _abi.MG_OK:
            raise SystemExit("mg_learned_step failed: %s" % L.mg_last_error(None).decode())

    K, W = args.steps * 10, args.warmup * 10
    for k in range(W):
        step(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(K):
        step(k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    avg = ms / K
    flops = LEARNED_FLOP_PER_PX * n * n
    achieved = flops / (avg * 1e-3) / 1e12
    res = dict(value=n * n * K / (ms * 1e-3), ms=ms / 10 * 1.0, cycles=K, unknowns=n * n, unit="pixel steps/s",
               metric="pixel updates/s of the fused learned step")
    res["roofline"] = {"bound": "mfma", "achieved": round(achieved, 2), "peak": MFMA_BF16_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 5), "traffic": None,
                       "kernel": "k_lstep_march", "flop_per_launch": flops, "avg_ms": round(avg, 5), "launches": K}
    res["cpu_baseline"] = None
    res["workload"] = ("the fused learned step (scaled residual, 1->16->16->16->1 3x3 convolutions on MFMA, "
                       "update) on a %dx%d 2D diffusion problem, %s state" % (n, n, st))
    res["dtype"] = "bf16 MFMA, FP32 accumulation (%s state)" % st
    res["data"] = "synthetic: He-normal weights seed 7000, a = exp(g) seed 5000, f ~ N(0,1) seed 5001"
    return res


def run_learned(args):
    """c5: train the network on the GPU, then time learned and plain solves of
    a held-out problem (coefficient seed 5000, rhs seed 5001)."""
    import numpy as np
    import torch

    import paper_1210_7774_amd as M
    import paper_1210_7774_amd.learned as L
    from paper_1210_7774_amd import inputs as I

    n = args.n or 1023
    a_np = I.lognormal_coef_2d(n, 5000)
    f_np = I.normal_rhs(n, 2, 5001)
    a = torch.from_numpy(a_np).to("cuda")
    f = torch.from_numpy(f_np).to("cuda")
    if args.weights:
        w = torch.from_numpy(np.load(args.weights).astype(np.float32)).to("cuda")
        train_info = {"weights": os.path.basename(args.weights)}
    else:
        t0 = time.time()
        log("generating %d training problems (n=%d)" % (args.c5_problems, n))
        probs = [(I.lognormal_coef_2d(n, 6000 + i), I.normal_rhs(n, 2, 6100 + i)) for i in range(args.c5_problems)]
        t1 = time.time()
        S, E, A = L.make_pairs(probs, cycles=10, crops=args.c5_crops, patch=64, seed=7200,
                               stages=("pre", "post", "noise"))
        torch.cuda.synchronize()
        t2 = time.time()
        log("pairs: %d in %.1f s; training %d epochs" % (S.shape[0], t2 - t1, args.c5_epochs))
        w = L.jacobi_start(0.8, 7001, 0.01)
        res = L.train(S, E, A, w, epochs=args.c5_epochs, batch=32, border=5, lr=1e-4)
        log("loss per epoch: " + " ".join("%.4f" % x for x in res.loss_hist))
        train_info = {"pairs": int(S.shape[0]), "epochs": args.c5_epochs, "adam_steps": res.steps,
                      "start": "damped-Jacobi network + 0.01 He noise", "lr": 1e-4,
                      "stages": "pre, post, noise",
                      "train_ms": round(res.ms, 1), "pairs_s": round(t2 - t1, 2), "problems_s": round(t1 - t0, 2),
                      "loss_first_epoch": round(res.loss_hist[0], 5), "loss_last_epoch": round(res.loss_hist[-1], 5)}
        del S, E, A
        if args.save_weights:
            np.save(args.save_weights, w.cpu().numpy())
    K, W = args.steps, args.warmup
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    forms = {}
    for name, kw in (("plain", dict(smoother="rbgs")), ("learned", dict(smoother="learned", learned=w))):
        solver = M.Solver(n, 2, a=a, precision="f32", use_graph=args.graph, max_cycles=200, **kw)
        per_tol = {}
        for rtol in (1e-8, args.rtol):
            def solve_once(k, rtol=rtol):
                u.zero_()
                rc, st = solver.solve(u, f, rtol=rtol)
                return rc, st.cycles, st.rel_res, st.rho_avg, st.fell_back
            prof = (not args.no_profile) and rtol == args.rtol
            ms, results, timings = timed(solve_once, K, W, solver, prof)
            rc, cyc, rel, rho, fb = results[-1]
            if rc not in (0, 2) or not (rel <= rtol):
                raise SystemExit("%s solve failed: status %d cycles %d rel %.3e" % (name, rc, cyc, rel))
            if not args.no_verify:
                import oracle as O
                got = u.cpu().numpy()
                rr = float(np.linalg.norm(O.residual(got, f_np, a=a_np)) / np.linalg.norm(f_np))
                if not rr <= rtol * 1.01:
                    raise SystemExit("%s verification failed: oracle residual %.3e" % (name, rr))
            per_tol[rtol] = dict(ms=ms / K, cycles=cyc, rho=rho, fell_back=fb, timings=timings)
            log("%-8s rtol %g: %.3f ms/solve, %d cycles, rho %.4f, fell_back %d"
                % (name, rtol, ms / K, cyc, rho, fb))
        forms[name] = per_tol
        solver.close()
    lt = forms["learned"][args.rtol]
    pl = forms["plain"][args.rtol]
    rows = kernel_table(lt["timings"]) if lt["timings"] else []
    out = dict(value=n * n / (lt["ms"] * 1e-3), ms=lt["ms"] * K, cycles=lt["cycles"], unknowns=n * n)
    # one timing launch of the learned class = nu (2) fused steps over n^2 pixels
    out["roofline"] = roofline_of(rows, learned_px_per_launch=2 * n * n) if rows else None
    out["cpu_baseline"] = None
    out["comparison"] = {
        name: {("%g" % t): {"ms": round(v["ms"], 4), "cycles": v["cycles"], "rho": round(v["rho"], 4),
                            "fell_back": v["fell_back"]} for t, v in forms[name].items()} for name in forms}
    out["speedup_vs_plain"] = {("%g" % t): round(forms["plain"][t]["ms"] / forms["learned"][t]["ms"], 3)
                               for t in forms["plain"]}
    out["training"] = train_info
    out["plain_value"] = n * n / (pl["ms"] * 1e-3)
    out["workload"] = ("2D diffusion %dx%d, a = exp(g), g Gaussian field sigma 1, correlation length 1/16 "
                       "(seed 5000), f ~ N(0,1) (seed 5001); V(2,2) whose finest-level sweeps are learned steps "
                       "(4-layer 3x3 conv, 16 channels, bf16, trained here), FP32 cycles in FP64 refinement; "
                       "value = learned solve to rtol %g" % (n, n, args.rtol))
    out["dtype"] = "f32 (FP64 outer); bf16 network"
    out["data"] = "synthetic: held-out seeds 5000/5001; training problems seeds 6000+i/6100+i"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="grid size (default: the configuration's)")
    ap.add_argument("--config", default="c3", choices=["c2", "c3", "c3-f32", "c3-bf16", "c4", "c4-f64", "c1", "c5", "jacobi", "vjacobi",
                                                        "stencil", "lstep"])
    ap.add_argument("--lstep-state", default="f32", choices=["f32", "bf16"], help="lstep: the state type")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--autotune", default="auto", choices=["auto", "on", "off"],
                    help="time the 2D launch shapes before the timed region (auto: on for 2D)")
    ap.add_argument("--graph", action="store_true", help="replay each cycle as a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="c3: skip the FP32 / bf16-state refinement solves")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--profile-all", action="store_true",
                    help="events around every launch, not only the finest level's (adds ~20%% to the time)")
    ap.add_argument("--c5-problems", type=int, default=20, help="c5: training problems")
    ap.add_argument("--c5-crops", type=int, default=34, help="c5: crops per problem, cycle and stage")
    ap.add_argument("--c5-epochs", type=int, default=30, help="c5: training epochs")
    ap.add_argument("--weights", default="", help="c5: load trained weights (.npy) instead of training")
    ap.add_argument("--save-weights", default="", help="c5: save the trained weights (.npy)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM counters) and exit")
    args = ap.parse_args()

    global PROFILE_ALL
    PROFILE_ALL = args.profile_all
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU only (it has no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        import torch
        nel = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nel * 8}))
        return

    if args.config.startswith("c4"):
        r = run_batch(args)
    elif args.config == "c5":
        r = run_learned(args)
    elif args.config == "jacobi":
        r = run_jacobi(args)
    elif args.config in ("vjacobi", "stencil"):
        r = run_vector(args)
    elif args.config == "lstep":
        r = run_lstep(args)
    else:
        r = run_single(args, CONFIGS[args.config])
    K = args.steps
    out = {
        "metric": r.get("metric", METRIC),
        "value": r["value"],
        "unit": r.get("unit", "unknowns/s"),
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": r["data"],
        "config": {"workload": r["workload"], "config": args.config, "cycles": r["cycles"],
                   "unknowns": r["unknowns"], "graph": bool(args.graph)},
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu_baseline"],
    }
    for key in ("comparison", "speedup_vs_plain", "training", "plain_value", "autotune", "paper", "forms",
                "speedup_vs_f64", "oracle_worst_rel_res", "engine"):
        if key in r:
            out[key] = r[key]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
