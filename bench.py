#!/usr/bin/env python3
"""Benchmark: unknowns/s of a full multigrid solve to a 1e-10 relative
residual on one MI355X.

Default workload: 2D Poisson, 5-point stencil on the unit square, 4095 x 4095
interior grid (16,769,025 unknowns), FP64, rhs i.i.d. N(0,1) (seed 2), red-black
Gauss-Seidel V(2,2), full weighting / bilinear transfers, 3x3 FP64 direct
coarsest solve.  One "step" is one complete solve from u = 0 to
||f - A u||_2 / ||f||_2 <= 1e-10 (every level operation of every cycle, the
stop test included), inputs resident in HBM.

Prints ONE JSON line (rank 0 only; this build runs on one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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


def oracle_baseline(f_np, cycles, n):
    """The oracle (plain C, one thread) on a bounded sample of the same
    workload: one V(2,2) cycle plus one residual norm on the full grid;
    the full solve is taken as `cycles` such units."""
    import numpy as np

    import oracle as O
    u = np.zeros_like(f_np)
    t0 = time.perf_counter()
    O.vcycle(u, f_np)
    r = O.residual(u, f_np)
    _ = float(np.sqrt((r * r).sum()))
    t = time.perf_counter() - t0
    per_solve = t * cycles
    return {"value": n * n / per_solve, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": "1 V(2,2) cycle + 1 residual norm on the %dx%d grid in %.1f s on one core (%s); "
                      "full solve = %d such cycles" % (n, n, t, cpu_model(), cycles)}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        csrc = os.path.join(ROOT, "paper_1210_7774_amd", "csrc")
        h = hashlib.sha256()
        for fn in ("k_march2d.inc", "k_march2d_f64.hip", "dev_common.h", "mg_internal.h"):
            h.update(open(os.path.join(csrc, fn), "rb").read())
        if h.hexdigest()[:16] != rec["source_hash"] or kernel not in rec["kernels"]:
            return None
        k = rec["kernels"][kernel]
        return k["read_bytes"] + k["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4095)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--graph", action="store_true", help="replay each cycle as a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM counters) and exit")
    args = ap.parse_args()

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

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the solver has no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1210_7774_amd as M
    from paper_1210_7774_amd import inputs as I

    n = args.n
    f_np = I.normal_rhs(n, 2, 2)
    f = torch.from_numpy(f_np).to("cuda")
    solver = M.Solver(n, 2, use_graph=args.graph)
    K, W = args.steps, args.warmup
    us = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for _ in range(K)]
    scratch = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    log("warmup %d solve(s)" % W)
    for _ in range(W):
        scratch.zero_()
        solver.solve(scratch, f, rtol=args.rtol)
    torch.cuda.synchronize()

    if not args.no_profile:
        solver.profile(True)
    stats = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(K):
        rc, st = solver.solve(us[k], f, rtol=args.rtol)
        stats.append((rc, st.cycles, st.rel_res))
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    timings = solver.kernel_timings() if not args.no_profile else {}
    solver.profile(False)
    log("timed %d solves: %.3f ms (events) / %.3f ms (wall)" % (K, ms, wall * 1e3))
    for rc, c, r in stats:
        if rc != 0 or not (r <= args.rtol):
            raise SystemExit("solve failed: status %d cycles %d rel %.3e" % (rc, c, r))
    cycles = stats[0][1]

    # per-kernel table and the dominant kernel's roofline
    if not timings:
        print(json.dumps({"ms_per_step": ms / K, "value": n * n * K / (ms * 1e-3), "cycles": cycles}), flush=True)
        return
    rows = sorted(timings.items(), key=lambda kv: -kv[1][0] * kv[1][1])
    tot = sum(v[0] * v[1] for v in timings.values())
    log("%-24s %8s %10s %10s %9s %7s" % ("kernel", "launches", "avg_us", "MB/launch", "GB/s", "share"))
    for name, (cnt, avg, b) in rows:
        gbs = b / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        log("%-24s %8d %10.2f %10.2f %9.1f %6.1f%%" % (name, cnt, avg * 1e3, b / 1e6, gbs, 100 * cnt * avg / tot))
    dom_name, (dom_cnt, dom_avg, dom_bytes) = rows[0]
    achieved = dom_bytes / (dom_avg * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom_name), "kernel": dom_name,
                "bytes_per_launch": dom_bytes, "avg_ms": round(dom_avg, 5), "launches": dom_cnt}

    if not args.no_verify:
        import oracle as O
        got = us[0].cpu().numpy()
        r = O.residual(got, f_np)
        relres = float(np.linalg.norm(r) / np.linalg.norm(f_np))
        log("oracle residual of the returned solution: %.3e" % relres)
        if not relres <= args.rtol * 1.01:
            raise SystemExit("verification failed: oracle residual %.3e" % relres)

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline (bounded sample)")
        cpu = oracle_baseline(f_np, cycles, n)

    value = n * n * K / (ms * 1e-3)
    out = {
        "metric": "unknowns/s solved to 1e-10 rel. residual; mixed/learned vs plain FP64",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: f ~ N(0,1) i.i.d., seed 2",
        "config": {"workload": "2D Poisson 5-point, %dx%d interior (%d unknowns), RB-GS V(2,2), full weighting/"
                               "bilinear, 3x3 FP64 coarsest solve, plain FP64, u0 = 0, rtol %g"
                               % (n, n, n * n, args.rtol),
                   "cycles": cycles, "form": "plain FP64", "graph": bool(args.graph)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
