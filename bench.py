#!/usr/bin/env python3
"""Throughput benchmark of the grid potential-flow solve on one MI355X.

Workload (one step = one full solve): flat plate of chord 1 at 20 deg,
Ns = 256 surface points, Kutta condition at both edges with one new vortex
per edge; 512 x 512 grid, dx = 0.005; 1e4 vortices from a Gaussian blob
behind the trailing edge.  The solve is R_v -> L^-1 -> E_s -> Schur and edge
constraints -> R_s -> L^-1 -> E_v.  The plan (LGF table, spectrum) and the
body (S^-1, f0) are resident; inputs are in HBM before the timed region.

Prints one JSON line: grid points solved per second (n^2 per full solve),
per-step latency p50/p99, the roofline of the dominant kernel from HIP
events on the launch stream, and the FP64 CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid points solved/sec (R -> L^-1 -> E) at FP32 vs plain; p50/p99 latency"


def kernel_bytes(n: int, nv: int, ns: int, m: int, w_fp64: bool) -> dict:
    """Algorithmic HBM bytes per launch of each kernel class.

    Convolution passes move their input and output once: pass 1 reads the
    n x n source and writes the n x (n+1) half spectrum; pass 2 reads and
    writes it and reads the (n+1)^2 real spectrum; pass 3 reads it and
    writes the n x n field.  FP32 complex = 8 B, FP64 complex = 16 B.
    """
    win = 8 if w_fp64 else 4
    return {
        "scatter": 24 * nv + 16 * 2 * win * nv,          # positions+strength, 16 RMW
        "rows_fwd": win * n * n + 8 * n * (n + 1),
        "cols": 16 * n * (n + 1) + 4 * (n + 1) ** 2,
        "rows_inv": 8 * n * (n + 1) + 4 * n * n,
        "rows_fwd64": 8 * n * n + 16 * n * (n + 1),
        "cols64": 32 * n * (n + 1) + 8 * (n + 1) ** 2,
        "rows_inv64": 16 * n * (n + 1) + 8 * n * n,
        "surface": 8 * ns * ns + 8 * ns * (4 + 3 * (1 + m)),
        "velocity": 24 * nv + 16 * nv,
    }


def cpu_baseline(case, budget_s: float = 12.0) -> dict:
    """The FP64 oracle, single-threaded, on a bounded sample of full solves."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.body import body_setup
    from oracle.lgf import lgf_table
    from oracle.operators import Grid
    from oracle.solve import Problem, solve

    with threadpool_limits(limits=1):
        grid = Grid.centered(case.n, case.dx)
        table = lgf_table(case.n)
        sf = case.surface
        body = body_setup(grid, sf.xs, sf.ys, sf.ds, table)
        p = Problem(grid=grid, X=case.X, Y=case.Y, G=case.G, u_inf=case.u_inf,
                    v_inf=case.v_inf, mode=case.mode, gamma_b=case.gamma_b,
                    edges=tuple(case.edges), znew=tuple(case.znew))
        solve(p, body, table)            # warm caches
        t0 = time.perf_counter()
        k = 0
        while True:
            solve(p, body, table)
            k += 1
            el = time.perf_counter() - t0
            if el >= budget_s or k >= 1000:
                break
    return {"value": case.n * case.n * k / el, "unit": "grid points/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{k} full solves of the same 512^2 plate workload (FP64 NumPy, one "
                      f"thread; plan and body set up beforehand), {el:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent problems shard one per GPU with no exchange).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2102_11910_amd import gpf
    from paper_2102_11910_amd import workloads as wl

    case = wl.config2()
    n = case.n
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] setup: {case.name}, nv={case.nv}, ns={case.surface.ns}")
    ctx = gpf.Context(0)
    t0 = time.perf_counter()
    solver = gpf.Solver(ctx, n, case.dx, case.surface, flags=gpf.GPF_POLICY_AUTO)
    info = solver.body.info()
    log(f"[bench] plan+body {time.perf_counter() - t0:.2f} s, body {info}")
    X, Y, G = solver.upload(case)
    inp = solver.inputs_for(case, X, Y, G)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.solve(inp, X)
    gpf.gpf_sync(solver.status)
    torch.cuda.synchronize()

    # timed region: K full solves, kernel classes bracketed by HIP events on
    # the launch stream, one event per step boundary for latency
    K = args.steps
    gpf.timing_enable(solver.plan, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        solver.solve(inp, X)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpf.gpf_sync(solver.status)
    kt = gpf.timing_read(solver.plan)
    gpf.timing_enable(solver.plan, False)
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])

    # same region without the kernel events (their cost is reported)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(K):
        solver.solve(inp, X)
    torch.cuda.synchronize()
    wall_noev = time.perf_counter() - t1

    ms_per_step = 1e3 * wall / K
    value = n * n * K / wall
    m = len(case.znew)
    w_fp64 = info["conv1_fp64"]
    kb = kernel_bytes(n, case.nv, case.surface.ns, m, w_fp64)
    per_kernel = {}
    for name, (cnt, ms) in kt.items():
        if cnt:
            avg_ms = ms / cnt
            per_kernel[name] = {"launches": cnt, "avg_us": 1e3 * avg_ms,
                                "share": ms / (1e3 * wall),
                                "GBps": kb[name] / (avg_ms * 1e-3) / 1e9}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"] * per_kernel[k]["launches"])
    d = per_kernel[dom]
    achieved = d["GBps"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": kb[dom], "avg_us": round(d["avg_us"], 3)}
    log("[bench] kernels: " + json.dumps({k: {kk: round(vv, 3) for kk, vv in v.items()}
                                          for k, v in per_kernel.items()}))

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "flat plate c=1 at 20 deg, Ns=256, Kutta at both edges with "
                               "new vortices; 512^2 grid dx=0.005; 1e4 vortices (Gaussian blob)",
                   "n": n, "nv": case.nv, "ns": case.surface.ns, "path": "plain",
                   "precision": "FP32 fields; FP64 first convolution (noise amplification "
                                f"{info['amp']:.3g} > 500), FP64 Schur/constraints"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "value_without_kernel_events": n * n * K / wall_noev,
        "roofline": roofline,
        "kernels": {k: {"avg_us": round(v["avg_us"], 3), "GBps": round(v["GBps"], 1),
                        "launches": v["launches"]} for k, v in per_kernel.items()},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host ...")
        res["cpu_baseline"] = cpu_baseline(case, args.cpu_budget)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
