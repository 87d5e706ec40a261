#!/usr/bin/env python3
"""Throughput benchmark of the grid potential-flow solve on one MI355X.

Workload: flat plate of chord 1 at 20 deg, Ns = 256 surface points, Kutta
condition at both edges with one new vortex per edge; 512 x 512 grid,
dx = 0.005; 1e4 vortices from a Gaussian blob behind the trailing edge.
One full solve is R_v -> L^-1 -> E_s -> Schur and edge constraints -> R_s
-> L^-1 -> E_v.  A step solves a batch of such problems (different vortex
seeds around the same plate) in shared launches; the plain path (one solve
per step, one launch per stage) is timed beside it.  The plan (LGF table,
spectrum) and the body (S^-1, f0) are resident; inputs are in HBM before
the timed region.

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


def kernel_bytes(n: int, nv: int, ns: int, m: int, w_fp64: bool, keep: float = 1.0) -> dict:
    """Algorithmic HBM bytes per launch of each kernel class.

    Convolution passes move their input and output once: pass 1 reads the
    n x n source and writes the n x (n+1) half spectrum; pass 2 reads and
    writes it and reads the (n+1)^2 real spectrum; pass 3 reads it and
    writes the n x n field.  FP32 complex = 8 B, FP64 complex = 16 B.  The
    first (FP64) convolution feeds only the surface stencils: its column
    pass writes, and its last pass reads and writes, the fraction `keep` of
    the rows.
    """
    win = 8 if w_fp64 else 4
    return {
        "scatter": 24 * nv + 16 * 2 * win * nv,          # positions+strength, 16 RMW
        "rows_fwd": win * n * n + 8 * n * (n + 1),
        "cols": 16 * n * (n + 1) + 4 * (n + 1) ** 2,
        "rows_inv": 8 * n * (n + 1) + 4 * n * n,
        "rows_fwd64": 8 * n * n + 16 * n * (n + 1),
        "cols64": 16 * n * (n + 1) * (1 + keep) + 8 * (n + 1) ** 2,
        "rows_inv64": keep * (16 * n * (n + 1) + 8 * n * n),
        "surface": 8 * ns * ns + 8 * ns * (4 + 3 * (1 + m)),
        "velocity": 24 * nv + 16 * nv,
    }


def kept_rows(case) -> float:
    """Fraction of grid rows the first convolution keeps: the rows of the
    surface stencils (base row floor(eta) - 1 to + 3), widened to whole
    16-row groups."""
    import numpy as np
    eta = (np.asarray(case.surface.ys, np.float64) - case.x0) / case.dx
    lo = int(np.floor(eta).min()) - 1
    hi = int(np.floor(eta).max()) + 2
    lo, hi = lo & ~15, min(case.n - 1, hi | 15)
    return (hi - lo + 1) / case.n


# kernel class -> (source file, kernel-name prefixes in a profiler trace)
KERNEL_SOURCES = {
    "scatter": ("transfer.hip", ("k_bin_count", "k_bin_place", "k_tile_scatter")),
    "rows_fwd": ("fft_conv.hip", ("k_rows_fwd<double, float",)),
    "cols": ("fft_conv.hip", ("k_cols_conv<float",)),
    "rows_inv": ("fft_conv.hip", ("k_rows_inv<float",)),
    "rows_fwd64": ("fft_conv.hip", ("k_rows_fwd<double, double",)),
    "cols64": ("fft_conv.hip", ("k_cols_conv<double", "k_cols_conv_split<double")),
    "rows_inv64": ("fft_conv.hip", ("k_rows_inv<double",)),
    "surface": ("schur.hip", ("k_surface_rhs", "k_schur_apply")),
    "velocity": ("transfer.hip", ("k_vortex_velocity",)),
}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "plate512_batch32_hbm_traffic.md")
COPY_BYTES = 1 << 28   # calibration copy: 256 MiB read + 256 MiB written


def source_hash(fname: str) -> str:
    """Hash of a kernel source file and of the descriptor structs its
    kernels read (ConvDesc, ProbDesc, SolveScalars in gpf_internal.h)."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2102_11910_amd", "csrc")
    with open(os.path.join(csrc, fname), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "gpf_internal.h")) as fh:
        hdr = fh.read()
    structs = ("ConvDesc",) if fname == "fft_conv.hip" else ("ConvDesc", "ProbDesc", "SolveScalars")
    for name in structs:
        mt = re.search(r"struct %s \{.*?\n\};" % name, hdr, re.S)
        h.update(mt.group(0).encode() if mt else b"")
    return h.hexdigest()[:16]


def _pmc_rows(d: str):
    import csv
    import glob
    fs = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not fs:
        raise SystemExit(f"no counter_collection.csv under {d}")
    with open(fs[0]) as fh:
        return list(csv.DictReader(fh))


def summarize_pmc(fetch_dir: str, write_dir: str, command: str) -> None:
    """Writes the HBM-traffic summary from two rocprofv3 --pmc runs of
    `bench.py --pmc-workload` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).
    Bytes are scaled by what each counter reads for the calibration copy."""
    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            acc.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        return ({k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()},
                {k: max(v) for k, v in acc.items()})

    fetch, cnt, fetch_max = per_kernel(_pmc_rows(fetch_dir), "FETCH_SIZE")
    write, _, write_max = per_kernel(_pmc_rows(write_dir), "WRITE_SIZE")
    # the calibration copy is the largest dispatch of a copy kernel
    copy = [k for k in fetch if "copy" in k.lower()]
    copy_k = max(copy, key=lambda k: fetch_max[k])
    ff, fw = fetch_max[copy_k] / COPY_BYTES, write_max.get(copy_k, COPY_BYTES) / COPY_BYTES
    lines = ["# HBM traffic per launch, 512^2 plate workload, batch of 32 problems", "",
             "Two rocprofv3 counter runs of the batched step (FETCH_SIZE, then WRITE_SIZE),",
             "each scaled by the reading of the same counter for a 256 MiB device copy.", "",
             f"command_fetch: {command.format(counter='FETCH_SIZE', out=fetch_dir)}",
             f"command_write: {command.format(counter='WRITE_SIZE', out=write_dir)}",
             f"copy_kernel: {copy_k}",
             f"copy_factor_fetch: {ff:.4f}", f"copy_factor_write: {fw:.4f}", ""]
    for cls, (src, prefixes) in KERNEL_SOURCES.items():
        ks = [k for k in fetch if any(p in k for p in prefixes)]
        if not ks:
            continue
        fb = sum(fetch[k] for k in ks) / ff
        wb = sum(write.get(k, 0.0) for k in ks) / fw
        matched = ",".join(p.replace(" ", "") for p in prefixes if any(p in k for k in ks))
        lines.append(f"class {cls}: fetch_bytes={fb:.0f} write_bytes={wb:.0f} "
                     f"source={src}@{source_hash(src)} kernels={len(ks)} matched={matched}")
    lines += ["", "| kernel | dispatches | FETCH (MB, raw) | WRITE (MB, raw) |", "|---|---|---|---|"]
    for k in sorted(fetch, key=lambda k: -fetch[k]):
        lines.append(f"| {k[:90]} | {cnt[k]} | {fetch[k] / 1e6:.2f} | {write.get(k, 0) / 1e6:.2f} |")
    with open(TRAFFIC_SUMMARY, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", TRAFFIC_SUMMARY)


def measured_traffic(cls: str, kernel_prefix=None):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None when it is absent, the kernel source changed since, or
    (kernel_prefix given) the counters belong to another kernel of the class
    than the one the timed run launched."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    src, _ = KERNEL_SOURCES[cls]
    with open(TRAFFIC_SUMMARY) as fh:
        for line in fh:
            if line.startswith(f"class {cls}:"):
                kv = dict(t.split("=", 1) for t in line.split(":", 1)[1].split() if "=" in t)
                if kv.get("source") != f"{src}@{source_hash(src)}":
                    return None
                if kernel_prefix is not None and kv.get("matched") != kernel_prefix.replace(" ", ""):
                    return None
                return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


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


def conv_roofline(gpf, torch, np, ctx, log, sizes=(1024, 2048), reps=20):
    """The LGF convolution alone (three passes, FP32) on large grids: achieved
    algorithmic GB/s (44 n^2 bytes per convolution) from HIP events."""
    out = {}
    for n in sizes:
        plan = gpf.Plan(ctx, n, 2.56 / n)
        g = torch.Generator(device="cpu").manual_seed(n)
        w = torch.randn((n, n), generator=g, dtype=torch.float32).to("cuda")
        s = torch.empty_like(w)
        gam = float(w.double().sum()) * (2.56 / n) ** 2
        for _ in range(3):
            gpf.gpf_convolve(plan, w, s, gam)
        torch.cuda.synchronize()
        gpf.timing_enable(plan, True)
        for _ in range(reps):
            gpf.gpf_convolve(plan, w, s, gam)
        kt = gpf.timing_read(plan)
        gpf.timing_enable(plan, False)
        kb = kernel_bytes(n, 0, 0, 0, False)
        passes, tot_us = {}, 0.0
        for name in ("rows_fwd", "cols", "rows_inv"):
            cnt, ms = kt[name]
            us = 1e3 * ms / cnt
            tot_us += us
            passes[name] = {"avg_us": round(us, 3), "GBps": round(kb[name] / (us * 1e-6) / 1e9, 1)}
        conv_bytes = kb["rows_fwd"] + kb["cols"] + kb["rows_inv"]
        gbps = conv_bytes / (tot_us * 1e-6) / 1e9
        out[str(n)] = {"us": round(tot_us, 2), "bytes": conv_bytes, "GBps": round(gbps, 1),
                       "frac_of_8TBps": round(gbps / HBM_PEAK_GBS, 4), "passes": passes}
        log(f"[bench] convolution {n}^2: {tot_us:.1f} us, {gbps:.0f} GB/s {passes}")
        del plan
    return out


def rk2_leg(gpf, torch, np, ctx, log, wl, steps=100):
    """Explicit-midpoint advection of the 1024^2 ellipse workload (1e5
    vortices), 100 steps (200 solves) from the same start: the step captured
    as one graph and launched eagerly (FP32 fields under the precision
    policy), and the plain FP64 path (every kernel in FP64, eager); ms per
    step of each and the final position difference of the FP32 graph run
    against the FP64 one (the dynamics is chaotic: a difference, not a
    parity check)."""
    case = wl.config3()
    dt = case.extra.get("dt", 0.5 * case.dx)
    dev = torch.device("cuda", 0)
    out = {"workload": f"{case.name}, nv={case.nv}, dt={dt}", "steps": steps}
    finals = {}
    for name, flags, use_graph in (("graph", gpf.GPF_POLICY_AUTO, True),
                                   ("eager", gpf.GPF_POLICY_AUTO, False),
                                   ("fp64_plain", gpf.GPF_FP64, False)):
        plan = gpf.Plan(ctx, case.n, case.dx, flags=flags)
        body = gpf.Body(plan, case.surface.xs, case.surface.ys, case.surface.ds)
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev)
        X, Y, G = t(case.X), t(case.Y), t(case.G)
        inp = gpf.make_inputs(X, Y, G, case.u_inf, case.v_inf, case.ub, case.vb, case.omega,
                              case.mode, case.gamma_b)
        # warm-up on a copy, then the timed run from the initial state
        Xw, Yw = X.clone(), Y.clone()
        rkw = gpf.Rk2(plan, body, inp, Xw, Yw, dt, use_graph=use_graph)
        rkw.run(2)
        rkw.sync()
        rkw.close()
        rk = gpf.Rk2(plan, body, inp, X, Y, dt, use_graph=use_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rk.run(steps)
        try:
            rk.sync()
        except gpf.GpfError as e:       # a vortex left the window: report, do not time
            out[f"{name}_error"] = str(e)
            rk.close()
            return out
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        out[f"{name}_ms_per_step"] = ms
        finals[name] = (X.cpu().numpy(), Y.cpu().numpy())
        log(f"[bench] rk2 {name}: {ms:.3f} ms/step")
        rk.close()
    xg, yg = finals["graph"]
    x64, y64 = finals["fp64_plain"]
    moved = float(np.max(np.hypot(x64 - case.X, y64 - case.Y)))
    out["final_position_diff_graph_vs_fp64"] = float(np.max(np.hypot(xg - x64, yg - y64)))
    out["max_displacement"] = moved
    return out


def shed_leg(gpf, torch, np, ctx, log, wl, steps=200):
    """Forward Euler shedding on the 512^2 plate (1e4 vortices, a new vortex
    at each edge per step, Kutta at both): ms per step with the state
    resident on the device."""
    case = wl.config2()
    dt = 0.0005      # the blob stays inside the window over the timed steps
    plan = gpf.Plan(ctx, case.n, case.dx, flags=gpf.GPF_POLICY_AUTO)
    sf = case.surface
    body = gpf.Body(plan, sf.xs, sf.ys, sf.ds, case.edges)
    dev = torch.device("cuda", 0)
    warm = 5
    cap = case.nv + 2 * (warm + steps)
    pad = lambda a: torch.as_tensor(np.r_[np.asarray(a, np.float64), np.zeros(cap - case.nv)],
                                    dtype=torch.float64).to(dev)
    X, Y, G = pad(case.X), pad(case.Y), pad(case.G)
    u = torch.zeros(cap, dtype=torch.float64, device=dev)
    v = torch.zeros(cap, dtype=torch.float64, device=dev)
    psi = torch.empty((case.n, case.n), dtype=plan.field_dtype, device=dev)
    sc = torch.zeros(gpf.N_SCALARS, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    inp = gpf.make_inputs(X, Y, G, case.u_inf, case.v_inf, 0.0, 0.0, 0.0, "shed", 0.0, case.znew)
    inp.nv = case.nv
    out = gpf.make_outputs(psi, u, v, None, None, sc, status)
    first = [(z[0] - sf.xs[k], z[1] - sf.ys[k]) for z, k in zip(case.znew, case.edges)]
    sh = gpf.Shed(plan, body, inp, out, X, Y, G, dt, first)
    sh.run(warm)
    sh.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sh.run(steps)
    sh.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    log(f"[bench] shedding: {ms:.3f} ms/step, {sh.nv} vortices at the end")
    res = {"workload": f"{case.name}, nv={case.nv}+2/step, dt={dt}", "ms_per_step": ms,
           "steps": steps, "nv_end": sh.nv}
    sh.close()
    return res


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def diagnostics_leg(gpf, torch, np, ctx, log, wl, reps=50):
    """The adjacent parts on the 512^2 plate workload: a solve with and
    without the impulse, the pressure (surface part, and with the grid
    pressure), and a several-body solve (the two plates of Fig. 16 at 256^2,
    four new vortices)."""
    dev = torch.device("cuda", 0)
    case = wl.config2()
    s = gpf.Solver(ctx, case.n, case.dx, case.surface, flags=gpf.GPF_POLICY_AUTO,
                   edges=tuple(case.edges))
    al = np.deg2rad(case.surface.params["alpha_deg"])
    ns = case.surface.ns
    s.body.set_normals(np.full(ns, np.sin(al)), np.full(ns, np.cos(al)), False)
    X, Y, G = s.upload(case)
    inp = s.inputs_for(case, X, Y, G)
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=dev)
    imp = z(3)
    out_plain = s.outputs(case.nv, velocities=True)
    out_imp = gpf.make_outputs(s.psi, s.u, s.v, s.f, s.ftilde, s.scalars, s.status, imp)
    res = {"workload": f"{case.name}, nv={case.nv}"}
    res["solve_ms"] = _timed(torch, lambda: gpf.gpf_solve(s.plan, s.body, inp, out_plain), reps)
    res["solve_with_impulse_ms"] = _timed(torch, lambda: gpf.gpf_solve(s.plan, s.body, inp, out_imp),
                                          reps)
    dphi, dp, P, side = z(ns), z(ns), z(case.n * case.n), z(2 * ns)
    res["pressure_surface_ms"] = _timed(
        torch, lambda: gpf.gpf_pressure(s.plan, s.body, inp, s.psi, s.f, dphi, dp), reps)
    res["pressure_with_field_ms"] = _timed(
        torch, lambda: gpf.gpf_pressure(s.plan, s.body, inp, s.psi, s.f, dphi, dp, P, side), reps)
    gpf.gpf_sync(s.status)
    mc = wl.two_plates_case()
    plan = gpf.Plan(ctx, mc.n, mc.dx, flags=gpf.GPF_POLICY_AUTO)
    body = gpf.Body(plan, mc.xs, mc.ys, mc.ds, mc.edges)
    body.set_parts(mc.part)
    t = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64).to(dev)
    Xm, Ym, Gm = t(mc.X), t(mc.Y), t(mc.G)
    psi = torch.empty((mc.n, mc.n), dtype=plan.field_dtype, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    minp = gpf.make_parts_inputs(Xm, Ym, Gm, mc.parts, mc.znew, (), mc.u_inf, mc.v_inf)
    mout = gpf.make_outputs(psi, z(mc.nv), z(mc.nv), z(len(mc.xs)), None, z(gpf.N_SCALARS), st)
    res["two_plates_workload"] = f"{mc.name}, nv={mc.nv}, ns={len(mc.xs)}, 4 new vortices"
    res["two_plates_solve_ms"] = _timed(torch, lambda: gpf.gpf_solve(plan, body, minp, mout), reps)
    gpf.gpf_sync(st)
    # the paper's airfoil demonstration: NACA 0012 at 20 deg started
    # impulsively, shedding at the trailing edge for 3 convective times
    nc = wl.naca0012_demo()
    nsteps = 40
    nplan = gpf.Plan(ctx, nc.n, nc.dx, flags=gpf.GPF_POLICY_AUTO)
    sfn = nc.surface
    nbody = gpf.Body(nplan, sfn.xs, sfn.ys, sfn.ds, tuple(nc.edges))
    Xn, Yn, Gn = z(nsteps), z(nsteps), z(nsteps)
    nsc = z(gpf.N_SCALARS)
    nout = gpf.make_outputs(torch.empty((nc.n, nc.n), dtype=nplan.field_dtype, device=dev),
                            z(nsteps), z(nsteps), z(sfn.ns), z(sfn.ns), nsc,
                            torch.zeros(1, dtype=torch.int32, device=dev))
    ninp = gpf.make_inputs(Xn, Yn, Gn, nc.u_inf, nc.v_inf, mode="shed", znew=nc.znew)
    ninp.nv = 0
    first = [(zz[0] - sfn.xs[k], zz[1] - sfn.ys[k]) for zz, k in zip(nc.znew, nc.edges)]
    shed = gpf.Shed(nplan, nbody, ninp, nout, Xn, Yn, Gn, nc.extra["dt"], first)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    shed.run(nsteps)
    shed.sync()
    torch.cuda.synchronize()
    res["naca0012_demo"] = {"workload": f"{nc.name}, ns={sfn.ns}, {nsteps} steps of dt U/c = "
                                        f"{nc.extra['dt']}", "ms_per_step":
                            1e3 * (time.perf_counter() - t0) / nsteps,
                            "gamma_b_end": float(nsc[3].item())}
    # the plate's Schur complement: the exact FP64 build of body creation
    # (host-timed, with the inversion and the probes), and the column build
    # from 256 unit sheets in batches of 32, FP32 and FP64 fields, against it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sb = gpf.Body(s.plan, case.surface.xs, case.surface.ys, case.surface.ds, tuple(case.edges))
    torch.cuda.synchronize()
    res["schur"] = {"body_create_ms": 1e3 * (time.perf_counter() - t0)}
    for fp64 in (False, True):
        rs, rf, ms = sb.schur_by_convolution(fp64=fp64, batch=32)
        res["schur"]["columns_" + ("fp64" if fp64 else "fp32")] = {
            "rel_S": rs, "rel_f_unit_flow": rf, "ms": ms}
    log(f"[bench] diagnostics: {res}")
    return res


def c4_leg(gpf, torch, np, ctx, log, wl, reps=10):
    """64 independent problems of uneven size (n 128..1024, 1e3..1e5 vortices,
    ellipses): grid points per second batched vs solved one after another."""
    cases = wl.config4()
    dev = torch.device("cuda", 0)
    plans = {}
    for c in cases:
        if c.n not in plans:
            plans[c.n] = gpf.Plan(ctx, c.n, c.dx, flags=gpf.GPF_POLICY_AUTO)
    bodies, ins, outs, keep = [], [], [], []
    for c in cases:
        sf = c.surface
        bodies.append(gpf.Body(plans[c.n], sf.xs, sf.ys, sf.ds))
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(dev) for a in (c.X, c.Y, c.G))
        keep.append((X, Y, G))
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, gamma_b=c.gamma_b))
        outs.append(gpf.Outputs(c.n, c.nv, sf.ns))
    batch = gpf.Batch(ctx, len(cases))
    pl = [plans[c.n] for c in cases]
    gp = float(sum(c.n * c.n for c in cases))
    # lane count and schedules of every group of the batch, tuned on the
    # batch itself
    batch.autotune(pl, bodies, ins, [o.struct for o in outs])
    log(f"[bench] C4 lanes chosen: {batch.lanes}")

    def batched():
        batch.solve(pl, bodies, ins, [o.struct for o in outs])

    def plain():
        for p, b, i, o in zip(pl, bodies, ins, outs):
            gpf.gpf_solve(p, b, i, o.struct)

    res = {"workload": f"{len(cases)} ellipse problems, n in {sorted(plans)}, "
                       f"nv {min(c.nv for c in cases)}..{max(c.nv for c in cases)}",
           "grid_points_per_batch": gp, "lanes": batch.lanes}
    for name, fn in (("batched", batched), ("plain", plain)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        # median of five rounds, so that a one-off host stall in a round
        # does not stand for the rate
        rounds = []
        for _ in range(5):
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            rounds.append((time.perf_counter() - t0) / reps)
        el = sorted(rounds)[len(rounds) // 2]
        res[name] = {"ms_per_batch": 1e3 * el, "grid_points_per_s": gp / el,
                     "rounds_ms": [round(1e3 * r, 3) for r in rounds]}
        log(f"[bench] C4 {name}: {1e3 * el:.3f} ms per 64 problems (median of rounds "
            f"{[round(1e3 * r, 3) for r in rounds]}), {gp / el:.3g} GP/s")
    for o in outs:
        gpf.gpf_sync(o.status)
    res["speedup"] = res["batched"]["grid_points_per_s"] / res["plain"]["grid_points_per_s"]
    return res


def c5_leg(gpf, torch, np, ctx, log, wl, npool=16, copies=6, nsat=480, nopen=960):
    """Serving: requests (n 256..2048, up to 1e6 vortices, cylinders with a
    prescribed circulation and plates with Kutta at both edges) through
    gpf_server with 32 slots and a 64 GiB budget.  A pool of distinct
    requests is cycled (each pool entry has `copies` output sets, so requests
    in flight never share outputs).  Closed loop: saturated throughput mu.
    Open loop: Poisson arrivals at 0.5 mu and 0.8 mu, latency from submission
    to observed completion (server clock), p50/p99."""
    rng = np.random.default_rng(5)
    pool = [wl.config5_request(rng) for _ in range(npool)]
    dev = torch.device("cuda", 0)
    srv = gpf.Server(ctx, 64 << 30, max_slots=32, flags=gpf.GPF_POLICY_AUTO)
    bodies, plans, ins, keep, outs = {}, [], [], [], []
    for c in pool:
        plan = srv.plan(c.n, c.dx)
        sf = c.surface
        key = (c.n, sf.kind, sf.ns, round(float(sf.xs[0]), 9), round(float(sf.ys[0]), 9))
        if key not in bodies:
            edges = tuple(c.edges) if c.mode == "shed" else ()
            bodies[key] = gpf.Body(plan, sf.xs, sf.ys, sf.ds, edges)
        plans.append((plan, bodies[key]))
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(dev) for a in (c.X, c.Y, c.G))
        keep.append((X, Y, G))
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, gamma_b=c.gamma_b,
                                   znew=c.znew))
        outs.append([gpf.Outputs(c.n, c.nv, sf.ns) for _ in range(copies)])
    window = npool * copies

    def run(count, arrivals=None):
        ids, lats = [], []
        t0 = time.perf_counter()
        for i in range(count):
            if i >= window:
                lats.append(srv.wait(ids[i - window]))
            if arrivals is not None:
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
            k = i % npool
            plan, body = plans[k]
            ids.append(srv.submit(plan, body, ins[k], outs[k][(i // npool) % copies].struct))
        for r in ids[max(0, count - window):]:
            lats.append(srv.wait(r))
        return time.perf_counter() - t0, np.array(lats)

    run(2 * window)                       # warm-up: plans, workspaces, first launches
    gp_req = np.mean([c.n * c.n for c in pool])
    el, _ = run(nsat)
    mu = nsat / el
    res = {"workload": f"{npool} distinct requests cycled: n {sorted(set(c.n for c in pool))}, "
                       f"nv {min(c.nv for c in pool)}..{max(c.nv for c in pool)}, "
                       f"{sum(c.mode == 'shed' for c in pool)} plates with Kutta x2, "
                       f"{sum(c.mode == 'circulation' for c in pool)} cylinders",
           "slots": 32, "saturated_requests_per_s": mu, "saturated_grid_points_per_s": mu * gp_req}
    log(f"[bench] C5 saturated: {mu:.0f} requests/s, {mu * gp_req:.3g} GP/s")
    for frac in (0.5, 0.8):
        lam = frac * mu
        arr = np.cumsum(rng.exponential(1.0 / lam, size=nopen))
        el, lats = run(nopen, arr)
        res[f"load_{frac}"] = {"offered_per_s": lam, "achieved_per_s": nopen / el,
                               "p50_ms": 1e3 * float(np.percentile(lats, 50)),
                               "p99_ms": 1e3 * float(np.percentile(lats, 99))}
        log(f"[bench] C5 at {frac} mu: p50 {res[f'load_{frac}']['p50_ms']:.3f} ms, "
            f"p99 {res[f'load_{frac}']['p99_ms']:.3f} ms")
    for o in outs:
        for x in o:
            gpf.gpf_sync(x.status)
    del bodies
    srv.close()
    return res


def timed(run_step, K, plan, gpf, torch, np, with_events=True):
    """K steps between synchronizations; per-step events and kernel events."""
    stream = torch.cuda.current_stream()
    if with_events:
        gpf.timing_enable(plan, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        run_step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = gpf.timing_read(plan) if with_events else {}
    if with_events:
        gpf.timing_enable(plan, False)
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    return wall, lat, kt


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=32, help="problems per batched step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--pmc-workload", action="store_true",
                    help="only a few batched steps and a 256 MiB copy, for counter runs")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM-traffic summary from two counter runs")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc,
                      command="rocprofv3 --pmc {counter} --output-format csv -d {out} -o pmc "
                              "-- python3 bench.py --pmc-workload")
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent problems shard one per GPU with no exchange).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2102_11910_amd import gpf
    from paper_2102_11910_amd import workloads as wl

    B = args.batch
    cases = [wl.config2(seed=2 + i) for i in range(B)]
    case = cases[0]
    n = case.n
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] setup: {case.name}, nv={case.nv}, ns={case.surface.ns}, batch={B}")
    ctx = gpf.Context(0)
    t0 = time.perf_counter()
    solver = gpf.Solver(ctx, n, case.dx, case.surface, flags=gpf.GPF_POLICY_AUTO)
    plan, body = solver.plan, solver.body
    info = body.info()
    log(f"[bench] plan+body {time.perf_counter() - t0:.2f} s, body {info}")
    dev = solver.dev
    # one set of inputs/outputs per problem of the batch
    ins, outs, keep = [], [], []
    for c in cases:
        X, Y, G = (torch.as_tensor(a, dtype=torch.float64).to(dev) for a in (c.X, c.Y, c.G))
        psi = torch.empty((n, n), dtype=torch.float32, device=dev)
        u = torch.empty(c.nv, dtype=torch.float64, device=dev)
        v = torch.empty_like(u)
        f = torch.empty(body.ns, dtype=torch.float64, device=dev)
        ft = torch.empty_like(f)
        sc = torch.zeros(gpf.N_SCALARS, dtype=torch.float64, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        ins.append(gpf.make_inputs(X, Y, G, c.u_inf, c.v_inf, mode=c.mode, znew=c.znew))
        outs.append(gpf.make_outputs(psi, u, v, f, ft, sc, st))
        keep.append((X, Y, G, psi, u, v, f, ft, sc, st))
    batch = gpf.Batch(ctx, B)
    plans, bodies = [plan] * B, [body] * B
    # convolution schedules of this workload, chosen by the library's
    # autotuner on the batched step itself before anything is timed (both
    # precisions the step uses: the FP64 first convolution and the FP32
    # second one).  The counter runs keep the default rules, so that their
    # dispatches are the three steps alone; the FP64 column kernel of the
    # rules is the split one, and the traffic is reported below only when
    # the tuned run launched that kernel too.
    if not args.pmc_workload:
        batch.autotune(plans, bodies, ins, outs)
    tuned = {"fp64": gpf.schedule_get(ctx, n, True, B), "fp32": gpf.schedule_get(ctx, n, False, B)}
    log(f"[bench] convolution schedules: {tuned}")

    def step_batched():
        batch.solve(plans, bodies, ins, outs)

    def step_plain():
        gpf.gpf_solve(plan, body, ins[0], outs[0])

    if args.pmc_workload:
        for _ in range(3):
            step_batched()
        torch.cuda.synchronize()
        a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] pmc workload done")
        return 0

    for _ in range(args.warmup):
        step_batched()
        step_plain()
    for k in keep:
        gpf.gpf_sync(k[-1])
    torch.cuda.synchronize()

    K = args.steps
    # batched: K steps of B problems, kernel events on the launch stream
    wall_b, lat_b, kt = timed(step_batched, K, plan, gpf, torch, np)
    wall_b_noev, _, _ = timed(step_batched, K, plan, gpf, torch, np, with_events=False)
    # plain: one problem per step, each stage its own launch
    Kp = 4 * K
    wall_p, lat_p, _ = timed(step_plain, Kp, plan, gpf, torch, np, with_events=False)
    for k in keep:
        gpf.gpf_sync(k[-1])

    value = B * n * n * K / wall_b_noev
    value_plain = n * n * Kp / wall_p
    m = len(case.znew)
    nv_mean = int(np.mean([c.nv for c in cases]))
    keep = kept_rows(case)
    kb1 = kernel_bytes(n, nv_mean, case.surface.ns, m, info["conv1_fp64"], keep)
    per_kernel = {}
    for name, (cnt, ms) in kt.items():
        if cnt:
            avg_ms = ms / cnt
            per_kernel[name] = {"launches": cnt, "avg_us": 1e3 * avg_ms,
                                "GBps": B * kb1[name] / (avg_ms * 1e-3) / 1e9}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"] * per_kernel[k]["launches"])
    # the kernel of the class this run launched, where a class has two
    dom_kernel = None
    if dom == "cols64":
        dom_kernel = "k_cols_conv<double" if tuned["fp64"]["cols"] == 1 else "k_cols_conv_split<double"
    d = per_kernel[dom]
    achieved = d["GBps"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, dom_kernel), "bytes_per_launch": int(B * kb1[dom]),
                "avg_us": round(d["avg_us"], 3)}
    # the batched step's convolutions as a whole (all row and column passes
    # of both): algorithmic bytes over the event-timed time of those passes
    conv_cls = [k for k in ("rows_fwd", "cols", "rows_inv", "rows_fwd64", "cols64", "rows_inv64")
                if k in per_kernel]
    conv_bytes = sum(B * kb1[k] for k in conv_cls)
    conv_us = sum(per_kernel[k]["avg_us"] for k in conv_cls)
    conv_batched = {"passes": conv_cls, "bytes_per_step": int(conv_bytes), "us_per_step": round(conv_us, 3),
                    "GBps": round(conv_bytes / (conv_us * 1e-6) / 1e9, 1),
                    "frac": round(conv_bytes / (conv_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"[bench] batched convolutions: {conv_bytes / 1e6:.1f} MB in {conv_us:.1f} us, "
        f"frac {conv_batched['frac']:.3f} of HBM peak")
    log("[bench] kernels (batched): " + json.dumps(
        {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in per_kernel.items()}))

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall_b_noev / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "flat plate c=1 at 20 deg, Ns=256, Kutta at both edges with "
                               "new vortices; 512^2 grid dx=0.005; 1e4 vortices (Gaussian blob); "
                               f"a step solves {B} such problems (different vortex seeds) in "
                               "shared launches",
                   "n": n, "nv": case.nv, "ns": case.surface.ns, "batch": B, "path": "batched",
                   "precision": "FP32 fields; FP64 first convolution (noise amplification "
                                f"{info['amp']:.3g} > 500), FP64 Schur/constraints; S built "
                                "exactly in FP64 from the LGF table (its build from 256 "
                                "batched unit sheets, FP32 and FP64, under diagnostics.schur)"},
        "latency_ms": {"p50": float(np.percentile(lat_b, 50)),
                       "p99": float(np.percentile(lat_b, 99)),
                       "per": f"batch of {B} solves"},
        "plain": {"value": value_plain, "ms_per_solve": 1e3 * wall_p / Kp,
                  "latency_ms": {"p50": float(np.percentile(lat_p, 50)),
                                 "p99": float(np.percentile(lat_p, 99))}},
        "speedup_vs_plain": value / value_plain,
        "schedules": tuned,
        "value_with_kernel_events": B * n * n * K / wall_b,
        "roofline": roofline,
        "convolution_batched": conv_batched,
        "kernels": {k: {"avg_us": round(v["avg_us"], 3), "GBps": round(v["GBps"], 1),
                        "launches": v["launches"]} for k, v in per_kernel.items()},
    }
    res["convolution"] = conv_roofline(gpf, torch, np, ctx, log)
    res["rk2"] = rk2_leg(gpf, torch, np, ctx, log, wl)
    res["shed"] = shed_leg(gpf, torch, np, ctx, log, wl)
    res["diagnostics"] = diagnostics_leg(gpf, torch, np, ctx, log, wl)
    res["c4"] = c4_leg(gpf, torch, np, ctx, log, wl)
    res["c5"] = c5_leg(gpf, torch, np, ctx, log, wl)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host ...")
        res["cpu_baseline"] = cpu_baseline(case, args.cpu_budget)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
