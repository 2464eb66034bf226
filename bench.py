"""Benchmark: semi-implicit Landau-Lifshitz time steps on one MI355X.

One step = assemble the 3x3-block operator for m^n, rebuild the aggregation
AMG hierarchy, solve with V-cycle-preconditioned FGMRES to rel. residual
1e-8, project.  Default workload: 2D 1024x1024 Neumann grid (3,145,728
unknowns), smoothed random unit field, alpha = 0.02, dt = 1e-4, FP64, the
hierarchy rebuilt every step; the same run is repeated with the FP32-AMG form.
Prints ONE JSON line (metric unknowns*steps/s).

  python bench.py [--gpus 1] [--steps 50] [--warmup 3]
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
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="rough2d_1024")
    p.add_argument("--forms", default="fp64:1:jacobi:factored,fp32_amg:1:jacobi:factored,fp64:1,fp32_amg:1,"
                                      "fp64:0:jacobi:factored",
                   help="comma list of precision:kcycle_depth[:smoother[:operator]] (depth 0 = V-cycle; "
                        "smoother jacobi or mcgs, default jacobi; grid-level operator bsr or factored, "
                        "default bsr); the first gives `value`")
    p.add_argument("--roofline-class", default="outer_spmv")
    p.add_argument("--alpha", type=float, default=None, help="override the workload's alpha")
    p.add_argument("--kdepth", type=int, default=None, help="override the K-cycle depth of every form")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=1)
    p.add_argument("--serve", action="store_true",
                   help="run the serving workload instead (Poisson arrivals of mixed-size simulations)")
    p.add_argument("--requests", type=int, default=32)
    p.add_argument("--workers", type=int, default=4)
    p.add_argument("--serve-steps", type=int, default=20)
    p.add_argument("--baselines", action="store_true",
                   help="compare the unpreconditioned Krylov solvers the paper uses (GMRES, BiCGstab, TFQMR, "
                        "max 1000 iterations) with the AMG-preconditioned FGMRES on the workload")
    p.add_argument("--field", action="store_true",
                   help="full model: exchange only vs Permalloy-like anisotropy, external and stray field")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain device copy of known size (for the PMC byte counters)")
    return p.parse_args()


def source_sha() -> str:
    """Hash of the sources the solve kernels are compiled from (the PMC
    summary is only valid for the kernel source it was taken on)."""
    h = hashlib.sha256()
    for f in ("k_solve.hip", "llg_internal.h"):
        with open(os.path.join(ROOT, "paper_2608_09102_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str, precision: str, operator: str):
    """HBM bytes per launch from the committed PMC summary, or None when the
    summary is missing, was taken on another form or on a different kernel
    source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s_%s.txt" % (kernel, workload, precision, operator))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha():
        return None
    if kv.get("precision", "fp64") != precision or kv.get("grid_operator", "bsr") != operator:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(cls: str, st, N: int, precision: str, operator: str = "bsr") -> float:
    """Bytes one launch of the kernel class must move at minimum (values,
    indices, input vector read once, output written once)."""
    nnzb0 = st.level_nnzb[0]
    if cls == "outer_spmv":
        zb = 4 if precision == "fp32_amg" else 8
        if operator == "factored":  # block recomputed from the frozen field (24 B per node), neighbours from the grid
            return 24.0 * N + 3.0 * zb * N + 24.0 * N
        return 72.0 * nnzb0 + 4.0 * nnzb0 + 3.0 * zb * N + 24.0 * N
    raise ValueError("no byte model for kernel class " + cls)


def forcing_list(torch, w, total: int):
    """Manufactured forcing F(t_{k+1}) for every step of the run, resident on
    the device before the timed region (None when the workload has none)."""
    if not w.forcing:
        return [None] * total
    import llg_inputs as I
    return [torch.from_numpy(I.manufactured_forcing(w.dim, w.n, (k + 1) * w.dt, w.alpha)).cuda()
            for k in range(total)]


def run_form(llg, torch, w, form: str, steps: int, warmup: int, cls: str, Fs, kdepth: int = 0,
             smoother: str = "jacobi", operator: str = "bsr"):
    opts = llg.default_opts(rtol=w.rtol, precision=form, kcycle_depth=kdepth, smoother=smoother,
                            fine_operator=operator)
    grid = llg.make_grid(w.dim, w.n)
    S = llg.Solver(grid, opts)
    m0 = torch.from_numpy(w.m0()).cuda()
    bufs = [m0.clone(), torch.empty_like(m0)]
    cur = 0
    for k in range(warmup):
        _, s, st = S.step(bufs[cur], w.alpha, w.dt, forcing=Fs[k], out=bufs[1 - cur])
        cur = 1 - cur
        log("  warmup %d: iters %d, %.1f ms" % (k, st.iters, st.ms_total))
    S.set_kernel_timing(cls)
    iters = []
    kms = 0.0
    klaunch = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        _, s, st = S.step(bufs[cur], w.alpha, w.dt, forcing=Fs[warmup + k], out=bufs[1 - cur])
        cur = 1 - cur
        if s != llg.OK:
            raise RuntimeError("step %d: %s" % (k, llg.status_str(s)))
        iters.append(st.iters)
        kms += st.kernel_ms
        klaunch += st.kernel_launches
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.set_kernel_timing("none")
    final = bufs[cur]
    err_exact = None
    if w.forcing:
        import llg_inputs as I
        me = torch.from_numpy(I.exact_solution(w.dim, w.n, (warmup + steps) * w.dt)).cuda()
        err_exact = float((final - me).abs().max())
    # single step from m0 for the cross-form comparison (outside the timed region)
    one, _, _ = S.step(m0, w.alpha, w.dt, forcing=Fs[0])
    res = {"seconds": el, "iters": iters, "kernel_ms": kms, "kernel_launches": klaunch, "stats": st,
           "one_step": one, "levels": st.levels, "level_nodes": list(st.level_nodes[:st.levels]),
           "level_nnzb": list(st.level_nnzb[:st.levels]), "err_vs_exact": err_exact,
           "workspace_GB": S.workspace_bytes / 1e9}
    S.close()
    del S
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w, nsteps: int, kdepth: int = 0, smoother: str = "jacobi"):
    """The oracle timed on `nsteps` steps of the workload from m0 (forcing of
    the first steps when the workload has one), with the cycle and smoother of
    the main form; also returns its first step."""
    import numpy as np
    import oracle
    import llg_inputs as I
    g = oracle.make_grid(w.dim, w.n)
    o = oracle.default_opts(rtol=w.rtol, kcycle_depth=kdepth, smoother=1 if smoother == "mcgs" else 0)
    m = w.m0()
    t0 = time.perf_counter()
    iters = []
    first = None
    for k in range(nsteps):
        F = I.manufactured_forcing(w.dim, w.n, (k + 1) * w.dt, w.alpha) if w.forcing else None
        rc, m, st = oracle.step(g, o, m, w.alpha, w.dt, F)
        iters.append(st.iters)
        if first is None:
            first = m.copy()
    el = time.perf_counter() - t0
    return {"value": 3.0 * w.nodes * nsteps / el, "unit": "unknowns*steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d step(s) of the %s workload (assembly, hierarchy, FGMRES to rtol %g with the %s, "
                      "projection), single-threaded C++ oracle, %.1f s, %s FGMRES iterations"
                      % (nsteps, w.name, w.rtol, "K-cycle on levels 1..%d" % kdepth if kdepth else "V-cycle",
                         el, iters),
            "host_threads_available": os.cpu_count()}, first


def baselines_bench(a, llg, torch, w):
    """Per solver: ms/step, iterations/step, steps that converged and the last
    true relative residual, over `steps` steps after one warm-up step; FP64,
    iteration cap 1000 for the baselines (as in the paper's tables)."""
    forms = [("fgmres_amg_k1", dict(kcycle_depth=1)), ("fgmres_amg_v", dict(kcycle_depth=0)),
             ("gmres", dict(krylov="gmres", max_iters=1000)), ("bicgstab", dict(krylov="bicgstab", max_iters=1000)),
             ("tfqmr", dict(krylov="tfqmr", max_iters=1000))]
    Fs = forcing_list(torch, w, a.steps + 1)
    out = {"metric": "Krylov baselines vs AMG-FGMRES", "workload": w.name, "unknowns": w.unknowns,
           "rtol": w.rtol, "steps": a.steps, "solvers": {}}
    for name, kw in forms:
        S = llg.Solver(llg.make_grid(w.dim, w.n), llg.default_opts(rtol=w.rtol, **kw))
        m = torch.from_numpy(w.m0()).cuda()
        nxt = torch.empty_like(m)
        m, nxt = S.step(m, w.alpha, w.dt, forcing=Fs[0], out=nxt, check=False)[0], m
        its, conv, rel = [], 0, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(a.steps):
            o, s, st = S.step(m, w.alpha, w.dt, forcing=Fs[k + 1], out=nxt, check=False)
            m, nxt = o, m
            its.append(st.iters)
            conv += int(s == llg.OK)
            rel = st.relres_true
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["solvers"][name] = {"ms_per_step": 1e3 * el / a.steps, "iters_per_step": sum(its) / len(its),
                                "iters": its, "converged_steps": conv, "relres_true_last": rel}
        log("  %-14s %9.2f ms/step  %7.1f its/step  converged %d/%d  relres %.1e"
            % (name, 1e3 * el / a.steps, sum(its) / len(its), conv, a.steps, rel))
    print(json.dumps(out), flush=True)


# reduced Permalloy parameters for a 1 um body (exchange constant 1.3e-11 J/m,
# anisotropy 100 J/m^3, saturation 8e5 A/m) and a weak in-plane external field
MU0_MS2 = 4e-7 * math.pi * 8.0e5 ** 2
PERMALLOY = dict(eps=1.3e-11 / (MU0_MS2 * 1e-12), q=100.0 / MU0_MS2, h_ext=(0.01, 0.0, 0.0))


def stray_bytes(n, pdims) -> float:
    """Algorithmic HBM bytes of one stray-field evaluation as the library does
    it: m~ packed into two complex planes on the n-box; forward line passes
    that read only lines holding data and write the padded extent; the
    product with the 6 real tensor planes (read 2 planes, write 2 planes);
    inverse passes that write only the n-box; the cropped output."""
    nx, ny, nz = n
    px, py, pz = pdims
    N, P = nx * ny * nz, px * py * pz
    c = 16.0 * 2  # one complex value in each of the two planes
    passes = [(N, px * ny * nz), (px * ny * nz, px * py * nz)]  # forward x, y: (read, write)
    if pz > 1:
        passes.append((px * py * nz, P))
    fwd = sum(r + w for r, w in passes)
    return (24.0 * N + c * N) + 2 * c * fwd + (c * P + 48.0 * P + c * P) + (c * N + 24.0 * N)


def field_bench(a, llg, torch, w, form: str, kdepth: int):
    """Per variant of the model: ms/step and iterations/step over `steps` steps
    after `warmup` steps, same main form; then the stray-field evaluation
    alone (host-timed calls, each synchronizing)."""
    variants = [("exchange_only", None), ("anisotropy_external", dict(PERMALLOY, stray=0)),
                ("anisotropy_external_stray", dict(PERMALLOY, stray=1))]
    out = {"metric": "full-model step time, %s" % form, "workload": w.name, "unknowns": w.unknowns,
           "rtol": w.rtol, "steps": a.steps, "warmup": a.warmup, "field": dict(PERMALLOY), "variants": {}}
    for name, kw in variants:
        S = llg.Solver(llg.make_grid(w.dim, w.n), llg.default_opts(rtol=w.rtol, precision=form,
                                                                  kcycle_depth=kdepth, stray_field=1))
        fld = llg.make_field(**kw) if kw else None
        bufs = [torch.from_numpy(w.m0()).cuda(), None]
        bufs[1] = torch.empty_like(bufs[0])
        cur = 0

        def one():
            nonlocal cur
            if fld is None:
                _, s, st = S.step(bufs[cur], w.alpha, w.dt, out=bufs[1 - cur])
            else:
                _, s, st = S.step_field(bufs[cur], w.alpha, w.dt, fld, out=bufs[1 - cur])
            if s != llg.OK:
                raise RuntimeError("%s: %s" % (name, llg.status_str(s)))
            cur = 1 - cur
            return st
        for _ in range(a.warmup):
            one()
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            its.append(one().iters)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["variants"][name] = {"ms_per_step": 1e3 * el / a.steps, "iters_per_step": sum(its) / len(its),
                                 "iters": its}
        log("  %-26s %8.2f ms/step %6.1f its/step" % (name, 1e3 * el / a.steps, sum(its) / len(its)))
        if name == "anisotropy_external_stray":
            m = bufs[cur]
            for _ in range(3):
                S.stray_field(m)
            reps = 20
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                S.stray_field(m)
            ms = 1e3 * (time.perf_counter() - t0) / reps
            n3 = (w.n, w.n, w.n if w.dim == 3 else 1)
            pd = tuple(1 << (2 * k - 2).bit_length() if k > 1 else 1 for k in n3)
            P = pd[0] * pd[1] * pd[2]
            nb = stray_bytes(n3, pd)
            out["stray_field"] = {"ms_per_call": ms, "padded_cells": P, "algorithmic_bytes": nb,
                                  "GBps_host_timed": nb / ms / 1e6}
            log("  stray field alone: %.3f ms/call, %.0f GB/s host-timed over %.2f GB" % (ms, nb / ms / 1e6, nb / 1e9))
        S.close()
        del S
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def serve_bench(a):
    """Serving workload: Poisson arrivals (8/s) of 20-step simulations, 2D n in
    128..2048 or 3D n in 32..192, FP32-AMG, admission by device footprint."""
    import llg_inputs as I
    from paper_2608_09102_amd.serve import HipRunner, Server, default_budget
    reqs = I.serving_requests(count=a.requests, steps=a.serve_steps)
    budget = default_budget(0.8)
    # FP32-AMG on the factored grid level; the K-cycle on level 1 in 2D, the
    # V-cycle in 3D (the faster cycle on each, as measured on the benchmark grids)
    runner = HipRunner(opts_kw=dict(rtol=1e-8, precision="fp32_amg", fine_operator="factored"), workers=a.workers,
                       opts_by_dim={2: dict(kcycle_depth=1), 3: dict(kcycle_depth=0)})
    log("[serve] %d requests, %d workers, budget %.1f GB" % (len(reqs), a.workers, budget / 1e9))
    rep = Server(runner, budget, a.workers).run(reqs, log=log)
    offered = sum(3 * r.nodes * r.steps for r in reqs) / max(r.arrival for r in reqs)
    out = {"metric": "serving step latency and throughput (FP32-AMG, rel.res 1e-8)",
           "value": rep["served_unknowns_steps_per_s"], "unit": "unknowns*steps/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "serving", "requests": len(reqs), "rate_per_s": 8, "steps": a.serve_steps,
                      "workers": a.workers, "budget_bytes": budget,
                      "solver": "FP32-AMG, factored grid level; K-cycle on level 1 (2D), V-cycle (3D)"},
           "offered_unknowns_steps_per_s": offered}
    for k, v in rep.items():
        if k != "outcomes":
            out[k] = v
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if a.calibrate_copy:
        # plain device copy of 1 GiB: the reference for the PMC byte counters
        # and the achievable copy bandwidth of the box
        n = 1 << 27
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": reps + 3,
                          "copy_ms": ms, "copy_GBps": 2 * n * 8 / ms / 1e6}))
        return
    import llg_inputs as I
    import paper_2608_09102_amd as llg
    if a.serve:
        serve_bench(a)
        return
    w = I.WORKLOADS[a.workload]
    if a.alpha is not None:
        w.alpha = a.alpha
    if a.baselines:
        baselines_bench(a, llg, torch, w)
        return
    if a.field:
        f0 = a.forms.split(",")[0].split(":")
        field_bench(a, llg, torch, w, f0[0], int(f0[1]) if len(f0) > 1 and f0[1] else 0)
        return
    forms = []
    for f in a.forms.split(","):
        if not f:
            continue
        parts = f.split(":")
        prec = parts[0]
        kd = int(parts[1]) if len(parts) > 1 and parts[1] else 0
        sm = parts[2] if len(parts) > 2 and parts[2] else "jacobi"
        op = parts[3] if len(parts) > 3 and parts[3] else "bsr"
        if a.kdepth is not None:
            kd = a.kdepth
        forms.append((f, prec, kd, sm, op))
    Fs = forcing_list(torch, w, a.warmup + a.steps)
    res = {}
    for key, prec, kd, sm, op in forms:
        log("[bench] %s %s kcycle_depth %d smoother %s operator %s: %d warmup + %d timed steps"
            % (w.name, prec, kd, sm, op, a.warmup, a.steps))
        res[key] = run_form(llg, torch, w, prec, a.steps, a.warmup, a.roofline_class, Fs, kd, sm, op)
        r = res[key]
        log("  %.3f s, %.2f ms/step, iters/step %.1f, %s kernel %.3f ms over %d launches"
            % (r["seconds"], 1e3 * r["seconds"] / a.steps, sum(r["iters"]) / len(r["iters"]),
               a.roofline_class, r["kernel_ms"], r["kernel_launches"]))
    main_key, main_form, main_kd, main_sm, main_op = forms[0]
    r = res[main_key]
    unknowns = w.unknowns
    value = unknowns * a.steps / r["seconds"]
    # roofline of the timed kernel class
    lb = algorithmic_bytes(a.roofline_class, r["stats"], w.nodes, main_form, main_op)
    avg_s = r["kernel_ms"] / 1e3 / max(1, r["kernel_launches"])
    achieved = lb / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = read_traffic(a.roofline_class, w.name, main_form, main_op)
    out = {
        "metric": "unknowns*steps/s (FP64 AMG-FGMRES, rel.res 1e-8)",
        "value": value,
        "unit": "unknowns*steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * r["seconds"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": "%dD %s" % (w.dim, "x".join([str(w.n)] * w.dim)),
                   "unknowns": unknowns, "alpha": w.alpha, "dt": w.dt, "rtol": w.rtol,
                   "form": main_form, "hierarchy": "rebuilt every step", "krylov": "FGMRES(30)",
                   "preconditioner": "aggregation AMG, %s (1,1), %s" % (
                       "damped block-Jacobi" if main_sm == "jacobi" else "multicolour block Gauss-Seidel",
                       "K-cycle on levels 1..%d" % main_kd if main_kd else "V-cycle"),
                   "grid_operator": "3x3-block sliced ELL" if main_op == "bsr" else "factored (one block per node)"},
        "iters_per_step": sum(r["iters"]) / len(r["iters"]),
        "iters": r["iters"],
        "levels": r["levels"],
        "workspace_GB": r["workspace_GB"],
        "level_nodes": r["level_nodes"],
        "roofline": {"bound": "hbm", "kernel": a.roofline_class, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": lb,
                     "avg_launch_us": avg_s * 1e6, "launches": r["kernel_launches"]},
    }
    def form_name(prec, kd, sm, op):
        return "%s_%s%s%s" % (prec, "k%d" % kd if kd else "vcycle", "" if sm == "jacobi" else "_" + sm,
                              "" if op == "bsr" else "_" + op)

    for key, prec, kd, sm, op in forms[1:]:
        rf = res[key]
        diff = float((rf["one_step"] - r["one_step"]).abs().max())
        name = form_name(prec, kd, sm, op)
        out[name] = {"value": unknowns * a.steps / rf["seconds"], "ms_per_step": 1e3 * rf["seconds"] / a.steps,
                     "iters_per_step": sum(rf["iters"]) / len(rf["iters"]), "iters": rf["iters"],
                     "err_vs_exact": rf["err_vs_exact"], "kcycle_depth": kd, "smoother": sm, "grid_operator": op,
                     "speedup_vs_main": (unknowns * a.steps / rf["seconds"]) / value,
                     "max_abs_diff_one_step_vs_main": diff}
    if r["err_vs_exact"] is not None:
        out["err_vs_exact"] = r["err_vs_exact"]
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline: oracle, %d step(s)" % a.cpu_steps)
        out["cpu_baseline"], ref = cpu_baseline(w, a.cpu_steps, main_kd, main_sm)
        # error of every form's first step against the FP64 oracle's (both at the workload's rtol)
        import numpy as np
        out["err_vs_oracle"] = float(np.abs(r["one_step"].cpu().numpy() - ref).max())
        for key, prec, kd, sm, op in forms[1:]:
            name = form_name(prec, kd, sm, op)
            out[name]["err_vs_oracle"] = float(np.abs(res[key]["one_step"].cpu().numpy() - ref).max())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
