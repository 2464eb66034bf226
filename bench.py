"""Benchmark: semi-implicit Landau-Lifshitz time steps on one MI355X.

One step = assemble the 3x3-block operator for m^n (+ dt F), rebuild the
aggregation AMG hierarchy, solve with AMG-preconditioned FGMRES to rel.
residual 1e-8, project.  Default workload: the 3D 256^3 manufactured solution
(50,331,648 unknowns, alpha = 0.1, dt = 1e-4, forcing F resident on the device),
timed in the FP32-AMG form (`value`) and the FP64 form over the same steps;
then, as secondary keys, the 2D 1024^2 rough-field forms and a short serving
run.  Prints ONE JSON line (metric unknowns*steps/s).

  python bench.py [--gpus 1] [--steps 20] [--warmup 5]
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

# forms timed per workload when --forms is not given (the first gives `value`):
# the metric compares FP32-AMG with FP64, both at rel.res 1e-8
# The 256^3 main forms rebuild the hierarchy structure before each step's
# assembly (+serial): with the rebuild overlapped on a second stream (the
# forms without the suffix, reported beside them) the step is about 5%
# faster, but its kernels share the device with the rebuild, which a kernel
# trace cannot show (the profiler serializes the streams), so the roofline
# kernel is timed in the serial form.
# +nuXY: X block-Jacobi sweeps before and Y after the coarse correction (the
# library default is one and one); the counts are the measured cheapest per
# workload (design notes, the smoothing study)
DEFAULT_FORMS = {
    "mms3d_256": "fp32_amg:1:jacobi:factored+serial+nu03,fp64:1:jacobi:factored+serial+nu03,"
                 "fp32_amg:1:jacobi:factored+nu03,fp64:1:jacobi:factored+nu03",
    "rough3d_128": "fp32_amg:0:jacobi:factored+nu02,fp64:0:jacobi:factored+nu02",
    "rough2d_1024": "fp32_amg:1:jacobi:factored+nu02,fp64:1:jacobi:factored+nu02",
    "vortex64": "fp64:1:jacobi:factored,fp32_amg:1:jacobi:factored",
}
# the oracle runs one step of the workload when it takes about 10-30 s on one
# host core; larger workloads are sampled on the same problem at half the grid
# points per axis
ORACLE_MAX_NODES = 2_200_000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="mms3d_256")
    p.add_argument("--forms", default=None,
                   help="comma list of precision:kcycle_depth[:smoother[:operator]] (depth 0 = V-cycle; "
                        "smoother jacobi or mcgs, default jacobi; grid-level operator bsr or factored, "
                        "default bsr); the first gives `value`.  Default: per workload (DEFAULT_FORMS)")
    p.add_argument("--no-secondary", action="store_true",
                   help="skip the secondary keys (the 1024^2 forms and the short serving run)")
    p.add_argument("--secondary-workload", default="rough2d_1024")
    p.add_argument("--serve-leg-requests", type=int, default=24,
                   help="requests of the serving run reported as a secondary key")
    p.add_argument("--roofline-class", default="level1",
                   help="kernel class of the roofline object: level1 (the level-1 products through the grid "
                        "blocks, k_l1, the largest kernel of the 256^3 forms) or outer_spmv")
    p.add_argument("--alpha", type=float, default=None, help="override the workload's alpha")
    p.add_argument("--kdepth", type=int, default=None, help="override the K-cycle depth of every form")
    p.add_argument("--nu", type=int, default=None, help="smoothing sweeps before and after the coarse correction "
                                                          "(every form; default 1)")
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
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s_%s.txt" % (kernel, workload, precision,
                                                                      operator.replace("+", "_")))
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


def algorithmic_bytes(cls: str, st, N: int, precision: str, operator: str = "bsr", r=None) -> float:
    """Bytes one launch of the kernel class must move at minimum (values,
    indices, input vector read once, output written once).  level1: the
    library adds up each timed launch's bytes by its mode (frozen field by
    member 24 B and neighbour aggregates 4 B per neighbour per grid node,
    member pointers, x, and per mode b / D1^-1 / the dot operands and the
    output); the figure is their mean per launch."""
    if cls == "level1":
        return r["kernel_bytes"] / max(1, r["kernel_launches"])
    nnzb0 = st.level_nnzb[0]
    if cls == "outer_spmv":
        zb = 4 if precision == "fp32_amg" else 8
        if operator.split("+")[0] == "factored":  # block recomputed from the frozen field (24 B per node), neighbours from the grid
            return 24.0 * N + 3.0 * zb * N + 24.0 * N
        return 72.0 * nnzb0 + 4.0 * nnzb0 + 3.0 * zb * N + 24.0 * N
    raise ValueError("no byte model for kernel class " + cls)


def forcing_list(torch, w, total: int):
    """Manufactured forcing F(t_{k+1}) for every step of the run, generated on
    the device and resident there before the timed region (None when the
    workload has none)."""
    if not w.forcing:
        return [None] * total
    import llg_inputs as I
    dev = torch.device("cuda")
    return [I.manufactured_forcing(w.dim, w.n, (k + 1) * w.dt, w.alpha, xp=torch, device=dev) for k in range(total)]


NU = None  # --nu: sweeps before and after the coarse correction, every form


def form_opts(llg, rtol: float, precision: str, kdepth: int, smoother: str, operator: str):
    """Options of a form.  operator[+serial|+reuse][+sliced][+nuXY]: the
    hierarchy structure rebuilt on a second stream beside the step (default),
    rebuilt at the start of each step (serial), or built once per context
    (reuse); +sliced: the large coarse levels' products on sliced-ELL values
    instead of the CSR-ordered blocks; +nuXY: X smoothing sweeps before and Y
    after the coarse correction (default one and one)."""
    base, *mods = operator.split("+")
    extra = {}
    for rb in mods:
        if rb.startswith("nu"):
            extra.update(nu_pre=int(rb[2]), nu_post=int(rb[3]))
            continue
        extra.update({"serial": dict(overlap_rebuild=0), "reuse": dict(rebuild_aggregates=0),
                      "sliced": dict(csr_levels=0)}[rb])
    if NU is not None:
        extra.update(nu_pre=NU, nu_post=NU)
    return llg.default_opts(rtol=rtol, precision=precision, kcycle_depth=kdepth, smoother=smoother,
                            fine_operator=base, **extra)


def run_form(llg, torch, w, form: str, steps: int, warmup: int, cls: str, Fs, kdepth: int = 0,
             smoother: str = "jacobi", operator: str = "bsr"):
    opts = form_opts(llg, w.rtol, form, kdepth, smoother, operator)
    grid = llg.make_grid(w.dim, w.n)
    t0 = time.perf_counter()
    S = llg.Solver(grid, opts)
    t_create = time.perf_counter() - t0
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
    kbytes = 0.0
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
        kbytes += st.kernel_bytes
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.set_kernel_timing("none")
    final = bufs[cur]
    err_exact = None
    if w.forcing:
        import llg_inputs as I
        me = I.exact_solution(w.dim, w.n, (warmup + steps) * w.dt, xp=torch, device=final.device)
        err_exact = float((final - me).abs().max())
        del me
    res = {"seconds": el, "iters": iters, "kernel_ms": kms, "kernel_launches": klaunch, "kernel_bytes": kbytes,
           "stats": st,
           "levels": st.levels, "level_nodes": list(st.level_nodes[:st.levels]),
           "level_nnzb": list(st.level_nnzb[:st.levels]), "err_vs_exact": err_exact,
           "workspace_GB": S.workspace_bytes / 1e9, "create_s": t_create,
           "ms_setup_last": st.ms_setup, "ms_solve_last": st.ms_solve}
    S.close()
    del S, bufs, m0, final
    torch.cuda.empty_cache()
    return res


def host_info() -> dict:
    """CPU model, logical CPUs and memory of the host the oracle runs on."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["mem_GB"] = round(int(line.split()[1]) / 1e6, 1)
                    break
    except OSError:
        pass
    return info


def sample_step(w, warmup: int):
    """The step the CPU baseline times: the workload's own step after the
    warm-up steps when the oracle takes it in about 10-30 s, else the same
    problem at half the grid points per axis.  Forced workloads start from
    the exact solution m_e(t_w) with the forcing F(t_w + dt); the others from
    the workload's m0.  Returns (dim, n, m, F, label)."""
    import llg_inputs as I
    n = w.n if w.nodes <= ORACLE_MAX_NODES else w.n // 2
    if w.forcing:
        t = warmup * w.dt
        m = I.exact_solution(w.dim, n, t)
        F = I.manufactured_forcing(w.dim, n, t + w.dt, w.alpha)
        label = "one step of the manufactured problem of the %s workload at %d^%d (alpha %g, dt %g, from the " \
                "exact m_e(t) at t = %d dt, forcing F(t + dt))" % (w.name, n, w.dim, w.alpha, w.dt, warmup)
    else:
        m = I.smooth_unit_field(w.dim, n, w.seed) if n != w.n else w.m0()
        F = None
        label = "the first step of the %s workload at %d^%d" % (w.name, n, w.dim)
    return w.dim, n, m, F, label


def form_nu(operator: str):
    """(sweeps before, sweeps after) of a form's operator string."""
    nu = (NU, NU) if NU is not None else (1, 1)
    for rb in operator.split("+")[1:]:
        if rb.startswith("nu"):
            nu = (int(rb[2]), int(rb[3]))
    return nu


def cpu_baseline(w, warmup: int, kdepth: int, smoother: str, nu=(1, 1)):
    """The oracle (single-threaded C++, FP64) timed on sample_step, with the
    workload's rtol and the main form's cycle, smoother and sweep counts."""
    import oracle
    dim, n, m, F, label = sample_step(w, warmup)
    g = oracle.make_grid(dim, n)
    o = oracle.default_opts(rtol=w.rtol, kcycle_depth=kdepth, smoother=1 if smoother == "mcgs" else 0,
                            nu_pre=nu[0], nu_post=nu[1])
    t0 = time.perf_counter()
    rc, out, st = oracle.step(g, o, m, w.alpha, w.dt, F)
    el = time.perf_counter() - t0
    unknowns = 3 * n ** dim
    res = {"value": unknowns / el, "unit": "unknowns*steps/s", "cores": 1, "kind": "oracle",
           "sample": "%s; assembly, hierarchy, FGMRES(30) to rtol %g with the %s, (%d,%d) smoothing sweeps, "
                     "projection; %d FGMRES iterations; %.1f s on 1 host core (single-threaded C++, -O2)" % (
                         label, w.rtol, "K-cycle on levels 1..%d" % kdepth if kdepth else "V-cycle", nu[0], nu[1],
                         st.iters, el),
           "seconds": el, "iters": st.iters, "host": host_info()}
    return res, (dim, n, m, F, out, st.iters)


def gpu_sample_error(llg, torch, w, sample, form: str, kdepth: int, smoother: str, operator: str):
    """The GPU's step (the given form) of the CPU baseline's sample step, and
    its max-norm difference from the oracle's."""
    import numpy as np
    dim, n, m, F, ref, _ = sample
    S = llg.Solver(llg.make_grid(dim, n), form_opts(llg, w.rtol, form, kdepth, smoother, operator))
    out, s, st = S.step(torch.from_numpy(m).cuda(), w.alpha, w.dt,
                        forcing=torch.from_numpy(F).cuda() if F is not None else None)
    d = float(np.abs(out.cpu().numpy() - ref).max())
    S.close()
    return d, st.iters


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


SERVE_SOLVER = "FP32-AMG, factored grid level; K-cycle on level 1 (2D), V-cycle (3D)"


def serve_inputs(count: int, steps: int):
    """The request stream and its initial fields, generated on the host by a
    process pool before anything touches the GPU."""
    import llg_inputs as I
    reqs = I.serving_requests(count=count, steps=steps)
    log("[serve] generating the initial fields of %d requests" % len(reqs))
    return reqs, I.serving_inputs(reqs)


def serve_report(count: int, steps: int, workers: int, prepared=None) -> dict:
    """The serving workload's request stream (Poisson arrivals at 8/s of
    `steps`-step simulations, 2D n in 128..2048 or 3D n in 32..192, initial
    fields from the input recipe with seed 5000 + r), served in FP32-AMG at
    rel.res 1e-8 with admission by device footprint within 0.9 of the free
    device memory."""
    import llg_inputs as I
    from paper_2608_09102_amd.serve import HipRunner, Server, default_budget
    reqs, inputs = prepared if prepared is not None else serve_inputs(count, steps)
    budget = default_budget(0.9)
    # FP32-AMG on the factored grid level, no sweep before and two after the
    # coarse correction; the K-cycle on level 1 in 2D, the V-cycle in 3D (the
    # faster settings on each, as measured on the 1024^2 and 128^3 grids)
    runner = HipRunner(opts_kw=dict(rtol=1e-8, precision="fp32_amg", fine_operator="factored", nu_pre=0,
                                    nu_post=2), workers=workers,
                       opts_by_dim={2: dict(kcycle_depth=1), 3: dict(kcycle_depth=0)}, inputs=inputs)
    log("[serve] %d requests, %d workers, budget %.1f GB" % (len(reqs), workers, budget / 1e9))
    rep = Server(runner, budget, workers).run(reqs, log=log)
    offered = sum(3 * r.nodes * r.steps for r in reqs) / max(r.arrival for r in reqs)
    out = {"requests": len(reqs), "rate_per_s": 8, "steps": steps, "workers": workers, "budget_bytes": budget,
           "solver": SERVE_SOLVER, "offered_unknowns_steps_per_s": offered}
    for k, v in rep.items():
        if k != "outcomes":
            out[k] = v
    return out


def serve_bench(a, prepared=None):
    rep = serve_report(a.requests, a.serve_steps, a.workers, prepared)
    out = {"metric": "serving step latency and throughput (FP32-AMG, rel.res 1e-8)",
           "value": rep["served_unknowns_steps_per_s"], "unit": "unknowns*steps/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "serving", "requests": rep["requests"], "rate_per_s": 8, "steps": a.serve_steps,
                      "workers": a.workers, "budget_bytes": rep["budget_bytes"], "solver": SERVE_SOLVER}}
    out.update({k: v for k, v in rep.items() if k not in out["config"]})
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    prepared = None
    if a.serve:
        prepared = serve_inputs(a.requests, a.serve_steps)
    elif not a.no_secondary and a.serve_leg_requests > 0 and not (a.baselines or a.field or a.calibrate_copy):
        prepared = serve_inputs(a.serve_leg_requests, a.serve_steps)
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
        serve_bench(a, prepared)
        return
    w = I.WORKLOADS[a.workload]
    global NU
    NU = a.nu
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
    for f in (a.forms or DEFAULT_FORMS[w.name]).split(","):
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
    log("[bench] generating the forcing of %d steps on the device" % (a.warmup + a.steps) if w.forcing else "")
    Fs = forcing_list(torch, w, a.warmup + a.steps)
    res = {}
    for key, prec, kd, sm, op in forms:
        log("[bench] %s %s kcycle_depth %d smoother %s operator %s: %d warmup + %d timed steps"
            % (w.name, prec, kd, sm, op, a.warmup, a.steps))
        res[key] = run_form(llg, torch, w, prec, a.steps, a.warmup, a.roofline_class, Fs, kd, sm, op)
        r = res[key]
        log("  %.3f s, %.2f ms/step, iters/step %.1f, %s kernel %.3f ms over %d launches, create %.2f s"
            % (r["seconds"], 1e3 * r["seconds"] / a.steps, sum(r["iters"]) / len(r["iters"]),
               a.roofline_class, r["kernel_ms"], r["kernel_launches"], r["create_s"]))
    del Fs
    torch.cuda.empty_cache()
    main_key, main_form, main_kd, main_sm, main_op = forms[0]
    r = res[main_key]
    unknowns = w.unknowns
    value = unknowns * a.steps / r["seconds"]
    # roofline of the timed kernel class
    lb = algorithmic_bytes(a.roofline_class, r["stats"], w.nodes, main_form, main_op, r)
    avg_s = r["kernel_ms"] / 1e3 / max(1, r["kernel_launches"])
    achieved = lb / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = read_traffic(a.roofline_class, w.name, main_form, main_op)

    def form_name(prec, kd, sm, op):
        return "%s_%s%s%s" % (prec, "k%d" % kd if kd else "vcycle", "" if sm == "jacobi" else "_" + sm,
                              "" if op == "bsr" else "_" + op.replace("+", "_"))

    def cycle(kd, sm, op="bsr"):
        return "aggregation AMG, %s (%d,%d), %s" % (("damped block-Jacobi" if sm == "jacobi" else
                                                      "multicolour block Gauss-Seidel",) + form_nu(op) +
                                                     ("K-cycle on levels 1..%d" % kd if kd else "V-cycle",))
    out = {
        "metric": "unknowns*steps/s, FP32-AMG vs FP64 at rel.res 1e-8" if main_form == "fp32_amg"
                  else "unknowns*steps/s (FP64 AMG-FGMRES, rel.res 1e-8)",
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
                   "forcing": "manufactured (resident on the device)" if w.forcing else None,
                   "form": main_form, "hierarchy": "rebuilt every step", "krylov": "FGMRES(30), FP64",
                   "preconditioner": cycle(main_kd, main_sm, main_op),
                   "grid_operator": "3x3-block sliced ELL" if main_op.startswith("bsr") else "factored (one block per node)",
                   "structure_rebuild": ("once per context" if "reuse" in main_op.split("+") else
                                         "every step, before the assembly" if "serial" in main_op.split("+") else
                                         "every step, on a second stream beside the step (double-buffered)"),
                   "large_coarse_levels": "sliced ELL" if "sliced" in main_op.split("+") else "CSR-ordered copy"},
        "iters_per_step": sum(r["iters"]) / len(r["iters"]),
        "iters": r["iters"],
        "levels": r["levels"],
        "workspace_GB": r["workspace_GB"],
        "level_nodes": r["level_nodes"],
        "level_nnzb": r["level_nnzb"],
        "roofline": {"bound": "hbm", "kernel": a.roofline_class, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": lb,
                     "avg_launch_us": avg_s * 1e6, "launches": r["kernel_launches"]},
    }
    if r["err_vs_exact"] is not None:
        out["err_vs_exact"] = r["err_vs_exact"]
        out["err_vs_exact_note"] = ("max-norm distance from the manufactured m_e after warmup + steps steps; the "
                                    "forcing uses the continuous Laplacian, so it holds the O(h^2) spatial error "
                                    "besides the O(dt) temporal one")
    for key, prec, kd, sm, op in forms[1:]:
        rf = res[key]
        name = form_name(prec, kd, sm, op)
        out[name] = {"value": unknowns * a.steps / rf["seconds"], "ms_per_step": 1e3 * rf["seconds"] / a.steps,
                     "iters_per_step": sum(rf["iters"]) / len(rf["iters"]), "iters": rf["iters"],
                     "err_vs_exact": rf["err_vs_exact"], "kcycle_depth": kd, "smoother": sm, "grid_operator": op,
                     "value_ratio_main_over_this": value / (unknowns * a.steps / rf["seconds"])}
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline: the oracle on one step")
        cb, sample = cpu_baseline(w, a.warmup, main_kd, main_sm, form_nu(main_op))
        out["cpu_baseline"] = cb
        log("  %s" % cb["sample"])
        # every form's step of the same sample against the oracle's (both at the workload's rtol)
        errs = {}
        for key, prec, kd, sm, op in forms:
            d, its = gpu_sample_error(llg, torch, w, sample, prec, kd, sm, op)
            errs[form_name(prec, kd, sm, op)] = {"max_abs_diff": d, "gpu_iters": its, "oracle_iters": sample[5]}
        out["err_vs_oracle_sample"] = errs
    if not a.no_secondary:
        if a.secondary_workload and a.secondary_workload != w.name:
            w2 = I.WORKLOADS[a.secondary_workload]
            sec = {}
            for f in DEFAULT_FORMS[w2.name].split(","):
                prec, kd, sm, op = f.split(":")
                log("[bench] secondary %s %s" % (w2.name, f))
                rf = run_form(llg, torch, w2, prec, a.steps, a.warmup, "none", [None] * (a.warmup + a.steps),
                              int(kd), sm, op)
                sec[form_name(prec, int(kd), sm, op)] = {
                    "value": w2.unknowns * a.steps / rf["seconds"], "ms_per_step": 1e3 * rf["seconds"] / a.steps,
                    "iters_per_step": sum(rf["iters"]) / len(rf["iters"]), "preconditioner": cycle(int(kd), sm, op)}
            out[w2.name] = sec
        if a.serve_leg_requests > 0:
            out["serving"] = serve_report(a.serve_leg_requests, a.serve_steps, a.workers, prepared)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
