"""Serving loop: continuous batching of independent Landau-Lifshitz simulations.

Requests (grid, alpha, dt, number of steps, initial field) arrive over time.
When a request arrives its exact device footprint is planned
(llg_workspace_bytes plus its two field buffers); it is admitted when a worker
slot is free and the footprint fits in the HBM budget next to the simulations
already running; admission is first-come first-served.  Planning runs the
field-independent aggregation once per grid shape on the device, in temporary
memory outside the budget (the budget is a fraction of the free memory that
leaves room for it).  Each
admitted simulation owns a context on the worker's own HIP stream, so its
field, its AMG hierarchy and its Krylov state stay resident on the device
between steps, and the steps of different simulations overlap on the GPU.  A
finished simulation frees its memory and slot at once, and the next queued
request is admitted.

Reported per run: p50/p99 step latency (one llg_step, including interference
from co-running simulations), p50/p99 request latency (arrival to last step),
p50/p99 queueing delay (arrival to admission), served unknowns*steps/s.

The scheduler is independent of the device: `Server(runner=...)` accepts any
object with `footprint(req)` and `run(req, worker, on_step)`; the default
`HipRunner` drives libllg.so.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Outcome:
    rid: int
    status: str = "queued"          # queued, running, done, failed, rejected
    arrival: float = 0.0            # seconds since the start of the run
    admitted: float = math.nan
    finished: float = math.nan
    step_ms: list = field(default_factory=list)
    iters: list = field(default_factory=list)
    unknowns: int = 0
    steps: int = 0
    worker: int = -1
    result: object = None           # final field (host float64 array) when kept
    error: str = ""


def percentile(xs, q):
    if not xs:
        return math.nan
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


class Server:
    """First-come first-served admission by device footprint, `workers` slots."""

    def __init__(self, runner, budget_bytes: int, workers: int = 4):
        self.runner = runner
        self.budget = int(budget_bytes)
        self.workers = int(workers)

    def run(self, requests, time_scale: float = 1.0, keep_results: bool = False, log=None) -> dict:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        out = {r.rid: Outcome(r.rid, arrival=r.arrival * time_scale, unknowns=3 * r.nodes, steps=r.steps)
               for r in reqs}
        foot = {}  # each request's footprint, planned when it arrives
        cv = threading.Condition()
        state = {"used": 0, "free": list(range(self.workers)), "active": 0, "next": 0}
        pending = []
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def work(r, wid):
            o = out[r.rid]
            try:
                def on_step(ms, iters):
                    o.step_ms.append(ms)
                    o.iters.append(iters)
                res = self.runner.run(r, wid, on_step)
                o.status = "done"
                if keep_results:
                    o.result = res
            except Exception as e:  # a failed request does not stop the others
                o.status = "failed"
                o.error = repr(e)
            with cv:
                o.finished = now()
                state["used"] -= foot[r.rid]
                state["free"].append(wid)
                state["active"] -= 1
                cv.notify_all()

        threads = []
        with cv:
            while True:
                t = now()
                while state["next"] < len(reqs) and reqs[state["next"]].arrival * time_scale <= t:
                    r = reqs[state["next"]]
                    state["next"] += 1
                    foot[r.rid] = int(self.runner.footprint(r))
                    if foot[r.rid] > self.budget:
                        out[r.rid].status = "rejected"
                        out[r.rid].error = "footprint %d exceeds the budget %d" % (foot[r.rid], self.budget)
                    else:
                        pending.append(r)
                # admit in arrival order while the head fits
                while pending and state["free"] and state["used"] + foot[pending[0].rid] <= self.budget:
                    r = pending.pop(0)
                    wid = state["free"].pop(0)
                    state["used"] += foot[r.rid]
                    state["active"] += 1
                    o = out[r.rid]
                    o.status, o.admitted, o.worker = "running", now(), wid
                    th = threading.Thread(target=work, args=(r, wid), daemon=True)
                    threads.append(th)
                    th.start()
                    if log:
                        log("admit %d at %.3f s (worker %d, %.2f GB in use)" % (r.rid, o.admitted, wid,
                                                                                  state["used"] / 1e9))
                if state["next"] >= len(reqs) and not pending and state["active"] == 0:
                    break
                wait = None
                if state["next"] < len(reqs):
                    wait = max(0.0, reqs[state["next"]].arrival * time_scale - now())
                cv.wait(timeout=wait if wait is not None else 1.0)
        for th in threads:
            th.join()
        makespan = now()
        return report(list(out.values()), makespan)


def report(outcomes, makespan: float) -> dict:
    done = [o for o in outcomes if o.status == "done"]
    steps = [ms for o in done for ms in o.step_ms]
    req_lat = [o.finished - o.arrival for o in done]
    queue = [o.admitted - o.arrival for o in done]
    served = sum(o.unknowns * len(o.step_ms) for o in done)
    return {
        "requests": len(outcomes), "done": len(done),
        "failed": sum(o.status == "failed" for o in outcomes),
        "rejected": sum(o.status == "rejected" for o in outcomes),
        "makespan_s": makespan,
        "step_ms_p50": percentile(steps, 50), "step_ms_p99": percentile(steps, 99),
        "request_s_p50": percentile(req_lat, 50), "request_s_p99": percentile(req_lat, 99),
        "queue_s_p50": percentile(queue, 50), "queue_s_p99": percentile(queue, 99),
        "served_unknowns_steps_per_s": served / makespan if makespan > 0 else math.nan,
        "steps_total": len(steps),
        "outcomes": outcomes,
    }


class HipRunner:
    """Runs a request through libllg.so: one context per simulation on the
    worker's stream, `steps` calls of llg_step, fields resident on the device.
    opts_kw applies to every request; opts_by_dim[d] adds options for grids of
    dimension d (e.g. the cycle that is fastest there)."""

    def __init__(self, opts_kw=None, device: int = 0, workers: int = 4, keep_device: bool = False,
                 opts_by_dim=None, inputs=None):
        import torch
        import paper_2608_09102_amd as llg
        self.llg = llg
        self.torch = torch
        self.opts_kw = dict(opts_kw or {})
        self.opts_by_dim = {int(k): dict(v) for k, v in (opts_by_dim or {}).items()}
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(workers)]
        self._plan_lock = threading.Lock()
        self.inputs = inputs  # rid -> initial field on the host (else generated from the request's recipe)

    def _grid_opts(self, r):
        llg = self.llg
        kw = dict(self.opts_kw)
        kw.update(self.opts_by_dim.get(r.dim, {}))
        return llg.make_grid(r.dim, r.n), llg.default_opts(**kw)

    def footprint(self, r) -> int:
        g, o = self._grid_opts(r)
        with self._plan_lock, self.torch.cuda.device(self.device):
            s, b = self.llg.workspace_bytes(g, o)
        if s != self.llg.OK:
            raise self.llg.LLGError(s, "llg_workspace_bytes")
        return b + 2 * 24 * r.nodes  # workspace + m^n and m^{n+1} (the initial field is copied into m^n)

    def run(self, r, wid: int, on_step):
        torch, llg = self.torch, self.llg
        st = self.streams[wid]
        g, o = self._grid_opts(r)
        with torch.cuda.device(self.device), torch.cuda.stream(st):
            S = llg.Solver(g, o, stream=st)
            h = self.inputs[r.rid] if self.inputs is not None else r.m0()
            m = torch.from_numpy(h).to(self.device)
            nxt = torch.empty_like(m)
            st.synchronize()
            for _ in range(r.steps):
                t = time.perf_counter()
                _, s, stt = S.step(m, r.alpha, r.dt, out=nxt)
                on_step(1e3 * (time.perf_counter() - t), stt.iters)
                m, nxt = nxt, m
            S.close()
            res = m.cpu().numpy()
            del S
        return res


def default_budget(fraction: float = 0.9, device: int = 0) -> int:
    import torch
    free, _ = torch.cuda.mem_get_info(device)
    return int(fraction * free)
