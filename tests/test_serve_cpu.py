"""Scheduler of the serving loop, on the CPU with a fake runner: admission by
footprint never exceeds the budget, at most `workers` simulations run at once,
admission is first-come first-served, oversized requests are rejected, and
every admitted request completes."""
import threading
import time

import pytest

from llg_inputs import Request
from paper_2608_09102_amd.serve import Server


class FakeRunner:
    def __init__(self, budget):
        self.lock = threading.Lock()
        self.used = 0
        self.active = 0
        self.max_used = 0
        self.max_active = 0
        self.starts = []
        self.budget = budget

    def footprint(self, r):
        return r.nodes * 100

    def run(self, r, wid, on_step):
        with self.lock:
            self.used += self.footprint(r)
            self.active += 1
            self.max_used = max(self.max_used, self.used)
            self.max_active = max(self.max_active, self.active)
            self.starts.append(r.rid)
        for _ in range(r.steps):
            time.sleep(0.002)
            on_step(2.0, 3)
        with self.lock:
            self.used -= self.footprint(r)
            self.active -= 1
        return r.rid


def _reqs():
    out = []
    t = 0.0
    for rid in range(24):
        n = 8 + (rid * 7) % 24
        out.append(Request(rid, t, 2, n, 0.1, 1e-3, 3 + rid % 4, 5000 + rid))
        t += 0.001
    out.append(Request(99, 0.005, 3, 200, 0.1, 1e-3, 2, 1))  # 8M nodes: larger than the budget
    return out


@pytest.mark.parametrize("workers", [1, 3, 6])
def test_admission_respects_budget_and_slots(workers):
    budget = 150_000
    fr = FakeRunner(budget)
    rep = Server(fr, budget, workers).run(_reqs(), keep_results=True)
    assert fr.max_used <= budget
    assert fr.max_active <= workers
    assert rep["done"] == 24 and rep["rejected"] == 1 and rep["failed"] == 0
    outs = {o.rid: o for o in rep["outcomes"]}
    assert outs[99].status == "rejected"
    # first-come first-served: admission order follows arrival order
    admitted = sorted((o.admitted, o.rid) for o in rep["outcomes"] if o.status == "done")
    assert [rid for _, rid in admitted] == sorted(rid for _, rid in admitted)
    for o in rep["outcomes"]:
        if o.status == "done":
            assert len(o.step_ms) == o.steps and o.result == o.rid
            assert o.admitted >= o.arrival - 1e-9 and o.finished >= o.admitted
    assert rep["step_ms_p50"] == 2.0 and rep["steps_total"] == sum(3 + r % 4 for r in range(24))


def test_failure_isolated():
    class Failing(FakeRunner):
        def run(self, r, wid, on_step):
            if r.rid == 5:
                raise RuntimeError("injected")
            return super().run(r, wid, on_step)

    fr = Failing(10**9)
    rep = Server(fr, 10**9, 4).run(_reqs()[:10])
    assert rep["failed"] == 1 and rep["done"] == 9
