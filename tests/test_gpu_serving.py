"""Serving loop on the GPU: continuous batching of simulations of different
sizes.  Each request's final field must be the same whether it ran alone or
in the mix (bitwise: every kernel is deterministic and contexts share nothing),
and a tight budget must queue requests instead of failing them."""
import sys

import numpy as np
import pytest

from llg_inputs import Request

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    rng = np.random.default_rng(11)
    out = []
    t = 0.0
    for rid in range(10):
        dim = 2 if rid % 2 == 0 else 3
        n = int(rng.integers(24, 90)) if dim == 2 else int(rng.integers(8, 18))
        alpha = float(np.exp(rng.uniform(np.log(0.01), 0.0)))
        dt = float(rng.uniform(1e-4, 1e-3))
        out.append(Request(rid, t, dim, n, alpha, dt, 5, 5000 + rid))
        t += 0.004
    return out


# the forms the serving run uses: FP32-AMG with the grid level stored per
# node; the K-cycle on level 1 in 2D, the V-cycle in 3D
SERVED = dict(precision="fp32_amg", fine_operator="factored", nu_pre=0, nu_post=2)
SERVED_BY_DIM = {2: dict(kcycle_depth=1), 3: dict(kcycle_depth=0)}


def test_alone_equals_mix():
    """The served forms at the serving tolerance: each request's final field
    is bitwise the same alone and in the mix."""
    from paper_2608_09102_amd.serve import HipRunner, Server
    say("[serving alone vs mix]")
    reqs = _requests()
    runner = HipRunner(opts_kw=dict(rtol=1e-8, **SERVED), workers=4, opts_by_dim=SERVED_BY_DIM)
    alone = {}
    for r in reqs:
        alone[r.rid] = runner.run(r, 0, lambda ms, it: None)
    rep = Server(runner, budget_bytes=40 * 2 ** 30, workers=4).run(reqs, keep_results=True)
    say("  done %d, step p50 %.2f ms p99 %.2f ms" % (rep["done"], rep["step_ms_p50"], rep["step_ms_p99"]))
    assert rep["done"] == len(reqs)
    for o in rep["outcomes"]:
        assert np.array_equal(o.result, alone[o.rid]), o.rid
        assert len(o.step_ms) == 5
        nrm = np.linalg.norm(o.result, axis=1)
        assert np.abs(nrm - 1).max() < 1e-12


def test_served_requests_match_oracle(orc):
    """The served forms through the serving loop, solved to rtol 1e-11: every
    request's field after its 5 steps (from its recipe's initial field,
    seed 5000 + r) within 1e-8 of the oracle's 5-step trajectory."""
    from paper_2608_09102_amd.serve import HipRunner, Server
    say("[served requests vs oracle]")
    reqs = _requests()
    runner = HipRunner(opts_kw=dict(rtol=1e-11, **SERVED), workers=4, opts_by_dim=SERVED_BY_DIM)
    rep = Server(runner, budget_bytes=40 * 2 ** 30, workers=4).run(reqs, keep_results=True)
    assert rep["done"] == len(reqs)
    by = {r.rid: r for r in reqs}
    for o in rep["outcomes"]:
        r = by[o.rid]
        g = orc.make_grid(r.dim, r.n)
        oo = orc.default_opts(rtol=1e-11, kcycle_depth=SERVED_BY_DIM[r.dim]["kcycle_depth"],
                              nu_pre=SERVED["nu_pre"], nu_post=SERVED["nu_post"])
        m = r.m0()
        for _ in range(r.steps):
            rc, m, _ = orc.step(g, oo, m, r.alpha, r.dt)
            assert rc == 0
        d = np.abs(o.result - m).max()
        say("  request %d (%dD n=%d): |gpu - oracle| = %.2e" % (o.rid, r.dim, r.n, d))
        assert d <= 1e-8, (o.rid, d)


def test_tight_budget_queues():
    from paper_2608_09102_amd.serve import HipRunner, Server
    say("[serving tight budget]")
    reqs = _requests()
    runner = HipRunner(opts_kw=dict(rtol=1e-8), workers=4)
    foot = [runner.footprint(r) for r in reqs]
    budget = max(foot) + min(foot) // 2
    rep = Server(runner, budget_bytes=budget, workers=4).run(reqs, keep_results=False)
    assert rep["done"] == len(reqs) and rep["rejected"] == 0
    assert rep["queue_s_p99"] > 0
    rep2 = Server(runner, budget_bytes=max(foot) - 1, workers=4).run(reqs)
    assert rep2["rejected"] >= 1 and rep2["done"] == len(reqs) - rep2["rejected"]
