"""GPU parity of the BDF2 step (m~ = 2 m^n - m^{n-1}, dt' = 2 dt / 3).

Bars: the assembled operator and every hierarchy level bit-exact against the
oracle's hierarchy at (m~, dt'); steps within 1e-8 of the oracle's BDF2 step
(both at rtol 1e-11); second-order convergence in time of the GPU path on a
manufactured solution.
"""
import sys

import numpy as np
import pytest

import llg_inputs as I
from helpers import laplacian

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    import paper_2608_09102_amd as llg
    assert torch.cuda.is_available()
    return llg


def _cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _history(dim, n):
    a = I.smooth_unit_field(dim, n, seed=21)
    b = I.smooth_unit_field(dim, n, seed=22)
    m_n = a + 0.1 * (b - a)
    return m_n / np.linalg.norm(m_n, axis=1, keepdims=True), a


@pytest.mark.parametrize("dim,n", [(2, 48), (3, 14)])
def test_bdf2_levels_bitwise(gpu, orc, dim, n):
    say("[bdf2_levels_bitwise]", dim, n)
    m_n, m_nm1 = _history(dim, n)
    alpha, dt = 0.1, 1e-3
    S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(rtol=1e-10, scheme="bdf2"))
    out, s, st = S.step(_cuda(m_n), alpha, dt, m_nm1=_cuda(m_nm1))
    assert s == gpu.OK
    mt = 2.0 * m_n - m_nm1
    H = orc.Hierarchy(orc.make_grid(dim, n), orc.default_opts(), mt, alpha, (2.0 * dt) / 3.0)
    assert S.num_levels == H.num_levels
    for l in range(-1, H.num_levels):
        rp, ci, val = S.level(l)
        R = H.level(l)
        assert np.array_equal(ci, R.ci) and np.array_equal(val, R.val), l


@pytest.mark.parametrize("precision", ["fp64", "fp32_amg"])
def test_bdf2_steps(gpu, orc, precision):
    """A BDF1 start step, then BDF2 steps: each step from the same history
    matches the oracle's step to 1e-8 (FP32-AMG: error stated, 1e-7 bound)."""
    say("[bdf2_steps]", precision)
    w = I.WORKLOADS["vortex64"]
    og = orc.make_grid(2, w.n)
    oo = orc.default_opts(rtol=1e-11)
    S = gpu.Solver(gpu.make_grid(2, w.n), gpu.default_opts(rtol=1e-11, scheme="bdf2", precision=precision))
    tol = 1e-8 if precision == "fp64" else 1e-7
    m0 = w.m0()
    out, s, st = S.step(_cuda(m0), w.alpha, w.dt)  # no history: BDF1
    rc, ref, _ = orc.step(og, oo, m0, w.alpha, w.dt)
    d = np.abs(out.cpu().numpy() - ref).max()
    say("  start (BDF1) iters %d diff %.2e" % (st.iters, d))
    assert s == gpu.OK and d <= tol
    prev, cur = m0, ref
    for k in range(4):
        out, s, st = S.step(_cuda(cur), w.alpha, w.dt, m_nm1=_cuda(prev))
        rc, ref, ost = orc.step2(og, oo, cur, prev, w.alpha, w.dt)
        assert s == gpu.OK and rc == 0
        d = np.abs(out.cpu().numpy() - ref).max()
        say("  BDF2 step %d iters gpu %d orc %d diff %.2e" % (k, st.iters, ost.iters, d))
        assert d <= tol
        prev, cur = cur, ref


def test_bdf2_second_order_on_gpu(gpu):
    """Manufactured solution with the forcing built from the discrete
    Laplacian: the GPU BDF2 path (unprojected) converges with order 2."""
    say("[bdf2_second_order_on_gpu]")
    dim, n, alpha, T = 2, 24, 0.1, 0.5
    L = laplacian(dim, n, 1.0 / n)
    x, y = I.cell_centres(dim, n)
    xbar = x * x * (1 - x) ** 2 + y * y * (1 - y) ** 2

    def forcing(t):
        me = I.exact_solution(dim, n, t)
        s, c = np.sin(t), np.cos(t)
        dme = np.stack([np.cos(xbar) * c, np.sin(xbar) * c, np.full(len(x), -s)], axis=1)
        mxl = np.cross(me, L @ me)
        return dme + mxl + alpha * np.cross(me, mxl)

    errs = []
    for nt in (8, 16, 32):
        dt = T / nt
        S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(rtol=1e-12, scheme="bdf2", project=0))
        prev = _cuda(I.exact_solution(dim, n, 0.0))
        cur = _cuda(I.exact_solution(dim, n, dt))
        for k in range(1, nt):
            nxt, s, _ = S.step(cur, alpha, dt, forcing=_cuda(forcing((k + 1) * dt)), m_nm1=prev)
            assert s == gpu.OK
            prev, cur = cur, nxt
        errs.append(float(np.abs(cur.cpu().numpy() - I.exact_solution(dim, n, T)).max()))
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    say("  errors", errs, "orders", orders)
    assert all(1.8 <= p <= 2.3 for p in orders), (errs, orders)
