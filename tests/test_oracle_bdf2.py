"""Pins for the oracle's BDF2 step (second-order backward differentiation with
second-order extrapolation m~ = 2 m^n - m^{n-1}; the first-order scheme of
Sec. 2.1 raised to second order, with the same operator structure).

- Scheme identity: the unprojected solution satisfies the BDF2 equation
  (3u - 4m^n + m^{n-1}) / (2dt) = -m~ x L u - alpha m~ x (m~ x L u) + F,
  with L the tensor-product Laplacian built here with scipy and the cross
  products taken with numpy.
- Special case: with m^{n-1} = m^n it is the BDF1 step with dt' = 2dt/3.
- Manufactured solution (forcing from the discrete Laplacian, so the error is
  purely temporal): second-order convergence in time.
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import laplacian


def _fields(dim, n):
    a = I.smooth_unit_field(dim, n, seed=11)
    b = I.smooth_unit_field(dim, n, seed=12)
    m_nm1 = a
    m_n = a + 0.05 * (b - a)
    m_n /= np.linalg.norm(m_n, axis=1, keepdims=True)
    return m_n, m_nm1


@pytest.mark.parametrize("dim,n", [(2, 14), (3, 6)])
def test_bdf2_scheme_identity(orc, dim, n):
    m_n, m_nm1 = _fields(dim, n)
    alpha, dt = 0.2, 2e-3
    rng = np.random.default_rng(4)
    F = rng.standard_normal(m_n.shape)
    g = orc.make_grid(dim, n)
    rc, u, st = orc.step2(g, orc.default_opts(rtol=1e-13, project=0, max_coarse=8), m_n, m_nm1, alpha, dt, F)
    assert rc == 0
    L = laplacian(dim, n, 1.0 / n)
    mt = 2 * m_n - m_nm1
    Lu = L @ u
    mxl = np.cross(mt, Lu)
    lhs = (3 * u - 4 * m_n + m_nm1) / (2 * dt)
    rhs = -mxl - alpha * np.cross(mt, mxl) + F
    scale = np.abs(lhs).max() + np.abs(rhs).max()
    assert np.abs(lhs - rhs).max() <= 1e-9 * scale


def test_bdf2_with_equal_history_is_bdf1(orc):
    dim, n = 2, 16
    m = I.smooth_unit_field(dim, n, seed=2)
    g = orc.make_grid(dim, n)
    o = orc.default_opts(rtol=1e-13)
    rc, a, _ = orc.step2(g, o, m, m, 0.1, 3e-3)
    rc2, b, _ = orc.step(g, o, m, 0.1, (2.0 * 3e-3) / 3.0)
    assert rc == 0 and rc2 == 0
    assert np.abs(a - b).max() <= 1e-12


def _mms_bdf2(orc, n, alpha, T, nt, project):
    dim = 2
    g = orc.make_grid(dim, n)
    L = laplacian(dim, n, 1.0 / n)
    dt = T / nt
    o = orc.default_opts(rtol=1e-13, project=project, max_coarse=16)
    x, y = I.cell_centres(dim, n)
    xbar = x * x * (1 - x) ** 2 + y * y * (1 - y) ** 2

    def forcing(t):
        me = I.exact_solution(dim, n, t)
        s, c = np.sin(t), np.cos(t)
        dme = np.stack([np.cos(xbar) * c, np.sin(xbar) * c, np.full(len(x), -s)], axis=1)
        mxl = np.cross(me, L @ me)
        return dme + mxl + alpha * np.cross(me, mxl)

    m_prev = I.exact_solution(dim, n, 0.0)
    # start-up: the exact value at t = dt (the error then measures the BDF2 steps alone)
    m = I.exact_solution(dim, n, dt)
    for k in range(1, nt):
        rc, m_new, _ = orc.step2(g, o, m, m_prev, alpha, dt, forcing((k + 1) * dt))
        assert rc == 0
        m_prev, m = m, m_new
    return np.abs(m - I.exact_solution(dim, n, T)).max()


@pytest.mark.parametrize("project", [0, 1])
def test_manufactured_second_order(orc, project):
    n, alpha, T = 16, 0.1, 0.5
    errs = [_mms_bdf2(orc, n, alpha, T, nt, project) for nt in (8, 16, 32, 64)]
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    if project == 0:
        assert all(1.8 <= p <= 2.3 for p in orders), (errs, orders)
    else:
        assert orders[-1] >= 1.7 and errs[-1] < errs[0], (errs, orders)
