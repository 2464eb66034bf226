"""Pins for the oracle's V-cycle (Sec. 3) and the scheme's temporal order.

T12: the preconditioner is a linear map; applied to unit vectors it must equal
the matrix built from the multigrid recursion written with dense numpy
operators (smoother S = omega D^{-1}, restriction P^T, prolongation P, exact
inverse at the coarsest level).
T9: a manufactured solution with the forcing evaluated by the discrete
Laplacian shows first-order convergence in time (BDF1, Sec. 2.1).
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import bsr_to_dense, laplacian


def _dense_vcycle(levels, omega, l=0):
    """Matrix B_l of the V-cycle with one pre- and one post-smoothing sweep."""
    A, Dinv, agg = levels[l]
    n3 = A.shape[0]
    if l == len(levels) - 1:
        return np.linalg.inv(A)
    S = omega * Dinv
    nc = int(agg.max()) + 1
    P = np.zeros((n3 // 3, nc))
    P[np.arange(n3 // 3), agg] = 1.0
    P3 = np.kron(P, np.eye(3))
    Bc = _dense_vcycle(levels, omega, l + 1)
    M1 = S
    M2 = M1 + P3 @ Bc @ P3.T @ (np.eye(n3) - A @ M1)
    return M2 + S @ (np.eye(n3) - A @ M2)


@pytest.mark.parametrize("dim,n,max_coarse", [(2, 10, 6), (3, 5, 8)])
def test_vcycle_matches_dense_recursion(orc, dim, n, max_coarse):
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=31)
    H = orc.Hierarchy(g, orc.default_opts(max_coarse=max_coarse), m, 0.1, 3e-3)
    assert H.num_levels >= 3
    levels = []
    for l in range(H.num_levels):
        L = H.level(l)
        A = bsr_to_dense(L.rp, L.ci, L.val)
        N = len(L.rp) - 1
        Dinv = np.zeros((3 * N, 3 * N))
        for i in range(N):
            Dinv[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.linalg.inv(A[3 * i:3 * i + 3, 3 * i:3 * i + 3])
        levels.append((A, Dinv, L.agg))
    omega = 4.0 / 5.0 if dim == 2 else 6.0 / 7.0
    B0 = _dense_vcycle(levels, omega)
    F = H.level(-1)
    Af = bsr_to_dense(F.rp, F.ci, F.val)
    N = n ** dim
    D0inv = np.zeros((3 * N, 3 * N))
    for i in range(N):
        D0inv[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.linalg.inv(Af[3 * i:3 * i + 3, 3 * i:3 * i + 3])
    Bref = B0 @ D0inv
    rng = np.random.default_rng(0)
    for _ in range(4):
        v = rng.standard_normal(3 * N)
        z = H.precond(v.reshape(N, 3)).ravel()
        ref = Bref @ v
        assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()


def _dense_cycle_apply(levels, omega, kdepth, l, b):
    """The cycle applied to b with dense operators: V-cycle recursion, except
    that the coarse equation of levels 1..kdepth (not the coarsest) is solved
    by two minimal-residual steps preconditioned by that level's cycle."""
    A, Dinv, agg = levels[l]
    n3 = A.shape[0]
    if l == len(levels) - 1:
        return np.linalg.solve(A, b)
    S = omega * Dinv
    nc = int(agg.max()) + 1
    P = np.zeros((n3 // 3, nc))
    P[np.arange(n3 // 3), agg] = 1.0
    P3 = np.kron(P, np.eye(3))
    x = S @ b
    rc = P3.T @ (b - A @ x)
    lc = l + 1
    if lc < len(levels) - 1 and lc <= kdepth:
        Ac = levels[lc][0]
        v1 = _dense_cycle_apply(levels, omega, kdepth, lc, rc)
        v2 = _dense_cycle_apply(levels, omega, kdepth, lc, rc - ((Ac @ v1) @ rc) / ((Ac @ v1) @ (Ac @ v1)) * (Ac @ v1))
        # e minimizes || rc - Ac e || over span{v1, v2}
        W = np.stack([Ac @ v1, Ac @ v2], 1)
        g = np.linalg.lstsq(W, rc, rcond=None)[0]
        ec = g[0] * v1 + g[1] * v2
    else:
        ec = _dense_cycle_apply(levels, omega, kdepth, lc, rc)
    x = x + P3 @ ec
    return x + S @ (b - A @ x)


@pytest.mark.parametrize("kdepth", [1, 2, 5])
def test_kcycle_matches_dense_recursion(orc, kdepth):
    dim, n = 2, 14
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=17)
    H = orc.Hierarchy(g, orc.default_opts(max_coarse=4, kcycle_depth=kdepth), m, 0.05, 4e-3)
    assert H.num_levels >= 4
    levels = []
    for l in range(H.num_levels):
        L = H.level(l)
        A = bsr_to_dense(L.rp, L.ci, L.val)
        N = len(L.rp) - 1
        Dinv = np.zeros((3 * N, 3 * N))
        for i in range(N):
            Dinv[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.linalg.inv(A[3 * i:3 * i + 3, 3 * i:3 * i + 3])
        levels.append((A, Dinv, L.agg))
    F = H.level(-1)
    Af = bsr_to_dense(F.rp, F.ci, F.val)
    N = n ** dim
    D0inv = np.zeros((3 * N, 3 * N))
    for i in range(N):
        D0inv[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.linalg.inv(Af[3 * i:3 * i + 3, 3 * i:3 * i + 3])
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.standard_normal(3 * N)
        z = H.precond(v.reshape(N, 3)).ravel()
        ref = _dense_cycle_apply(levels, 0.8, kdepth, 0, D0inv @ v)
        assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()


def test_kcycle_reduces_iterations(orc):
    """Regression band: on a rough field at large dt/h^2 the K-cycle needs
    clearly fewer FGMRES iterations than the V-cycle."""
    n, c = 64, 104.9
    g = orc.make_grid(2, n)
    m = I.smooth_unit_field(2, n, seed=2)
    for _ in range(8):  # let the field evolve: the V-cycle degrades on it
        rc, m, _ = orc.step(g, orc.default_opts(rtol=1e-8), m, 0.02, c / n ** 2)
    its = []
    for kd in (0, 2):
        rc, _, st = orc.step(g, orc.default_opts(rtol=1e-8, kcycle_depth=kd), m, 0.02, c / n ** 2)
        assert rc == 0
        its.append(st.iters)
    assert its[1] < 0.6 * its[0], its


def _mms_run(orc, n, alpha, T, nt, project):
    dim = 2
    g = orc.make_grid(dim, n)
    L = laplacian(dim, n, 1.0 / n)
    dt = T / nt
    m = I.exact_solution(dim, n, 0.0)
    o = orc.default_opts(rtol=1e-13, project=project, max_coarse=16)
    x, y = I.cell_centres(dim, n)
    xbar = x * x * (1 - x) ** 2 + y * y * (1 - y) ** 2
    for k in range(nt):
        t1 = (k + 1) * dt
        me = I.exact_solution(dim, n, t1)
        s, c = np.sin(t1), np.cos(t1)
        # d/dt m_e = (cos(xbar) cos t, sin(xbar) cos t, -sin t)
        dme = np.stack([np.cos(xbar) * c, np.sin(xbar) * c, np.full(len(x), -s)], axis=1)
        lm = L @ me
        mxl = np.cross(me, lm)
        F = dme + mxl + alpha * np.cross(me, mxl)
        rc, m, _ = orc.step(g, o, m, alpha, dt, F)
        assert rc == 0
    return np.abs(m - I.exact_solution(dim, n, T)).max()


@pytest.mark.parametrize("project", [0, 1])
def test_manufactured_first_order(orc, project):
    n, alpha, T = 16, 0.1, 0.5
    errs = [_mms_run(orc, n, alpha, T, nt, project) for nt in (8, 16, 32, 64)]
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    if project == 0:
        assert all(0.85 <= p <= 1.25 for p in orders), (errs, orders)
    else:
        assert orders[-1] >= 0.85, (errs, orders)
        assert errs[-1] < errs[0]
