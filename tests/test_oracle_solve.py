"""Pins for the oracle's solve and step.

T1 dense LU, T6 discrete energy identity, T8 constant-field fixed point,
T10 FGMRES versus the preconditioned GCR of Algorithm 1, T11 projection,
plus iteration-count regression bands for the workloads.
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import apply_scheme, dense_scheme_matrix, laplacian


@pytest.mark.parametrize("dim,n,max_coarse,alpha,dt", [
    (2, 4, 256, 0.1, 1e-2),     # single level: exact dense solve
    (2, 12, 8, 0.1, 1e-2),      # several levels
    (2, 16, 4, 0.02, 5e-2),
    (3, 4, 256, 1.0, 1e-2),
    (3, 6, 6, 0.01, 1e-2),
])
def test_step_matches_dense_lu(orc, dim, n, max_coarse, alpha, dt):
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=21, sweeps=2)
    o = orc.default_opts(rtol=1e-13, project=0, max_coarse=max_coarse)
    rc, u, st = orc.step(g, o, m, alpha, dt)
    assert rc == 0
    A = dense_scheme_matrix(laplacian(dim, n, 1.0 / n), m, alpha, dt)
    x = np.linalg.solve(A, m.ravel())
    assert np.abs(x - u.ravel()).max() <= 1e-11 * np.abs(x).max()
    if max_coarse < n ** dim:
        assert st.levels >= 2


def test_energy_identity(orc):
    """E(u) - E(m) + E(u - m) = -alpha dt sum |m x L u|^2 with E(v) = 1/2 <v, -L v>
    (dot product of the damped scheme with -L u)."""
    dim, n, alpha, dt = 2, 20, 0.2, 2e-3
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=4, sweeps=4)
    o = orc.default_opts(rtol=1e-14, project=0, max_coarse=16)
    rc, u, _ = orc.step(g, o, m, alpha, dt)
    assert rc == 0
    L = laplacian(dim, n, 1.0 / n)

    def E(v):
        return 0.5 * float((v * (-(L @ v))).sum())

    lhs = E(u) - E(m) + E(u - m)
    rhs = -alpha * dt * float((np.cross(m, L @ u) ** 2).sum())
    assert abs(lhs - rhs) <= 1e-10 * abs(E(m))


def test_constant_field_is_fixed(orc):
    """L m = 0 for a constant field, so m^{n+1} = m^n (the e3 initial state)."""
    for dim, n in [(2, 20), (3, 8)]:
        g = orc.make_grid(dim, n)
        m = np.tile(np.array([0.0, 0.0, 1.0]), (n ** dim, 1))
        rc, m1, st = orc.step(g, orc.default_opts(), m, 0.1, 1e-3)
        assert rc == 0
        assert st.iters == 0
        assert np.array_equal(m1, m)


def test_projection_unit_length(orc):
    dim, n = 2, 32
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=8)
    rc, m1, _ = orc.step(g, orc.default_opts(), m, 0.1, 1e-3)
    assert rc == 0
    nrm = np.sqrt((m1 * m1).sum(1))
    assert np.abs(nrm - 1.0).max() <= 4 * np.finfo(float).eps


def test_nodal_identity_of_solution(orc):
    """m . u = m . b node by node holds for the exact solution, and for an
    iterate up to the residual."""
    dim, n = 2, 24
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=3)
    o = orc.default_opts(rtol=1e-13, project=0)
    rc, u, _ = orc.step(g, o, m, 0.05, 2e-3)
    assert rc == 0
    assert np.abs((m * u).sum(1) - 1.0).max() <= 1e-10


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_fgmres_equals_gcr(orc, k):
    """Algorithm 1 (GCR) and FGMRES minimize the same residual over the same
    space for a fixed linear preconditioner, so their k-th iterates agree."""
    dim, n = 2, 24
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=13)
    b = m.copy()
    res = []
    for kry in (0, 1):
        o = orc.default_opts(rtol=1e-30, restart=30, max_iters=k, krylov=kry, max_coarse=16)
        H = orc.Hierarchy(g, o, m, 0.1, 5e-3)
        rc, u, st = H.solve(b, m)
        assert st.iters == k
        res.append(u)
    assert np.abs(res[0] - res[1]).max() <= 1e-12 * np.abs(res[0]).max()


def test_not_converged_reports(orc):
    dim, n = 2, 32
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=1)
    rc, m1, st = orc.step(g, orc.default_opts(rtol=1e-14, max_iters=1), m, 0.1, 1e-2)
    assert rc == orc.LLGO_ERR_NOT_CONVERGED
    assert st.iters == 1 and st.converged == 0
    assert np.isfinite(m1).all()


def test_nonfinite_input(orc):
    g = orc.make_grid(2, 8)
    m = np.tile(np.array([0.0, 0.0, 1.0]), (64, 1))
    m[5, 1] = np.nan
    rc, _, _ = orc.step(g, orc.default_opts(), m, 0.1, 1e-3)
    assert rc == orc.LLGO_ERR_NONFINITE


def test_vortex64_iteration_band(orc):
    """Regression band for the 64x64 vortex workload (not a paper number)."""
    w = I.WORKLOADS["vortex64"]
    g = orc.make_grid(2, w.n)
    rc, _, st = orc.step(g, orc.default_opts(rtol=w.rtol), w.m0(), w.alpha, w.dt)
    assert rc == 0
    assert 20 <= st.iters <= 45
    assert st.levels == 5
