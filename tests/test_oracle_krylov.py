"""Pins for the oracle's Krylov baselines, the unpreconditioned solvers the
paper compares its multigrid solve against (GMRES, BiCGstab, TFQMR, Sec. 4).

- Each converges to the dense LU solution of the assembled system.
- Iterate by iterate they follow scipy's independent implementations of the
  same published algorithms: BiCGstab and TFQMR from the same start with the
  shadow vector r^ = r_0, and one restart cycle of GMRES(R) (the minimal
  residual over the same Krylov space).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import llg_inputs as I
from helpers import bsr_to_scipy


DT = 2e-4  # dt / h^2 = 0.03: a regime where all three baselines converge


def _system(orc, n=12, alpha=0.1, dt=DT, seed=4):
    """The assembled operator and a random right-hand side.  (With b = m^n and
    a zero start the shadow vector r^ = m would satisfy r^T A = r^T, since
    m_i^T M_i = 0, and BiCGstab would break down after one step.)"""
    g = orc.make_grid(2, n)
    m = I.smooth_unit_field(2, n, seed=seed)
    H = orc.Hierarchy(g, orc.default_opts(), m, alpha, dt)
    F = H.level(-1)
    A = bsr_to_scipy(F.rp, F.ci, F.val).tocsr()
    b = np.random.default_rng(seed).standard_normal(3 * n * n)
    return g, m, H, A, b


@pytest.mark.parametrize("krylov", [2, 3, 4])
def test_baselines_converge_to_lu(orc, krylov):
    g, m, _, A, b = _system(orc)
    H = orc.Hierarchy(g, orc.default_opts(krylov=krylov, rtol=1e-12, max_iters=5000), m, 0.1, DT)
    rc, u, st = H.solve(b.reshape(-1, 3), np.zeros_like(b).reshape(-1, 3))
    assert rc == 0 and st.converged
    x = np.linalg.solve(A.toarray(), b)
    assert np.abs(u.ravel() - x).max() <= 1e-9 * np.abs(x).max()
    assert np.linalg.norm(b - A @ u.ravel()) <= 1e-12 * np.linalg.norm(b)


def _iterates(fn, A, b, x0, n, **kw):
    xs = []
    fn(A, b, x0=x0.copy(), rtol=1e-300, atol=0.0, maxiter=n, callback=lambda xk: xs.append(np.array(xk)), **kw)
    return xs


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_bicgstab_follows_scipy(orc, k):
    g, m, _, A, b = _system(orc)
    x0 = np.zeros_like(b)
    xs = _iterates(spl.bicgstab, A, b, x0, k)
    H = orc.Hierarchy(g, orc.default_opts(krylov=3, rtol=1e-300, max_iters=k), m, 0.1, DT)
    rc, u, st = H.solve(b.reshape(-1, 3), x0.reshape(-1, 3))
    assert st.iters == k
    assert np.abs(u.ravel() - xs[k - 1]).max() <= 1e-11 * np.abs(xs[k - 1]).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_tfqmr_follows_scipy(orc, k):
    """scipy counts half-steps; one oracle iteration is two of them."""
    g, m, _, A, b = _system(orc)
    x0 = np.zeros_like(b)
    xs = _iterates(spl.tfqmr, A, b, x0, 2 * k)
    H = orc.Hierarchy(g, orc.default_opts(krylov=4, rtol=1e-300, max_iters=k), m, 0.1, DT)
    rc, u, st = H.solve(b.reshape(-1, 3), x0.reshape(-1, 3))
    assert st.iters == k
    assert np.abs(u.ravel() - xs[2 * k - 1]).max() <= 1e-11 * np.abs(xs[2 * k - 1]).max()


@pytest.mark.parametrize("R", [3, 8])
def test_gmres_cycle_is_minimal_residual(orc, R):
    g, m, _, A, b = _system(orc)
    x0 = np.zeros_like(b)
    H = orc.Hierarchy(g, orc.default_opts(krylov=2, rtol=1e-300, max_iters=R, restart=R), m, 0.1, DT)
    rc, u, st = H.solve(b.reshape(-1, 3), x0.reshape(-1, 3))
    assert st.iters == R
    # minimal residual over the Krylov space K_R(A, b), from an explicit basis
    K = np.empty((len(b), R))
    v = b / np.linalg.norm(b)
    for j in range(R):
        K[:, j] = v
        v = A @ v
        for q in range(j + 1):  # orthonormalize (twice) for a well-conditioned basis
            v -= (K[:, q] @ v) * K[:, q]
        for q in range(j + 1):
            v -= (K[:, q] @ v) * K[:, q]
        v /= np.linalg.norm(v)
    y = np.linalg.lstsq(A @ K, b, rcond=None)[0]
    xr = K @ y
    assert np.abs(u.ravel() - xr).max() <= 1e-10 * np.abs(xr).max()


def test_bicgstab_breaks_down_from_zero_on_m(orc):
    """The structural breakdown: b = m^n, start 0, r^ = r_0 = m^n gives
    (r_1, r^) = 0 up to rounding after the first step."""
    g, m, _, A, _ = _system(orc)
    b = m.ravel()
    r0 = b.copy()
    v = A @ r0
    alpha = (r0 @ r0) / (v @ r0)
    s = r0 - alpha * v
    t = A @ s
    omega = (t @ s) / (t @ t)
    r1 = s - omega * t
    assert abs(r1 @ r0) <= 1e-12 * np.linalg.norm(r1) * np.linalg.norm(r0)
