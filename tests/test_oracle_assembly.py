"""Pins for the oracle's block assembly (damped semi-implicit system, Sec. 2.1).

The oracle assembles each 3x3 block from the component-wise form.  These
tests check it against the scheme written with vector operations instead:
A u = u + dt m x (L u) + alpha dt m x (m x (L u)), with L the Neumann
Laplacian built from Kronecker products, plus closed-form properties of the
operator.
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import apply_scheme, bsr_to_dense, laplacian


def _grid(orc, dim, n):
    return orc.make_grid(dim, n)


@pytest.mark.parametrize("dim,n,alpha,dt", [(2, 7, 0.1, 1e-3), (2, 12, 0.0, 5e-3), (3, 5, 1.0, 2e-3),
                                            (3, 4, 0.01, 1e-2)])
def test_blocks_match_cross_product_form(orc, dim, n, alpha, dt):
    g = _grid(orc, dim, n)
    N = n ** dim
    m = I.smooth_unit_field(dim, n, seed=11, sweeps=2)
    rp, ci, val = orc.assemble(g, m, alpha, dt)
    A = bsr_to_dense(rp, ci, val)
    L = laplacian(dim, n, 1.0 / n)
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal((N, 3))
        ref = apply_scheme(L, m, alpha, dt, u).ravel()
        got = A @ u.ravel()
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_pattern_sorted_with_diagonal(orc):
    for dim, n in [(2, 6), (3, 4)]:
        g = _grid(orc, dim, n)
        m = I.smooth_unit_field(dim, n, seed=1, sweeps=1)
        rp, ci, val = orc.assemble(g, m, 0.1, 1e-3)
        N = n ** dim
        L = laplacian(dim, n, 1.0)
        for i in range(N):
            cols = ci[rp[i]:rp[i + 1]]
            assert list(cols) == sorted(cols)
            assert i in cols
            assert set(cols) == set(L[i].indices)


def test_skew_part_constant_field_alpha0(orc):
    """alpha = 0, constant m: every off-diagonal block is s [m]x, so
    A + A^T = 2 I holds exactly (the commented remark after the undamped
    block form in Sec. 2.1)."""
    for dim, n in [(2, 8), (3, 4)]:
        g = _grid(orc, dim, n)
        N = n ** dim
        v = np.array([0.3, -0.5, 0.8])
        m = np.tile(v / np.linalg.norm(v), (N, 1))
        rp, ci, val = orc.assemble(g, m, 0.0, 1e-2)
        A = bsr_to_dense(rp, ci, val)
        assert np.array_equal(A + A.T, 2.0 * np.eye(3 * N))


def test_nodal_identity(orc):
    """m_i . (A u)_i = m_i . u_i for every u: m^T [m]x = 0 and
    m^T (m m^T - |m|^2 I) = 0 when |m| = 1."""
    dim, n = 2, 10
    g = _grid(orc, dim, n)
    m = I.smooth_unit_field(dim, n, seed=5, sweeps=3)
    rp, ci, val = orc.assemble(g, m, 0.3, 1e-3)
    A = bsr_to_dense(rp, ci, val)
    u = np.random.default_rng(0).standard_normal((n * n, 3))
    Au = (A @ u.ravel()).reshape(-1, 3)
    lhs = (m * Au).sum(1)
    rhs = (m * u).sum(1)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(Au).max()


@pytest.mark.parametrize("alpha", [0.0, 0.05, 1.0])
def test_nonsingular(orc, alpha):
    """A u = 0 forces <u, -L u> = -alpha dt sum |m x L u|^2 <= 0, so u is
    constant and then u = 0: the smallest singular value is positive."""
    dim, n = 2, 6
    g = _grid(orc, dim, n)
    m = I.smooth_unit_field(dim, n, seed=9, sweeps=0)
    rp, ci, val = orc.assemble(g, m, alpha, 4e-2)
    A = bsr_to_dense(rp, ci, val)
    s = np.linalg.svd(A, compute_uv=False)
    assert s.min() > 1e-3
