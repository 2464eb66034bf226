"""Pins for the oracle's full field (Sec. 2: exchange coefficient, uniaxial
anisotropy, external field, stray field) and its entry into the scheme.

- Demagnetizing tensor: a cubic cell's self term is I/3 and every cuboid's has
  trace 1; the tensor has the parities of its components; beyond the switch
  distance it is the point-dipole tensor, and just inside it agrees with the
  dipole to the order of the next multipole; for cells at least one side apart
  it equals the defining cell average of the point kernel, evaluated by
  Gauss-Legendre quadrature in numpy, to about 1e-15 absolute.
- Sum rule: the cell-averaged tensors of the cells of a box, summed over one
  cell and averaged over all, are the box's demagnetizing tensor; for a cube
  that is I/3, for any box its trace is 1.
- The step: for a uniform field the Laplacian vanishes and the solution is the
  explicit update m - dt (m x f + alpha m x (m x f)) in closed form; on a
  general field the unprojected solution satisfies the scheme of Sec. 2.1 with
  the full field, checked with a scipy Laplacian and numpy cross products.
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import laplacian


def test_demag_self_terms(orc):
    N = orc.demag_tensor(0, 0, 0, 1.0, 1.0, 1.0)
    assert np.allclose(N[:3], 1.0 / 3.0, atol=1e-14) and np.allclose(N[3:], 0.0, atol=1e-15)
    for d in [(1.0, 1.0, 0.1), (2.0, 0.5, 1.0), (1.0, 3.0, 0.2)]:
        N = orc.demag_tensor(0, 0, 0, *d)
        assert abs(N[:3].sum() - 1.0) <= 1e-12 and np.abs(N[3:]).max() <= 1e-13


def test_demag_parities(orc):
    X, Y, Z = 2.0, -3.0, 1.0
    N = orc.demag_tensor(X, Y, Z, 1, 1, 1)
    for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]:
        M = orc.demag_tensor(sx * X, sy * Y, sz * Z, 1, 1, 1)
        assert np.allclose(M[:3], N[:3], rtol=1e-12)
        assert np.isclose(M[3], sx * sy * N[3], rtol=1e-12)
        assert np.isclose(M[4], sx * sz * N[4], rtol=1e-12)
        assert np.isclose(M[5], sy * sz * N[5], rtol=1e-12)


def _dipole(X, Y, Z, V=1.0):
    r = np.array([X, Y, Z], float)
    r2 = r @ r
    T = -(V / (4 * np.pi)) * (3 * np.outer(r, r) / r2 - np.eye(3)) / r2 ** 1.5
    return np.array([T[0, 0], T[1, 1], T[2, 2], T[0, 1], T[0, 2], T[1, 2]])


def test_demag_far_field(orc):
    for X, Y, Z in [(20.0, 3.0, -2.0), (0.0, 17.0, 5.0)]:
        assert np.allclose(orc.demag_tensor(X, Y, Z, 1, 1, 1), _dipole(X, Y, Z), rtol=1e-12, atol=1e-18)
    for X, Y, Z in [(15.0, 4.0, 2.0), (10.0, 10.0, 0.5)]:  # Newell inside the switch: next multipole small
        N = orc.demag_tensor(X, Y, Z, 1, 1, 1)
        D = _dipole(X, Y, Z)
        assert np.abs(N - D).max() <= 2e-3 * np.abs(D).max()


def _cell_average(X, Y, Z, d, nodes=16):
    """The defining integral of the cell-averaged tensor between two cuboid
    cells of sides d whose centres are (X, Y, Z) apart: the average over one
    cell of the field of the other, uniformly magnetized, is
    -1/(4 pi V) int prod_a (d_a - |u_a|) K(r + u) du with the point kernel
    K_ab(y) = (3 y_a y_b - delta_ab |y|^2) / |y|^5 (the tent is the
    autocorrelation of the cell).  For cells more than one side apart along
    some axis the integrand is analytic on the domain, and tensor-product
    Gauss-Legendre quadrature (each axis folded onto [0, d_a], the tent
    becoming a weight) converges to the last digit."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (x + 1.0)
    wt = 0.5 * w * (1.0 - t)
    s = np.concatenate([t, -t])
    ws = np.concatenate([wt, wt])
    A, B, C = np.meshgrid(s * d[0] + X, s * d[1] + Y, s * d[2] + Z, indexing="ij")
    W = ws[:, None, None] * ws[None, :, None] * ws[None, None, :]
    r2 = A * A + B * B + C * C
    r5 = r2 * r2 * np.sqrt(r2)
    K = [(3 * A * A - r2) / r5, (3 * B * B - r2) / r5, (3 * C * C - r2) / r5, 3 * A * B / r5, 3 * A * C / r5,
         3 * B * C / r5]
    # u = d s: du = V ds and prod (d_a - |u_a|) = V prod (1 - |s_a|), so the
    # integral over the folded unit tents carries V^2 / V = V
    V = d[0] * d[1] * d[2]
    return np.array([-V * (W * k).sum() / (4 * np.pi) for k in K])


@pytest.mark.parametrize("off", [(2, 0, 0), (2, 1, 0), (0, 2, 1), (2, 2, 2), (3, 1, -2), (-5, 3, 2), (8, 0, 0),
                                 (11, -9, 5), (12, 7, 0), (16, 0, 0), (16, 3, -1), (16, 16, 16), (0, 0, 9)])
def test_demag_against_cell_average_quadrature(orc, off):
    """The closed form (cubic cells) equals the defining cell average up to
    the switch, to a few units in the last place of the largest entry (I/3):
    a dropped term, a wrong sign or a permuted argument in f, g or the
    second difference shows up far above this bar."""
    N = orc.demag_tensor(float(off[0]), float(off[1]), float(off[2]), 1.0, 1.0, 1.0)
    Q = _cell_average(*off, d=(1.0, 1.0, 1.0))
    assert np.abs(N - Q).max() <= 1e-15, (N, Q)


@pytest.mark.parametrize("off,d", [((5.0, 0.0, 0.0), (2.0, 0.5, 1.0)), ((1.0, 3.0, 2.0), (1.0, 1.0, 0.25)),
                                   ((4.0, -1.0, 0.5), (1.5, 0.5, 0.5))])
def test_demag_cuboid_against_cell_average_quadrature(orc, off, d):
    """Cuboid cells (the spacings enter f, g and the second difference)."""
    N = orc.demag_tensor(*off, *d)
    Q = _cell_average(*off, d=d)
    assert np.abs(N - Q).max() <= 1e-14, (N, Q)


@pytest.mark.parametrize("n", [(4, 4, 4), (6, 3, 2)])
def test_demag_sum_rule(orc, n):
    nx, ny, nz = n
    acc = np.zeros(6)
    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for a in cells:
        for b in cells:
            acc += orc.demag_tensor(a[0] - b[0], a[1] - b[1], a[2] - b[2], 1, 1, 1)
    acc /= len(cells)
    assert abs(acc[:3].sum() - 1.0) <= 1e-12 and np.abs(acc[3:]).max() <= 1e-12
    if nx == ny == nz:
        assert np.allclose(acc[:3], 1.0 / 3.0, atol=1e-12)


def test_stray_field_of_uniform_cube(orc):
    n = 5
    g = orc.make_grid(3, n)
    m = np.tile(np.array([0.6, 0.0, 0.8]), (n ** 3, 1))
    h = orc.stray_field(g, m)
    assert np.allclose(h.mean(axis=0), -m[0] / 3.0, atol=1e-12)


def _explicit(m, f, alpha, dt):
    c1 = np.cross(m, f)
    return m - dt * (c1 + alpha * np.cross(m, c1))


@pytest.mark.parametrize("stray", [0, 1])
def test_uniform_field_step_closed_form(orc, stray):
    n, alpha, dt = 8, 0.3, 0.02
    g = orc.make_grid(2, n)
    m0 = np.array([0.36, 0.48, 0.8])
    m = np.tile(m0, (n * n, 1))
    fld = orc.make_field(eps=0.7, q=0.5, h_ext=(0.1, -0.2, 0.3), stray=stray)
    rc, u, st = orc.step_field(g, orc.default_opts(rtol=1e-13, project=0), m, alpha, dt, fld)
    assert rc == 0
    f = np.tile(np.array([0.1, -0.2, 0.3]), (n * n, 1)) - 0.5 * np.stack([0 * m[:, 0], m[:, 1], m[:, 2]], 1)
    if stray:
        f = f + orc.stray_field(g, m)
        # a uniform magnetization's stray field is not uniform: only the cell-wise closed form holds
        # when the Laplacian of the solution vanishes, so compare through the scheme residual below
        L = laplacian(2, n, 1.0 / n)
        ff = f
        lu = L @ u
        lhs = (u - m) / dt
        rhs = -np.cross(m, 0.7 * lu + ff) - alpha * np.cross(m, np.cross(m, 0.7 * lu + ff))
        assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(lhs).max()
    else:
        assert np.allclose(u, _explicit(m, f, alpha, dt), rtol=0, atol=1e-12)  # solved to rtol 1e-13


@pytest.mark.parametrize("bdf2", [False, True])
def test_field_scheme_identity(orc, bdf2):
    dim, n, alpha, dt = 2, 10, 0.2, 2e-3
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=13)
    mp = I.smooth_unit_field(dim, n, seed=14) if bdf2 else None
    eps, q, he = 0.5, 0.8, np.array([0.05, 0.1, -0.2])
    fld = orc.make_field(eps=eps, q=q, h_ext=tuple(he), stray=1)
    rc, u, st = orc.step_field(g, orc.default_opts(rtol=1e-13, project=0, max_coarse=8), m, alpha, dt, fld,
                               m_nm1=mp)
    assert rc == 0
    mt = 2 * m - mp if bdf2 else m
    f = he - q * np.stack([0 * mt[:, 0], mt[:, 1], mt[:, 2]], 1) + orc.stray_field(g, mt)
    L = laplacian(dim, n, 1.0 / n)
    hx = eps * (L @ u) + f
    lhs = (3 * u - 4 * m + mp) / (2 * dt) if bdf2 else (u - m) / dt
    rhs = -np.cross(mt, hx) - alpha * np.cross(mt, np.cross(mt, hx))
    assert np.abs(lhs - rhs).max() <= 1e-9 * (np.abs(lhs).max() + np.abs(rhs).max())


@pytest.mark.parametrize("dim,n", [(2, (13, 9)), (3, (5, 4, 6))])
def test_stray_field_at_is_the_full_sum(orc, dim, n):
    """The pointwise form sums the same terms in the same order as the full
    form: equal to the bit at every cell, so the pins of the full form carry
    over to the sampled one used at sizes the full form cannot reach."""
    N = int(np.prod(n))
    rng = np.random.default_rng(5)
    m = rng.standard_normal((N, 3))
    g = orc.make_grid(dim, n)
    full = orc.stray_field(g, m)
    cells = np.array([0, N - 1, N // 2, 1, n[0] - 1] + list(rng.integers(0, N, 5)))
    assert np.array_equal(orc.stray_field_at(g, m, cells), full[cells])
    assert orc.stray_field_at(g, m, []).shape == (0, 3)
