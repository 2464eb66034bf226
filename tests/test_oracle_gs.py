"""Pins for the oracle's multicolour block Gauss-Seidel smoother variant
(Sec. 3 names Gauss-Seidel smoothing; the colour classes make it parallel).

- The colouring: level 0 is the parity of i + j + k; every coarse level is
  reproduced bit for bit by Jones-Plassmann rounds written here in pure
  Python (a node is coloured in the round where every neighbour of smaller
  priority is coloured, and takes the smallest colour they do not use), and it
  is a proper colouring of the level's matrix pattern.
- The smoother: the cycle with forward pre-sweeps and backward post-sweeps is
  the linear map built from dense block triangular solves on the operator
  permuted by colour class, (D + L)^{-1} forward and (D + U)^{-1} backward.
"""
import numpy as np
import pytest

import llg_inputs as I
from helpers import MASK, bsr_to_dense, sm64


def _prio(v, salt):
    return (sm64((((v << 32) | v) ^ salt) & MASK), v)


def jones_plassmann(rp, ci, salt):
    n = len(rp) - 1
    pr = [_prio(v, salt) for v in range(n)]
    nbr = [[int(j) for j in ci[rp[v]:rp[v + 1]] if j != v] for v in range(n)]
    col = [-1] * n
    while any(c < 0 for c in col):
        ready = [v for v in range(n) if col[v] < 0 and
                 all(col[u] >= 0 for u in nbr[v] if pr[u] < pr[v])]
        assert ready
        new = {}
        for v in ready:
            used = {col[u] for u in nbr[v] if col[u] >= 0}
            c = 0
            while c in used:
                c += 1
            new[v] = c
        for v, c in new.items():
            col[v] = c
    return np.array(col, np.int32)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 7)])
def test_colouring(orc, dim, n):
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=5)
    H = orc.Hierarchy(g, orc.default_opts(max_coarse=4, smoother=1), m, 0.1, 2e-3)
    assert H.num_levels >= 3
    for l in range(H.num_levels - 1):
        L = H.level(l)
        col, k = H.colour(l)
        assert col.min() == 0 and col.max() == k - 1
        # proper: no block of the pattern joins two rows of one class
        for i in range(len(L.rp) - 1):
            for j in L.ci[L.rp[i]:L.rp[i + 1]]:
                assert j == i or col[i] != col[j]
        if l == 0:
            idx = np.arange(n ** dim)
            par = (idx % n + (idx // n) % n + (idx // n // n)) & 1
            assert np.array_equal(col, par.astype(np.int32))
            assert k == 2
        else:
            salt = (l << 8) | 0x80
            assert np.array_equal(col, jones_plassmann(L.rp, L.ci, salt))


def _block_tri(A, order_pos, lower):
    n = A.shape[0] // 3
    pi = order_pos[:, None]
    pj = order_pos[None, :]
    mask = (pi >= pj) if lower else (pi <= pj)
    return A * np.kron(mask, np.ones((3, 3)))


def _dense_gs_cycle(levels, l=0):
    A, col, agg = levels[l]
    n3 = A.shape[0]
    if l == len(levels) - 1:
        return np.linalg.inv(A)
    n = n3 // 3
    pos = np.empty(n, np.int64)
    pos[np.lexsort((np.arange(n), col))] = np.arange(n)
    Sf = np.linalg.inv(_block_tri(A, pos, True))
    Sb = np.linalg.inv(_block_tri(A, pos, False))
    nc = int(agg.max()) + 1
    P = np.zeros((n, nc))
    P[np.arange(n), agg] = 1.0
    P3 = np.kron(P, np.eye(3))
    Bc = _dense_gs_cycle(levels, l + 1)
    M1 = Sf
    M2 = M1 + P3 @ Bc @ P3.T @ (np.eye(n3) - A @ M1)
    return M2 + Sb @ (np.eye(n3) - A @ M2)


@pytest.mark.parametrize("dim,n,max_coarse", [(2, 10, 6), (3, 5, 8)])
def test_gs_cycle_matches_dense_triangular_solves(orc, dim, n, max_coarse):
    g = orc.make_grid(dim, n)
    m = I.smooth_unit_field(dim, n, seed=41)
    H = orc.Hierarchy(g, orc.default_opts(max_coarse=max_coarse, smoother=1), m, 0.1, 3e-3)
    assert H.num_levels >= 3
    levels = []
    for l in range(H.num_levels):
        L = H.level(l)
        A = bsr_to_dense(L.rp, L.ci, L.val)
        col = H.colour(l)[0] if l < H.num_levels - 1 else None
        levels.append((A, col, L.agg))
    B0 = _dense_gs_cycle(levels)
    F = H.level(-1)
    N = n ** dim
    D0inv = np.zeros((3 * N, 3 * N))
    for i in range(N):
        D0inv[3 * i:3 * i + 3, 3 * i:3 * i + 3] = F.dinv[i]
    Bref = B0 @ D0inv
    rng = np.random.default_rng(3)
    for _ in range(4):
        v = rng.standard_normal(3 * N)
        z = H.precond(v.reshape(N, 3)).ravel()
        ref = Bref @ v
        assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()


def test_gs_reduces_iterations(orc):
    """Regression band: on the evolved rough 64^2 field Gauss-Seidel smoothing
    needs fewer FGMRES iterations than block Jacobi, V- and K-cycle alike."""
    n, c = 64, 104.9
    g = orc.make_grid(2, n)
    m = I.smooth_unit_field(2, n, seed=2)
    for _ in range(8):
        rc, m, _ = orc.step(g, orc.default_opts(rtol=1e-8), m, 0.02, c / n ** 2)
    for kd in (0, 1):
        its = []
        for sm in (0, 1):
            rc, _, st = orc.step(g, orc.default_opts(rtol=1e-8, kcycle_depth=kd, smoother=sm), m, 0.02, c / n ** 2)
            assert rc == 0
            its.append(st.iters)
        assert its[1] < its[0], (kd, its)
