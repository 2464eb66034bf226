"""Hierarchy values bit for bit on grids large enough for the setup kernels
that only run on large levels (eq. galerkin, eq. Ac_direct, Sec. 3.1.1): the
Galerkin products of coarse levels of 65,536 nodes or more (one workgroup per
coarse slice from the grid level, stored as sliced ELL or per node; row by
row, a group of lanes per coarse row, from a coarse level's CSR-ordered copy),
the coarse-graph rows of more than 32 candidates (3D coarse levels), and the
matching rounds over many workgroups.

Bars: every level's pattern and FP64 values equal the oracle's (both sides add
the same blocks in the same order without contraction); the aggregates equal
the oracle's; FP32-AMG levels equal between the sliced-ELL and the per-node
grid form.
"""
import sys

import numpy as np
import pytest

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


def _rough(N, seed=7):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((N, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


# 3d_96: level 2 (about 70,000 nodes) is formed row by row from level 1's
# CSR-ordered blocks
CASES = [("2d_512", 2, 512, 0.05, 2e-5), ("3d_64", 3, 64, 0.3, 1e-3), ("3d_96", 3, 96, 0.3, 1e-3)]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_large_levels_bitwise(gpu, orc, case):
    name, dim, n, alpha, dt = case
    say("[large_levels_bitwise]", name)
    N = n ** dim
    m = _rough(N)
    H = orc.Hierarchy(orc.make_grid(dim, n), orc.default_opts(kcycle_depth=1), m, alpha, dt)
    nl = H.num_levels
    sizes = [len(H.level(l).rp) - 1 for l in range(nl)]
    say("  oracle levels", sizes)
    assert sizes[1] >= 65536  # level 1 is formed by the slice-parallel product
    forms = {}
    for op in ("bsr", "factored"):
        for prec in ("fp64", "fp32_amg"):
            S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(kcycle_depth=1, fine_operator=op, precision=prec))
            assert S.setup(_cuda(m), alpha, dt) == gpu.OK
            assert S.num_levels == nl
            forms[(op, prec)] = [S.level(l) for l in range(nl)]
            if prec == "fp64":
                for l in range(nl - 1):
                    assert np.array_equal(S.aggregates(l), H.level(l).agg), (op, l)
            S.close()
    for op in ("bsr", "factored"):
        for l in range(nl):
            rp, ci, val = forms[(op, "fp64")][l]
            R = H.level(l)
            assert np.array_equal(rp, R.rp) and np.array_equal(ci, R.ci), (op, l)
            assert np.array_equal(val, R.val), (op, l, np.abs(val - R.val).max())
    for l in range(nl):
        a, b = forms[("bsr", "fp32_amg")][l], forms[("factored", "fp32_amg")][l]
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), l
        # FP32-AMG levels are the FP64 ones rounded, up to the rounding of the
        # coarse sums formed in FP32
        rel = np.abs(a[2] - forms[("bsr", "fp64")][l][2]).max() / np.abs(forms[("bsr", "fp64")][l][2]).max()
        assert rel <= 1e-5, (l, rel)
    say("  %d levels equal" % nl)


# Large coarse levels applied from their CSR-ordered blocks (opts.csr_levels):
# grids with a level of at least 32768 nodes below the K-cycle levels (and
# below level 1 of the per-node grid form, which is applied through the grid
# blocks) and above the coarsest.
CSR_CASES = [
    # name, dim, n, alpha, dt, grid-level storage, K-cycle depth
    ("2d_512_bsr_v", 2, 512, 0.05, 2e-5, "bsr", 0),
    ("3d_96_factored_k1", 3, 96, 0.3, 1e-3, "factored", 1),
]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", CSR_CASES, ids=[c[0] for c in CSR_CASES])
def test_csr_levels_cycle(gpu, orc, case):
    """The cycle with the large levels' row products on the CSR-ordered copy
    against the oracle's cycle (FP64, 1e-12 relative, the V-cycle bar of the
    small grids) and against the sliced-ELL products (FP32-AMG: the two add a
    row's blocks in different orders)."""
    name, dim, n, alpha, dt, op, kd = case
    say("[csr_levels_cycle]", name)
    m = _rough(n ** dim)
    H = orc.Hierarchy(orc.make_grid(dim, n), orc.default_opts(kcycle_depth=kd), m, alpha, dt)
    sizes = [len(H.level(l).rp) - 1 for l in range(H.num_levels)]
    say("  oracle levels", sizes)
    first = max(2 if op == "factored" else 1, kd + 1)
    assert any(s >= 32768 for s in sizes[first:-1])
    v = np.random.default_rng(5).standard_normal(m.shape)
    zr = H.precond(v)
    out = {}
    for csr in (1, 0):
        for prec in ("fp64", "fp32_amg"):
            S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(kcycle_depth=kd, fine_operator=op, precision=prec,
                                                                   csr_levels=csr))
            assert S.setup(_cuda(m), alpha, dt) == gpu.OK
            out[(csr, prec)] = S.precond(_cuda(v)).cpu().numpy()
            S.close()
    for csr in (1, 0):
        d = np.abs(out[(csr, "fp64")] - zr).max() / np.abs(zr).max()
        say("  csr_levels %d: fp64 cycle vs oracle %.2e" % (csr, d))
        assert d <= 1e-12, (csr, d)
    d = np.abs(out[(1, "fp32_amg")] - out[(0, "fp32_amg")]).max() / np.abs(out[(0, "fp32_amg")]).max()
    say("  fp32_amg cycle, CSR vs sliced products %.2e" % d)
    assert d <= 1e-5, d
