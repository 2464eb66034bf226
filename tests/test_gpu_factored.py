"""GPU parity of the factored grid-level operator (one 3x3 block per node).

Bars:
- every hierarchy level bit-exact against the BSR form and the oracle (the
  per-node block is the value every off-diagonal slot holds, and the Galerkin
  sums keep their order);
- the outer operator A within 4 ulp-scale rounding of the oracle's BSR product:
  |Az - (Az)_ref| <= 1e-14 (|z| + (dt/h^2)|M||z| (2 deg)) per entry, taken as
  1e-13 of max|Az| on these inputs;
- the preconditioner within 1e-11 relative, steps within 1e-8 (the target).
"""
import sys

import numpy as np
import pytest

import llg_inputs as I

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


CASES = [
    ("vortex64", 2, (64, 64, 1), 1 / 64, 0.1, 1e-3),
    ("rect2d_37x23", 2, (37, 23, 1), 1 / 37, 0.05, 2e-3),
    ("box3d_9x7x5", 3, (9, 7, 5), 1 / 9, 1.0, 1e-2),
    ("cube3d_20", 3, (20, 20, 20), 1 / 20, 0.01, 5e-4),
]


def _rough(n, seed=7):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((int(np.prod(n)), 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32_amg"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_factored_levels_and_products(gpu, orc, case, precision):
    name, dim, n, h, alpha, dt = case
    say("[factored_levels_and_products]", name, precision)
    m = I.vortex_field(64, seed=1) if name == "vortex64" else _rough(n)
    g = gpu.make_grid(dim, n, h)
    Sf = gpu.Solver(g, gpu.default_opts(fine_operator="factored", precision=precision, kcycle_depth=1))
    Sb = gpu.Solver(g, gpu.default_opts(precision=precision, kcycle_depth=1))
    assert Sf.setup(_cuda(m), alpha, dt) == gpu.OK and Sb.setup(_cuda(m), alpha, dt) == gpu.OK
    H = orc.Hierarchy(orc.make_grid(dim, n, h), orc.default_opts(kcycle_depth=1), m, alpha, dt)
    assert Sf.num_levels == Sb.num_levels == H.num_levels
    for l in range(0, H.num_levels):
        rf, cf, vf = Sf.level(l)
        rb, cb, vb = Sb.level(l)
        assert np.array_equal(cf, cb) and np.array_equal(vf, vb), l
        if precision == "fp64":
            assert np.array_equal(vf, H.level(l).val), l
    rf, cf, vf = Sf.level(-1)
    R = H.level(-1)
    assert np.array_equal(cf, R.ci)
    assert np.abs(vf - R.val).max() <= 1e-14 * np.abs(R.val).max()
    rng = np.random.default_rng(3)
    for _ in range(2):
        v = rng.standard_normal(m.shape)
        y = Sf.apply_A(_cuda(v)).cpu().numpy()
        yr = H.apply_A(v)
        assert np.abs(y - yr).max() <= 1e-13 * np.abs(yr).max()
        z = Sf.precond(_cuda(v)).cpu().numpy()
        zb = Sb.precond(_cuda(v)).cpu().numpy()
        tol = 1e-11 if precision == "fp64" else 1e-4
        assert np.abs(z - zb).max() <= tol * np.abs(zb).max()
        if precision == "fp64":
            zr = H.precond(v)
            assert np.abs(z - zr).max() <= 1e-11 * np.abs(zr).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32_amg"])
@pytest.mark.parametrize("dim,n", [(2, 384), (3, 56)])
def test_level1_products_from_grid_blocks(gpu, orc, dim, n, precision):
    """Grids whose level 1 has at least 32768 nodes: there the factored form
    applies level 1 through the grid level's blocks, (A1 x)_I = |I| x_I +
    sum_i K_i sum_{j~i} x_agg(j), while the BSR form multiplies the stored
    Galerkin blocks.  The K-cycle preconditioner (level 1 visited by the
    residual, the post-smoothing sweep and the K-cycle products) agrees with
    the BSR form's and with the oracle's to 1e-11 relative (FP64)."""
    say("[level1_products_from_grid_blocks]", dim, n, precision)
    nn = (n, n, n if dim == 3 else 1)
    m = _rough(nn, seed=11)
    alpha, dt = 0.1, 2e-4
    g = gpu.make_grid(dim, n)
    Sf = gpu.Solver(g, gpu.default_opts(fine_operator="factored", precision=precision, kcycle_depth=1))
    Sb = gpu.Solver(g, gpu.default_opts(precision=precision, kcycle_depth=1))
    assert Sf.setup(_cuda(m), alpha, dt) == gpu.OK and Sb.setup(_cuda(m), alpha, dt) == gpu.OK
    assert Sf.level_info(1)[0] >= 32768 and Sf.num_levels > 2
    rng = np.random.default_rng(5)
    v = rng.standard_normal(m.shape)
    z = Sf.precond(_cuda(v)).cpu().numpy()
    zb = Sb.precond(_cuda(v)).cpu().numpy()
    d = np.abs(z - zb).max() / np.abs(zb).max()
    say("  level-1 nodes %d, |z - z_bsr| / |z| = %.2e" % (Sf.level_info(1)[0], d))
    assert d <= (1e-11 if precision == "fp64" else 1e-4)
    if precision == "fp64":
        H = orc.Hierarchy(orc.make_grid(dim, n), orc.default_opts(kcycle_depth=1), m, alpha, dt)
        zr = H.precond(v)
        assert np.abs(z - zr).max() <= 1e-11 * np.abs(zr).max()


def test_factored_steps(gpu, orc):
    """Vortex trajectory (rtol 1e-10 on the GPU, 1e-12 in the oracle) and an
    evolved rough field with the K-cycle (both at 1e-11): within 1e-8."""
    say("[factored_steps]")
    w = I.WORKLOADS["vortex64"]
    S = gpu.Solver(gpu.make_grid(2, w.n), gpu.default_opts(rtol=w.rtol, fine_operator="factored"))
    og = orc.make_grid(2, w.n)
    oo = orc.default_opts(rtol=1e-12)
    m = w.m0()
    for k in range(w.steps):
        out, s, st = S.step(_cuda(m), w.alpha, w.dt)
        rc, ref, ost = orc.step(og, oo, m, w.alpha, w.dt)
        d = np.abs(out.cpu().numpy() - ref).max()
        assert s == gpu.OK and d <= 1e-8, (k, d)
        m = out.cpu().numpy()
    say("  vortex 10 steps ok, last iters %d diff %.2e" % (st.iters, d))
    n, c = 96, 104.9
    m = I.smooth_unit_field(2, n, seed=2)
    og = orc.make_grid(2, n)
    for _ in range(6):
        rc, m, _ = orc.step(og, orc.default_opts(rtol=1e-8), m, 0.02, c / n ** 2)
    for kw in (dict(kcycle_depth=1), dict(kcycle_depth=1, smoother="mcgs"), dict(precision="fp32_amg")):
        S = gpu.Solver(gpu.make_grid(2, n), gpu.default_opts(rtol=1e-11, fine_operator="factored", **kw))
        out, s, st = S.step(_cuda(m), 0.02, c / n ** 2)
        okw = {k: (1 if v == "mcgs" else v) for k, v in kw.items() if k != "precision"}
        rc, ref, ost = orc.step(og, orc.default_opts(rtol=1e-11, **okw), m, 0.02, c / n ** 2)
        d = np.abs(out.cpu().numpy() - ref).max()
        say("  evolved 96^2 %s iters gpu %d orc %d diff %.2e" % (kw, st.iters, ost.iters, d))
        assert s == gpu.OK and d <= 1e-8


def test_factored_bdf2_3d(gpu, orc):
    say("[factored_bdf2_3d]")
    dim, n, alpha = 3, 16, 0.1
    a = I.smooth_unit_field(dim, n, seed=31)
    b = I.smooth_unit_field(dim, n, seed=32)
    m_n = a + 0.1 * (b - a)
    m_n /= np.linalg.norm(m_n, axis=1, keepdims=True)
    dt = 8.19 / n ** 2
    S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(rtol=1e-11, scheme="bdf2", fine_operator="factored",
                                                           precision="fp32_amg", kcycle_depth=1))
    out, s, st = S.step(_cuda(m_n), alpha, dt, m_nm1=_cuda(a))
    rc, ref, ost = orc.step2(orc.make_grid(dim, n), orc.default_opts(rtol=1e-11), m_n, a, alpha, dt)
    d = np.abs(out.cpu().numpy() - ref).max()
    say("  iters gpu %d orc %d diff %.2e" % (st.iters, ost.iters, d))
    assert s == gpu.OK and d <= 1e-8


def test_factored_unsupported_without_left_scale(gpu):
    s, _ = gpu.workspace_bytes(gpu.make_grid(2, 32), gpu.default_opts(fine_operator="factored", left_scale=0))
    assert s == gpu.ERR_UNSUPPORTED
