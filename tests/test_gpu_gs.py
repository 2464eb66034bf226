"""GPU parity of the multicolour block Gauss-Seidel smoother variant.

Bars: colour classes bit-exact on every level (integer work); the cycle
within 1e-12 of the oracle's (FP64); steps within 1e-8 (the target's
tolerance) with both sides at rtol 1e-11.
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
    # name, dim, n, h, alpha, dt
    ("vortex64", 2, (64, 64, 1), 1 / 64, 0.1, 1e-3),
    ("rect2d_37x23", 2, (37, 23, 1), 1 / 37, 0.05, 2e-3),
    ("box3d_9x7x5", 3, (9, 7, 5), 1 / 9, 1.0, 1e-2),
    ("cube3d_20", 3, (20, 20, 20), 1 / 20, 0.01, 5e-4),
]


def _rough(n, seed=7):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((int(np.prod(n)), 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


@pytest.mark.parametrize("kdepth", [0, 2])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gs_colours_and_cycle(gpu, orc, case, kdepth):
    name, dim, n, h, alpha, dt = case
    say("[gs_colours_and_cycle]", name, "kcycle_depth", kdepth)
    m = I.vortex_field(64, seed=1) if name == "vortex64" else _rough(n)
    S = gpu.Solver(gpu.make_grid(dim, n, h), gpu.default_opts(smoother="mcgs", kcycle_depth=kdepth))
    assert S.setup(_cuda(m), alpha, dt) == gpu.OK
    H = orc.Hierarchy(orc.make_grid(dim, n, h), orc.default_opts(smoother=1, kcycle_depth=kdepth), m, alpha, dt)
    assert S.num_levels == H.num_levels
    for l in range(H.num_levels - 1):
        cg, kg = S.colours(l)
        co, ko = H.colour(l)
        assert kg == ko and np.array_equal(cg, co), (name, l)
        assert np.array_equal(S.aggregates(l), H.level(l).agg), (name, l)
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.standard_normal(m.shape)
        z = S.precond(_cuda(v)).cpu().numpy()
        zr = H.precond(v)
        err = np.abs(z - zr).max() / np.abs(zr).max()
        assert err <= 1e-12, err


@pytest.mark.parametrize("kdepth", [0, 1])
def test_gs_steps(gpu, orc, kdepth):
    """Steps of the vortex workload and of an evolved rough 96^2 field with
    Gauss-Seidel smoothing match the oracle to 1e-8 (both at rtol 1e-11) with
    the same iteration counts up to 2."""
    say("[gs_steps] kcycle_depth", kdepth)
    w = I.WORKLOADS["vortex64"]
    S = gpu.Solver(gpu.make_grid(2, w.n), gpu.default_opts(rtol=1e-11, smoother="mcgs", kcycle_depth=kdepth))
    og = orc.make_grid(2, w.n)
    oo = orc.default_opts(rtol=1e-11, smoother=1, kcycle_depth=kdepth)
    m = w.m0()
    for k in range(3):
        out, s, st = S.step(_cuda(m), w.alpha, w.dt)
        assert s == gpu.OK
        rc, ref, ost = orc.step(og, oo, m, w.alpha, w.dt)
        d = np.abs(out.cpu().numpy() - ref).max()
        say("  vortex step %d iters gpu %d orc %d diff %.2e" % (k, st.iters, ost.iters, d))
        assert d <= 1e-8 and abs(st.iters - ost.iters) <= 2
        m = ref
    n, c = 96, 104.9
    m = I.smooth_unit_field(2, n, seed=2)
    og = orc.make_grid(2, n)
    for _ in range(6):
        rc, m, _ = orc.step(og, orc.default_opts(rtol=1e-8), m, 0.02, c / n ** 2)
    S = gpu.Solver(gpu.make_grid(2, n), gpu.default_opts(rtol=1e-11, smoother="mcgs", kcycle_depth=kdepth))
    out, s, st = S.step(_cuda(m), 0.02, c / n ** 2)
    rc, ref, ost = orc.step(og, orc.default_opts(rtol=1e-11, smoother=1, kcycle_depth=kdepth), m, 0.02, c / n ** 2)
    d = np.abs(out.cpu().numpy() - ref).max()
    say("  evolved 96^2 iters gpu %d orc %d diff %.2e" % (st.iters, ost.iters, d))
    assert s == gpu.OK and d <= 1e-8 and abs(st.iters - ost.iters) <= 2


def test_gs_fp32_amg_3d(gpu, orc):
    """FP32 hierarchy with Gauss-Seidel smoothing reaches the FP64 outer
    tolerance on a 3D field; error against the tight FP64 oracle stated."""
    dim, n, alpha = 3, 24, 0.01
    say("[gs_fp32_amg_3d]")
    m = I.smooth_unit_field(dim, n, seed=3)
    dt = 8.19 / n ** 2
    S = gpu.Solver(gpu.make_grid(dim, n), gpu.default_opts(rtol=1e-8, precision="fp32_amg", smoother="mcgs"))
    out, s, st = S.step(_cuda(m), alpha, dt)
    assert s == gpu.OK and st.relres_true <= 1e-8
    rc, ref, ost = orc.step(orc.make_grid(dim, n), orc.default_opts(rtol=1e-12, smoother=1), m, alpha, dt)
    e = np.abs(out.cpu().numpy() - ref).max()
    say("  iters gpu %d orc %d err %.2e" % (st.iters, ost.iters, e))
    assert e <= 1e-7


def test_gs_graphs_match_eager(gpu):
    say("[gs_graphs_match_eager]")
    m = I.smooth_unit_field(2, 80, seed=9)
    outs = []
    for graphs in (0, 1):
        S = gpu.Solver(gpu.make_grid(2, 80), gpu.default_opts(rtol=1e-9, graphs=graphs, smoother="mcgs",
                                                              kcycle_depth=1))
        x = _cuda(m)
        for _ in range(3):
            x, s, st = S.step(x, 0.05, 2e-3)
            assert s == gpu.OK
        outs.append((x.cpu().numpy(), st.iters))
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])
