"""The 256^3 manufactured-solution workload at full size (50,331,648
unknowns), in the forms the benchmark times (FP32-AMG and FP64; grid level
stored per node; K-cycle on level 1; no smoothing sweep before the coarse
correction and three after it).

Bars:
- the aggregates of every level bit for bit against the oracle's aggregation
  hierarchy of the grid graph (field independent, so the oracle builds it
  without matrix values: its full hierarchy would need about 50 GB of host
  memory and a few minutes here);
- the unprojected solution of the first step, solved to rtol 1e-8, through its
  true residual ||b - A u|| / ||b|| <= 1e-8, with A applied by an operator
  built independently of both sides (scipy Kronecker Laplacian and numpy cross
  products, the scheme of Sec. 2.1) and b = m^n + dt F;
- the projected step of both forms within 1e-6 of each other and within the
  manufactured solution's error band (the exact m_e one step on).
"""
import sys

import numpy as np
import pytest

import llg_inputs as I
from helpers import apply_scheme, laplacian

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


@pytest.mark.timeout(1500)
def test_full_size_mms3d_256(gpu, orc):
    import torch
    w = I.WORKLOADS["mms3d_256"]
    say("[full_size_mms3d_256] oracle aggregation hierarchy of the 256^3 grid graph")
    sizes, maps = orc.aggregate_levels(orc.make_grid(3, w.n), orc.default_opts())
    say("  oracle levels", sizes)
    m = w.m0()
    F = I.manufactured_forcing(3, w.n, w.dt, w.alpha)
    b = m + w.dt * F
    L = laplacian(3, w.n, 1.0 / w.n)
    bn = np.linalg.norm(b.ravel())
    outs = {}
    for prec in ("fp32_amg", "fp64"):
        say("  %s: step" % prec)
        S = gpu.Solver(gpu.make_grid(3, w.n), gpu.default_opts(rtol=w.rtol, project=0, kcycle_depth=1,
                                                              fine_operator="factored", precision=prec,
                                                              nu_pre=0, nu_post=3))
        u, s, st = S.step(torch.from_numpy(m).cuda(), w.alpha, w.dt, forcing=torch.from_numpy(F).cuda())
        assert s == gpu.OK
        assert S.num_levels == len(sizes), (S.num_levels, sizes)
        for l in range(len(sizes) - 1):
            assert np.array_equal(S.aggregates(l), maps[l]), l
        u = u.cpu().numpy()
        S.close()
        del S
        torch.cuda.empty_cache()
        res = np.linalg.norm((b - apply_scheme(L, m, w.alpha, w.dt, u)).ravel()) / bn
        say("  %s: iters %d levels %d, true relres (independent operator) %.2e" % (prec, st.iters, st.levels, res))
        assert res <= 1e-8
        outs[prec] = u / np.linalg.norm(u, axis=1, keepdims=True)
    d = np.abs(outs["fp32_amg"] - outs["fp64"]).max()
    me = I.exact_solution(3, w.n, w.dt)
    e = np.abs(outs["fp64"] - me).max()
    say("  |fp32_amg - fp64| = %.2e, |fp64 - m_e(dt)| = %.2e" % (d, e))
    assert d <= 1e-6 and e <= 1e-6
