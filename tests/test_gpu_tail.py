"""GPU: the V-cycle of the small coarse levels in one workgroup (opts.tail_nodes).

The fused cycle takes every step of the per-level kernels in the same order
and precision (row products with the level's lane groups, restriction sums in
member order, the coarsest solve's unfused dot products), so the
preconditioner and whole steps are bit-identical to the per-level path
(tail_nodes = 0), across smoothing counts, K-cycle depths, precisions and
both storages of the grid level; the per-level path itself is pinned to the
oracle by the parity tests.
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


def _rough(n, seed=7):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((int(np.prod(n)), 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


# (name, dim, n, alpha, dt)
CASES = [
    ("vortex64", 2, (64, 64, 1), 0.1, 1e-3),
    ("rect2d_97x61", 2, (97, 61, 1), 0.05, 2e-4),
    ("cube3d_20", 3, (20, 20, 20), 0.01, 5e-4),
    ("box3d_33x17x9", 3, (33, 17, 9), 1.0, 1e-3),
]
# (precision, kcycle_depth, nu_pre, nu_post, fine_operator)
FORMS = [
    ("fp64", 0, 1, 1, "bsr"),
    ("fp64", 1, 1, 1, "factored"),
    ("fp32_amg", 1, 1, 1, "factored"),
    ("fp64", 2, 2, 2, "bsr"),
    ("fp64", 0, 0, 1, "bsr"),
    ("fp32_amg", 0, 1, 0, "bsr"),
    ("fp64", 1, 3, 1, "factored"),
]


def _pair(gpu, dim, n, h, form, **kw):
    prec, kd, nu_pre, nu_post, op = form
    g = gpu.make_grid(dim, n, h)
    base = dict(precision=prec, kcycle_depth=kd, nu_pre=nu_pre, nu_post=nu_post, fine_operator=op, **kw)
    Sa = gpu.Solver(g, gpu.default_opts(tail_nodes=1 << 20, **base))
    Sb = gpu.Solver(g, gpu.default_opts(tail_nodes=0, **base))
    return Sa, Sb


@pytest.mark.parametrize("form", FORMS, ids=["-".join(map(str, f)) for f in FORMS])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tail_cycle_bit_identical(gpu, case, form):
    name, dim, n, alpha, dt = case
    say("[tail_cycle_bit_identical]", name, form)
    h = 1.0 / n[0]
    m = I.vortex_field(64, seed=1) if name == "vortex64" else _rough(n)
    Sa, Sb = _pair(gpu, dim, n, h, form, rtol=1e-10)
    assert Sa.setup(_cuda(m), alpha, dt) == gpu.OK and Sb.setup(_cuda(m), alpha, dt) == gpu.OK
    rng = np.random.default_rng(13)
    for _ in range(2):
        v = _cuda(rng.standard_normal(m.shape))
        za = Sa.precond(v).cpu().numpy()
        zb = Sb.precond(v).cpu().numpy()
        assert np.isfinite(za).all()
        assert np.array_equal(za, zb), np.abs(za - zb).max() / np.abs(zb).max()
    ua, sa, ta = Sa.step(_cuda(m), alpha, dt)
    ub, sb, tb = Sb.step(_cuda(m), alpha, dt)
    say("  levels %d, tail from level %d, nodes %s, its %d/%d" %
        (ta.levels, ta.tail_level, list(ta.level_nodes[:ta.levels]), ta.iters, tb.iters))
    assert ta.tail_level >= 1 and tb.tail_level == 0
    assert ta.tail_level > form[1]  # below the K-cycle levels
    assert sa == sb == gpu.OK and ta.iters == tb.iters
    assert np.array_equal(ua.cpu().numpy(), ub.cpu().numpy())
    Sa.close()
    Sb.close()


def test_tail_respects_node_limit_and_lds(gpu):
    """tail_nodes bounds the fused levels: every fused level has at most that
    many nodes and the level above the first fused one has more (or is a
    K-cycle level, or level 1 applied through the grid level)."""
    say("[tail_respects_node_limit_and_lds]")
    n = (256, 256, 1)
    m = _rough(n, seed=3)
    for limit in (64, 300, 1024, 1 << 20):
        S = gpu.Solver(gpu.make_grid(2, n), gpu.default_opts(tail_nodes=limit, kcycle_depth=1,
                                                               fine_operator="factored", rtol=1e-8))
        _, s, st = S.step(_cuda(m), 0.02, 2e-4)
        nodes = list(st.level_nodes[:st.levels])
        say("  limit %d: tail from %d, nodes %s, its %d" % (limit, st.tail_level, nodes, st.iters))
        assert s == gpu.OK
        if st.tail_level:
            t = st.tail_level
            assert t >= 2 and all(x <= limit for x in nodes[t:-1])
            vb = lambda k: -(-3 * k * 8 // 16) * 16  # noqa: E731  (FP64 vector bytes, 16-byte aligned)
            lds = 2 * vb(nodes[-1]) + sum(3 * vb(x) for x in nodes[t:-1])
            assert lds <= 152 * 1024
            assert nodes[t - 1] > limit or t == 2 or lds + 3 * vb(nodes[t - 1]) > 152 * 1024
        else:
            assert nodes[-2] > limit
        S.close()


def test_tail_full_size_steps(gpu):
    """rough2d_1024 with the headline form: the fused and the per-level cycle
    give the same step, bit for bit, at the same iteration count."""
    say("[tail_full_size_steps]")
    w = I.WORKLOADS["rough2d_1024"]
    m = _cuda(w.m0())
    res = []
    for limit in (1024, 0):
        S = gpu.Solver(gpu.make_grid(w.dim, w.n), gpu.default_opts(rtol=w.rtol, kcycle_depth=1,
                                                                     fine_operator="factored", tail_nodes=limit))
        u, s, st = S.step(m, w.alpha, w.dt)
        say("  tail_nodes %d: tail from %d, its %d, %.1f ms" % (limit, st.tail_level, st.iters, st.ms_total))
        res.append((u.cpu().numpy(), st.iters, st.tail_level))
        S.close()
    assert res[0][2] > 0 and res[1][2] == 0
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])
