"""GPU: the pipelined FGMRES loop (opts.pipeline).

The head of iteration j + 1 (preconditioner and product) is enqueued before
the host tests iteration j; it writes only z_{j+1} and w, which a finished
cycle never reads, so every step is bit-identical to the unpipelined loop:
same iterate, iteration and restart counts, residuals, with and without
graphs, with kernel timing on (its events are harvested in two parts), across
restart boundaries and when the iteration cap ends the solve.  (A head
enqueued ahead of an iteration that converges is wasted work; with kernel
timing on it shows as one more timed product.)
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


# (name, dim, n, alpha, dt, steps, opts)
CASES = [
    ("vortex64", 2, (64, 64, 1), 0.1, 1e-3, 3, dict(rtol=1e-10)),
    ("rough2d_256_restart5", 2, (256, 256, 1), 0.02, 2e-4, 2, dict(rtol=1e-9, restart=5, kcycle_depth=1,
                                                                     fine_operator="factored")),
    ("rough2d_256_fp32_graphs", 2, (256, 256, 1), 0.02, 2e-4, 2, dict(rtol=1e-8, precision="fp32_amg",
                                                                        kcycle_depth=1, graphs=1)),
    ("cube3d_24_bdf2", 3, (24, 24, 24), 0.1, 1e-3, 3, dict(rtol=1e-10, scheme="bdf2")),
    ("rough2d_128_capped", 2, (128, 128, 1), 0.02, 5e-4, 1, dict(rtol=1e-12, max_iters=9, restart=4)),
    ("rough2d_128_timed", 2, (128, 128, 1), 0.02, 5e-4, 2, dict(rtol=1e-9, restart=7)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pipelined_loop_bit_identical(gpu, case):
    name, dim, n, alpha, dt, steps, kw = case
    say("[pipelined_loop_bit_identical]", name)
    h = 1.0 / n[0]
    m0 = I.vortex_field(64, seed=1) if name == "vortex64" else _rough(n, seed=5)
    runs = []
    for pipe in (1, 0):
        S = gpu.Solver(gpu.make_grid(dim, n, h), gpu.default_opts(pipeline=pipe, **kw))
        if name.endswith("timed"):
            S.set_kernel_timing("outer_spmv")
        m, prev = _cuda(m0), None
        out = []
        for _ in range(steps):
            u, s, st = S.step(m, alpha, dt, m_nm1=prev)
            out.append((u.cpu().numpy(), s, st.iters, st.restarts, st.relres_true, st.relres_est,
                        st.kernel_launches))
            prev, m = m, u
        runs.append(out)
        S.close()
    for k, (a, b) in enumerate(zip(*runs)):
        say("  step %d: status %d, its %d, restarts %d, relres %.2e, timed launches %d/%d" %
            (k, a[1], a[2], a[3], a[4], a[6], b[6]))
        assert a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
        assert a[4] == b[4] and a[5] == b[5]
        assert np.array_equal(a[0], b[0])
        if name.endswith("timed"):
            # one timed outer product per iteration; the pipelined loop may add
            # the product of a head enqueued ahead of a converged iteration
            assert b[6] == a[2] and b[6] <= a[6] <= b[6] + a[3] + 1
    if name.endswith("capped"):
        assert runs[0][0][1] == gpu.ERR_NOT_CONVERGED and runs[0][0][2] == 9
