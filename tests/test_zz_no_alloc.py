"""The stray field's no-allocation entry point (llg_stray_field_noalloc),
through the C ABI, against the context entry point llg_stray_field on the
same inputs: bit for bit (same kernels, same tensor), over consecutive calls
whose grids change size (the second smaller), repeat, and change dimension,
so the static scratch is reused with new contents each time; and a grid too
large for the scratch is refused."""
import sys

import numpy as np
import pytest

import llg_inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_stray_field_matches_context():
    import torch
    import paper_2608_09102_amd as llg
    assert torch.cuda.is_available()
    cases = [(3, (40, 40, 40)), (3, (20, 16, 12)), (3, (20, 16, 12)), (2, (100, 70)), (3, (40, 40, 40))]
    for dim, n in cases:
        say("[noalloc stray field]", dim, n)
        N = int(np.prod(n))
        rng = np.random.default_rng(N)
        m = rng.standard_normal((N, 3))
        m /= np.linalg.norm(m, axis=1, keepdims=True)
        mt = torch.from_numpy(m).cuda()
        g = llg.make_grid(dim, n)
        h0, s = llg.stray_field_noalloc(g, mt)
        assert s == llg.OK, llg.status_str(s)
        S = llg.Solver(llg.make_grid(dim, n), llg.default_opts(stray_field=1))
        ref = S.stray_field(mt)
        S.close()
        assert bool(torch.equal(h0, ref))
        say("  max|h| %.3e equal" % float(ref.abs().max()))
    big = llg.make_grid(3, 80)
    mb = torch.zeros((80 ** 3, 3), dtype=torch.float64, device="cuda")
    _, s = llg.stray_field_noalloc(big, mb)
    assert s == llg.ERR_UNSUPPORTED
