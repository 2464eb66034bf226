"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point declared in include/llg.h, and rejects bad arguments on the host
before any device work."""
import ctypes

import pytest

import paper_2608_09102_amd as llg


def test_exports_every_declared_symbol():
    names = llg.declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(llg.lib(), n), n


def test_default_opts():
    o = llg.default_opts()
    assert o.restart == 30 and o.max_iters == 1000 and o.npass == 2
    assert (o.beta_num, o.beta_den) == (1, 4)
    assert o.max_coarse == 40 and o.left_scale == 1 and o.project == 1 and o.rebuild_aggregates == 1
    assert o.precision == llg.PREC_FP64


def test_status_strings():
    for s in range(7):
        assert llg.status_str(s)


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(dim=2, n=(1, 8, 1)), dict(dim=2, n=(8, 8, 2)), dict(dim=3, n=(8, 8, 1)), dict(h=0.0),
    dict(h=float("nan")),
])
def test_workspace_bytes_rejects_bad_grid(bad):
    g = llg.make_grid(bad.get("dim", 2), bad.get("n", 8))
    if "h" in bad:
        g.h = bad["h"]
    s, _ = llg.workspace_bytes(g, llg.default_opts())
    assert s == llg.ERR_INVALID_ARG


@pytest.mark.parametrize("bad", [dict(restart=0), dict(restart=33), dict(npass=0), dict(npass=4),
                                 dict(max_levels=41), dict(precision=7), dict(beta_den=0), dict(nu_pre=5),
                                 dict(rtol=-1.0)])
def test_workspace_bytes_rejects_bad_opts(bad):
    g = llg.make_grid(2, 8)
    s, _ = llg.workspace_bytes(g, llg.default_opts(**bad))
    assert s == llg.ERR_INVALID_ARG


def test_unsupported_bc():
    g = llg.make_grid(2, 8, bc=1)
    s, _ = llg.workspace_bytes(g, llg.default_opts())
    assert s == llg.ERR_UNSUPPORTED


def test_null_arguments():
    L = llg.lib()
    assert L.llg_workspace_bytes(None, None, None) == llg.ERR_INVALID_ARG
    assert L.llg_step(None, None, None, 0.1, 1e-3, None, None, None) == llg.ERR_INVALID_ARG
    assert L.llg_destroy(None) == llg.ERR_INVALID_ARG
    g = llg.make_grid(2, 8)
    o = llg.default_opts()
    ctx = ctypes.c_void_p()
    # null workspace is rejected before any device call
    assert L.llg_create(ctypes.byref(g), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == llg.ERR_INVALID_ARG
