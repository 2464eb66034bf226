"""FP64 CPU oracle for one semi-implicit BDF1 Landau-Lifshitz step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It wraps ``llgo.cpp``
(plain single-threaded C++, FP64, -ffp-contract=off) with ctypes and numpy; it
shares no code with the HIP library.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against a definition that does not come from this code (dense LU, brute-force
matching, explicit Kronecker-product operators, closed forms, the energy
identity, the manufactured solution); the test module names the pin.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "llgo.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

LLGO_OK = 0
LLGO_ERR_ARG = -1
LLGO_ERR_UNSUPPORTED = -2
LLGO_ERR_NOT_CONVERGED = -5
LLGO_ERR_NONFINITE = -6


def build(force: bool = True) -> str:
    """Compile llgo.cpp into liboracle.so with g++ (-O2 -ffp-contract=off)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, _SRC]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("omega", ctypes.c_double),
        ("npass", ctypes.c_int32), ("beta_num", ctypes.c_int32), ("beta_den", ctypes.c_int32),
        ("max_coarse", ctypes.c_int32), ("stagnation", ctypes.c_double),
        ("max_levels", ctypes.c_int32), ("max_dense", ctypes.c_int32),
        ("left_scale", ctypes.c_int32), ("project", ctypes.c_int32), ("x0_is_mn", ctypes.c_int32),
        ("agg_salt", ctypes.c_uint64), ("krylov", ctypes.c_int32), ("kcycle_depth", ctypes.c_int32),
        ("smoother", ctypes.c_int32),
    ]


class Field(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("q", ctypes.c_double), ("h_ext", ctypes.c_double * 3),
                ("stray", ctypes.c_int32)]


def make_field(eps=1.0, q=0.0, h_ext=(0.0, 0.0, 0.0), stray=0) -> Field:
    f = Field()
    f.eps, f.q = eps, q
    f.h_ext[0], f.h_ext[1], f.h_ext[2] = h_ext
    f.stray = int(stray)
    return f


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres_est", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.llgo_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.llgo_splitmix64.argtypes = [ctypes.c_uint64]
        L.llgo_splitmix64.restype = ctypes.c_uint64
        L.llgo_match_pass.argtypes = [i64, P, P, P, ctypes.c_uint64, i32, i32, P, P, P]
        L.llgo_galerkin.argtypes = [i64, P, P, P, P, i64, P, P, P, P]
        L.llgo_aggregate_levels.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), P, P, P, i64]
        L.llgo_assemble_nnzb.argtypes = [ctypes.POINTER(Grid), P]
        L.llgo_assemble.argtypes = [ctypes.POINTER(Grid), P, ctypes.c_double, ctypes.c_double, P, P, P]
        L.llgo_setup.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), P, ctypes.c_double,
                                 ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.llgo_setup.restype = P
        L.llgo_free.argtypes = [P]
        L.llgo_num_levels.argtypes = [P]
        L.llgo_level_info.argtypes = [P, ctypes.c_int, P, P]
        L.llgo_level_matrix.argtypes = [P, ctypes.c_int, P, P, P]
        L.llgo_level_dinv.argtypes = [P, ctypes.c_int, P]
        L.llgo_level_agg.argtypes = [P, ctypes.c_int, P]
        L.llgo_level_colour.argtypes = [P, ctypes.c_int, P, P]
        L.llgo_apply_A.argtypes = [P, P, P]
        L.llgo_precond.argtypes = [P, P, P]
        L.llgo_solve.argtypes = [P, P, P, P, ctypes.POINTER(Stats)]
        L.llgo_step.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), P, ctypes.c_double,
                                ctypes.c_double, P, P, ctypes.POINTER(Stats)]
        L.llgo_step2.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), P, P, ctypes.c_double,
                                 ctypes.c_double, P, P, ctypes.POINTER(Stats)]
        L.llgo_demag_tensor.argtypes = [ctypes.c_double] * 6 + [P]
        L.llgo_stray_field.argtypes = [ctypes.POINTER(Grid), P, P]
        L.llgo_stray_field_at.argtypes = [ctypes.POINTER(Grid), P, P, ctypes.c_int64, P]
        L.llgo_step_field.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), P, P, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(Field), P, P, ctypes.POINTER(Stats)]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_grid(dim: int, n, h: float | None = None) -> Grid:
    """Grid with n points per axis (int or tuple); h defaults to 1/n[0]."""
    if isinstance(n, int):
        n = (n, n, n if dim == 3 else 1)
    n = tuple(int(v) for v in n)
    if len(n) == 2:
        n = (n[0], n[1], 1)
    g = Grid()
    g.dim = dim
    g.n[0], g.n[1], g.n[2] = n
    g.h = float(h) if h is not None else 1.0 / n[0]
    return g


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().llgo_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def splitmix64(x: int) -> int:
    return int(lib().llgo_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def match_pass(rp, ci, w, salt: int, beta=(1, 4)):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int64)
    n = len(rp) - 1
    agg = np.empty(n, np.int32)
    mate = np.empty(n, np.int32)
    nc = ctypes.c_int64(0)
    rc = lib().llgo_match_pass(n, _p(rp), _p(ci), _p(w), ctypes.c_uint64(salt), beta[0], beta[1],
                               _p(agg), _p(mate), ctypes.byref(nc))
    assert rc == 0
    return agg, mate, int(nc.value)


def aggregate_levels(grid: Grid, opts: Opts):
    """The aggregation hierarchy of the grid graph alone (no matrix values):
    the list of level sizes and the aggregate map of every level but the
    coarsest."""
    N = int(grid.n[0]) * int(grid.n[1]) * int(grid.n[2])
    cap = 2 * N  # the level sizes shrink by at least the stagnation factor
    agg = np.empty(cap, np.int32)
    sizes = np.zeros(max(int(opts.max_levels), 1) + 1, np.int64)
    nl = ctypes.c_int32(0)
    rc = lib().llgo_aggregate_levels(ctypes.byref(grid), ctypes.byref(opts), ctypes.byref(nl), _p(sizes), _p(agg),
                                     cap)
    assert rc == 0, rc
    L = int(nl.value)
    maps, off = [], 0
    for l in range(L - 1):
        n = int(sizes[l])
        maps.append(agg[off:off + n].copy())
        off += n
    return [int(v) for v in sizes[:L]], maps


def galerkin(rp, ci, val, agg, nc):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    n = len(rp) - 1
    nz = ctypes.c_int64(0)
    L = lib()
    rc = L.llgo_galerkin(n, _p(rp), _p(ci), _p(val), _p(agg), nc, ctypes.byref(nz), None, None, None)
    assert rc == 0
    rpc = np.empty(nc + 1, np.int64)
    cic = np.empty(nz.value, np.int32)
    vc = np.empty((nz.value, 3, 3), np.float64)
    rc = L.llgo_galerkin(n, _p(rp), _p(ci), _p(val), _p(agg), nc, ctypes.byref(nz), _p(rpc), _p(cic), _p(vc))
    assert rc == 0
    return rpc, cic, vc


def assemble(grid: Grid, m_tilde: np.ndarray, alpha: float, dt: float):
    m_tilde = np.ascontiguousarray(m_tilde, dtype=np.float64)
    nz = ctypes.c_int64(0)
    L = lib()
    assert L.llgo_assemble_nnzb(ctypes.byref(grid), ctypes.byref(nz)) == 0
    N = grid.n[0] * grid.n[1] * grid.n[2]
    rp = np.empty(N + 1, np.int64)
    ci = np.empty(nz.value, np.int32)
    val = np.empty((nz.value, 3, 3), np.float64)
    rc = L.llgo_assemble(ctypes.byref(grid), _p(m_tilde), alpha, dt, _p(rp), _p(ci), _p(val))
    assert rc == 0
    return rp, ci, val


@dataclass
class LevelData:
    rp: np.ndarray
    ci: np.ndarray
    val: np.ndarray
    dinv: np.ndarray
    agg: np.ndarray | None


class Hierarchy:
    """Oracle setup for one frozen field: A, D^{-1}, and the AMG levels."""

    def __init__(self, grid: Grid, opts: Opts, m_tilde: np.ndarray, alpha: float, dt: float):
        self.grid, self.opts = grid, opts
        self.N = grid.n[0] * grid.n[1] * grid.n[2]
        m_tilde = np.ascontiguousarray(m_tilde, dtype=np.float64).reshape(self.N, 3)
        st = ctypes.c_int(0)
        self._h = lib().llgo_setup(ctypes.byref(grid), ctypes.byref(opts), _p(m_tilde), alpha, dt,
                                   ctypes.byref(st))
        self.status = st.value
        if not self._h:
            raise RuntimeError("llgo_setup failed with status %d" % st.value)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().llgo_free(self._h)
            self._h = None

    @property
    def num_levels(self) -> int:
        return lib().llgo_num_levels(self._h)

    def level(self, l: int) -> LevelData:
        """l = -1: unscaled fine operator A; l >= 0: hierarchy level l."""
        L = lib()
        n = ctypes.c_int64(0)
        nz = ctypes.c_int64(0)
        assert L.llgo_level_info(self._h, l, ctypes.byref(n), ctypes.byref(nz)) == 0
        rp = np.empty(n.value + 1, np.int64)
        ci = np.empty(nz.value, np.int32)
        val = np.empty((nz.value, 3, 3), np.float64)
        assert L.llgo_level_matrix(self._h, l, _p(rp), _p(ci), _p(val)) == 0
        dinv = np.empty((n.value, 3, 3), np.float64)
        assert L.llgo_level_dinv(self._h, l, _p(dinv)) == 0
        agg = None
        if 0 <= l < self.num_levels - 1:
            agg = np.empty(n.value, np.int32)
            assert L.llgo_level_agg(self._h, l, _p(agg)) == 0
        return LevelData(rp, ci, val, dinv, agg)

    def colour(self, l: int):
        """(colour class per node, number of classes) of level l, multicolour
        Gauss-Seidel only."""
        L = lib()
        n = ctypes.c_int64(0)
        nz = ctypes.c_int64(0)
        assert L.llgo_level_info(self._h, l, ctypes.byref(n), ctypes.byref(nz)) == 0
        col = np.empty(n.value, np.int32)
        k = ctypes.c_int32(0)
        assert L.llgo_level_colour(self._h, l, _p(col), ctypes.byref(k)) == 0
        return col, int(k.value)

    def apply_A(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        assert lib().llgo_apply_A(self._h, _p(x), _p(y)) == 0
        return y

    def precond(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        z = np.empty_like(v)
        assert lib().llgo_precond(self._h, _p(v), _p(z)) == 0
        return z

    def solve(self, b: np.ndarray, u0: np.ndarray):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        u = np.empty_like(b)
        st = Stats()
        rc = lib().llgo_solve(self._h, _p(b), _p(u0), _p(u), ctypes.byref(st))
        return rc, u, st


def step(grid: Grid, opts: Opts, m_n: np.ndarray, alpha: float, dt: float, F: np.ndarray | None = None):
    """One oracle step; returns (status, m_np1[N,3], Stats)."""
    N = grid.n[0] * grid.n[1] * grid.n[2]
    m_n = np.ascontiguousarray(m_n, dtype=np.float64).reshape(N, 3)
    out = np.empty_like(m_n)
    st = Stats()
    Fp = None
    if F is not None:
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(N, 3)
        Fp = _p(F)
    rc = lib().llgo_step(ctypes.byref(grid), ctypes.byref(opts), _p(m_n), alpha, dt, Fp, _p(out),
                         ctypes.byref(st))
    return rc, out, st


def step2(grid: Grid, opts: Opts, m_n: np.ndarray, m_nm1: np.ndarray, alpha: float, dt: float,
          F: np.ndarray | None = None):
    """One oracle BDF2 step from (m^n, m^{n-1}); returns (status, m_np1[N,3], Stats)."""
    N = grid.n[0] * grid.n[1] * grid.n[2]
    m_n = np.ascontiguousarray(m_n, dtype=np.float64).reshape(N, 3)
    m_nm1 = np.ascontiguousarray(m_nm1, dtype=np.float64).reshape(N, 3)
    out = np.empty_like(m_n)
    st = Stats()
    Fp = None
    if F is not None:
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(N, 3)
        Fp = _p(F)
    rc = lib().llgo_step2(ctypes.byref(grid), ctypes.byref(opts), _p(m_n), _p(m_nm1), alpha, dt, Fp, _p(out),
                          ctypes.byref(st))
    return rc, out, st


def demag_tensor(X, Y, Z, dx, dy, dz) -> np.ndarray:
    """[xx, yy, zz, xy, xz, yz] of the cell-averaged demagnetizing tensor."""
    N = np.empty(6, np.float64)
    lib().llgo_demag_tensor(X, Y, Z, dx, dy, dz, _p(N))
    return N


def stray_field(grid: Grid, m: np.ndarray) -> np.ndarray:
    N = grid.n[0] * grid.n[1] * grid.n[2]
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(N, 3)
    h = np.empty_like(m)
    assert lib().llgo_stray_field(ctypes.byref(grid), _p(m), _p(h)) == 0
    return h


def stray_field_at(grid: Grid, m: np.ndarray, cells) -> np.ndarray:
    """Stray field at the given cell indices only, [len(cells), 3]."""
    N = grid.n[0] * grid.n[1] * grid.n[2]
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(N, 3)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    h = np.empty((len(cells), 3), np.float64)
    assert lib().llgo_stray_field_at(ctypes.byref(grid), _p(m), _p(cells), len(cells), _p(h)) == 0
    return h


def step_field(grid: Grid, opts: Opts, m_n: np.ndarray, alpha: float, dt: float, field: Field,
               m_nm1: np.ndarray | None = None, F: np.ndarray | None = None):
    """One step of the full model (BDF1, or BDF2 with m_nm1); returns (status, m_np1, Stats)."""
    N = grid.n[0] * grid.n[1] * grid.n[2]
    m_n = np.ascontiguousarray(m_n, dtype=np.float64).reshape(N, 3)
    prev = None
    if m_nm1 is not None:
        m_nm1 = np.ascontiguousarray(m_nm1, dtype=np.float64).reshape(N, 3)
        prev = _p(m_nm1)
    Fp = None
    if F is not None:
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(N, 3)
        Fp = _p(F)
    out = np.empty_like(m_n)
    st = Stats()
    rc = lib().llgo_step_field(ctypes.byref(grid), ctypes.byref(opts), _p(m_n), prev, alpha, dt, ctypes.byref(field),
                               Fp, _p(out), ctypes.byref(st))
    return rc, out, st
