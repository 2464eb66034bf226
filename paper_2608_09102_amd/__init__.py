"""Python binding of libllg.so: one semi-implicit Landau-Lifshitz step on MI355X.

Argument marshalling only.  Every step of the computation (assembly,
aggregation, Galerkin, V-cycle, FGMRES, projection) runs in the HIP kernels of
libllg.so; PyTorch provides device memory (the workspace, the fields) and the
stream.  There is no CPU fallback: if libllg.so is missing or does not load,
importing this package raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # loads the HIP runtime that libllg.so then binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libllg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "llg.h")

if not os.path.exists(LIB_PATH):
    raise ImportError("libllg.so is not built (run __graft_entry__.build() or "
                      "python paper_2608_09102_amd/build.py); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

MAX_LEVELS = 40

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_NONFINITE = range(7)
PREC_FP64, PREC_FP32_AMG = 0, 1
SMOOTHER_JACOBI, SMOOTHER_MCGS = 0, 1
SCHEME_BDF1, SCHEME_BDF2 = 0, 1
FINE_BSR, FINE_FACTORED = 0, 1
ARNOLDI_CGS2, ARNOLDI_DCGS2 = 0, 1
KRYLOV_FGMRES_AMG, KRYLOV_GMRES, KRYLOV_BICGSTAB, KRYLOV_TFQMR = 0, 2, 3, 4
KT_NONE, KT_OUTER_SPMV, KT_SMOOTH, KT_RESIDUAL, KT_ARNOLDI, KT_GALERKIN, KT_ASSEMBLE = range(7)
KERNEL_CLASSES = {"none": 0, "outer_spmv": 1, "smooth": 2, "residual": 3, "arnoldi": 4, "galerkin": 5, "level1": 7,
                  "assemble": 6}


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("bc", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
        ("omega", ctypes.c_double), ("npass", ctypes.c_int32), ("beta_num", ctypes.c_int32),
        ("beta_den", ctypes.c_int32), ("max_coarse", ctypes.c_int32), ("stagnation", ctypes.c_double),
        ("max_levels", ctypes.c_int32), ("max_dense", ctypes.c_int32), ("left_scale", ctypes.c_int32),
        ("project", ctypes.c_int32), ("x0_is_mn", ctypes.c_int32), ("agg_salt", ctypes.c_uint64),
        ("rebuild_aggregates", ctypes.c_int32), ("kcycle_depth", ctypes.c_int32),
        ("graphs", ctypes.c_int32), ("smoother", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("fine_operator", ctypes.c_int32), ("arnoldi", ctypes.c_int32), ("krylov", ctypes.c_int32),
        ("stray_field", ctypes.c_int32), ("tail_nodes", ctypes.c_int32),
        ("pipeline", ctypes.c_int32), ("overlap_rebuild", ctypes.c_int32), ("csr_levels", ctypes.c_int32),
    ]


class Field(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("q", ctypes.c_double), ("h_ext", ctypes.c_double * 3),
                ("stray", ctypes.c_int32)]


def make_field(eps=1.0, q=0.0, h_ext=(0.0, 0.0, 0.0), stray=0) -> Field:
    f = Field()
    f.eps, f.q = float(eps), float(q)
    f.h_ext[0], f.h_ext[1], f.h_ext[2] = (float(v) for v in h_ext)
    f.stray = int(stray)
    return f


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("converged", ctypes.c_int32), ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
        ("level_nodes", ctypes.c_int64 * MAX_LEVELS), ("level_nnzb", ctypes.c_int64 * MAX_LEVELS),
        ("ms_setup", ctypes.c_double), ("ms_solve", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_int64), ("reorth_passes", ctypes.c_int32),
        ("tail_level", ctypes.c_int32), ("kernel_bytes", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        L = self.levels
        return {"iters": self.iters, "restarts": self.restarts, "levels": L, "converged": bool(self.converged),
                "relres_est": self.relres_est, "relres_true": self.relres_true,
                "level_nodes": list(self.level_nodes[:L]), "level_nnzb": list(self.level_nnzb[:L]),
                "ms_setup": self.ms_setup, "ms_solve": self.ms_solve, "ms_total": self.ms_total,
                "kernel_ms": self.kernel_ms, "kernel_launches": self.kernel_launches,
                "reorth_passes": self.reorth_passes, "tail_level": self.tail_level,
                "kernel_bytes": self.kernel_bytes}


_P = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
_lib.llg_default_opts.argtypes = [ctypes.POINTER(Opts)]
_lib.llg_default_opts.restype = None
_lib.llg_workspace_bytes.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)]
_lib.llg_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P,
                            ctypes.POINTER(_P)]
_lib.llg_step.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, ctypes.POINTER(Stats)]
_lib.llg_setup.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double]
_lib.llg_num_levels.argtypes = [_P, ctypes.POINTER(_i32)]
_lib.llg_level_info.argtypes = [_P, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.llg_get_level.argtypes = [_P, _i32, _P, _P, _P, _i64]
_lib.llg_get_aggregates.argtypes = [_P, _i32, _P, _i64]
_lib.llg_get_colours.argtypes = [_P, _i32, _P, _i64, _P]
_lib.llg_step_field.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Field), _P, _P,
                                ctypes.POINTER(Stats)]
_lib.llg_stray_field.argtypes = [_P, _P, _P]
_lib.llg_get_demag_tensor.argtypes = [_P, _P, _i64]
_lib.llg_stray_field_noalloc.argtypes = [ctypes.POINTER(Grid), _P, _P, _P]
_lib.llg_apply_precond.argtypes = [_P, _P, _P]
_lib.llg_apply_A.argtypes = [_P, _P, _P]
_lib.llg_set_kernel_timing.argtypes = [_P, _i32]
_lib.llg_ctx_bytes.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
_lib.llg_destroy.argtypes = [_P]
_lib.llg_status_str.argtypes = [_i32]
_lib.llg_status_str.restype = ctypes.c_char_p
_lib.llg_last_error.argtypes = []
_lib.llg_last_error.restype = ctypes.c_char_p
for _f in ("llg_workspace_bytes", "llg_create", "llg_step", "llg_setup", "llg_num_levels", "llg_level_info",
           "llg_get_level", "llg_get_aggregates", "llg_get_colours", "llg_step_field", "llg_stray_field",
           "llg_get_demag_tensor", "llg_stray_field_noalloc",
           "llg_apply_precond", "llg_apply_A", "llg_set_kernel_timing",
           "llg_ctx_bytes", "llg_destroy"):
    getattr(_lib, _f).restype = _i32


def lib() -> ctypes.CDLL:
    return _lib


def declared_symbols() -> list:
    """Entry points declared in include/llg.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(llg_[a-z_0-9]+)\s*\(", text)))


class LLGError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.llg_status_str(status).decode()
        detail = _lib.llg_last_error().decode()
        super().__init__("%s: %s%s" % (where, msg, (" (" + detail + ")") if detail and status == ERR_DEVICE else ""))
        self.status = status


def status_str(s: int) -> str:
    return _lib.llg_status_str(s).decode()


def make_grid(dim: int, n, h: float | None = None, bc: int = 0) -> Grid:
    if isinstance(n, int):
        n = (n, n, n if dim == 3 else 1)
    n = tuple(int(v) for v in n)
    if len(n) == 2:
        n = (n[0], n[1], 1)
    g = Grid()
    g.dim = dim
    g.n[0], g.n[1], g.n[2] = n
    g.h = float(h) if h is not None else 1.0 / n[0]
    g.bc = bc
    return g


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.llg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "precision" and isinstance(v, str):
            v = {"fp64": PREC_FP64, "fp32_amg": PREC_FP32_AMG}[v]
        if k == "smoother" and isinstance(v, str):
            v = {"jacobi": SMOOTHER_JACOBI, "mcgs": SMOOTHER_MCGS}[v]
        if k == "scheme" and isinstance(v, str):
            v = {"bdf1": SCHEME_BDF1, "bdf2": SCHEME_BDF2}[v]
        if k == "fine_operator" and isinstance(v, str):
            v = {"bsr": FINE_BSR, "factored": FINE_FACTORED}[v]
        if k == "arnoldi" and isinstance(v, str):
            v = {"cgs2": ARNOLDI_CGS2, "dcgs2": ARNOLDI_DCGS2}[v]
        if k == "krylov" and isinstance(v, str):
            v = {"fgmres_amg": KRYLOV_FGMRES_AMG, "gmres": KRYLOV_GMRES, "bicgstab": KRYLOV_BICGSTAB,
                 "tfqmr": KRYLOV_TFQMR}[v]
        setattr(o, k, v)
    return o


def stray_field_noalloc(grid: Grid, m, out=None, stream=None):
    """h_s(m) without a context: the library's static device scratch holds
    the tensor and work planes (llg_stray_field_noalloc); m and out are
    (N, 3) float64 CUDA tensors.  Returns (out, status)."""
    if out is None:
        out = torch.empty_like(m)
    st = stream if stream is not None else torch.cuda.current_stream(m.device)
    with torch.cuda.device(m.device):
        s = _lib.llg_stray_field_noalloc(ctypes.byref(grid), _ptr(m), _ptr(out), ctypes.c_void_p(st.cuda_stream))
    return out, s


def workspace_bytes(grid: Grid, opts: Opts) -> tuple:
    b = ctypes.c_size_t(0)
    s = _lib.llg_workspace_bytes(ctypes.byref(grid), ctypes.byref(opts), ctypes.byref(b))
    return s, int(b.value)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """A context: grid, options, a torch-owned workspace and a HIP stream."""

    def __init__(self, grid: Grid, opts: Opts | None = None, device: int | None = None,
                 stream: torch.cuda.Stream | None = None, workspace: torch.Tensor | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the library runs only on the GPU")
        self.grid = grid
        self.opts = opts if opts is not None else default_opts()
        self.device = torch.device("cuda", device if device is not None else torch.cuda.current_device())
        self.N = grid.n[0] * grid.n[1] * grid.n[2]
        self.stream = stream
        self._ctx = None
        with torch.cuda.device(self.device):
            s, nbytes = workspace_bytes(grid, self.opts)
            if s != OK:
                raise LLGError(s, "llg_workspace_bytes")
            self.workspace_bytes = nbytes
            if workspace is None:
                workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.workspace = workspace
            ctx = ctypes.c_void_p()
            sh = self._stream_handle()
            s = _lib.llg_create(ctypes.byref(grid), ctypes.byref(self.opts), _ptr(workspace),
                                workspace.numel(), sh, ctypes.byref(ctx))
            if s != OK:
                raise LLGError(s, "llg_create")
            self._ctx = ctx

    def _stream_handle(self):
        st = self.stream if self.stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(st.cuda_stream)

    def close(self):
        if self._ctx is not None:
            _lib.llg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, x, name):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
                and x.numel() == 3 * self.N):
            raise ValueError("%s must be a contiguous float64 CUDA tensor with %d entries" % (name, 3 * self.N))
        return x

    def step(self, m_n, alpha: float, dt: float, forcing=None, out=None, m_nm1=None, check: bool = True):
        """One time step; returns (m_np1, status, Stats).  m_nm1 (m^{n-1}) is
        read by BDF2 contexts; without it their step is a BDF1 step."""
        self._field(m_n, "m_n")
        if m_nm1 is not None:
            self._field(m_nm1, "m_nm1")
        if forcing is not None:
            self._field(forcing, "forcing")
        if out is None:
            out = torch.empty_like(m_n)
        self._field(out, "out")
        st = Stats()
        with torch.cuda.device(self.device):
            s = _lib.llg_step(self._ctx, _ptr(m_n), _ptr(m_nm1), float(alpha), float(dt), _ptr(forcing),
                              _ptr(out), ctypes.byref(st))
        if check and s not in (OK, ERR_NOT_CONVERGED):
            raise LLGError(s, "llg_step")
        return out, s, st

    def step_field(self, m_n, alpha: float, dt: float, field: "Field", forcing=None, out=None, m_nm1=None,
                   check: bool = True):
        """One step of the full model (anisotropy, external and stray field)."""
        self._field(m_n, "m_n")
        if m_nm1 is not None:
            self._field(m_nm1, "m_nm1")
        if forcing is not None:
            self._field(forcing, "forcing")
        if out is None:
            out = torch.empty_like(m_n)
        self._field(out, "out")
        st = Stats()
        with torch.cuda.device(self.device):
            s = _lib.llg_step_field(self._ctx, _ptr(m_n), _ptr(m_nm1), float(alpha), float(dt), ctypes.byref(field),
                                    _ptr(forcing), _ptr(out), ctypes.byref(st))
        if check and s not in (OK, ERR_NOT_CONVERGED):
            raise LLGError(s, "llg_step_field")
        return out, s, st

    def stray_field(self, m):
        self._field(m, "m")
        h = torch.empty_like(m)
        with torch.cuda.device(self.device):
            s = _lib.llg_stray_field(self._ctx, _ptr(m), _ptr(h))
        if s != OK:
            raise LLGError(s, "llg_stray_field")
        return h

    def demag_tensor(self):
        """The device's demagnetizing tensor for every cell offset, as a host
        array [6][2nz-1][2ny-1][2nx-1] (xx, yy, zz, xy, xz, yz; offset k at
        index k + n - 1 per axis)."""
        import numpy as np
        nx, ny, nz = (int(self.grid.n[0]), int(self.grid.n[1]), int(self.grid.n[2]))
        out = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
        with torch.cuda.device(self.device):
            s = _lib.llg_get_demag_tensor(self._ctx, out.ctypes.data, out.size)
        if s != OK:
            raise LLGError(s, "llg_get_demag_tensor")
        return out

    def setup(self, m_tilde, alpha: float, dt: float) -> int:
        self._field(m_tilde, "m_tilde")
        with torch.cuda.device(self.device):
            return _lib.llg_setup(self._ctx, _ptr(m_tilde), float(alpha), float(dt))

    @property
    def num_levels(self) -> int:
        v = _i32(0)
        s = _lib.llg_num_levels(self._ctx, ctypes.byref(v))
        if s != OK:
            raise LLGError(s, "llg_num_levels")
        return v.value

    def level_info(self, level: int):
        n, nz = _i64(0), _i64(0)
        s = _lib.llg_level_info(self._ctx, level, ctypes.byref(n), ctypes.byref(nz))
        if s != OK:
            raise LLGError(s, "llg_level_info")
        return n.value, nz.value

    def level(self, level: int):
        """Host BSR copy (row_ptr int32, col int32, vals float64 [nnzb,3,3])."""
        import numpy as np
        n, nz = self.level_info(level)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nz, np.int32)
        val = np.empty((nz, 3, 3), np.float64)
        with torch.cuda.device(self.device):
            s = _lib.llg_get_level(self._ctx, level, rp.ctypes.data_as(_P), ci.ctypes.data_as(_P),
                                   val.ctypes.data_as(_P), nz)
        if s != OK:
            raise LLGError(s, "llg_get_level")
        return rp, ci, val

    def aggregates(self, level: int):
        import numpy as np
        n, _ = self.level_info(level)
        a = np.empty(n, np.int32)
        with torch.cuda.device(self.device):
            s = _lib.llg_get_aggregates(self._ctx, level, a.ctypes.data_as(_P), n)
        if s != OK:
            raise LLGError(s, "llg_get_aggregates")
        return a

    def colours(self, level: int):
        """(colour class of every node, number of classes) of a level smoothed
        by multicolour Gauss-Seidel."""
        import numpy as np
        n, _ = self.level_info(level)
        a = np.empty(n, np.int32)
        k = ctypes.c_int32(0)
        with torch.cuda.device(self.device):
            s = _lib.llg_get_colours(self._ctx, level, a.ctypes.data_as(_P), n, ctypes.cast(ctypes.byref(k), _P))
        if s != OK:
            raise LLGError(s, "llg_get_colours")
        return a, int(k.value)

    def precond(self, v):
        self._field(v, "v")
        z = torch.empty_like(v)
        with torch.cuda.device(self.device):
            s = _lib.llg_apply_precond(self._ctx, _ptr(v), _ptr(z))
        if s != OK:
            raise LLGError(s, "llg_apply_precond")
        return z

    def apply_A(self, x):
        self._field(x, "x")
        y = torch.empty_like(x)
        with torch.cuda.device(self.device):
            s = _lib.llg_apply_A(self._ctx, _ptr(x), _ptr(y))
        if s != OK:
            raise LLGError(s, "llg_apply_A")
        return y

    def set_kernel_timing(self, cls) -> None:
        if isinstance(cls, str):
            cls = KERNEL_CLASSES[cls]
        s = _lib.llg_set_kernel_timing(self._ctx, int(cls))
        if s != OK:
            raise LLGError(s, "llg_set_kernel_timing")

    def ctx_bytes(self) -> int:
        b = ctypes.c_size_t(0)
        _lib.llg_ctx_bytes(self._ctx, ctypes.byref(b))
        return int(b.value)
