"""Seeded synthetic inputs for the semi-implicit Landau-Lifshitz step.

This module is shared by the oracle side (tests, CPU baseline) and the HIP side
(binding tests, benchmark, serving).  It holds only input recipes: grids,
initial magnetizations, the manufactured exact solution with its forcing, and
the serving request stream.  It contains none of the solver's arithmetic (no
discrete operator, no assembly, no aggregation, no Krylov step).

Fields are float64 arrays of shape (N, 3), node-major, node index
p = i + nx*(j + ny*k) with x fastest; node p sits at the cell centre
((i + 1/2) h, (j + 1/2) h, (k + 1/2) h) of the unit square or cube, h = 1/n.

The workloads follow the paper's setting: the damped Landau-Lifshitz equation
on the unit square/cube with Neumann boundaries and unit-length initial data
(Sec. 2, Sec. 4.2-4.4), at the grid sizes of the benchmark configurations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def normalize(m: np.ndarray) -> np.ndarray:
    """Scale every node's vector to unit length."""
    nrm = np.sqrt((m * m).sum(axis=-1, keepdims=True))
    return m / nrm


def cell_centres(dim: int, n: int, xp=np, device=None):
    """Coordinates (x, y[, z]) of the cell centres, flattened in node order.
    xp is numpy (default) or torch (then on `device`)."""
    if xp is np:
        c = (np.arange(n, dtype=np.float64) + 0.5) / n
        grids = np.meshgrid(*([c] * dim), indexing="ij")
    else:
        c = (xp.arange(n, dtype=xp.float64, device=device) + 0.5) / n
        grids = xp.meshgrid(*([c] * dim), indexing="ij")
    # the slowest index comes first: (y, x) in 2D, (z, y, x) in 3D
    return tuple(g.reshape(-1) for g in reversed(grids))


def _stack(xp, arrs):
    return np.stack(arrs, axis=1) if xp is np else xp.stack(arrs, dim=1)


def _cross(xp, a, b):
    return np.cross(a, b) if xp is np else xp.linalg.cross(a, b, dim=1)


def smooth_unit_field(dim: int, n: int, seed: int, sweeps: int = 20) -> np.ndarray:
    """Random unit vectors smoothed by neighbour averaging, then normalized.

    Each sweep replaces every node by 1/2 itself + 1/2 the mean of its in-grid
    neighbours (all nodes updated from the previous sweep's values), which
    gives a spatially correlated field with a wide range of length scales.
    """
    rng = np.random.default_rng(seed)
    shape = (n, n, 3) if dim == 2 else (n, n, n, 3)
    m = normalize(rng.standard_normal(size=shape))
    for _ in range(sweeps):
        acc = np.zeros_like(m)
        cnt = np.zeros(shape[:-1] + (1,), dtype=np.float64)
        for ax in range(dim):
            lo = [slice(None)] * (dim + 1)
            hi = [slice(None)] * (dim + 1)
            lo[ax] = slice(0, n - 1)
            hi[ax] = slice(1, n)
            lo, hi = tuple(lo), tuple(hi)
            acc[lo] += m[hi]
            acc[hi] += m[lo]
            cnt[lo] += 1.0
            cnt[hi] += 1.0
        m = 0.5 * m + 0.5 * (acc / cnt)
    m = normalize(m)
    return np.ascontiguousarray(m.reshape(-1, 3))


def vortex_field(n: int, seed: int, sigma: float = 0.01) -> np.ndarray:
    """2D field (cos pi x sin pi y, sin pi x sin pi y, cos pi y) plus seeded
    N(0, sigma^2) noise per component, normalized."""
    x, y = cell_centres(2, n)
    m = np.stack([np.cos(np.pi * x) * np.sin(np.pi * y), np.sin(np.pi * x) * np.sin(np.pi * y),
                  np.cos(np.pi * y)], axis=1)
    rng = np.random.default_rng(seed)
    m = m + rng.normal(0.0, sigma, size=m.shape)
    return np.ascontiguousarray(normalize(m))


def _xbar(dim: int, n: int, xp=np, device=None):
    """xbar = sum_d x_d^2 (1 - x_d)^2 with its gradient norm^2 and Laplacian."""
    cs = cell_centres(dim, n, xp, device)
    xb = xp.zeros_like(cs[0])
    grad2 = xp.zeros_like(cs[0])
    lap = xp.zeros_like(cs[0])
    for c in cs:
        xb += c * c * (1 - c) * (1 - c)
        d1 = 2 * c * (1 - c) * (1 - 2 * c)
        grad2 += d1 * d1
        lap += 2 * (1 - 6 * c + 6 * c * c)
    return xb, grad2, lap


def exact_solution(dim: int, n: int, t: float, xp=np, device=None):
    """Manufactured m_e = (cos(xbar) sin t, sin(xbar) sin t, cos t), |m_e| = 1.
    xp is numpy (default) or torch (then on `device`)."""
    xb, _, _ = _xbar(dim, n, xp, device)
    s = math.sin(t)
    m = _stack(xp, [xp.cos(xb) * s, xp.sin(xb) * s, xp.full_like(xb, math.cos(t))])
    return np.ascontiguousarray(m) if xp is np else m.contiguous()


def manufactured_forcing(dim: int, n: int, t: float, alpha: float, xp=np, device=None):
    """F = d/dt m_e + m_e x Lap m_e + alpha m_e x (m_e x Lap m_e), with the
    continuous Laplacian of m_e in closed form, so that m_e solves the damped
    equation of Sec. 2 with forcing F.  xbar has zero normal derivative on
    the boundary, so m_e meets the Neumann condition.  The discrete solution
    therefore carries the O(h^2) error of the 5-/7-point Laplacian besides
    the first-order error in time.  xp is numpy (default) or torch (then on
    `device`)."""
    xb, g2, lap = _xbar(dim, n, xp, device)
    s, c = math.sin(t), math.cos(t)
    m = _stack(xp, [xp.cos(xb) * s, xp.sin(xb) * s, xp.full_like(xb, c)])
    dm = _stack(xp, [xp.cos(xb) * c, xp.sin(xb) * c, xp.full_like(xb, -s)])
    # Lap cos(xbar) = -sin(xbar) Lap xbar - cos(xbar) |grad xbar|^2, same for sin
    lm = _stack(xp, [(-xp.sin(xb) * lap - xp.cos(xb) * g2) * s, (xp.cos(xb) * lap - xp.sin(xb) * g2) * s,
                     xp.zeros_like(xb)])
    mxl = _cross(xp, m, lm)
    F = dm + mxl + alpha * _cross(xp, m, mxl)
    return np.ascontiguousarray(F) if xp is np else F.contiguous()


@dataclass
class Workload:
    name: str
    dim: int
    n: int
    alpha: float
    dt: float
    steps: int
    rtol: float
    seed: int
    precision: str = "fp64"          # "fp64" or "fp32_amg"
    alphas: tuple = ()               # extra alpha values swept by the workload
    forcing: bool = False
    notes: str = ""

    @property
    def nodes(self) -> int:
        return self.n ** self.dim

    @property
    def unknowns(self) -> int:
        return 3 * self.nodes

    @property
    def h(self) -> float:
        return 1.0 / self.n

    def m0(self) -> np.ndarray:
        if self.name == "vortex64":
            return vortex_field(self.n, self.seed)
        if self.forcing:
            return exact_solution(self.dim, self.n, 0.0)
        return smooth_unit_field(self.dim, self.n, self.seed)


WORKLOADS = {
    "vortex64": Workload("vortex64", 2, 64, 0.1, 1e-3, 10, 1e-10, 1,
                         notes="2D 64x64, vortex field + N(0, 0.01^2) noise, 12,288 unknowns"),
    "rough2d_1024": Workload("rough2d_1024", 2, 1024, 0.02, 1e-4, 50, 1e-8, 2,
                             notes="2D 1024x1024, smoothed random unit field, 3,145,728 unknowns"),
    "rough3d_128": Workload("rough3d_128", 3, 128, 0.01, 5e-4, 20, 1e-8, 3, precision="fp32_amg",
                            alphas=(0.01, 0.1, 1.0),
                            notes="3D 128^3, smoothed random unit field, 6,291,456 unknowns"),
    "mms3d_256": Workload("mms3d_256", 3, 256, 0.1, 1e-4, 10, 1e-8, 4, precision="fp32_amg",
                          forcing=True, notes="3D 256^3, manufactured solution, 50,331,648 unknowns"),
}


@dataclass
class Request:
    rid: int
    arrival: float
    dim: int
    n: int
    alpha: float
    dt: float
    steps: int
    seed: int

    @property
    def nodes(self) -> int:
        return self.n ** self.dim

    def m0(self) -> np.ndarray:
        return smooth_unit_field(self.dim, self.n, self.seed)


def serving_requests(count: int = 256, rate: float = 8.0, seed: int = 5, steps: int = 20,
                     n2d=(128, 2048), n3d=(32, 192)) -> list:
    """Poisson arrivals of independent simulations with mixed grid sizes.

    Inter-arrival Exp(1/rate); 2D or 3D with probability 1/2; n uniform on the
    given integer ranges; alpha log-uniform on [0.01, 1]; dt uniform on
    [1e-4, 1e-3]; request r's initial field uses seed 5000 + r.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.random() < 0.5 else 3
        lo, hi = n2d if dim == 2 else n3d
        n = int(rng.integers(lo, hi + 1))
        alpha = float(math.exp(rng.uniform(math.log(0.01), math.log(1.0))))
        dt = float(rng.uniform(1e-4, 1e-3))
        out.append(Request(r, t, dim, n, alpha, dt, steps, 5000 + r))
    return out


def _request_field(args):
    dim, n, seed = args
    return smooth_unit_field(dim, n, seed)


def serving_inputs(requests, workers: int | None = None) -> dict:
    """The initial field of every request (request r: seed 5000 + r), generated
    on the host by a pool of `workers` processes (default: up to 16), as a
    dict rid -> array."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    args = [(r.dim, r.n, r.seed) for r in requests]
    if workers == 1 or len(args) <= 1:
        fields = [_request_field(a) for a in args]
    else:
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            fields = list(ex.map(_request_field, args))
    return {r.rid: f for r, f in zip(requests, fields)}
