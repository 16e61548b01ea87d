"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes and samples* problem data: grid sizes, per-element
coefficient fields, random right-hand sides and manufactured source terms
sampled at points.  It contains none of the solver's arithmetic (no basis
functions, no quadrature weights, no operators), so the CPU oracle and the GPU
library can both consume its output without sharing any method code.

Layout conventions (the same ones the C-ABI documents):
  * elements of a uniform n^d grid on the unit box are numbered
    lexicographically with x fastest: e = ix + n*iy + n*n*iz;
  * a coefficient vector is element-major: [element][dof];
  * per-element coefficient fields (viscosity) are one double per element.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Callable, Optional

import numpy as np

BASE_SEED = 20241216


# --------------------------------------------------------------------------
# Workload descriptions (named by what they are, with their sizes)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    n: int
    p: int
    system: str = "poisson"        # "poisson" | "stokes"
    basis: str = "legendre"        # "legendre" | "gl_nodal"
    gamma: int = 0                 # Stokes form: 0 standard, 1 stress
    smoother: str = "sai"          # "jacobi" | "gs" | "sai"
    sai_level: int = 1
    order: str = "OI"
    krylov: str = "cg"             # "cg" | "gmres"
    precision: str = "fp32"        # V-cycle precision: "fp64" | "fp32"
    mu_kind: str = "const"         # "const" | "sphere" | "disc"
    mu_radius: float = 0.0
    mu_contrast: float = 1.0
    zeta: float = 0.1
    rhs: str = "normal"            # "normal" | "mms_plus_normal"

    def as_dict(self):
        return asdict(self)


POISSON2D_P2_N16 = Workload(
    name="poisson2d_p2_n16_glnodal_jacobi", dim=2, n=16, p=2, basis="gl_nodal",
    smoother="jacobi", order="OI", krylov="cg", precision="fp64",
    rhs="mms_plus_normal")
POISSON3D_P3_N64 = Workload(
    name="poisson3d_p3_n64_sai1", dim=3, n=64, p=3, smoother="sai", sai_level=1,
    order="OI", krylov="cg", precision="fp32")
INTERFACE3D_P2_N96 = Workload(
    name="interface3d_p2_n96_sphere1e4_sai1", dim=3, n=96, p=2, smoother="sai",
    sai_level=1, order="OI", krylov="cg", precision="fp32", mu_kind="sphere",
    mu_radius=0.3, mu_contrast=1e4)
STOKES2D_P2_N256 = Workload(
    name="stokes2d_stress_p2_n256_disc1e3_sai1", dim=2, n=256, p=2,
    system="stokes", gamma=1, smoother="sai", sai_level=1, order="OI",
    krylov="gmres", precision="fp32", mu_kind="disc", mu_radius=0.25,
    mu_contrast=1e3, zeta=0.131)

WORKLOADS = {w.name: w for w in
             (POISSON2D_P2_N16, POISSON3D_P3_N64, INTERFACE3D_P2_N96,
              STOKES2D_P2_N256)}


def scaled(w: Workload, n: int, **kw) -> Workload:
    """The same workload on a different grid (for oracle-sized parity runs)."""
    d = w.as_dict()
    d.update(kw)
    d["n"] = n
    d["name"] = f"{w.name}@n{n}"
    return Workload(**d)


# --------------------------------------------------------------------------
# Per-element coefficient fields
# --------------------------------------------------------------------------
def element_centres(dim: int, n: int) -> np.ndarray:
    """Centres of the n^dim elements, shape [n^dim, dim], x fastest."""
    c1 = (np.arange(n) + 0.5) / n
    grids = np.meshgrid(*([c1] * dim), indexing="ij")
    # meshgrid with 'ij' gives axis 0 = first coordinate; reorder so x fastest
    pts = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1)
                    for g in grids], axis=1)
    return pts


def mu_field(dim: int, n: int, kind: str = "const", radius: float = 0.0,
             contrast: float = 1.0) -> np.ndarray:
    """Piecewise-constant viscosity per element.

    kind "const": all ones.  kind "sphere"/"disc": `contrast` on elements whose
    centre lies strictly inside the ball of `radius` about the box centre,
    1 elsewhere.  Returns float64 [n^dim].
    """
    ne = n ** dim
    if kind == "const":
        return np.ones(ne)
    c = element_centres(dim, n)
    r2 = np.sum((c - 0.5) ** 2, axis=1)
    inside = r2 < radius * radius
    mu = np.ones(ne)
    mu[inside] = contrast
    return mu


def mu_for(w: Workload) -> np.ndarray:
    return mu_field(w.dim, w.n, w.mu_kind, w.mu_radius, w.mu_contrast)


def mu_box(dim: int, n: int, inner: float, outer: float = 1.0,
           lo: float = 0.25, hi: float = 0.75) -> np.ndarray:
    """Inner axis-aligned box (lo,hi)^dim with viscosity `inner`, `outer`
    elsewhere (element-centre test)."""
    c = element_centres(dim, n)
    inside = np.all((c > lo) & (c < hi), axis=1)
    mu = np.full(n ** dim, float(outer))
    mu[inside] = inner
    return mu


# --------------------------------------------------------------------------
# Random right-hand sides
# --------------------------------------------------------------------------
def rhs_normal(ndofs: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) coefficients, float64, drawn in element-major order."""
    return np.random.default_rng(seed).standard_normal(ndofs)


def rhs_normal_device(ndofs: int, seed: int, device="cuda"):
    """Seeded N(0,1) coefficients, float64, drawn by torch's generator on
    `device` (a request's right-hand side already resident in device memory;
    not the same numbers as rhs_normal)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn(ndofs, generator=g, device=device, dtype=torch.float64)


def rhs_uniform(ndofs: int, seed: int) -> np.ndarray:
    """Seeded U[-1,1] coefficients (the distribution the paper draws from)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, ndofs)


def stokes_body_force(dim: int, n: int, bs_scalar: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) on the velocity coefficients, zero on the pressure ones.

    Per element the unknowns are ordered [u_1 .. u_dim, p], each a block of
    bs_scalar coefficients."""
    ne = n ** dim
    bs = (dim + 1) * bs_scalar
    b = np.zeros((ne, bs))
    b[:, : dim * bs_scalar] = np.random.default_rng(seed).standard_normal(
        (ne, dim * bs_scalar))
    return b.reshape(-1)


# --------------------------------------------------------------------------
# Source terms sampled at points
# --------------------------------------------------------------------------
def gauss_points_1d(nq: int) -> np.ndarray:
    """The nq Gauss-Legendre abscissae on [-1,1] (sample locations only)."""
    x, _ = np.polynomial.legendre.leggauss(nq)
    return x


def sample_on_elements(dim: int, n: int, nq: int,
                       func: Callable[..., np.ndarray]) -> np.ndarray:
    """Evaluate func(x, y[, z]) at the nq^dim tensor Gauss-Legendre points of
    every element.  Result shape [n^dim, nq^dim], points ordered with the
    x index fastest inside an element."""
    xi = gauss_points_1d(nq)
    h = 1.0 / n
    idx = np.arange(n)
    # physical coordinate of point q in element i along one axis
    coord = (idx[:, None] + 0.5 * (xi[None, :] + 1.0)) * h      # [n, nq]
    if dim == 2:
        X = coord[None, :, None, :]      # ix, qx
        Y = coord[:, None, :, None]      # iy, qy
        X = np.broadcast_to(X, (n, n, nq, nq))
        Y = np.broadcast_to(Y, (n, n, nq, nq))
        F = func(X, Y)                   # [iy, ix, qy, qx]
        return np.ascontiguousarray(F).reshape(n * n, nq * nq)
    X = np.broadcast_to(coord[None, None, :, None, None, :], (n, n, n, nq, nq, nq))
    Y = np.broadcast_to(coord[None, :, None, None, :, None], (n, n, n, nq, nq, nq))
    Z = np.broadcast_to(coord[:, None, None, :, None, None], (n, n, n, nq, nq, nq))
    F = func(X, Y, Z)                    # [iz, iy, ix, qz, qy, qx]
    return np.ascontiguousarray(F).reshape(n ** 3, nq ** 3)


def mms_source_2d(x, y):
    """-Laplacian of sin(2 pi x) sin(3 pi y) (unit viscosity)."""
    return 13.0 * math.pi ** 2 * np.sin(2 * math.pi * x) * np.sin(3 * math.pi * y)


def mms_solution_2d(x, y):
    return np.sin(2 * math.pi * x) * np.sin(3 * math.pi * y)


# --------------------------------------------------------------------------
# Serving workload: a seeded stream of requests with Poisson arrivals
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float          # seconds after stream start
    kind: str               # "poisson" | "interface"
    dim: int
    n: int
    p: int
    contrast: float
    seed: int


def serving_requests(count: int = 512, rate: float = 100.0, seed: int = BASE_SEED,
                     grids2d=(32, 64, 128, 256), grids3d=(16, 24, 32, 48),
                     degrees=(1, 2, 3), contrasts=(1.0, 10.0, 1e2, 1e3, 1e4)):
    """Poisson arrivals at `rate` per second; each request draws its shape from
    a finite catalogue so that hierarchies can be shared between requests."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.random() < 0.5 else 3
        n = int(rng.choice(grids2d if dim == 2 else grids3d))
        p = int(rng.choice(degrees))
        contrast = float(rng.choice(contrasts))
        kind = "poisson" if contrast == 1.0 else "interface"
        out.append(Request(i, t, kind, dim, n, p, contrast, BASE_SEED + i))
    return out
