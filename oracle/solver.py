"""Build hierarchy + smoother + Krylov for a workload (oracle; test infrastructure).

Glue only: the arithmetic lives in the other oracle modules.  Defaults follow
the paper: nu1 = nu2 = 3 (Section 2.2), Jacobi w = 0.8, coloured GS w = 1
(Section 2.3), Stokes balancing zeta from tab:zeta when not given.
"""
from __future__ import annotations

import numpy as np

from . import hierarchy, stokes, vcycle, krylov

# tab:zeta (tuned zeta, tensor-product Legendre basis), keyed (gamma, dim) -> p=1..5
TAB_ZETA = {
    (0, 2): [0.0382, 0.131, 0.0990, 0.153, 0.142],
    (0, 3): [0.0462, 0.107, 0.113],
    (1, 2): [0.118, 0.131, 0.0814, 0.123, 0.0745],
    (1, 3): [0.0384, 0.0928, 0.0930],
}

DEFAULT_TAU0 = 1.0
DEFAULT_CP = 0.1


def build(dim, n, p, system="poisson", mu=None, bc=None, basis="legendre",
          gamma=1, smoother="sai", sai_level=1, order="OI", nu1=3, nu2=3,
          omega=None, zeta=None, tau0=DEFAULT_TAU0, cp=DEFAULT_CP, rho=None, delta=0.0):
    if system == "poisson":
        levels = hierarchy.scalar_levels(dim, n, p, mu, bc, basis, tau0)
        vc = vcycle.build_mg(levels, smoother, sai_level, order, nu1, nu2, omega,
                             balance="scalar")
    else:
        levels = stokes.stokes_levels(dim, n, p, mu, bc, gamma, basis, tau0, cp, rho, delta)
        if zeta is None:
            zeta = TAB_ZETA[(gamma, dim)][p - 1]
        vc = vcycle.build_mg(levels, smoother, sai_level, order, nu1, nu2, omega,
                             balance="stokes", zeta=zeta, dim=dim)
    return levels, vc


def solve(levels, vc, b, krylov_kind="cg", rtol=1e-10, maxit=200):
    A = levels[0].A.tocsr()
    if krylov_kind == "cg":
        return krylov.pcg(A, b, vc.apply, rtol, maxit)
    return krylov.gmres_left(A, b, vc.apply, rtol, min(maxit, 100))
