"""Mesh hierarchy, transfers and factor coarsening (oracle; test infrastructure).

Section 2.2 ("Multigrid schemes"):
  * nested hierarchy E_h, E_2h, ... by agglomerating 2^d children;
  * interpolation I_{2h}^h = polynomial injection, one tensor product of 1-D
    child matrices P^(c) per child;
  * restriction of the residual by (I_{2h}^h)^T (mass-basis Galerkin form,
    footnote to Algorithm 1);
  * coarse operators by operator coarsening, which the paper states is
    equivalent to re-discretising on the coarse mesh.  Reading taken: each
    factor of A is coarsened on its own,
        G_k^{2h}  = (M^{2h})^{-1} I^T M^h G_k^h I     (L2 projection of G I)
        M_mu^{2h} = I^T M_mu^h I
        E^{2h}    = 1/2 I^T E^h I                      (tau ~ 1/h)
        E_p^{2h}  = 2   I^T E_p^h I                    (pressure tau ~ h)
        M_rho^{2h} = I^T M_rho^h I                     (unsteady Stokes; delta is kept)
    and A^{2h} is formed from the coarse factors exactly as on the fine grid.
  * levels: halve n while n is even and n > 2; the last level is the bottom.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .basis import kron_dims
from .ldg import Grid, ElementMatrices, to_bsr, combine, assemble_scalar


@dataclass
class Level:
    grid: Grid
    em: ElementMatrices
    G: list
    Mmu: sp.spmatrix
    M: sp.spmatrix
    E: sp.spmatrix
    Ep: Optional[sp.spmatrix]
    A: sp.spmatrix
    bs: int                        # unknowns per element
    system: str = "poisson"
    gamma: int = 0
    I: Optional[sp.spmatrix] = None   # injection from the next coarser level into this one
    ncomp: int = 1                 # scalar fields per element (Stokes: d+1)
    Mrho: Optional[sp.spmatrix] = None   # density-weighted mass (unsteady Stokes), else None
    delta: float = 0.0                    # time-step parameter of eq:blockformunsteady (0: steady)


def level_sizes(n: int) -> List[int]:
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] > 2:
        sizes.append(sizes[-1] // 2)
    return sizes


def injection(fine: Grid, em: ElementMatrices, ncomp: int = 1) -> sp.bsr_matrix:
    """I : coarse coefficients -> fine coefficients (block rows = fine elements)."""
    coarse_n = fine.n // 2
    bss = em.bs
    P = em.ref.P
    blocks_data = []
    indices = []
    for e in range(fine.ne):
        idx = fine.index(e)
        cpos = [i % 2 for i in idx]
        parent_idx = [i // 2 for i in idx]
        pe = 0
        for k in reversed(range(fine.dim)):
            pe = pe * coarse_n + parent_idx[k]
        blk = kron_dims([P[c] for c in cpos])
        if ncomp > 1:
            blk = np.kron(np.eye(ncomp), blk)
        blocks_data.append(blk)
        indices.append(pe)
    bs = bss * ncomp
    data = np.array(blocks_data).reshape(-1, bs, bs)
    return sp.bsr_matrix((data, np.array(indices), np.arange(fine.ne + 1)),
                         shape=(fine.ne * bs, coarse_n ** fine.dim * bs))


def coarsen_factors(lv: Level, tau_scale_E=0.5, tau_scale_Ep=2.0):
    """Coarse factors of one level (scalar fields; Stokes uses the same scalar
    factors for every component)."""
    g = lv.grid
    cg = Grid(g.dim, g.n // 2, g.bc)
    cem = ElementMatrices(g.dim, lv.em.p, cg.h, lv.em.ref.kind)
    I = injection(g, lv.em, 1).tocsr()
    It = I.T.tocsr()
    Mf = lv.M.tocsr()
    bsz = lv.em.bs
    Mc_inv = sp.block_diag([cem.Minv] * cg.ne, format="csr")
    G = [to_bsr(Mc_inv @ (It @ (Mf @ (Gk.tocsr() @ I))), bsz) for Gk in lv.G]
    Mmu = to_bsr(It @ lv.Mmu.tocsr() @ I, bsz)
    M = sp.block_diag([cem.M] * cg.ne, format="bsr")
    E = to_bsr(tau_scale_E * (It @ lv.E.tocsr() @ I), bsz)
    Ep = None if lv.Ep is None else to_bsr(tau_scale_Ep * (It @ lv.Ep.tocsr() @ I), bsz)
    if lv.Mrho is not None:      # M_rho^{2h} = I^T M_rho^h I, like the viscosity-weighted mass
        return cg, cem, G, Mmu, M, E, Ep, to_bsr(It @ lv.Mrho.tocsr() @ I, bsz)
    return cg, cem, G, Mmu, M, E, Ep


def scalar_levels(dim: int, n: int, p: int, mu=None, bc=None, basis="legendre",
                  tau0: float = 1.0) -> List[Level]:
    """Level list for the scalar (Poisson / elliptic interface) problem."""
    op = assemble_scalar(dim, n, p, mu, bc, basis, tau0)
    lv = Level(op.grid, op.em, op.G, op.Mmu, op.M, op.E, None, op.A, op.em.bs)
    levels = [lv]
    for _ in level_sizes(n)[1:]:
        cg, cem, G, Mmu, M, E, _ = coarsen_factors(levels[-1])[:7]
        A = combine(G, Mmu, E, cem.bs)
        levels[-1].I = injection(levels[-1].grid, levels[-1].em, 1)
        levels.append(Level(cg, cem, G, Mmu, M, E, None, A, cem.bs))
    return levels
