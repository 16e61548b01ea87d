"""Stokes LDG saddle-point operator (oracle; test infrastructure).

Section 3.1 ("LDG schemes") and eq:components: unknowns (u_1..u_d, p), and

    [ A_ij        -G_i^T M ]        A_ij = delta_ij (sum_k G_k^T M_mu G_k)
    [ -M G_j      -E_p     ]               + gamma G_j^T M_mu G_i + delta_ij E

with G the (viscosity-upwinded) discrete gradient of the scalar problem, M the
plain block-diagonal mass, M_mu the viscosity-weighted mass, E the scalar
velocity penalty and E_p a pressure-only penalty.  gamma = 0 standard form,
gamma = 1 stress form.  Velocity Dirichlet boundary conditions use the same
one-sided gradient as the scalar problem (its divergence is the same G).

Pressure penalty (parity unpinned in absolute terms: the paper takes its
constants from an earlier work): E_p = sum over interior faces of
c_p * h / max(mu_L, mu_R) * int_F [p][q]; this has the h^d / mu scaling the
paper states in Section 3.3.

Per element the unknowns are ordered [u_1 (bs_s), .., u_d (bs_s), p (bs_s)]
with bs_s = (p+1)^d, so the element block has (d+1) bs_s unknowns
(Section 3.2: a block is velocity and pressure together).
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp

from .ldg import (Grid, ElementMatrices, assemble_gradient, assemble_penalty,
                  block_diag, to_bsr, volume_load, dirichlet_lifting, face_load)
from .hierarchy import Level, level_sizes, injection, coarsen_factors


def _perm_comp_to_elem(ne: int, bss: int, ncomp: int) -> np.ndarray:
    """perm[i_elem_major] = index in component-major ordering."""
    e = np.arange(ne)[:, None, None]
    c = np.arange(ncomp)[None, :, None]
    a = np.arange(bss)[None, None, :]
    return (c * ne * bss + e * bss + a).reshape(-1)


def stokes_matrix(G, Mmu, M, E, Ep, gamma: int, ne: int, bss: int, Mrho=None, delta: float = 0.0):
    """Assemble the element-major saddle-point matrix from scalar factors;
    with Mrho and delta > 0 the velocity blocks gain (1/delta) M_rho
    (eq:blockformunsteady)."""
    d = len(G)
    Gc = [g.tocsr() for g in G]
    Mmu = Mmu.tocsr()
    M = M.tocsr()
    lap = E.tocsr()
    for k in range(d):
        lap = lap + Gc[k].T @ Mmu @ Gc[k]
    if Mrho is not None and delta > 0:
        lap = lap + Mrho.tocsr() / delta
    rows = []
    for i in range(d):
        row = []
        for j in range(d):
            blk = lap if i == j else sp.csr_matrix(lap.shape)
            if gamma:
                blk = blk + gamma * (Gc[j].T @ Mmu @ Gc[i])
            row.append(blk)
        row.append(-(Gc[i].T @ M))
        rows.append(row)
    rows.append([-(M @ Gc[j]) for j in range(d)] + [-Ep.tocsr()])
    K = sp.bmat(rows, format="csr")
    perm = _perm_comp_to_elem(ne, bss, d + 1)
    K = K[perm][:, perm]
    return to_bsr(K, (d + 1) * bss)


def pressure_penalty(grid: Grid, em: ElementMatrices, mu, cp: float, rho=None, delta: float = 0.0):
    """E_p with weight c_p h / max(mu_eff,L, mu_eff,R) on interior faces.
    Steady: mu_eff = mu.  Unsteady (delta > 0; the blending rule of the work
    the paper cites is not reproduced in it, so this is a reading, parity
    unpinned in absolute terms): mu_eff = mu + rho h^2 / delta, so that the
    weight is c_p h / mu where viscosity dominates and c_p delta / (rho h),
    the penalty of the pressure-Poisson (projection) limit, where rho / delta
    dominates."""
    mu = np.asarray(mu, dtype=np.float64)
    if rho is not None and delta > 0:
        mu = mu + np.asarray(rho, dtype=np.float64) * grid.h ** 2 / delta
    return assemble_penalty(grid, em, mu, 0.0,
                            interior_tau=lambda ml, mr: cp * grid.h / max(ml, mr),
                            dirichlet=False)


def stokes_levels(dim: int, n: int, p: int, mu=None, bc=None, gamma: int = 1,
                  basis: str = "legendre", tau0: float = 1.0, cp: float = 1.0,
                  rho=None, delta: float = 0.0) -> List[Level]:
    """Stokes hierarchy; with delta > 0 the unsteady operator of
    eq:blockformunsteady: (1/delta) M_rho added to every velocity block, rho
    per element (None: 1), delta kept on every level."""
    grid = Grid(dim, n, bc)
    em = ElementMatrices(dim, p, grid.h, basis)
    mu = np.ones(grid.ne) if mu is None else np.asarray(mu, dtype=np.float64)
    unsteady = delta > 0
    rho_v = np.ones(grid.ne) if rho is None else np.asarray(rho, dtype=np.float64)
    G = assemble_gradient(grid, em, mu)
    Mmu = block_diag(grid, [mu[e] * em.M for e in range(grid.ne)])
    M = block_diag(grid, [em.M] * grid.ne)
    E = assemble_penalty(grid, em, mu, tau0)
    Ep = pressure_penalty(grid, em, mu, cp, rho_v if unsteady else None, delta)
    Mrho = block_diag(grid, [rho_v[e] * em.M for e in range(grid.ne)]) if unsteady else None
    ncomp = dim + 1
    A = stokes_matrix(G, Mmu, M, E, Ep, gamma, grid.ne, em.bs, Mrho, delta)
    lv = Level(grid, em, G, Mmu, M, E, Ep, A, ncomp * em.bs, "stokes", gamma, None, ncomp, Mrho, delta)
    levels = [lv]
    for _ in level_sizes(n)[1:]:
        out = coarsen_factors(levels[-1])
        cg, cem, Gc, Mmuc, Mc, Ec, Epc = out[:7]
        Mrc = out[7] if unsteady else None
        Ac = stokes_matrix(Gc, Mmuc, Mc, Ec, Epc, gamma, cg.ne, cem.bs, Mrc, delta)
        levels[-1].I = injection(levels[-1].grid, levels[-1].em, ncomp)
        levels.append(Level(cg, cem, Gc, Mmuc, Mc, Ec, Epc, Ac, ncomp * cem.bs,
                            "stokes", gamma, None, ncomp, Mrc, delta))
    return levels


def pressure_kernel(level: Level) -> np.ndarray:
    """Coefficient vector of (u = 0, p = 1): the kernel of the velocity-Dirichlet
    operator.  The constant's coefficients are m^-1 int psi_i per dimension."""
    ref = level.em.ref
    c1 = np.linalg.solve(ref.mass, _ones_moments(ref))
    from .basis import kron_dims
    cp = kron_dims([c1[:, None]] * level.grid.dim)[:, 0]
    bss = level.em.bs
    d = level.grid.dim
    k = np.zeros((level.grid.ne, (d + 1) * bss))
    k[:, d * bss:] = cp
    return k.reshape(-1)


def _ones_moments(ref):
    from .basis import gauss_legendre
    t, w = gauss_legendre(ref.p + 2)
    return ref.basis.eval(t) @ w


def stokes_rhs(level: Level, mu, f_qp=None, nq: int = 8, g=None,
               tau0: float = 1.0) -> np.ndarray:
    """Right-hand side of eq:components with a body force and velocity
    Dirichlet data (Section 3.1; the scalar data terms of Section 2.1 applied
    per velocity component).

    f_qp: list of d arrays [ne, nq^d], f_i at the tensor Gauss points;
    g:    list of d callables, the boundary velocity.
    Moving the data part of each velocity gradient, G_k^full u_i =
    G_k u_i + L_k g_i, to the right-hand side gives
      b_{u_i} = int f_i v - sum_k G_k^T M_mu L_k g_i
                - gamma sum_j G_j^T M_mu L_i g_j + sum_{F Dirichlet} tau_F int_F g_i v,
      b_p     = sum_j M L_j g_j
    (the continuity row of eq:components is -sum_j M G_j^full u_j - E_p p = 0).
    Returns the element-major vector [u_1 .. u_d, p] per element."""
    grid, em = level.grid, level.em
    d, bss, ne = grid.dim, em.bs, grid.ne
    mu = np.asarray(mu, dtype=np.float64)
    comp = np.zeros((d + 1, ne * bss))
    if f_qp is not None:
        for i in range(d):
            comp[i] += volume_load(em, f_qp[i], nq)
    if g is not None:
        G = [Gk.tocsr() for Gk in level.G]
        Mmu = level.Mmu.tocsr()
        M = level.M.tocsr()
        L = [dirichlet_lifting(level, g[i], nq) for i in range(d)]   # L[i][k] = L_k g_i
        for i in range(d):
            for k in range(d):
                comp[i] -= G[k].T @ (Mmu @ L[i][k])
                comp[i] -= level.gamma * (G[k].T @ (Mmu @ L[k][i]))
            for e in range(ne):
                for k in range(d):
                    for side in (-1, 1):
                        if grid.neighbour(e, k, side) is None and \
                                grid.boundary_type(k, side) == "D":
                            tau = tau0 * mu[e] / grid.h
                            comp[i, e * bss:(e + 1) * bss] += \
                                tau * face_load(grid, em, e, k, side, g[i], nq)
        for j in range(d):
            comp[d] += M @ L[j][j]
    return comp.reshape(d + 1, ne, bss).transpose(1, 0, 2).reshape(-1)
