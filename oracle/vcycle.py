"""Multigrid V-cycle (oracle; test infrastructure).

Algorithm 1 of the paper, V(E_h, x_h, b_h):
  bottom level: solve A x = b with the bottom direct solver;
  otherwise: pre-smooth nu1 times; restricted residual r_2h = I^T (b - A x);
             x_2h = V(E_2h, 0, r_2h); x <- x + I x_2h; post-smooth nu2 times.
Section 2.2 (bullet "Bottom solver"): a precomputed symmetric
eigendecomposition of the bottom A, used as a pseudo-inverse on its kernel.
Reading for the kernel threshold: eigenvalues with |lambda| <= 1e-12 max|lambda|
are treated as zero.  nu1 = nu2 = 3 (Section 2.2).

Pre/post orderings (Section 2.4): the first letter is the pre-smoother, the
second the post-smoother; "O" = forward (eq:B1, or Gauss-Seidel colours in
order), "I" = reverse (eq:BT, or colours backwards).  Block Jacobi ignores the
ordering (it is symmetric).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import smoothers as sm


def bottom_pinv(A) -> np.ndarray:
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    lam, Q = np.linalg.eigh(0.5 * (Ad + Ad.T))
    thr = 1e-12 * np.abs(lam).max()
    inv = np.where(np.abs(lam) > thr, 1.0 / np.where(lam == 0, 1.0, lam), 0.0)
    return (Q * inv) @ Q.T


@dataclass
class SmootherData:
    kind: str                       # "jacobi" | "gs" | "sai"
    Dinv: Optional[np.ndarray] = None
    colours: Optional[np.ndarray] = None
    B: Optional[sp.spmatrix] = None
    omega: float = 0.8


@dataclass
class MGLevel:
    A: sp.csr_matrix
    bs: int
    I: Optional[sp.csr_matrix]      # coarse -> this level (None on the bottom)
    sm: Optional[SmootherData]
    pinv: Optional[np.ndarray] = None


class VCycle:
    def __init__(self, levels: List[MGLevel], order: str = "OI", nu1: int = 3, nu2: int = 3):
        self.levels = levels
        self.order = order
        self.nu1, self.nu2 = nu1, nu2

    def smooth(self, lv: MGLevel, x, b, forward: bool):
        s = lv.sm
        if s.kind == "jacobi":
            return x + s.omega * sm.block_diag_apply(s.Dinv, b - lv.A @ x)
        if s.kind == "gs":
            return sm.gs_sweep(lv.A, s.Dinv, s.colours, x, b, lv.bs,
                               reverse=not forward, omega=s.omega)
        if s.kind == "sai":
            r = b - lv.A @ x                 # x - B(Ax - b) = x + B(b - Ax)
            return x + (s.B @ r if forward else s.B.T @ r)
        raise ValueError(s.kind)

    def apply(self, b, level: int = 0):
        """x = V(E_level, 0, b)."""
        lv = self.levels[level]
        if lv.pinv is not None:
            return lv.pinv @ b
        x = np.zeros_like(b)
        pre_fwd = self.order[0] == "O"
        post_fwd = self.order[1] == "O"
        for _ in range(self.nu1):
            x = self.smooth(lv, x, b, pre_fwd)
        rc = lv.I.T @ (b - lv.A @ x)
        xc = self.apply(rc, level + 1)
        x = x + lv.I @ xc
        for _ in range(self.nu2):
            x = self.smooth(lv, x, b, post_fwd)
        return x

    def matrix(self) -> np.ndarray:
        """Dense matrix of the linear operator V (tiny problems only)."""
        n = self.levels[0].A.shape[0]
        return np.column_stack([self.apply(e) for e in np.eye(n)])


def build_mg(levels, smoother: str = "sai", sai_level: int = 1, order: str = "OI",
             nu1: int = 3, nu2: int = 3, omega: float = None, balance: str = "scalar",
             zeta: float = 0.1, dim: int = None):
    """Smoother data for every level of an oracle hierarchy and the V-cycle."""
    mls = []
    nsai_unique = []
    for li, lv in enumerate(levels):
        A = sp.csr_matrix(lv.A)
        bottom = li == len(levels) - 1
        if bottom:
            mls.append(MGLevel(A, lv.bs, None, None, pinv=bottom_pinv(A)))
            continue
        if smoother == "jacobi":
            sd = SmootherData("jacobi", Dinv=sm.block_inverses(A, lv.bs),
                              omega=0.8 if omega is None else omega)
        elif smoother == "gs":
            sd = SmootherData("gs", Dinv=sm.block_inverses(A, lv.bs),
                              colours=sm.greedy_colours(sm.block_pattern(A, lv.bs)),
                              omega=1.0 if omega is None else omega)
        elif smoother == "sai":
            if balance == "stokes":
                alpha = sm.balance_stokes(A, lv.bs, dim, zeta)
            elif balance == "scalar":
                alpha = sm.balance_scalar(A, lv.bs)
            else:
                alpha = None
            B, nu = sm.sai(A, lv.bs, sai_level, alpha)
            nsai_unique.append(nu)
            sd = SmootherData("sai", B=sp.csr_matrix(B))
        else:
            raise ValueError(smoother)
        mls.append(MGLevel(A, lv.bs, sp.csr_matrix(lv.I), sd))
    vc = VCycle(mls, order, nu1, nu2)
    vc.sai_unique = nsai_unique
    return vc
