"""Single block rows of the operator and single SAI columns on grids too large
to assemble whole (oracle; test infrastructure).

The same definitions as `ldg` / `stokes` / `smoothers`, evaluated only where
they are needed: row K of A = sum_k G_k^T M_mu G_k + E (Section 2.1) needs the
G_k rows of K and of the face neighbours whose flux is sourced from K; the
Stokes rows (eq:components) add the stress-form coupling G_j^T M_mu G_i, the
pressure gradient -G_i^T M, the divergence -M G_j and -E_p; a balanced SAI
column (Section 2.3.3 / 3.3) needs the rows of A on the two-step neighbourhood
of the column.  Only factors on the finest grid are available here, so these
functions cover the fine level of a hierarchy.
"""
from __future__ import annotations

import numpy as np

from .ldg import Grid, ElementMatrices, gradient_row, penalty_row, _add
from . import smoothers as sm


class LocalOperator:
    def __init__(self, dim, n, p, mu=None, bc=None, basis="legendre", tau0=1.0,
                 system="poisson", gamma=1, cp=0.1):
        self.grid = Grid(dim, n, bc)
        self.em = ElementMatrices(dim, p, self.grid.h, basis)
        self.mu = np.ones(self.grid.ne) if mu is None else np.asarray(mu, dtype=np.float64)
        self.tau0, self.system, self.gamma, self.cp = tau0, system, gamma, cp
        self.bss = self.em.bs
        self.ncomp = dim + 1 if system == "stokes" else 1
        self.bs = self.ncomp * self.bss
        self._grow = {}

    def grad_row(self, e, k):
        key = (e, k)
        if key not in self._grow:
            self._grow[key] = gradient_row(self.grid, self.em, self.mu, e, k)
        return self._grow[key]

    def _sources(self, K, k):
        """Rows L of G_k with a block in column K (K and its neighbours along e_k)."""
        out = [K]
        for side in (-1, 1):
            L = self.grid.neighbour(K, k, side)
            if L is not None and L not in out:
                out.append(L)
        return [L for L in out if K in self.grad_row(L, k)]

    def gram_row(self, K, ka, kb):
        """Row K of G_ka^T M_mu G_kb."""
        M = self.em.M
        blocks = {}
        for L in self._sources(K, ka):
            GLK = self.grad_row(L, ka)[K]
            for J, GLJ in self.grad_row(L, kb).items():
                _add(blocks, J, GLK.T @ (self.mu[L] * M) @ GLJ)
        return blocks

    def row(self, K):
        """{J: A_KJ} for one block row of the system matrix."""
        d, bss = self.grid.dim, self.bss
        lap = {}
        for k in range(d):
            for J, B in self.gram_row(K, k, k).items():
                _add(lap, J, B)
        for J, B in penalty_row(self.grid, self.em, self.mu, K, self.tau0).items():
            _add(lap, J, B)
        if self.system == "poisson":
            return lap
        bs = self.bs
        out = {}

        def put(J, ci, cj, B):
            if J not in out:
                out[J] = np.zeros((bs, bs))
            out[J][ci * bss:(ci + 1) * bss, cj * bss:(cj + 1) * bss] += B

        for J, B in lap.items():
            for i in range(d):
                put(J, i, i, B)
        if self.gamma:
            for i in range(d):
                for j in range(d):
                    for J, B in self.gram_row(K, j, i).items():
                        put(J, i, j, self.gamma * B)
        M = self.em.M
        for i in range(d):
            # -G_i^T M: (K, J) = -(G_i)_{J,K}^T M
            for L in self._sources(K, i):
                put(L, i, d, -(self.grad_row(L, i)[K].T @ M))
            # -M G_i: (K, J) = -M (G_i)_{K,J}
            for J, B in self.grad_row(K, i).items():
                put(J, d, i, -(M @ B))
        h = self.grid.h
        cp = self.cp
        for J, B in penalty_row(self.grid, self.em, self.mu, K, 0.0,
                                interior_tau=lambda a, b: cp * h / max(a, b),
                                dirichlet=False).items():
            put(J, d, d, -B)
        return out

    def apply_rows(self, rows, x):
        """(A x) restricted to the block rows `rows` -> array [len(rows), bs]."""
        bs = self.bs
        xv = x.reshape(-1, bs)
        return np.array([sum(B @ xv[J] for J, B in self.row(K).items()) for K in rows])

    # --- balanced SAI column (fine level) ------------------------------------
    def alpha(self, e, zeta=None):
        D = self.row(e)[e]
        if self.system == "poisson":
            return np.full(self.bs, np.linalg.norm(D) ** -0.5)
        nv = self.grid.dim * self.bss
        nA = np.linalg.norm(D[:nv, :nv])
        nD = np.linalg.norm(D[nv:, :nv])
        a = np.empty(self.bs)
        a[:nv] = nA ** -0.5
        a[nv:] = zeta * nA ** 0.5 / nD
        return a

    def sai_column(self, i, ell=1, zeta=None):
        """Block column i of the balanced SAI B (Section 2.3.3): returns
        {j: B_ji} for j in the pattern of column i of A^ell."""
        rows_cache = {}

        def row(K):
            if K not in rows_cache:
                rows_cache[K] = self.row(K)
            return rows_cache[K]

        J = {i}
        for _ in range(ell):
            J = set().union(*[set(row(j).keys()) for j in J])
        J = sorted(J)
        I = sorted(set().union(*[set(row(j).keys()) for j in J]))   # symmetric pattern
        al = {e: self.alpha(e, zeta) for e in set(I) | set(J)}
        bs = self.bs
        C = np.zeros((len(I) * bs, len(J) * bs))
        for a_, K in enumerate(I):
            rK = row(K)
            for b_, Jb in enumerate(J):
                if Jb in rK:
                    C[a_ * bs:(a_ + 1) * bs, b_ * bs:(b_ + 1) * bs] = \
                        al[K][:, None] * rK[Jb] * al[Jb][None, :]
        Erhs = np.zeros((len(I) * bs, bs))
        pos = I.index(i)
        Erhs[pos * bs:(pos + 1) * bs] = np.eye(bs)
        X = sm.lstsq_qr(C, Erhs)
        return {Jb: al[Jb][:, None] * X[b_ * bs:(b_ + 1) * bs] * al[i][None, :]
                for b_, Jb in enumerate(J)}
