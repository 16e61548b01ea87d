"""1-D bases, quadrature and reference matrices (oracle; test infrastructure).

Section 2.1 ("LDG schemes"): the approximation space is the tensor-product
space Q_p on every element, with a tensor-product Legendre modal basis (the
paper's choice) or a nodal basis ("practically any reasonable basis").
Here two 1-D bases on the reference interval [-1, 1]:

  * "legendre": psi_i = sqrt((2i+1)/2) P_i, orthonormal in L2(-1,1);
  * "gl_nodal": Lagrange polynomials through the p+1 Gauss-Legendre points.

All reference integrals use (p+2)-point Gauss-Legendre quadrature, which is
exact for the degree-(2p+1) integrands that occur.

Section 2.2 ("Multigrid schemes"): the interpolation operator is polynomial
injection from a coarse element into its children; the 1-D factor for child c
(c = 0 lower half, c = 1 upper half) is P^(c) with
    P^(c)_{ij} = (m^-1 int_{-1}^{1} psi_i(t) psi_j(phi_c(t)) dt)_{ij}
where phi_c maps the child's reference interval onto its half of the parent's.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule on [-1,1] (library primitive)."""
    return npleg.leggauss(q)


class Basis1D:
    """Evaluates one of the two 1-D bases of degree p and their derivatives."""

    def __init__(self, p: int, kind: str = "legendre"):
        if p < 0:
            raise ValueError("degree must be >= 0")
        if kind not in ("legendre", "gl_nodal"):
            raise ValueError(kind)
        self.p = p
        self.kind = kind
        if kind == "gl_nodal":
            self.nodes, _ = gauss_legendre(p + 1)

    def eval(self, t: np.ndarray) -> np.ndarray:
        """V[i, k] = psi_i(t_k)."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        p = self.p
        V = np.zeros((p + 1, t.size))
        if self.kind == "legendre":
            for i in range(p + 1):
                c = np.zeros(i + 1)
                c[i] = 1.0
                V[i] = np.sqrt((2 * i + 1) / 2.0) * npleg.legval(t, c)
        else:
            z = self.nodes
            for i in range(p + 1):
                v = np.ones_like(t)
                for j in range(p + 1):
                    if j != i:
                        v = v * (t - z[j]) / (z[i] - z[j])
                V[i] = v
        return V

    def deriv(self, t: np.ndarray) -> np.ndarray:
        """D[i, k] = psi_i'(t_k)."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        p = self.p
        D = np.zeros((p + 1, t.size))
        if self.kind == "legendre":
            for i in range(p + 1):
                c = np.zeros(i + 1)
                c[i] = 1.0
                D[i] = np.sqrt((2 * i + 1) / 2.0) * npleg.legval(t, npleg.legder(c)) \
                    if i > 0 else 0.0
        else:
            z = self.nodes
            for i in range(p + 1):
                s = np.zeros_like(t)
                for m in range(p + 1):          # product rule: drop factor m
                    if m == i:
                        continue
                    term = np.full_like(t, 1.0 / (z[i] - z[m]))
                    for j in range(p + 1):
                        if j != i and j != m:
                            term = term * (t - z[j]) / (z[i] - z[j])
                    s = s + term
                D[i] = s
        return D


class RefMatrices:
    """Reference 1-D matrices on [-1,1] for a basis of degree p.

    mass[i,j]  = int psi_i psi_j
    adv[i,j]   = int psi_i psi_j'        (test i, differentiated trial j)
    tm[i]      = psi_i(-1),  tp[i] = psi_i(+1)
    P[c][i,j]  = injection of coarse psi_j into child c, in child coefficients
    """

    def __init__(self, p: int, kind: str = "legendre"):
        self.p = p
        self.kind = kind
        b = Basis1D(p, kind)
        t, w = gauss_legendre(p + 2)
        V = b.eval(t)
        Dv = b.deriv(t)
        self.mass = (V * w) @ V.T
        self.adv = (V * w) @ Dv.T
        self.tm = b.eval(np.array([-1.0]))[:, 0]
        self.tp = b.eval(np.array([1.0]))[:, 0]
        minv = np.linalg.inv(self.mass)
        self.P = []
        for c in (0, 1):
            tc = 0.5 * (t + (2 * c - 1))        # child point -> parent coordinate
            Vc = b.eval(tc)                     # coarse basis at those points
            self.P.append(minv @ ((V * w) @ Vc.T))
        self.basis = b


def kron_dims(mats):
    """Tensor-product operator for a dof index with dimension 0 fastest:
    mats[k] acts on the index of dimension k."""
    out = np.array([[1.0]])
    for m in mats:                  # later dims become slower (outer) factors
        out = np.kron(m, out)
    return out
