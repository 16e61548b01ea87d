"""Scalar LDG discretisation on a uniform Cartesian grid (oracle; test infrastructure).

Follows Section 2.1 ("LDG schemes") of the paper:

  (i)   a discrete gradient G = (G_1..G_d) built with viscosity-upwinded
        one-sided numerical fluxes, taking Dirichlet data into account;
  (ii)  sigma = L2 projection of mu * tau, i.e. the mu-weighted mass M_mu;
  (iii) the adjoint of the gradient as (negative) divergence;
  (iv)  penalty stabilisation E;
giving the symmetric operator  A = sum_k G_k^T M_mu G_k + E.

Flux rule (Section 2.1, first bullet): on a face between two elements the
numerical trace u-hat is taken from the *more viscous* side; sigma-hat then
comes from the other side, which the adjoint construction produces by itself.
Reading for ties (equal viscosity): u-hat from the lower-coordinate side.

Penalty (parity unpinned in absolute terms; the constants live in works the
paper cites but does not reproduce): tau_F = tau0 * mu_F / h with
mu_F = min(mu_L, mu_R) on interior faces and mu_K on Dirichlet faces,
E = sum_F tau_F int_F [u][v].

Conventions: elements lexicographic with x fastest; inside an element the
dof index has the x-degree fastest; BC codes per face ordered
(x-, x+, y-, y+, z-, z+), each "D" (Dirichlet), "N" (Neumann) or "P" (periodic).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np
import scipy.sparse as sp

from .basis import RefMatrices, kron_dims, gauss_legendre


class Grid:
    def __init__(self, dim: int, n: int, bc: Sequence[str] = None):
        self.dim = dim
        self.n = n
        self.ne = n ** dim
        self.h = 1.0 / n
        if bc is None:
            bc = ["D"] * (2 * dim)
        self.bc = list(bc)
        for k in range(dim):
            if (self.bc[2 * k] == "P") != (self.bc[2 * k + 1] == "P"):
                raise ValueError("periodic must be set on both faces of a dimension")

    def index(self, e: int):
        """Multi-index (i_0, .., i_{d-1}) of element e."""
        out = []
        for _ in range(self.dim):
            out.append(e % self.n)
            e //= self.n
        return out

    def elem(self, idx) -> int:
        e = 0
        for k in reversed(range(self.dim)):
            e = e * self.n + idx[k]
        return e

    def neighbour(self, e: int, k: int, side: int) -> Optional[int]:
        """Neighbour of e across its face in dimension k (side -1 lower, +1
        upper); None on a non-periodic boundary."""
        idx = self.index(e)
        j = idx[k] + side
        if 0 <= j < self.n:
            idx[k] = j
            return self.elem(idx)
        if self.bc[2 * k] == "P":
            idx[k] = j % self.n
            return self.elem(idx)
        return None

    def boundary_type(self, k: int, side: int) -> str:
        return self.bc[2 * k + (0 if side < 0 else 1)]


class ElementMatrices:
    """Physical element matrices of Q_p on a cube of side h."""

    def __init__(self, dim: int, p: int, h: float, kind: str = "legendre"):
        self.dim, self.p, self.h = dim, p, h
        self.ref = ref = RefMatrices(p, kind)
        self.bs = (p + 1) ** dim
        j = h / 2.0
        self.M = j ** dim * kron_dims([ref.mass] * dim)
        self.Minv = np.linalg.inv(self.M)
        self.D = []       # int_K w d_k u
        for k in range(dim):
            mats = [ref.mass] * dim
            mats = list(mats)
            mats[k] = ref.adv
            self.D.append(j ** (dim - 1) * kron_dims(mats))
        trace = {-1: ref.tm, +1: ref.tp}
        self.T = {}       # T[k, s_test, s_trial] = int_F w|_{s_test} u|_{s_trial}
        for k in range(dim):
            for s1 in (-1, 1):
                for s2 in (-1, 1):
                    mats = [ref.mass] * dim
                    mats = list(mats)
                    mats[k] = np.outer(trace[s1], trace[s2])
                    self.T[k, s1, s2] = j ** (dim - 1) * kron_dims(mats)


def _bsr(blocks: dict, nb: int, bs: int) -> sp.bsr_matrix:
    """Block dict {(I,J): dense bs x bs} -> BSR matrix (nb*bs square)."""
    rows = {}
    for (I, J), blk in blocks.items():
        rows.setdefault(I, []).append((J, blk))
    indptr = [0]
    indices = []
    data = []
    for I in range(nb):
        for J, blk in sorted(rows.get(I, []), key=lambda t: t[0]):
            indices.append(J)
            data.append(blk)
        indptr.append(len(indices))
    data = np.array(data, dtype=np.float64).reshape(-1, bs, bs) if data else \
        np.zeros((0, bs, bs))
    return sp.bsr_matrix((data, np.array(indices, dtype=np.int64),
                          np.array(indptr, dtype=np.int64)),
                         shape=(nb * bs, nb * bs))


def _add(blocks, key, val):
    if key in blocks:
        blocks[key] = blocks[key] + val
    else:
        blocks[key] = np.array(val, dtype=np.float64)


def flux_source_lower_face(grid: Grid, mu, e: int, k: int):
    """Element that supplies u-hat on the lower face of e in dimension k
    (Section 2.1: from the more viscous side; ties -> lower side).  Returns
    ('nbr', L), ('self', e), ('dirichlet', None) or ('neumann', None)."""
    L = grid.neighbour(e, k, -1)
    if L is None:
        return ("dirichlet" if grid.boundary_type(k, -1) == "D" else "neumann", None)
    return ("nbr", L) if mu[L] >= mu[e] else ("self", e)


def flux_source_upper_face(grid: Grid, mu, e: int, k: int):
    R = grid.neighbour(e, k, +1)
    if R is None:
        return ("dirichlet" if grid.boundary_type(k, +1) == "D" else "neumann", None)
    return ("self", e) if mu[e] >= mu[R] else ("nbr", R)


@dataclass
class ScalarLDG:
    """The factors of A = sum_k G_k^T M_mu G_k + E on one grid."""
    grid: Grid
    em: ElementMatrices
    mu: np.ndarray
    G: list            # G_k as BSR (dof level)
    Mmu: sp.spmatrix   # mu-weighted block-diagonal mass
    M: sp.spmatrix     # plain block-diagonal mass
    E: sp.spmatrix     # penalty
    A: sp.spmatrix = None

    @property
    def bs(self):
        return self.em.bs


def gradient_row(grid: Grid, em: ElementMatrices, mu, e: int, k: int) -> dict:
    """Block row e of G_k: M (G_k u)_e = int_e d_k u w + sum over the two faces
    of e normal to e_k of int_F (u-hat - u_e) w n_k, with u-hat from the flux
    rule; on Dirichlet faces the operator part of u-hat is 0 (the data part is
    `dirichlet_lifting`).  Returns {column element: block}."""
    blocks = {}
    _add(blocks, e, em.D[k])
    # lower face, outward normal -e_k
    src, L = flux_source_lower_face(grid, mu, e, k)
    if src == "nbr":          # -(u_L - u_e)
        _add(blocks, L, -em.T[k, -1, +1])
        _add(blocks, e, em.T[k, -1, -1])
    elif src == "dirichlet":  # -(0 - u_e)
        _add(blocks, e, em.T[k, -1, -1])
    # upper face, outward normal +e_k
    src, R = flux_source_upper_face(grid, mu, e, k)
    if src == "nbr":          # +(u_R - u_e)
        _add(blocks, R, em.T[k, +1, -1])
        _add(blocks, e, -em.T[k, +1, +1])
    elif src == "dirichlet":  # +(0 - u_e)
        _add(blocks, e, -em.T[k, +1, +1])
    return {J: em.Minv @ B for J, B in blocks.items()}


def assemble_gradient(grid: Grid, em: ElementMatrices, mu) -> list:
    """G_k for k = 1..d as BSR matrices, row by row (`gradient_row`)."""
    G = []
    for k in range(grid.dim):
        blocks = {}
        for e in range(grid.ne):
            for J, B in gradient_row(grid, em, mu, e, k).items():
                blocks[(e, J)] = B
        G.append(_bsr(blocks, grid.ne, em.bs))
    return G


def penalty_row(grid: Grid, em: ElementMatrices, mu, e: int, tau0: float,
                interior_tau=None, dirichlet=True) -> dict:
    """Block row e of E = sum_F tau_F int_F [u][v]: interior tau = tau0 min(mu)/h
    and Dirichlet tau = tau0 mu_e / h (reading of the penalty; see module
    docstring).  `interior_tau(mu_lower, mu_upper)` overrides the interior
    weight and `dirichlet=False` drops the boundary faces (pressure penalty)."""
    h = grid.h
    tau_of = (lambda a, b: tau0 * min(mu[a], mu[b]) / h) if interior_tau is None else \
        (lambda a, b: interior_tau(mu[a], mu[b]))
    blocks = {e: np.zeros((em.bs, em.bs))}
    for k in range(grid.dim):
        L = grid.neighbour(e, k, -1)
        if L is not None:          # face (L, e): e is the upper side
            tau = tau_of(L, e)
            _add(blocks, e, tau * em.T[k, -1, -1])
            _add(blocks, L, -tau * em.T[k, -1, +1])
        elif dirichlet and grid.boundary_type(k, -1) == "D":
            _add(blocks, e, tau0 * mu[e] / h * em.T[k, -1, -1])
        R = grid.neighbour(e, k, +1)
        if R is not None:          # face (e, R): e is the lower side
            tau = tau_of(e, R)
            _add(blocks, e, tau * em.T[k, +1, +1])
            _add(blocks, R, -tau * em.T[k, +1, -1])
        elif dirichlet and grid.boundary_type(k, +1) == "D":
            _add(blocks, e, tau0 * mu[e] / h * em.T[k, +1, +1])
    return blocks


def assemble_penalty(grid: Grid, em: ElementMatrices, mu, tau0: float,
                     interior_tau=None, dirichlet=True) -> sp.bsr_matrix:
    """E as a BSR matrix, row by row (`penalty_row`)."""
    blocks = {}
    for e in range(grid.ne):
        for J, B in penalty_row(grid, em, mu, e, tau0, interior_tau, dirichlet).items():
            blocks[(e, J)] = B
    return _bsr(blocks, grid.ne, em.bs)


def block_diag(grid: Grid, blocks_per_elem) -> sp.bsr_matrix:
    bs = blocks_per_elem[0].shape[0]
    return _bsr({(e, e): blocks_per_elem[e] for e in range(grid.ne)}, grid.ne, bs)


def to_bsr(A, bs: int) -> sp.bsr_matrix:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    return A.tobsr(blocksize=(bs, bs))


def combine(G, Mmu, E, bs):
    """A = sum_k G_k^T M_mu G_k + E (Section 2.1)."""
    A = E.tocsr()
    for Gk in G:
        Gc = Gk.tocsr()
        A = A + Gc.T @ (Mmu.tocsr() @ Gc)
    return to_bsr(A, bs)


def assemble_scalar(dim: int, n: int, p: int, mu=None, bc=None,
                    basis: str = "legendre", tau0: float = 1.0) -> ScalarLDG:
    grid = Grid(dim, n, bc)
    em = ElementMatrices(dim, p, grid.h, basis)
    mu = np.ones(grid.ne) if mu is None else np.asarray(mu, dtype=np.float64)
    G = assemble_gradient(grid, em, mu)
    Mmu = block_diag(grid, [mu[e] * em.M for e in range(grid.ne)])
    M = block_diag(grid, [em.M] * grid.ne)
    E = assemble_penalty(grid, em, mu, tau0)
    op = ScalarLDG(grid, em, mu, G, Mmu, M, E)
    op.A = combine(G, Mmu, E, em.bs)
    return op


# ----------------------------------------------------------------------------
# Right-hand side (Section 2.1: b collects f, g and h)
# ----------------------------------------------------------------------------
def volume_load(em: ElementMatrices, f_qp: np.ndarray, nq: int) -> np.ndarray:
    """b_K[a] = int_K f psi_a from f sampled at the nq^d tensor Gauss-Legendre
    points of every element (points ordered x fastest)."""
    t, w = gauss_legendre(nq)
    V = em.ref.basis.eval(t) * w              # [(p+1), nq]
    B = kron_dims([V] * em.dim)               # [(p+1)^d, nq^d]
    scale = (em.h / 2.0) ** em.dim
    return (scale * (np.asarray(f_qp).reshape(-1, nq ** em.dim) @ B.T)).reshape(-1)


def _face_points(grid: Grid, e: int, k: int, side: int, nq: int):
    """Physical quadrature points and weights on the face of e at (k, side),
    plus the tangential reference abscissae for basis evaluation."""
    t, w = gauss_legendre(nq)
    idx = grid.index(e)
    h = grid.h
    dims = [j for j in range(grid.dim) if j != k]
    grids = np.meshgrid(*([t] * len(dims)), indexing="ij") if dims else []
    # points with the first tangential dim fastest
    coords = np.zeros((nq ** len(dims), grid.dim))
    wts = np.ones(nq ** len(dims))
    refs = np.zeros((nq ** len(dims), grid.dim))
    for q in range(nq ** len(dims)):
        rem = q
        for j in dims:
            iq = rem % nq
            rem //= nq
            refs[q, j] = t[iq]
            coords[q, j] = (idx[j] + 0.5 * (t[iq] + 1.0)) * h
            wts[q] *= w[iq]
        refs[q, k] = float(side)
        coords[q, k] = (idx[k] + (0.0 if side < 0 else 1.0)) * h
    return coords, wts * (h / 2.0) ** (grid.dim - 1), refs


def _basis_at(em: ElementMatrices, refs: np.ndarray) -> np.ndarray:
    """psi_a at reference points refs [nq, d] -> [bs, nq]."""
    d = em.dim
    vals = [em.ref.basis.eval(refs[:, j]) for j in range(d)]   # [(p+1), nq]
    out = np.ones((1, refs.shape[0]))
    for j in range(d):
        out = (vals[j][:, None, :] * out[None, :, :]).reshape(-1, refs.shape[0])
    return out


def face_load(grid: Grid, em: ElementMatrices, e: int, k: int, side: int,
              func: Callable, nq: int) -> np.ndarray:
    """int_F func psi_a over the face of e at (k, side)."""
    X, W, R = _face_points(grid, e, k, side, nq)
    Phi = _basis_at(em, R)
    vals = func(*[X[:, j] for j in range(grid.dim)])
    return Phi @ (W * vals)


def dirichlet_lifting(op: ScalarLDG, g: Callable, nq: int):
    """Coefficients of L_k g: M (L_k g)_K = sum_{Dirichlet faces} int_F g w n_k."""
    grid, em = op.grid, op.em
    out = []
    for k in range(grid.dim):
        v = np.zeros(grid.ne * em.bs)
        for e in range(grid.ne):
            for side in (-1, 1):
                if grid.neighbour(e, k, side) is None and grid.boundary_type(k, side) == "D":
                    v[e * em.bs:(e + 1) * em.bs] += side * face_load(grid, em, e, k, side, g, nq)
        out.append((v.reshape(-1, em.bs) @ em.Minv.T).reshape(-1))
    return out


def rhs(op: ScalarLDG, f_qp=None, nq: int = 8, g: Callable = None,
        hflux: Callable = None, tau0: float = 1.0) -> np.ndarray:
    """b = int f v - sum_k G_k^T M_mu L_k g + sum_{F in Dirichlet} tau_F int_F g v
           + sum_{F in Neumann} int_F h v."""
    grid, em = op.grid, op.em
    b = np.zeros(grid.ne * em.bs)
    if f_qp is not None:
        b += volume_load(em, f_qp, nq)
    if g is not None:
        Lg = dirichlet_lifting(op, g, nq)
        for k in range(grid.dim):
            b -= op.G[k].T @ (op.Mmu @ Lg[k])
        for e in range(grid.ne):
            for k in range(grid.dim):
                for side in (-1, 1):
                    if grid.neighbour(e, k, side) is None and grid.boundary_type(k, side) == "D":
                        tau = tau0 * op.mu[e] / grid.h
                        b[e * em.bs:(e + 1) * em.bs] += tau * face_load(grid, em, e, k, side, g, nq)
    if hflux is not None:
        for e in range(grid.ne):
            for k in range(grid.dim):
                for side in (-1, 1):
                    if grid.neighbour(e, k, side) is None and grid.boundary_type(k, side) == "N":
                        b[e * em.bs:(e + 1) * em.bs] += face_load(grid, em, e, k, side, hflux, nq)
    return b


def evaluate(op: ScalarLDG, u: np.ndarray, nq: int):
    """Values of the discrete function u at the tensor Gauss points of every
    element: [ne, nq^d] (x fastest), plus the points' quadrature weights."""
    t, w = gauss_legendre(nq)
    V = op.em.ref.basis.eval(t)
    B = kron_dims([V] * op.grid.dim)           # [bs, nq^d]
    W = kron_dims([w[None, :]] * op.grid.dim)[0] * (op.grid.h / 2.0) ** op.grid.dim
    return u.reshape(op.grid.ne, -1) @ B, W
