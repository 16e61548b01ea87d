"""Element-wise block smoothers (oracle; test infrastructure).

Section 2.3 ("Element-wise block smoothers"); every block is the set of
unknowns of one element.

  * Block Jacobi, eq:Jsmooth:  x_i <- (1-w) x_i + w A_ii^{-1}(b_i - sum_{j!=i} A_ij x_j),
    A_ii^{-1} from a symmetric eigendecomposition of A_ii; w = 0.8.
  * Multi-coloured block Gauss-Seidel (Section 2.3.2 (i)): a greedy colouring of
    the block graph of A (red-black on 5/7-point stencils); colours processed in
    turn, in place, w = 1.  "Reverse" ordering visits the colours backwards.
  * Block SAI (Section 2.3.3): B_l = argmin_{B in M_A^l} ||A B - I||_F, where
    M_A^l has the block pattern of A^l, one independent least-squares problem
    per block column; with balancing alpha_{i,j} = ||A_ii||_F^{-1/2},
    A~ = diag(a) A diag(a), B = diag(a) B~ diag(a).  For Stokes the balancing
    of Section 3.3 (velocity/pressure sub-blocks and zeta) is used instead.
    Updates: eq:B1  x <- x - B (A x - b);  eq:BT  x <- x - B^T (A x - b).
    Representative-solution caching (Section 4, item (i)) is done by exact
    byte equality of the balanced local least-squares problem.
"""
from __future__ import annotations

import hashlib
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def diag_blocks(A: sp.bsr_matrix, bs: int) -> np.ndarray:
    A = sp.bsr_matrix(A, blocksize=(bs, bs))
    nb = A.shape[0] // bs
    out = np.zeros((nb, bs, bs))
    for i in range(nb):
        for s in range(A.indptr[i], A.indptr[i + 1]):
            if A.indices[s] == i:
                out[i] += A.data[s]
    return out


def sym_inverse_eig(Aii: np.ndarray) -> np.ndarray:
    """Inverse of a symmetric block through its eigendecomposition (eq:Jsmooth
    and the Stokes block smoothers cache an eigendecomposition of A_ii)."""
    lam, Q = np.linalg.eigh(0.5 * (Aii + Aii.T))
    return (Q / lam) @ Q.T


def block_inverses(A, bs) -> np.ndarray:
    return np.array([sym_inverse_eig(D) for D in diag_blocks(A, bs)])


def block_diag_apply(Dinv: np.ndarray, r: np.ndarray) -> np.ndarray:
    nb, bs, _ = Dinv.shape
    return np.einsum("iab,ib->ia", Dinv, r.reshape(nb, bs)).reshape(-1)


# ---------------------------------------------------------------------------
# Block pattern helpers
# ---------------------------------------------------------------------------
def block_pattern(A, bs) -> sp.csr_matrix:
    """Boolean block-level sparsity pattern of A (nb x nb)."""
    A = sp.bsr_matrix(A, blocksize=(bs, bs))
    nb = A.shape[0] // bs
    P = sp.csr_matrix((np.ones(len(A.indices)), A.indices.copy(), A.indptr.copy()),
                      shape=(nb, nb))
    P.sum_duplicates()
    P.data[:] = 1.0
    return P


def pattern_power(P: sp.csr_matrix, ell: int) -> sp.csr_matrix:
    nb = P.shape[0]
    out = sp.identity(nb, format="csr")
    for _ in range(ell):
        out = out @ P
        out.data[:] = 1.0
    out.sort_indices()
    return out


# ---------------------------------------------------------------------------
# Multi-coloured Gauss-Seidel
# ---------------------------------------------------------------------------
def greedy_colours(P: sp.csr_matrix) -> np.ndarray:
    """Visit elements in index order, give each the smallest colour not used by
    an already coloured neighbour (Section 2.3.2 (i))."""
    nb = P.shape[0]
    col = -np.ones(nb, dtype=np.int64)
    for i in range(nb):
        used = {col[j] for j in P.indices[P.indptr[i]:P.indptr[i + 1]] if j != i and col[j] >= 0}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def gs_sweep(A, Dinv, colours, x, b, bs, reverse=False, omega=1.0):
    """One multi-coloured block GS sweep: for each colour, every element of that
    colour is updated x_i <- (1-w)x_i + w A_ii^{-1}(b_i - sum_{j!=i} A_ij x_j)
    using the current x."""
    x = x.copy()
    ncol = colours.max() + 1
    order = range(ncol - 1, -1, -1) if reverse else range(ncol)
    A = A.tocsr()
    for c in order:
        mask = np.repeat(colours == c, bs)
        r = b - A @ x
        upd = block_diag_apply(Dinv, r)
        x[mask] += omega * upd[mask]
    return x


# ---------------------------------------------------------------------------
# Balanced block SAI
# ---------------------------------------------------------------------------
def balance_scalar(A, bs) -> np.ndarray:
    """alpha_{i,j} = ||A_ii||_F^{-1/2} (Section 2.3.3)."""
    D = diag_blocks(A, bs)
    a = np.array([np.linalg.norm(Di) ** -0.5 for Di in D])
    return np.repeat(a, bs)


def balance_stokes(A, bs, dim, zeta) -> np.ndarray:
    """Section 3.3: alpha_u = ||A_ii||_F^{-1/2} on the velocity unknowns and
    alpha_p = zeta ||A_ii||_F^{1/2} ||D_ii||_F^{-1} on the pressure unknowns of
    element i, A_ii the velocity-velocity and D_ii the (negated) divergence
    sub-block of the diagonal block."""
    D = diag_blocks(A, bs)
    nv = dim * (bs // (dim + 1))
    out = np.zeros((D.shape[0], bs))
    for i, Di in enumerate(D):
        nA = np.linalg.norm(Di[:nv, :nv])
        nD = np.linalg.norm(Di[nv:, :nv])
        out[i, :nv] = nA ** -0.5
        out[i, nv:] = zeta * nA ** 0.5 / nD
    return out.reshape(-1)


def sai(A, bs: int, ell: int, alpha: Optional[np.ndarray] = None,
        use_cache: bool = True):
    """Balanced block SAI B (as BSR) with the pattern of A^ell.

    Column block i:  J = rows of the pattern of column i,  I = block rows where
    A~[:, J] is nonzero;  X = argmin ||A~[I,J] X - E[I,i]||_F  by Householder QR
    (numpy's QR, i.e. LAPACK); fall back to a minimum-norm SVD solution when the
    problem is rank deficient.  B~[J, i] = X, then B = diag(a) B~ diag(a).
    """
    A = sp.bsr_matrix(A, blocksize=(bs, bs))
    nb = A.shape[0] // bs
    if alpha is None:
        alpha = np.ones(nb * bs)
    At = sp.diags(alpha) @ A.tocsr() @ sp.diags(alpha)
    At = At.tocsc()
    P = block_pattern(A, bs)
    Pl = pattern_power(P, ell).tocsc()          # column i of pattern -> J
    Pc = P.tocsc()
    cache = {}
    rows, cols, vals = [], [], []
    for i in range(nb):
        J = np.sort(Pl.indices[Pl.indptr[i]:Pl.indptr[i + 1]])
        Iset = set()
        for j in J:
            Iset.update(Pc.indices[Pc.indptr[j]:Pc.indptr[j + 1]].tolist())
        I = np.array(sorted(Iset))
        ri = np.concatenate([np.arange(k * bs, (k + 1) * bs) for k in I])
        ci = np.concatenate([np.arange(k * bs, (k + 1) * bs) for k in J])
        C = At[:, ci][ri, :].toarray()
        pos = int(np.where(I == i)[0][0])
        key = None
        if use_cache:
            hsh = hashlib.sha1(C.tobytes())
            hsh.update(np.array([len(I), len(J), pos]).tobytes())
            key = hsh.digest()
        if key is not None and key in cache:
            X = cache[key]
        else:
            Erhs = np.zeros((len(I) * bs, bs))
            Erhs[pos * bs:(pos + 1) * bs] = np.eye(bs)
            X = lstsq_qr(C, Erhs)
            if key is not None:
                cache[key] = X
        for jj, j in enumerate(J):
            blk = X[jj * bs:(jj + 1) * bs]          # B~_{j i}
            rr, cc = np.meshgrid(np.arange(j * bs, (j + 1) * bs),
                                 np.arange(i * bs, (i + 1) * bs), indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(blk.ravel())
    Bt = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=A.shape)
    B = sp.diags(alpha) @ Bt @ sp.diags(alpha)
    B = sp.csr_matrix(B)
    B.sort_indices()
    return B.tobsr(blocksize=(bs, bs)), len(cache)


def lstsq_qr(C: np.ndarray, R: np.ndarray) -> np.ndarray:
    """min ||C X - R||_F by Householder QR; min-norm SVD fallback if the
    triangular factor is numerically singular."""
    Q, Rf = np.linalg.qr(C, mode="reduced")
    d = np.abs(np.diag(Rf))
    if d.min() <= 1e-13 * d.max():
        return np.linalg.lstsq(C, R, rcond=None)[0]
    return sla.solve_triangular(Rf, Q.T @ R, lower=False)
