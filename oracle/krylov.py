"""Krylov outer solvers and the convergence-speed metric (oracle; test infrastructure).

Section 2.2 (paragraph after the bullets): the V-cycle with zero initial guess
is a linear operator V used as the preconditioner of CG (needs a symmetric V)
or as a left preconditioner of GMRES (solve V A x = V b).
Section 2.4 and its footnote: zero initial guess; the residual norm recorded
per iteration is the Krylov method's own: sqrt(r^T V r) for preconditioned CG,
||V (A x_k - b)||_2 for left-preconditioned GMRES; rho from a straight-line fit
of log r_k against k; eq:eta  eta = log(0.1) / log(rho).

Stopping rule (reading of "1e-10 relative residual"): CG stops when the
recursively updated ||r_k||_2 <= rtol ||b||_2; GMRES when
||V r_k||_2 <= rtol ||V b||_2.  Both report the true ||b - A x||_2 / ||b||_2.
GMRES: no restart, modified Gram-Schmidt, Givens rotations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: List[float]        # Krylov-native residual norms r_0, r_1, ...
    rel_res_true: float
    eta: float


def eta_from_history(hist) -> float:
    """eq:eta with rho from least squares on log10 r_k versus k."""
    h = np.asarray(hist, dtype=np.float64)
    h = h[h > 0]
    if h.size < 2:
        return float("nan")
    k = np.arange(h.size, dtype=np.float64)
    slope = np.polyfit(k, np.log10(h), 1)[0]     # log10 rho
    if slope >= 0:
        return float("inf")
    return -1.0 / slope


def pcg(A, b, V: Callable, rtol=1e-10, maxit=200) -> SolveResult:
    """Preconditioned CG (Hestenes-Stiefel form), x0 = 0, z = V r.  The
    history holds sqrt(r_k^T V r_k) for k = 0 .. iters-1 (no V-cycle is spent
    on the converged residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    z = V(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [np.sqrt(abs(rz))]
    it = 0
    converged = np.linalg.norm(r) <= rtol * nb
    while not converged and it < maxit:
        q = A @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * nb:
            converged = True
            break
        z = V(r)
        rz_new = float(r @ z)
        hist.append(np.sqrt(abs(rz_new)))
        p = z + (rz_new / rz) * p
        rz = rz_new
    rel = np.linalg.norm(b - A @ x) / nb
    return SolveResult(x, it, converged, hist, rel, eta_from_history(hist))


def gmres_left(A, b, V: Callable, rtol=1e-10, maxit=100) -> SolveResult:
    """Left-preconditioned GMRES on V A x = V b, x0 = 0, no restart, MGS."""
    n = b.size
    r0 = V(b)
    beta = np.linalg.norm(r0)
    Q = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    hist = [beta]
    if beta == 0:
        return SolveResult(np.zeros_like(b), 0, True, hist, 0.0, float("nan"))
    Q[0] = r0 / beta
    k = 0
    converged = False
    for j in range(maxit):
        w = V(A @ Q[j])
        for i in range(j + 1):
            H[i, j] = Q[i] @ w
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            Q[j + 1] = w / H[j + 1, j]
        for i in range(j):                 # apply previous rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= rtol * beta:
            converged = True
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = Q[:k].T @ y
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    return SolveResult(x, k, converged, hist, rel, eta_from_history(hist))
