"""Pins of the oracle's 1-D basis and transfer matrices against closed forms."""
import numpy as np
import pytest

from oracle.basis import Basis1D, RefMatrices, kron_dims, gauss_legendre


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_legendre_closed_forms(p):
    r = RefMatrices(p, "legendre")
    # orthonormal Legendre: identity mass
    assert np.allclose(r.mass, np.eye(p + 1), atol=1e-14)
    # P_i(1) = 1, P_i(-1) = (-1)^i
    s = np.sqrt((2 * np.arange(p + 1) + 1) / 2.0)
    assert np.allclose(r.tp, s, atol=1e-14)
    assert np.allclose(r.tm, s * (-1.0) ** np.arange(p + 1), atol=1e-14)
    # int P_i P_j' = 2 when j > i and i + j odd, else 0
    ref = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            if j > i and (i + j) % 2 == 1:
                ref[i, j] = 2.0 * s[i] * s[j]
    assert np.allclose(r.adv, ref, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gl_nodal_closed_forms(p):
    r = RefMatrices(p, "gl_nodal")
    t, w = gauss_legendre(p + 1)
    # Lagrange at the p+1 Gauss points: the exact mass is diag(weights)
    assert np.allclose(r.mass, np.diag(w), atol=1e-14)
    # cardinal property
    assert np.allclose(Basis1D(p, "gl_nodal").eval(t), np.eye(p + 1), atol=1e-13)
    # integration by parts: adv + adv^T = tp tp^T - tm tm^T
    assert np.allclose(r.adv + r.adv.T, np.outer(r.tp, r.tp) - np.outer(r.tm, r.tm), atol=1e-13)


@pytest.mark.parametrize("kind", ["legendre", "gl_nodal"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_injection_reproduces_coarse_polynomials(kind, p):
    """P^(c) maps coarse coefficients to the child coefficients of the same
    polynomial: check by evaluation at random points (brute force)."""
    r = RefMatrices(p, kind)
    b = Basis1D(p, kind)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(p + 1)
    t = rng.uniform(-1, 1, 17)
    for ch in (0, 1):
        parent_t = 0.5 * (t + (2 * ch - 1))
        lhs = (r.P[ch] @ c) @ b.eval(t)
        rhs = c @ b.eval(parent_t)
        assert np.allclose(lhs, rhs, atol=1e-13)
    # restriction of an injection is the identity: sum_c P_c^T m P_c = 2 m
    S = sum(r.P[ch].T @ r.mass @ r.P[ch] for ch in (0, 1))
    assert np.allclose(S, 2 * r.mass, atol=1e-13)


def test_kron_dims_ordering():
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    e = np.eye(2)
    K = kron_dims([a, e])           # acts on dim 0 (fastest)
    x = np.arange(4.0)              # x[a0 + 2 a1]
    y = K @ x
    X = x.reshape(2, 2)             # [a1, a0]
    assert np.allclose(y.reshape(2, 2), X @ a.T)
