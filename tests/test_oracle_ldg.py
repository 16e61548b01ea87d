"""Pins of the oracle's LDG discretisation (Section 2.1; Section 3.1)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from ldg_inputs import sample_on_elements, mms_source_2d, mms_solution_2d, mu_box
from oracle import ldg, hierarchy, stokes
from oracle.basis import kron_dims


def _solve(A, b):
    return spla.spsolve(A.tocsc(), b)


@pytest.mark.parametrize("basis", ["legendre", "gl_nodal"])
@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_polynomial_reproduction_dirichlet(basis, dim, p):
    """u in Q_p globally with u = g on the boundary and f = -Lap u exactly
    integrated is reproduced exactly (G u = grad u, no jumps)."""
    n = 3
    op = ldg.assemble_scalar(dim, n, p, basis=basis)
    if dim == 2:
        u = lambda x, y: x ** p * y + 0.5 * y ** p - x + 1.0
        f = lambda x, y: -(p * (p - 1) * x ** max(p - 2, 0) * y
                           + 0.5 * p * (p - 1) * y ** max(p - 2, 0))
    else:
        u = lambda x, y, z: x ** p * y * z + z - 2 * y
        f = lambda x, y, z: -(p * (p - 1) * x ** max(p - 2, 0) * y * z)
    nq = p + 3
    b = ldg.rhs(op, f_qp=sample_on_elements(dim, n, nq, f), nq=nq, g=u)
    x = _solve(op.A, b)
    vals, _ = ldg.evaluate(op, x, nq)
    assert np.abs(vals - sample_on_elements(dim, n, nq, u)).max() < 1e-11


def test_polynomial_reproduction_neumann_mixed():
    """Dirichlet on x faces, Neumann (flux data) on y faces."""
    dim, p, n = 2, 2, 4
    op = ldg.assemble_scalar(dim, n, p, bc=["D", "D", "N", "N"])
    u = lambda x, y: x * x - y * y + 3 * x * y + 0.25
    f = lambda x, y: 0.0 * x
    # outward flux mu du/dn on y = 0 (n = -y) and y = 1 (n = +y)
    hflux = lambda x, y: np.where(y < 0.5, -(-2 * y + 3 * x), (-2 * y + 3 * x))
    b = ldg.rhs(op, f_qp=sample_on_elements(dim, n, 5, f), nq=5, g=u, hflux=hflux)
    x = _solve(op.A, b)
    vals, _ = ldg.evaluate(op, x, 5)
    assert np.abs(vals - sample_on_elements(dim, n, 5, u)).max() < 1e-11


@pytest.mark.parametrize("ratio", [1e-4, 1e4])
def test_polynomial_reproduction_planar_interface(ratio):
    """Face-aligned interface x = 1/2: u piecewise linear in x with
    mu u' continuous is reproduced exactly for any viscosity ratio."""
    dim, p, n = 2, 2, 4
    grid_mu = np.array([ratio if (e % n) < n // 2 else 1.0 for e in range(n * n)])
    op = ldg.assemble_scalar(dim, n, p, mu=grid_mu)
    s_left = 1.0 / ratio                          # mu u' = 1 on both sides
    u = lambda x, y: np.where(x < 0.5, s_left * x, s_left * 0.5 + (x - 0.5)) + 0.0 * y
    f = lambda x, y: 0.0 * x
    b = ldg.rhs(op, f_qp=sample_on_elements(dim, n, 5, f), nq=5, g=u)
    x = _solve(op.A, b)
    vals, _ = ldg.evaluate(op, x, 5)
    ex = sample_on_elements(dim, n, 5, u)
    assert np.abs(vals - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


def test_mms_convergence_order_p2():
    """Config-1 manufactured solution sin(2 pi x) sin(3 pi y): the L2 error
    decays at order p + 1 = 3 (Section 2.1, last bullet)."""
    p, nq = 2, 6
    errs = []
    for n in (8, 16, 32):
        op = ldg.assemble_scalar(2, n, p, basis="gl_nodal")
        b = ldg.rhs(op, f_qp=sample_on_elements(2, n, nq, mms_source_2d), nq=nq)
        x = _solve(op.A, b)
        vals, W = ldg.evaluate(op, x, nq)
        ex = sample_on_elements(2, n, nq, mms_solution_2d)
        errs.append(math.sqrt(np.sum((vals - ex) ** 2 * W[None, :])))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.7 < r < 3.4 for r in rates), rates


@pytest.mark.parametrize("dim,n,p", [(2, 2, 1), (2, 3, 2), (2, 4, 3), (3, 2, 1), (3, 3, 2)])
def test_symmetric_definite_dirichlet(dim, n, p):
    A = ldg.assemble_scalar(dim, n, p).A.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("bc", ["P", "N"])
def test_semidefinite_kernel_is_constant(bc):
    dim, n, p = 2, 4, 2
    op = ldg.assemble_scalar(dim, n, p, bc=[bc] * 4)
    A = op.A.toarray()
    lam, Q = np.linalg.eigh(A)
    assert abs(lam[0]) < 1e-12 * lam[-1] and lam[1] > 1e-8 * lam[-1]
    # constant function in the Legendre basis: only the (0,0) mode, equal on all elements
    v = Q[:, 0].reshape(op.grid.ne, -1)
    v = v / v[0, 0]
    assert np.allclose(v[:, 0], 1.0, atol=1e-10) and np.abs(v[:, 1:]).max() < 1e-10


def test_stokes_inertia_velocity_dirichlet():
    """Saddle point with velocity Dirichlet: n_u positive, n_p - 1 negative and
    one zero eigenvalue (constant pressure)."""
    dim, n, p = 2, 3, 1
    lv = stokes.stokes_levels(dim, n, p, gamma=1, cp=0.1)
    A = lv[0].A.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    lam = np.linalg.eigvalsh(A)
    tol = 1e-10 * np.abs(lam).max()
    nbs = (p + 1) ** dim
    n_u, n_p = dim * nbs * n ** dim, nbs * n ** dim
    assert (lam > tol).sum() == n_u
    assert (lam < -tol).sum() == n_p - 1
    assert (np.abs(lam) <= tol).sum() == 1
    k = stokes.pressure_kernel(lv[0])
    assert np.abs(A @ k).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("system", ["poisson", "stokes"])
def test_factor_coarsening_equals_rediscretisation(system):
    """Constant viscosity: the factor-coarsened A_2h equals A assembled directly
    on the n/2 grid (Section 2.2: the two approaches are equivalent)."""
    dim, n, p = 2, 8, 2
    if system == "poisson":
        lv = hierarchy.scalar_levels(dim, n, p)
        direct = ldg.assemble_scalar(dim, n // 2, p).A
    else:
        lv = stokes.stokes_levels(dim, n, p, gamma=1, cp=0.1)
        direct = stokes.stokes_levels(dim, n // 2, p, gamma=1, cp=0.1)[0].A
    diff = (lv[1].A - direct).toarray()
    assert np.abs(diff).max() <= 1e-12 * np.abs(direct.toarray()).max()


def test_transfer_identities():
    """I^T M^h I = M^2h and restriction-of-injection = identity."""
    lv = hierarchy.scalar_levels(2, 8, 3)
    I = lv[0].I.tocsr()
    Mh, M2h = lv[0].M.tocsr(), lv[1].M.tocsr()
    assert np.abs((I.T @ Mh @ I - M2h).toarray()).max() < 1e-14
    R = np.linalg.inv(M2h.toarray()) @ (I.T @ Mh).toarray()
    assert np.allclose(R @ I.toarray(), np.eye(M2h.shape[0]), atol=1e-12)


def _l2_coefficients(level, funcs, nq):
    """Element-wise L2 projection of each callable onto Q_p (per component),
    stacked element-major [u_1 .. u_d, p]."""
    em, n, dim = level.em, level.grid.n, level.grid.dim
    cols = [ldg.volume_load(em, sample_on_elements(dim, n, nq, f), nq).reshape(-1, em.bs)
            @ em.Minv.T for f in funcs]
    return np.stack(cols, axis=1).reshape(-1)


def _stokes_exactness_residual(dim, n, p, gamma, mu, u, pres, f, nq):
    """max |A x_ex - b| / max(|A||x_ex| + |b|) for the exact solution's
    coefficients x_ex (a solution in the discrete space satisfies the
    discrete equations exactly: LDG consistency, Section 3.1)."""
    lv = stokes.stokes_levels(dim, n, p, mu=mu, gamma=gamma, cp=0.1)[0]
    fq = [sample_on_elements(dim, n, nq, fi) for fi in f]
    b = stokes.stokes_rhs(lv, mu, fq, nq, u)
    x = _l2_coefficients(lv, list(u) + [pres], nq)
    A = lv.A.tocsr()
    r = A @ x - b
    return np.abs(r).max() / (abs(A) @ np.abs(x) + np.abs(b)).max(), lv, b


@pytest.mark.parametrize("gamma", [0, 1])
def test_stokes_polynomial_reproduction_2d(gamma):
    """Divergence-free u in Q_2^2 (u = curl of x^2 y^2) and p = x y in Q_2 with
    unit viscosity, velocity Dirichlet data g = u and f = -Lap u + grad p (the
    stress term gamma grad(div u) vanishes): the discrete Stokes system of
    eq:components is solved exactly, in standard (gamma = 0) and stress
    (gamma = 1) form.  Both the residual of the exact coefficients and the
    solution of the singular system (bordered with the pressure kernel) are
    checked; the pressure is compared modulo its constant."""
    dim, n, p, nq = 2, 3, 2, 5
    u = [lambda x, y: 2 * x ** 2 * y, lambda x, y: -2 * x * y ** 2]
    pres = lambda x, y: x * y
    f = [lambda x, y: -4 * y + y, lambda x, y: 4 * x + x]
    res, lv, b = _stokes_exactness_residual(dim, n, p, gamma, np.ones(n * n), u, pres, f, nq)
    assert res < 1e-13
    A = lv.A.toarray()
    k = stokes.pressure_kernel(lv)
    N = A.shape[0]
    K = np.block([[A, k[:, None]], [k[None, :], np.zeros((1, 1))]])
    x = np.linalg.solve(K, np.concatenate([b, [0.0]]))
    assert abs(x[N]) < 1e-12 * np.abs(b).max()      # b is consistent (orthogonal to the kernel)
    X = x[:N].reshape(n * n, dim + 1, -1)
    for i, fn in enumerate(list(u) + [pres]):
        vals, W = ldg.evaluate(lv, X[:, i].reshape(-1), nq)
        ex = sample_on_elements(dim, n, nq, fn)
        if i == dim:
            vals = vals - (vals * W).sum() / (W.sum() * n * n)
            ex = ex - (ex * W).sum() / (W.sum() * n * n)
        assert np.abs(vals - ex).max() < 1e-11


@pytest.mark.parametrize("gamma", [0, 1])
def test_stokes_polynomial_reproduction_3d(gamma):
    """3D: u = (2x^2yz, -2xy^2z, xy) (divergence free, Q_2^3), p = x + yz."""
    u = [lambda x, y, z: 2 * x ** 2 * y * z, lambda x, y, z: -2 * x * y ** 2 * z,
         lambda x, y, z: x * y + 0 * z]
    pres = lambda x, y, z: x + y * z
    f = [lambda x, y, z: -4 * y * z + 1 + 0 * x, lambda x, y, z: 4 * x * z + z + 0 * y,
         lambda x, y, z: y + 0 * x]
    res, _, _ = _stokes_exactness_residual(3, 2, 2, gamma, np.ones(8), u, pres, f, 4)
    assert res < 1e-13


@pytest.mark.parametrize("ratio", [1e-4, 1e4, 10.0])
def test_stokes_stress_form_planar_interface(ratio):
    """Stress form across the face-aligned interface x = 1/2 (viscosity
    `ratio` left, 1 right): u = (c y, b(x)) with b piecewise linear is
    divergence free and force free in the bulk, and the traction
    mu (grad u + grad u^T) e_x is continuous iff mu_L (b_L' + c) =
    mu_R (b_R' + c).  That solution is reproduced exactly by the stress form
    only: the same data do not satisfy the standard form (whose traction is
    mu grad u e_x), and a stress term with its indices swapped
    (gamma G_i^T M_mu G_j, a grad-div term) leaves a residual of 2-5e-2."""
    dim, n, p, nq = 2, 4, 2, 5
    mu = np.array([ratio if (e % n) < n // 2 else 1.0 for e in range(n * n)])
    c, sR = 1.0, 1.0
    sL = (sR + c) / ratio - c
    u = [lambda x, y: c * y + 0 * x,
         lambda x, y: np.where(x < 0.5, sL * x, sL * 0.5 + sR * (x - 0.5)) + 0 * y]
    zero = lambda x, y: 0 * x
    res, _, _ = _stokes_exactness_residual(dim, n, p, 1, mu, u, zero, [zero, zero], nq)
    assert res < 1e-13
    res0, _, _ = _stokes_exactness_residual(dim, n, p, 0, mu, u, zero, [zero, zero], nq)
    assert res0 > 1e-7


@pytest.mark.parametrize("system", ["poisson", "stokes"])
@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1)])
@pytest.mark.parametrize("ratio", [1e-4, 1e4])
def test_factor_coarsening_variable_mu_aligned_box(system, dim, p, ratio):
    """Inner box (1/4,3/4)^d at viscosity ratio 1e+-4 on n = 8, whose faces lie
    on faces of the n = 4 grid: the factor-coarsened A_2h (upwinded G, mu-mass,
    1/2 I^T E I, 2 I^T E_p I) equals A assembled directly on the n = 4 grid
    with the same box (Section 2.2: operator coarsening is equivalent to
    re-discretisation)."""
    n = 8
    mu_f, mu_c = mu_box(dim, n, ratio), mu_box(dim, n // 2, ratio)
    if system == "poisson":
        lv = hierarchy.scalar_levels(dim, n, p, mu=mu_f)
        direct = ldg.assemble_scalar(dim, n // 2, p, mu=mu_c).A
    else:
        lv = stokes.stokes_levels(dim, n, p, mu=mu_f, gamma=1, cp=0.1)
        direct = stokes.stokes_levels(dim, n // 2, p, mu=mu_c, gamma=1, cp=0.1)[0].A
    D = direct.toarray()
    assert np.abs(lv[1].A.toarray() - D).max() <= 1e-13 * np.abs(D).max()


def _unsteady_residual(dim, n, p, gamma, mu, rho, delta, u, pres, f, nq, cp=0.1):
    lv = stokes.stokes_levels(dim, n, p, mu=mu, gamma=gamma, cp=cp, rho=rho, delta=delta)[0]
    fq = [sample_on_elements(dim, n, nq, fi) for fi in f]
    b = stokes.stokes_rhs(lv, mu, fq, nq, u)
    x = _l2_coefficients(lv, list(u) + [pres], nq)
    A = lv.A.tocsr()
    return np.abs(A @ x - b).max() / (abs(A) @ np.abs(x) + np.abs(b)).max()


@pytest.mark.parametrize("gamma", [0, 1])
def test_unsteady_stokes_polynomial_reproduction(gamma):
    """eq:govern1unsteady with delta = 0.1 h, rho = 3: the discrete system of
    eq:blockformunsteady reproduces u = curl(x^2 y^2), p = x y with
    f = (rho / delta) u - Lap u + grad p, in standard and stress form."""
    n, p, nq = 3, 2, 5
    rho, delta = 3.0, 0.1 / n
    u = [lambda x, y: 2 * x ** 2 * y, lambda x, y: -2 * x * y ** 2]
    pres = lambda x, y: x * y
    f = [lambda x, y: rho / delta * 2 * x ** 2 * y - 4 * y + y,
         lambda x, y: -rho / delta * 2 * x * y ** 2 + 4 * x + x]
    res = _unsteady_residual(2, n, p, gamma, np.ones(n * n), np.full(n * n, rho), delta, u, pres, f, nq)
    assert res < 1e-13
    # the density term belongs to the velocity rows only: the steady operator
    # with the same data leaves an O(1) residual
    res_s = _unsteady_residual(2, n, p, gamma, np.ones(n * n), None, 0.0, u, pres, f, nq)
    assert res_s > 1e-3


def test_unsteady_stokes_water_gas_planar_interface():
    """Water (rho 1, mu 1) left of x = 1/2, gas (rho 1e-3, mu 2e-4) right, stress
    form, delta = 0.1 h: u = (c y, b(x)) with the stress-form traction
    condition and f = (rho / delta) u, piecewise by phase, is reproduced
    exactly (the density jumps with the phase, element by element)."""
    dim, n, p, nq = 2, 4, 2, 5
    left = np.array([(e % n) < n // 2 for e in range(n * n)])
    mu = np.where(left, 1.0, 2e-4)
    rho = np.where(left, 1.0, 1e-3)
    delta = 0.1 / n
    c, sR = 1.0, 1.0
    sL = 2e-4 * (sR + c) / 1.0 - c
    b_of = lambda x: np.where(x < 0.5, sL * x, sL * 0.5 + sR * (x - 0.5))
    u = [lambda x, y: c * y + 0 * x, lambda x, y: b_of(x) + 0 * y]
    r_of = lambda x: np.where(x < 0.5, 1.0, 1e-3)
    f = [lambda x, y: r_of(x) / delta * c * y, lambda x, y: r_of(x) / delta * b_of(x) + 0 * y]
    res = _unsteady_residual(dim, n, p, 1, mu, rho, delta, u, lambda x, y: 0 * x, f, nq)
    assert res < 1e-12


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1)])
def test_unsteady_density_mass_coarsening(dim, p):
    """The coarsened density mass I^T M_rho I with delta kept equals the term
    assembled directly on the coarse grid (box of densities 1e-3 / 1 aligned
    with the n = 4 grid; the pressure penalty, which depends on h through its
    blending, is switched off on both sides)."""
    n = 8
    delta = 0.1 / n
    lv = stokes.stokes_levels(dim, n, p, mu=mu_box(dim, n, 2e-4), rho=mu_box(dim, n, 1e-3), delta=delta,
                              gamma=1, cp=0.0)
    direct = stokes.stokes_levels(dim, n // 2, p, mu=mu_box(dim, n // 2, 2e-4), rho=mu_box(dim, n // 2, 1e-3),
                                  delta=delta, gamma=1, cp=0.0)[0].A
    D = direct.toarray()
    assert np.abs(lv[1].A.toarray() - D).max() <= 1e-13 * np.abs(D).max()
