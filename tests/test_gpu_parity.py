"""GPU parity: every V-cycle kernel, the V-cycle and the Krylov solves of the
HIP library (called through the C-ABI) against the CPU oracle, on the same
seeded inputs.

Tolerances (derived from the arithmetic, not tuned):
  * FP64 level operations: |y - y_ref| <= 1e-12 max(|A||x| + |b|): the host
    setups agree to ~1e-15 and a row sums at most a few hundred products
    (block inverses: 20 kappa(A_ii) eps64, since both sides invert A_ii).
  * FP32 block storage (vectors and accumulation stay FP64): the only new
    error is the rounding of each stored entry, |fl(a) - a| <= u32 |a|, so
    |y - y_ref| <= 4 u32 |A||x| (u32 = 2^-24, with slack for the FP64 sums).
  * BF16 SAI storage ("bf16s": FP32 operators, BF16 B): the SAI applies, the
    smoothing steps and the V-cycle are compared with the oracle's own code
    run on its matrices rounded exactly as stored (tests/gpu_common), so the
    FP32 bounds above apply; the solve is compared with the unrounded oracle.
  * smoothing steps: the first-order bound |dx| <= u |S| (|b| + |A||x|) of
    one step (u = unit roundoff of the stored entries; once per colour for
    Gauss-Seidel), with a factor 64 of slack for the FP64 sums.
  * bottom solve and V-cycle: the two setups compute the bottom pseudo-inverse
    independently, so they agree only to ~kappa eps64 (kappa = condition number
    of the bottom operator on its range, computed from the oracle's matrix;
    ~2e9 for the multiphase Stokes case).  Bottom within 20 kappa eps64; V-cycle
    within 1e-10 (FP64) or 1e-5 (FP32 storage) plus 100 kappa eps64.
  * Solves: iteration count within +-1 of the oracle; solution within 1e-9
    relative of the oracle's in FP64 mode and 1e-8 with FP32 / BF16 storage
    (Stokes: modulo the constant pressure); the difference of the two
    solutions has an A-image within the sum of their true residuals; CG true
    FP64 residual <= 2e-10; GMRES (stops on ||V r||) true residual within 10x
    of the oracle's.
Sizes span several workgroups and ragged tails on every level.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from ldg_inputs import rhs_normal, stokes_body_force
from tests.gpu_common import lib_kwargs, oracle_build, smoother_matrix, stored_vcycle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
EPS64 = 2.0 ** -52

CASES = [
    dict(id="p2d-p2-gl-jacobi", dim=2, n=16, p=2, basis="gl_nodal", smoother="jacobi"),
    dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai", sai_level=1),
    dict(id="i3d-p2-sphere-sai1", dim=3, n=8, p=2, smoother="sai", mu=("sphere", 0.3, 1e4)),
    dict(id="i2d-p1-box-gs", dim=2, n=12, p=1, smoother="gs", mu=("box", 0.0, 1e-4)),
    dict(id="i3d-p1-n12-sphere-sai1", dim=3, n=12, p=1, smoother="sai", mu=("sphere", 0.3, 1e4)),
    dict(id="p2d-p3-sai2", dim=2, n=8, p=3, smoother="sai", sai_level=2),
    dict(id="s2d-p2-stress-disc-sai1", dim=2, n=8, p=2, system="stokes", gamma=1,
         smoother="sai", mu=("disc", 0.25, 1e3), krylov="gmres"),
    dict(id="s2d-p1-std-gs", dim=2, n=8, p=1, system="stokes", gamma=0, smoother="gs",
         order="OO", krylov="gmres"),
    # unsteady stress-form Stokes (eq:blockformunsteady): a gas bubble (rho 1e-3, mu 2e-4) in
    # water, delta = 0.1 h
    dict(id="s2d-p2-unsteady-gas-in-water", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("box", 0.0, 2e-4), rho=("box", 0.0, 1e-3), delta=0.1 / 8, krylov="gmres"),
]


def _dev():
    return torch.device("cuda:0")


def _variants(case):
    """(precision, device storage) pairs: every kernel instantiation the case reaches."""
    v = [("fp64", "auto"), ("fp32", "expanded"), ("fp32", "pooled"), ("fp32", "tiled")]
    if case["smoother"] == "sai":
        v += [("bf16s", "expanded"), ("bf16s", "pooled"), ("bf16s", "tiled")]
    return v


_ORACLE = {}


def _oracle(case):
    if case["id"] not in _ORACLE:
        _ORACLE.clear()                    # cases come in order: keep one
        _ORACLE[case["id"]] = oracle_build(case)
    return _ORACLE[case["id"]]


@pytest.fixture(scope="module",
                params=[(c, pr, st) for c in CASES for pr, st in _variants(c)],
                ids=lambda cp: f"{cp[0]['id']}-{cp[1]}-{cp[2]}")
def built(request):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, storage = request.param
    print(f"\n[case {case['id']} {prec} {storage}]", flush=True)
    s = L.Solver(storage=storage, **lib_kwargs(case, prec))
    lv, vc = _oracle(case)
    yield case, prec, s, lv, vc
    s.close()


def _kappa_bottom(vc):
    """Condition number of the bottom operator on its range (oracle side): the
    two independent pseudo-inverses can differ by ~kappa * eps."""
    lam = np.abs(np.linalg.eigvalsh(vc.levels[-1].A.toarray()))
    nz = lam[lam > 1e-12 * lam.max()]
    return lam.max() / nz.min()


def _t(a, prec=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(_dev())


def _round(a, prec):
    return a


def _tol_op(prec, A):
    return 1e-12 if prec == "fp64" else 4 * U32


def test_level_operations(built):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, s, lv, vc = built
    vs = stored_vcycle(vc, prec) if prec == "bf16s" else vc    # references for S and smoothing
    rng = np.random.default_rng(1234)
    nl = len(lv)
    assert s.nlevels == nl
    for l in range(nl):
        A = vc.levels[l].A
        N = A.shape[0]
        x = _round(rng.standard_normal(N), prec)
        b = _round(rng.standard_normal(N), prec)
        xt, bt = _t(x, prec), _t(b, prec)
        out = torch.empty_like(xt)
        absAx = abs(A) @ np.abs(x)
        tol = _tol_op(prec, A)
        # residual and operator apply (a1)
        L.ldgmg_level_op(s.handle, l, "residual", xt, bt, out)
        torch.cuda.synchronize()
        ref = b - A @ x
        err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(absAx + np.abs(b))
        assert err <= tol, (l, "residual", err, tol)
        if l == nl - 1:
            L.ldgmg_level_op(s.handle, l, "bottom", bt, None, out)
            torch.cuda.synchronize()
            ref = vc.levels[l].pinv @ b
            err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(vc.levels[l].pinv) @ np.abs(b))
            assert err <= max(1e-11, 20 * _kappa_bottom(vc) * EPS64), (l, "bottom", err)
            continue
        # smoother matrix forward / transposed (a2, a3).  Block inverses are
        # computed independently by both setups: they agree to ~kappa(A_ii) eps64.
        S = smoother_matrix(vs, l)
        stol = _tol_op(prec, S)
        if vc.levels[l].sm.kind != "sai":
            kd = max(np.linalg.cond(D) for D in np.linalg.inv(vc.levels[l].sm.Dinv))
            stol = max(stol, 20 * kd * EPS64)
        for op, M in (("apply_s", S), ("apply_st", S.T.tocsr())):
            L.ldgmg_level_op(s.handle, l, op, xt, None, out)
            torch.cuda.synchronize()
            ref = M @ x
            err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(abs(M) @ np.abs(x))
            assert err <= stol, (l, op, err, stol)
        # smoothing steps (a2 / a3 / a4).  First-order bound for stored-entry
        # rounding u: |dx| <= u |S| (|b| + |A||x|) per step (per colour for GS)
        ncol = vc.levels[l].sm.colours.max() + 1 if vc.levels[l].sm.kind == "gs" else 1
        mag = abs(S) @ (np.abs(b) + absAx) + np.abs(x)
        u = 1e-14 if prec == "fp64" else U32
        if vc.levels[l].sm.kind != "sai":
            u = max(u, kd * EPS64)
        for op, fwd in (("smooth_fwd", True), ("smooth_rev", False)):
            L.ldgmg_level_op(s.handle, l, op, xt, bt, out)
            torch.cuda.synchronize()
            ref = vs.smooth(vs.levels[l], x, b, fwd)
            err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(mag)
            assert err <= 4 * ncol * u * 16, (l, op, err)
        # transfers (a5, a6)
        I = vc.levels[l].I
        Nc = I.shape[1]
        rc = torch.empty(Nc, dtype=torch.float64, device=_dev())
        L.ldgmg_level_op(s.handle, l, "restrict", xt, None, rc)
        torch.cuda.synchronize()
        ref = I.T @ x
        err = np.max(np.abs(rc.cpu().numpy() - ref)) / np.max(abs(I.T) @ np.abs(x))
        assert err <= 1e-13, (l, "restrict", err)
        xc = _round(rng.standard_normal(Nc), prec)
        o2 = xt.clone()
        L.ldgmg_level_op(s.handle, l, "prolong_add", _t(xc, prec), None, o2)
        torch.cuda.synchronize()
        ref = x + I @ xc
        err = np.max(np.abs(o2.cpu().numpy() - ref)) / np.max(np.abs(x) + abs(I) @ np.abs(xc))
        assert err <= 1e-13, (l, "prolong", err)
    # FP64 Krylov operator on the fine level (a10)
    A = vc.levels[0].A
    x = rng.standard_normal(A.shape[0])
    xt = torch.from_numpy(x).to(_dev())
    out = torch.empty_like(xt)
    L.ldgmg_level_op(s.handle, 0, "apply_a64", xt, None, out)
    torch.cuda.synchronize()
    err = np.max(np.abs(out.cpu().numpy() - A @ x)) / np.max(abs(A) @ np.abs(x))
    assert err <= 1e-12


def _rhs(case, N, seed):
    if case.get("system") == "stokes":
        return stokes_body_force(case["dim"], case["n"], (case["p"] + 1) ** case["dim"], seed)
    return rhs_normal(N, seed)


def test_vcycle(built):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, s, lv, vc = built
    N = lv[0].A.shape[0]
    b = _rhs(case, N, 7)
    bt = torch.from_numpy(b).to(_dev())
    xt = torch.empty_like(bt)
    L.ldgmg_vcycle(s.handle, bt, xt)
    torch.cuda.synchronize()
    ref = (stored_vcycle(vc, prec) if prec == "bf16s" else vc).apply(b)
    err = np.linalg.norm(xt.cpu().numpy() - ref) / np.linalg.norm(ref)
    tol = (1e-10 if prec == "fp64" else 1e-5) + 100 * _kappa_bottom(vc) * EPS64
    assert err <= tol, (err, tol)
    # a second call on the same handle gives the same result (no stale state)
    xt2 = torch.empty_like(bt)
    L.ldgmg_vcycle(s.handle, bt, xt2)
    torch.cuda.synchronize()
    assert torch.equal(xt, xt2)


def test_solve(built):
    from paper_2412_12506_amd import ldgmg as L
    from oracle import solver as osolver
    case, prec, s, lv, vc = built
    N = lv[0].A.shape[0]
    b = _rhs(case, N, 11)
    krylov = case.get("krylov", "cg")
    ref = osolver.solve(lv, vc, b, krylov)
    bt = torch.from_numpy(b).to(_dev())
    xt = torch.empty_like(bt)
    info = L.ldgmg_solve(s.handle, bt, xt, krylov, 1e-10, 200)
    assert info["converged"] and ref.converged
    assert abs(info["iters"] - ref.iters) <= 1, (info["iters"], ref.iters)
    x = xt.cpu().numpy()
    if case.get("system") == "stokes":     # compare modulo the constant-pressure kernel
        from oracle import stokes
        k = stokes.pressure_kernel(lv[0])
        proj = lambda v: v - (v @ k) / (k @ k) * k
        x, xr = proj(x), proj(ref.x)
    else:
        xr = ref.x
    # x - x_ref = A^-1 (r_ref - r): its A-image is bounded by the two true
    # residuals, whatever the conditioning
    d = xt.cpu().numpy() - ref.x
    ares = np.linalg.norm(lv[0].A @ d) / np.linalg.norm(b)
    rel = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    print(f"\n[solve {case['id']} {prec}] iters gpu {info['iters']} oracle {ref.iters}; solution rel diff "
          f"{rel:.2e}; A-residual of the difference {ares:.2e}", flush=True)
    assert ares <= 1.01 * (info["rel_res_true"] + ref.rel_res_true) + 1e-12
    # the stated solution tolerance: 1e-9 relative in FP64 mode; with FP32 / BF16
    # storage the V-cycle is another (fixed) preconditioner, so the two Krylov
    # iterates reach the 1e-10 residual along different paths: 1e-8
    assert rel <= (1e-9 if prec == "fp64" else 1e-8), rel
    if krylov == "cg":     # CG stops on the FP64 residual itself
        assert info["rel_res_true"] <= 2e-10
    else:                  # left-preconditioned GMRES stops on ||V r||: compare with the oracle
        assert info["rel_res_krylov"] <= 1e-10
        assert info["rel_res_true"] <= 10 * ref.rel_res_true + 1e-12
    if prec == "fp64":
        assert abs(info["eta"] - ref.eta) <= 0.05 * ref.eta


@pytest.mark.parametrize("dim,n,p,basis,nq", [(2, 16, 2, "gl_nodal", 6), (3, 6, 3, "legendre", 5),
                                              (2, 9, 1, "legendre", 4)])
def test_rhs_volume(dim, n, p, basis, nq):
    """ldgmg_rhs_volume (the int f v part of b_h, Section 2.1) against the
    oracle's volume_load on the same sampled source: the manufactured source
    of the 2D workload, or seeded N(0,1) point values.  Both sides sum nq^d
    weighted products per entry in FP64: |b - b_ref| <= 1e-13 max |b_ref|."""
    from paper_2412_12506_amd import ldgmg as L
    from ldg_inputs import sample_on_elements, mms_source_2d
    from oracle import ldg
    if dim == 2 and basis == "gl_nodal":
        fq = sample_on_elements(dim, n, nq, mms_source_2d)
    else:
        fq = np.random.default_rng(5).standard_normal((n ** dim, nq ** dim))
    s = L.Solver(dim=dim, n=n, p=p, basis=basis, smoother="jacobi", precision="fp64")
    try:
        bt = torch.zeros(s.ndofs, dtype=torch.float64, device=_dev())
        L.ldgmg_rhs_volume(s.handle, fq, nq, bt)
        torch.cuda.synchronize()
        em = ldg.ElementMatrices(dim, p, 1.0 / n, basis)
        ref = ldg.volume_load(em, fq, nq)
        err = np.max(np.abs(bt.cpu().numpy() - ref)) / np.max(np.abs(ref))
        print(f"\n[rhs_volume {dim}D n={n} p={p} {basis}] max error / max |b| {err:.2e}", flush=True)
        assert err <= 1e-13
    finally:
        s.close()
