"""FP32 products on the matrix cores (ldgmg_fp32_products) against the oracle.

With the mode on, every tiled operator and smoother apply of the V-cycle rounds
its input to FP32 and multiplies and sums in FP32; the result is combined with
the FP64 vectors in FP64.  Tolerances, from that arithmetic:
  * level operations (operator and smoother applies, smoothing steps, whose
    residual is written in FP32 where the level is tiled with 16 | bs), entry
    by entry: a row of n stored terms summed in FP32
    from an FP32-rounded input is within (n + 3) u32 (|M||x|)_i of the FP64
    product of the stored matrix (u32 = 2^-24: n - 1 sums, the products, the
    input rounding, and one unit for a stored entry that the two independent
    setups round to neighbouring FP32 values); in a smoothing step whose BF16
    B reads the FP32 residual (32 | bs) the residual is split exactly into
    three BF16 parts, each product exact, so n becomes 3n for that apply;
  * V-cycle: against the oracle's V-cycle with FP32 products
    (tests/gpu_common.fp32_products_vcycle; the same roundings, another
    summation order) within 1e-4 relative: each apply agrees to n u32 <= 3e-5
    relative per entry for n <= 448 terms;
  * solves: CG converges to a true FP64 residual <= 2e-10; its iteration count
    is within +-1 of the oracle's CG preconditioned by that FP32-product
    V-cycle, and on Poisson also within +-1 of the plain FP64 oracle's; the
    solution differs from the FP64 oracle's by a vector whose residual is
    within the two solves' residuals (<= 4e-10 ||b||);
  * a level that is not tiled is not affected: with pooled storage the results
    are bitwise those without the mode.
"""
import numpy as np
import pytest

from ldg_inputs import rhs_normal
from tests.gpu_common import (fp32_products_vcycle, lib_kwargs, oracle_build, round_bf16, round_fp32,
                              smoother_matrix)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24

CASES = [
    (dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"), "fp32", True),
    (dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"), "bf16s", True),
    (dict(id="p2d-p2-sai1", dim=2, n=32, p=2, smoother="sai"), "fp32", True),
    (dict(id="i3d-p2-sphere-sai1", dim=3, n=8, p=2, smoother="sai", mu=("sphere", 0.3, 1e4)), "fp32", False),
]

_ORACLE = {}


def _oracle(case):
    if case["id"] not in _ORACLE:
        _ORACLE.clear()
        _ORACLE[case["id"]] = oracle_build(case)
    return _ORACLE[case["id"]]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]['id']}-{c[1]}")
def built(request):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, poisson = request.param
    print(f"\n[fp32 products {case['id']} {prec}]", flush=True)
    s = L.Solver(storage="tiled", fp32_products=True, **lib_kwargs(case, prec))
    lv, vc = _oracle(case)
    yield case, prec, poisson, s, lv, vc
    s.close()


def _split_terms(prec, bs):
    """Summed terms per stored entry in a smoothing step's B apply: 3 where a
    BF16 B meets the FP32 residual on the BF16 matrix cores (the residual split
    exactly into three BF16 parts; 32 | bs), else 1."""
    return 3 if prec == "bf16s" and bs % 32 == 0 else 1


def _check_rows(y, ref, M, x, what):
    """Entry-wise FP32-product bound; M is the stored matrix (FP64 values)."""
    M = M.tocsr()
    n = np.diff(M.indptr)
    bound = (n + 3) * U32 * (abs(M) @ np.abs(x))
    err = np.abs(y - ref)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    assert worst <= 1.0, (what, worst)
    return worst


def test_level_operations(built):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, poisson, s, lv, vc = built
    rng = np.random.default_rng(77)
    for l in range(len(lv) - 1):
        st = L.ldgmg_level_storage(s.handle, l)
        assert st["tiled_A"] and st["tiled_S"], (l, st)
        A = round_fp32(vc.levels[l].A)
        S = smoother_matrix(vc, l)
        S = round_bf16(S) if prec == "bf16s" else round_fp32(S)
        N = A.shape[0]
        x = rng.standard_normal(N)
        b = rng.standard_normal(N)
        xt, bt = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
        out = torch.empty_like(xt)
        L.ldgmg_level_op(s.handle, l, "residual", xt, bt, out)
        torch.cuda.synchronize()
        _check_rows(b - out.cpu().numpy(), A @ x, A, x, (l, "residual"))
        for op, M in (("apply_a", A), ("apply_s", S), ("apply_st", S.T)):
            L.ldgmg_level_op(s.handle, l, op, xt, None, out)
            torch.cuda.synchronize()
            w = _check_rows(out.cpu().numpy(), M @ x, M, x, (l, op))
            print(f"  level {l} {op}: worst error / bound {w:.3f}", flush=True)
        # smoothing steps x + B (b - A x): the residual is rounded to FP32 once
        # (written in FP32 where the level keeps an FP32 residual), then B's
        # FP32 products; entry-wise first-order bound from both products
        nA, nS = np.diff(A.tocsr().indptr), np.diff(S.tocsr().indptr)
        absAx = abs(A) @ np.abs(x)
        ks = _split_terms(prec, s.bs)
        for op, M, n in (("smooth_fwd", S, ks * nS), ("smooth_rev", S.T.tocsr(), ks * np.diff(S.T.tocsr().indptr))):
            L.ldgmg_level_op(s.handle, l, op, xt, bt, out)
            torch.cuda.synchronize()
            ref = x + M @ (b - A @ x)
            bound = (n + 3) * U32 * (abs(M) @ (np.abs(b) + absAx)) + abs(M) @ ((nA + 3) * U32 * absAx)
            err = np.abs(out.cpu().numpy() - ref)
            worst = float(np.max(err / np.maximum(bound, 1e-300)))
            print(f"  level {l} {op}: worst error / bound {worst:.3f}", flush=True)
            assert worst <= 1.0, (l, op, worst)


def test_vcycle(built):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, poisson, s, lv, vc = built
    b = rhs_normal(lv[0].A.shape[0], 5)
    bt = torch.from_numpy(b).cuda()
    xt = torch.empty_like(bt)
    L.ldgmg_vcycle(s.handle, bt, xt)
    torch.cuda.synchronize()
    ref = fp32_products_vcycle(vc, prec).apply(b)
    err = np.linalg.norm(xt.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  V-cycle relative difference {err:.2e}", flush=True)
    assert err <= 1e-4
    xt2 = torch.empty_like(bt)
    L.ldgmg_vcycle(s.handle, bt, xt2)
    torch.cuda.synchronize()
    assert torch.equal(xt, xt2)            # deterministic


def test_solve(built):
    from paper_2412_12506_amd import ldgmg as L
    from oracle import krylov, solver as osolver
    case, prec, poisson, s, lv, vc = built
    b = rhs_normal(lv[0].A.shape[0], 11)
    bt = torch.from_numpy(b).cuda()
    xt = torch.empty_like(bt)
    info = L.ldgmg_solve(s.handle, bt, xt, "cg", 1e-10, 200)
    torch.cuda.synchronize()
    vm = fp32_products_vcycle(vc, prec)
    model = krylov.pcg(lv[0].A.tocsr(), b, vm.apply)
    ref = osolver.solve(lv, vc, b, "cg")
    print(f"  iterations: GPU {info['iters']}, FP32-product model {model.iters}, FP64 oracle {ref.iters}",
          flush=True)
    assert info["converged"] and info["rel_res_true"] <= 2e-10
    assert abs(info["iters"] - model.iters) <= 1
    if poisson:
        assert abs(info["iters"] - ref.iters) <= 1
    # two CG runs converged to 1e-10 from V-cycles that differ in their FP32
    # roundings: their solutions differ by A^-1 of two residuals each <= 2e-10 ||b||
    d = xt.cpu().numpy() - ref.x
    res = np.linalg.norm(lv[0].A @ d) / np.linalg.norm(b)
    print(f"  solution difference {np.linalg.norm(d) / np.linalg.norm(ref.x):.2e}, A-residual of it {res:.2e}",
          flush=True)
    assert res <= 4e-10


def test_untiled_levels_unaffected():
    from paper_2412_12506_amd import ldgmg as L
    case = dict(dim=3, n=6, p=3, smoother="sai")
    a = L.Solver(storage="pooled", fp32_products=True, **lib_kwargs(case, "fp32"))
    c = L.Solver(storage="pooled", **lib_kwargs(case, "fp32"))
    try:
        b = torch.from_numpy(rhs_normal(a.ndofs, 3)).cuda()
        xa, xc = torch.empty_like(b), torch.empty_like(b)
        L.ldgmg_vcycle(a.handle, b, xa)
        L.ldgmg_vcycle(c.handle, b, xc)
        torch.cuda.synchronize()
        assert torch.equal(xa, xc)
    finally:
        a.close()
        c.close()


def test_jacobi_block_inverse_apply():
    """Block Jacobi on tiled storage: the first pre-smoothing step applies the
    block inverses (x = w D^-1 b) on the matrix cores with FP32 products; that
    apply meets the entry-wise bound against the stored D^-1, and CG still
    converges to a true FP64 residual <= 2e-10 within +-1 iteration of FP64
    products on the same handle."""
    from paper_2412_12506_amd import ldgmg as L
    case = dict(id="p2d-p2-gl-jacobi", dim=2, n=16, p=2, basis="gl_nodal", smoother="jacobi")
    lv, vc = oracle_build(case)
    s = L.Solver(storage="tiled", **lib_kwargs(case, "fp32"))
    try:
        b = torch.from_numpy(rhs_normal(s.ndofs, 17)).cuda()
        x = torch.empty_like(b)
        ref = L.ldgmg_solve(s.handle, b, x, "cg", 1e-10, 200)
        L.ldgmg_fp32_products(s.handle, True)
        assert L.ldgmg_level_storage(s.handle, 0)["tiled_S"]
        rng = np.random.default_rng(8)
        D = round_fp32(smoother_matrix(vc, 0))
        xn = rng.standard_normal(D.shape[0])
        out = torch.empty(D.shape[0], dtype=torch.float64, device="cuda")
        L.ldgmg_level_op(s.handle, 0, "apply_s", torch.from_numpy(xn).cuda(), None, out)
        torch.cuda.synchronize()
        _check_rows(out.cpu().numpy(), D @ xn, D, xn, "jacobi apply_s")
        info = L.ldgmg_solve(s.handle, b, x, "cg", 1e-10, 200)
        torch.cuda.synchronize()
        assert info["converged"] and info["rel_res_true"] <= 2e-10
        assert abs(info["iters"] - ref["iters"]) <= 1, (info["iters"], ref["iters"])
    finally:
        s.close()


def test_batch_matches_single():
    """The batched serving step with FP32 products: each right-hand side
    converges to a true residual <= 2e-10 within +-1 iteration of its single
    solve, and the two solutions agree to 1e-8 (two converged CG runs whose
    FP32 V-cycle inputs differ in their last bits)."""
    from paper_2412_12506_amd import ldgmg as L
    case = dict(dim=3, n=6, p=3, smoother="sai")
    s = L.Solver(storage="tiled", fp32_products=True, **lib_kwargs(case, "bf16s"))
    try:
        bs = [torch.from_numpy(rhs_normal(s.ndofs, 40 + q)).cuda() for q in range(3)]
        xs = [torch.empty_like(b) for b in bs]
        infos = L.ldgmg_solve_batch(s.handle, bs, xs, 1e-10, 200)
        torch.cuda.synchronize()
        for q in range(3):
            x1 = torch.empty_like(bs[q])
            one = L.ldgmg_solve(s.handle, bs[q], x1, "cg", 1e-10, 200)
            torch.cuda.synchronize()
            assert infos[q]["converged"] and abs(infos[q]["iters"] - one["iters"]) <= 1
            assert infos[q]["rel_res_true"] <= 2e-10
            rel = float(torch.linalg.norm(xs[q] - x1) / torch.linalg.norm(x1))
            assert rel <= 1e-8, (q, rel)
    finally:
        s.close()


def test_headline_path_fine_level_n12():
    """The benchmark's path on a grid whose fine-level launches span 27
    workgroups (3D Q_3, 12^3 = 1,728 block rows, 64 rows per workgroup): BF16
    SAI storage, tiled storage, FP32 products, the FP32 smoothing residual
    (16 | bs, A and B tiled), the 4-step k layout of B and B^T and the XCD
    tile order (24 workgroups remapped, a tail of 3).  Every fine-level apply
    and both smoothing steps against the oracle's fine operator and balanced
    SAI_1 matrix (rounded as stored), entry by entry within the bounds of
    test_level_operations."""
    from paper_2412_12506_amd import ldgmg as L
    from oracle import ldg, smoothers as sm
    dim, n, p = 3, 12, 3
    A64 = ldg.assemble_scalar(dim, n, p).A
    bs = (p + 1) ** dim
    B64, _ = sm.sai(A64, bs, 1, sm.balance_scalar(A64, bs))
    A, S = round_fp32(A64), round_bf16(B64)
    s = L.Solver(dim=dim, n=n, p=p, smoother="sai", precision="bf16s", storage="tiled", fp32_products=True)
    try:
        st = L.ldgmg_level_storage(s.handle, 0)
        assert st["tiled_A"] and st["tiled_S"], st
        rng = np.random.default_rng(2024)
        N = A.shape[0]
        x, b = rng.standard_normal(N), rng.standard_normal(N)
        xt, bt = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
        out = torch.empty_like(xt)
        L.ldgmg_level_op(s.handle, 0, "residual", xt, bt, out)
        torch.cuda.synchronize()
        _check_rows(b - out.cpu().numpy(), A @ x, A, x, "residual n12")
        for op, M in (("apply_a", A), ("apply_s", S), ("apply_st", S.T)):
            L.ldgmg_level_op(s.handle, 0, op, xt, None, out)
            torch.cuda.synchronize()
            w = _check_rows(out.cpu().numpy(), M @ x, M, x, (op, "n12"))
            print(f"  12^3 {op}: worst error / bound {w:.3f}", flush=True)
        nA = np.diff(A.tocsr().indptr)
        absAx = abs(A) @ np.abs(x)
        for op, M in (("smooth_fwd", S.tocsr()), ("smooth_rev", S.T.tocsr())):
            L.ldgmg_level_op(s.handle, 0, op, xt, bt, out)
            torch.cuda.synchronize()
            nM = _split_terms("bf16s", bs) * np.diff(M.indptr)
            ref = x + M @ (b - A @ x)
            bound = (nM + 3) * U32 * (abs(M) @ (np.abs(b) + absAx)) + abs(M) @ ((nA + 3) * U32 * absAx)
            worst = float(np.max(np.abs(out.cpu().numpy() - ref) / np.maximum(bound, 1e-300)))
            print(f"  12^3 {op}: worst error / bound {worst:.3f}", flush=True)
            assert worst <= 1.0, (op, worst)
    finally:
        s.close()


def _dense_round(B, how):
    return (round_bf16 if how == "bf16" else round_fp32)(B).toarray()


@pytest.mark.parametrize("n", [32, 64])
def test_headline_path_fine_level_sampled(n):
    """The benchmark's launch configurations at sizes the oracle cannot
    assemble whole, 3D Q_3 with BF16 SAI, tiled storage and FP32 products:
    32^3 (32,768 block rows, over 2,048 tiles: the unsplit tiled launches, one
    tile per wavefront) and 64^3 (262,144 block rows: two tiles per wavefront
    for the FP32 A, the benchmark's own grid), both in the XCD tile order with
    padded tiles.  Sampled rows
    (corners, edges, faces, random) of the residual, apply_s, apply_st and
    both smoothing steps (whose residual is the FP32-x, FP32-out launch)
    against the oracle's local rows and local least-squares SAI columns,
    rounded as stored, within the bounds of test_level_operations; then a CG
    solve with FP32 products takes the iterations of FP64 products (+-1) to a
    true FP64 residual <= 2e-10."""
    from paper_2412_12506_amd import ldgmg as L
    from oracle.local import LocalOperator
    dim, p = 3, 3
    bs = (p + 1) ** dim
    lo = LocalOperator(dim, n, p)
    s = L.Solver(dim=dim, n=n, p=p, smoother="sai", precision="bf16s", storage="tiled", fp32_products=True)
    try:
        st = L.ldgmg_level_storage(s.handle, 0)
        assert st["tiled_A"] and st["tiled_S"], st
        ne = lo.grid.ne
        rng = np.random.default_rng(2000 + n)
        rows = sorted({0, n - 1, n * n - 1, ne - 1, n // 2, n * n // 2 + 3, ne // 2 + n // 2 + 1,
                       *rng.choice(ne, 6, replace=False).tolist()})
        N = ne * bs
        x, b = rng.standard_normal(N), rng.standard_normal(N)
        xv, bv = x.reshape(-1, bs), b.reshape(-1, bs)
        xt, bt = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
        outs = {}
        for op in ("residual", "apply_s", "apply_st", "smooth_fwd", "smooth_rev"):
            out = torch.empty_like(xt)
            L.ldgmg_level_op(s.handle, 0, op, xt, bt if op in ("residual", "smooth_fwd", "smooth_rev") else None, out)
            torch.cuda.synchronize()
            outs[op] = out.cpu().numpy().reshape(-1, bs)
        arows, acache, scols = {}, {}, {}

        def arow(K):                        # {J: A_KJ}, FP32 as stored
            if K not in arows:
                arows[K] = {J: _dense_round(B, "fp32") for J, B in lo.row(K).items()}
            return arows[K]

        def ax(K):                          # (A x)_K, (|A||x|)_K, terms per row
            if K not in acache:
                blocks = arow(K)
                acache[K] = (sum(B @ xv[J] for J, B in blocks.items()),
                             sum(np.abs(B) @ np.abs(xv[J]) for J, B in blocks.items()), bs * len(blocks))
            return acache[K]

        def scol(J):                        # {I: S_IJ}, BF16 as stored
            if J not in scols:
                scols[J] = {I: _dense_round(B, "bf16") for I, B in lo.sai_column(J, 1).items()}
            return scols[J]

        worst = {}
        for K in rows:
            AxK, absK, nA = ax(K)
            err = np.abs((bv[K] - outs["residual"][K]) - AxK)
            w = float(np.max(err / np.maximum((nA + 3) * U32 * absK, 1e-300)))
            worst["residual"] = max(worst.get("residual", 0.0), w)
            assert w <= 1.0, ("residual", K, w)
            srow = {J: scol(J)[K] for J in arow(K)}          # row K of S (the pattern of A is symmetric)
            ref_s = sum(B @ xv[J] for J, B in srow.items())
            mag_s = sum(np.abs(B) @ np.abs(xv[J]) for J, B in srow.items())
            nS = bs * len(srow)
            w = float(np.max(np.abs(outs["apply_s"][K] - ref_s) / np.maximum((nS + 3) * U32 * mag_s, 1e-300)))
            worst["apply_s"] = max(worst.get("apply_s", 0.0), w)
            assert w <= 1.0, ("apply_s", K, w)
            stcol = scol(K)                                   # row K of S^T = column K of S
            ref_t = sum(B.T @ xv[I] for I, B in stcol.items())
            mag_t = sum(np.abs(B.T) @ np.abs(xv[I]) for I, B in stcol.items())
            nT = bs * len(stcol)
            w = float(np.max(np.abs(outs["apply_st"][K] - ref_t) / np.maximum((nT + 3) * U32 * mag_t, 1e-300)))
            worst["apply_st"] = max(worst.get("apply_st", 0.0), w)
            assert w <= 1.0, ("apply_st", K, w)
            for op, Mrow in (("smooth_fwd", srow), ("smooth_rev", {I: B.T for I, B in stcol.items()})):
                ref = xv[K].copy()
                bound = np.zeros(bs)
                nM = _split_terms("bf16s", bs) * bs * len(Mrow)
                for J, B in Mrow.items():
                    AxJ, absJ, nAJ = ax(J)
                    ref += B @ (bv[J] - AxJ)
                    bound += (nM + 3) * U32 * (np.abs(B) @ (np.abs(bv[J]) + absJ))
                    bound += np.abs(B) @ ((nAJ + 3) * U32 * absJ)
                w = float(np.max(np.abs(outs[op][K] - ref) / np.maximum(bound, 1e-300)))
                worst[op] = max(worst.get(op, 0.0), w)
                assert w <= 1.0, (op, K, w)
        print(f"  {n}^3 sampled rows " + ", ".join(f"{k} {v:.3f}" for k, v in worst.items()), flush=True)
        b = torch.from_numpy(rhs_normal(N, 7)).cuda()
        its = {}
        for fp32p in (False, True):
            L.ldgmg_fp32_products(s.handle, fp32p)
            xs = torch.empty_like(b)
            info = L.ldgmg_solve(s.handle, b, xs, "cg", 1e-10, 100)
            torch.cuda.synchronize()
            assert info["converged"] and info["rel_res_true"] <= 2e-10, (fp32p, info)
            its[fp32p] = info["iters"]
        assert abs(its[True] - its[False]) <= 1, its
        print(f"  {n}^3 CG iterations: FP64 products {its[False]}, FP32 products {its[True]}", flush=True)
    finally:
        s.close()


def test_stokes3d_q1_bs32_bf16_core_smoothing():
    """Block size 32 (3D stress-form Stokes, Q_1: 4 x 8 unknowns per element),
    the other block size with 32 | bs: BF16 SAI, tiled storage, FP32 products.
    Its smoothing steps read the FP32 residual into the BF16-core apply with a
    single 32-wide k group; both steps entry by entry against the oracle's
    matrices (rounded as stored) within the bounds of test_level_operations,
    and the V-cycle within 1e-4 of the FP32-product emulation."""
    from paper_2412_12506_amd import ldgmg as L
    case = dict(id="s3d-p1-stress-sai1", dim=3, n=4, p=1, system="stokes", gamma=1, smoother="sai")
    lv, vc = oracle_build(case)
    s = L.Solver(storage="tiled", fp32_products=True, **lib_kwargs(case, "bf16s"))
    try:
        assert s.bs == 32, s.bs
        st = L.ldgmg_level_storage(s.handle, 0)
        assert st["tiled_A"] and st["tiled_S"], st
        A = round_fp32(vc.levels[0].A)
        S = round_bf16(smoother_matrix(vc, 0))
        rng = np.random.default_rng(32)
        N = A.shape[0]
        x, b = rng.standard_normal(N), rng.standard_normal(N)
        xt, bt = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
        out = torch.empty_like(xt)
        nA = np.diff(A.tocsr().indptr)
        absAx = abs(A) @ np.abs(x)
        ks = _split_terms("bf16s", s.bs)
        assert ks == 3
        for op, M in (("smooth_fwd", S.tocsr()), ("smooth_rev", S.T.tocsr())):
            L.ldgmg_level_op(s.handle, 0, op, xt, bt, out)
            torch.cuda.synchronize()
            n = ks * np.diff(M.indptr)
            ref = x + M @ (b - A @ x)
            bound = (n + 3) * U32 * (abs(M) @ (np.abs(b) + absAx)) + abs(M) @ ((nA + 3) * U32 * absAx)
            worst = float(np.max(np.abs(out.cpu().numpy() - ref) / np.maximum(bound, 1e-300)))
            print(f"  bs=32 {op}: worst error / bound {worst:.3f}", flush=True)
            assert worst <= 1.0, (op, worst)
        bv = rhs_normal(N, 9)
        bvt = torch.from_numpy(bv).cuda()
        xv = torch.empty_like(bvt)
        L.ldgmg_vcycle(s.handle, bvt, xv)
        torch.cuda.synchronize()
        ref = fp32_products_vcycle(vc, "bf16s").apply(bv)
        err = np.linalg.norm(xv.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"  bs=32 V-cycle relative difference {err:.2e}", flush=True)
        assert err <= 1e-4
    finally:
        s.close()
