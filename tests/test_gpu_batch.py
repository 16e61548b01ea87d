"""Batched serving step: k right-hand sides of one hierarchy solved together
(every matrix block streamed once per batch).  Each right-hand side must match
the oracle exactly as a single solve does (iterations +-1, solution within
1e-9 relative in FP64 mode and 1e-8 with FP32 / BF16 storage), and the batched V-cycle must equal k single V-cycles to rounding
(same arithmetic, summation order aside: 1e-12 relative)."""
import numpy as np
import pytest

from ldg_inputs import rhs_normal
from tests.gpu_common import lib_kwargs, oracle_build

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"),
    dict(id="i3d-p2-sphere-sai1", dim=3, n=8, p=2, smoother="sai", mu=("sphere", 0.3, 1e4)),
    dict(id="p2d-p2-gl-jacobi", dim=2, n=16, p=2, basis="gl_nodal", smoother="jacobi"),
    dict(id="i2d-p1-box-gs", dim=2, n=12, p=1, smoother="gs", mu=("box", 0.0, 1e4)),
]


def _variants(case):
    """(precision, device storage): tiled storage runs the batched products on
    the matrix cores, the others on the vector units."""
    v = [("fp64", "auto"), ("fp32", "auto"), ("fp32", "tiled")]
    if case["smoother"] == "sai":
        v += [("bf16s", "auto"), ("bf16s", "tiled")]
    return v


@pytest.fixture(scope="module", params=[(c, pr, st) for c in CASES for pr, st in _variants(c)],
                ids=lambda cp: f"{cp[0]['id']}-{cp[1]}-{cp[2]}")
def built(request):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, storage = request.param
    print(f"\n[batch {case['id']} {prec} {storage}]", flush=True)
    s = L.Solver(storage=storage, **lib_kwargs(case, prec))
    lv, vc = oracle_build(case)
    yield case, prec, s, lv, vc
    s.close()


@pytest.mark.parametrize("k", [1, 3, 8])
def test_vcycle_batch_equals_single(built, k):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, s, lv, vc = built
    bs = [torch.from_numpy(rhs_normal(s.ndofs, 100 + q)).cuda() for q in range(k)]
    xs = [torch.empty_like(b) for b in bs]
    L.ldgmg_vcycle_batch(s.handle, bs, xs)
    torch.cuda.synchronize()
    for q in range(k):
        x1 = torch.empty_like(bs[q])
        L.ldgmg_vcycle(s.handle, bs[q], x1)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(xs[q] - x1) / torch.linalg.norm(x1))
        assert err <= 1e-12, (q, err)


def test_solve_batch_matches_oracle(built):
    from paper_2412_12506_amd import ldgmg as L
    from oracle import solver as osolver
    case, prec, s, lv, vc = built
    k = 5
    bnp = [rhs_normal(s.ndofs, 200 + q) for q in range(k)]
    bs = [torch.from_numpy(b).cuda() for b in bnp]
    xs = [torch.empty_like(b) for b in bs]
    infos = L.ldgmg_solve_batch(s.handle, bs, xs, 1e-10, 200)
    for q in range(k):
        ref = osolver.solve(lv, vc, bnp[q], "cg")
        assert infos[q]["converged"] and ref.converged
        assert abs(infos[q]["iters"] - ref.iters) <= 1, (q, infos[q]["iters"], ref.iters)
        x = xs[q].cpu().numpy()
        # the solution tolerance of the single solves (tests/test_gpu_parity.py):
        # 1e-9 relative in FP64 mode, 1e-8 with FP32 / BF16 storage
        rel = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
        assert rel <= (1e-9 if prec == "fp64" else 1e-8), (q, prec, rel)
        assert infos[q]["rel_res_true"] <= 2e-10
        # the same right-hand side alone gives the same iterations
        xa = torch.empty_like(bs[q])
        alone = L.ldgmg_solve(s.handle, bs[q], xa, "cg", 1e-10, 200)
        assert alone["iters"] == infos[q]["iters"]
        assert float(torch.linalg.norm(xa - xs[q]) / torch.linalg.norm(xa)) <= 1e-10
