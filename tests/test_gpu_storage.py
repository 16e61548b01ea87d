"""Pooled and tiled against expanded device storage (GPU).

Both storages hold the same block values (the setup builds every matrix as a
pool of distinct blocks; pooled storage keeps the pool and a block id per slot,
expanded storage copies each slot's block), and the kernels do the same
arithmetic in the same order, so every result must be bitwise equal: level
operations, the V-cycle, single and batched solves.  The bytes ldgmg_upload
allocates equal ldgmg_upload_bytes exactly in every storage.  Tiled storage
applies the same blocks on the FP64 matrix cores: its products and sums are
FP64 in another order, so it agrees with pooled storage to a few FP64 units
per row sum (1e-13 of |M||x|) and gives the same CG iterations.
"""
import numpy as np
import pytest

from ldg_inputs import rhs_normal, stokes_body_force
from tests.gpu_common import lib_kwargs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    (dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"), "fp32"),
    (dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"), "bf16s"),
    (dict(id="p3d-p2-sai1-fp64", dim=3, n=6, p=2, smoother="sai"), "fp64"),
    (dict(id="i3d-p2-sphere-sai1", dim=3, n=8, p=2, smoother="sai", mu=("sphere", 0.3, 1e4)), "fp32"),
    (dict(id="p2d-p2-gl-jacobi", dim=2, n=16, p=2, basis="gl_nodal", smoother="jacobi"), "fp32"),
    (dict(id="i2d-p1-box-gs", dim=2, n=12, p=1, smoother="gs", mu=("box", 0.0, 1e4)), "fp32"),
    (dict(id="s2d-p2-stress-disc-sai1", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
          mu=("disc", 0.25, 1e3), krylov="gmres"), "fp32"),
]


@pytest.fixture(scope="module", params=CASES, ids=lambda cp: f"{cp[0]['id']}-{cp[1]}")
def pair(request):
    from paper_2412_12506_amd import ldgmg as L
    case, prec = request.param
    print(f"\n[storage {case['id']} {prec}]", flush=True)
    out = {}
    for st in ("expanded", "pooled", "tiled"):
        s = L.Solver(storage=st, **lib_kwargs(case, prec))
        torch.cuda.synchronize()
        out[st] = s
    yield case, prec, out
    for s in out.values():
        s.close()


def test_upload_bytes_exact(pair):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, sv = pair
    for st, s in sv.items():
        assert s.device_bytes == s.upload_bytes, (st, s.device_bytes, s.upload_bytes)
    assert sv["pooled"].upload_bytes < sv["expanded"].upload_bytes
    st = L.ldgmg_level_storage(sv["tiled"].handle, 0)
    assert st["tiled_A"] and st["pool_A"] > 0


def _rhs(case, s, seed):
    if case.get("system") == "stokes":
        return stokes_body_force(case["dim"], case["n"], (case["p"] + 1) ** case["dim"], seed)
    return rhs_normal(s.ndofs, seed)


def test_level_ops_bitwise(pair):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, sv = pair
    e, p = sv["expanded"], sv["pooled"]
    rng = np.random.default_rng(3)
    for l in range(e.nlevels):
        info = L.ldgmg_level_info(e.handle, l)
        N = info["nelem"] * e.bs
        x = torch.from_numpy(rng.standard_normal(N)).cuda()
        b = torch.from_numpy(rng.standard_normal(N)).cuda()
        bottom = l == e.nlevels - 1
        ops = ["residual", "apply_a"] + ([] if bottom else ["apply_s", "apply_st", "smooth_fwd", "smooth_rev"])
        for op in ops:
            outs = []
            for s in (e, p):
                o = torch.empty_like(x)
                L.ldgmg_level_op(s.handle, l, op, x, b if op in ("residual", "smooth_fwd", "smooth_rev") else None, o)
                torch.cuda.synchronize()
                outs.append(o)
            assert torch.equal(outs[0], outs[1]), (l, op)
    x = torch.from_numpy(rng.standard_normal(e.ndofs)).cuda()
    outs = []
    for s in (e, p):
        o = torch.empty_like(x)
        L.ldgmg_level_op(s.handle, 0, "apply_a64", x, None, o)
        torch.cuda.synchronize()
        outs.append(o)
    assert torch.equal(outs[0], outs[1])


def test_vcycle_and_solve_bitwise(pair):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, sv = pair
    e, p = sv["expanded"], sv["pooled"]
    b = torch.from_numpy(_rhs(case, e, 21)).cuda()
    xs = []
    for s in (e, p):
        x = torch.empty_like(b)
        L.ldgmg_vcycle(s.handle, b, x)
        torch.cuda.synchronize()
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
    krylov = case.get("krylov", "cg")
    res = []
    for s in (e, p):
        x = torch.empty_like(b)
        info = L.ldgmg_solve(s.handle, b, x, krylov, 1e-10, 200)
        torch.cuda.synchronize()
        res.append((info, x))
    assert res[0][0]["converged"] and res[0][0]["iters"] == res[1][0]["iters"]
    assert torch.equal(res[0][1], res[1][1])


def test_batch_bitwise(pair):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, sv = pair
    if case.get("krylov", "cg") != "cg":
        pytest.skip("the batched solve is CG")
    e, p = sv["expanded"], sv["pooled"]
    bs = [torch.from_numpy(_rhs(case, e, 30 + q)).cuda() for q in range(3)]
    outs = []
    for s in (e, p):
        xs = [torch.empty_like(b) for b in bs]
        infos = L.ldgmg_solve_batch(s.handle, bs, xs, 1e-10, 200)
        torch.cuda.synchronize()
        outs.append((infos, xs))
    for q in range(3):
        assert outs[0][0][q]["iters"] == outs[1][0][q]["iters"]
        assert torch.equal(outs[0][1][q], outs[1][1][q])


def test_tiled_close_to_pooled(pair):
    from paper_2412_12506_amd import ldgmg as L
    case, prec, sv = pair
    p, t = sv["pooled"], sv["tiled"]
    rng = np.random.default_rng(4)
    for l in range(p.nlevels):
        info = L.ldgmg_level_info(p.handle, l)
        N = info["nelem"] * p.bs
        xn = rng.standard_normal(N)
        x = torch.from_numpy(xn).cuda()
        bottom = l == p.nlevels - 1
        A = abs(L.export_bsr(p.handle, l, "A").tocsr())
        S = None if bottom else abs(L.export_bsr(p.handle, l, "S").tocsr())
        for op, M in [("apply_a", A)] + ([] if bottom else [("apply_s", S), ("apply_st", S.T.tocsr())]):
            outs = []
            for s in (p, t):
                o = torch.empty_like(x)
                L.ldgmg_level_op(s.handle, l, op, x, None, o)
                torch.cuda.synchronize()
                outs.append(o.cpu().numpy())
            # the same FP64 products summed in another order: a few hundred
            # terms per row, each sum within (terms) u64 of |M||x|
            mag = np.max(M @ np.abs(xn))
            err = np.max(np.abs(outs[0] - outs[1]))
            assert err <= 1e-13 * mag, (l, op, err, mag)
    b = torch.from_numpy(_rhs(case, p, 22)).cuda()
    krylov = case.get("krylov", "cg")
    res = []
    for s in (p, t):
        x = torch.empty_like(b)
        info = L.ldgmg_solve(s.handle, b, x, krylov, 1e-10, 200)
        torch.cuda.synchronize()
        res.append((info, x))
    assert res[0][0]["converged"] and res[1][0]["converged"]
    assert abs(res[0][0]["iters"] - res[1][0]["iters"]) <= 1
    rel = float(torch.linalg.norm(res[0][1] - res[1][1]) / torch.linalg.norm(res[0][1]))
    assert rel <= 1e-8, rel
