"""The boundary's allocator hooks, singular-operator handling and the
multi-hierarchy batched solve, through the C-ABI:

  * dev_alloc / dev_free (torch's caching allocator): the hierarchy's device
    memory is counted by torch, every block is handed back on unload, and the
    solve is bitwise that of hipMalloc'd storage;
  * Stokes with velocity Dirichlet data (Section 3.1: the pressure is defined
    up to a constant) and a scalar problem with Neumann faces only: the kernel
    found at upload is the constant of the oracle's kernel vector; a
    right-hand side with a kernel component is projected on the range (the
    solution equals that of the projected right-hand side, within the solve
    tolerance), the returned pressure (scalar field) has zero mean, and
    ldgmg_rhs_check turns an inconsistent right-hand side into
    LDGMG_ESINGULAR while accepting a consistent one;
  * ldgmg_solve_batch over several handles (different sizes and problems,
    interleaved): every right-hand side gets the result of its single solve
    (CG: +-1 iteration and 1e-8 relative, the batch grouping its products
    differently; GMRES runs one by one: bitwise).
"""
import numpy as np
import pytest

from ldg_inputs import rhs_normal, stokes_body_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solve(s, b, krylov="cg"):
    from paper_2412_12506_amd import ldgmg as L
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xt = torch.empty_like(bt)
    info = L.ldgmg_solve(s.handle, bt, xt, krylov, 1e-10, 200)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), info


def test_torch_allocator():
    from paper_2412_12506_amd import ldgmg as L
    kw = dict(dim=3, n=8, p=2, smoother="sai", precision="bf16s")
    ref = L.Solver(**kw)
    alloc = L.TorchAllocator()
    before = torch.cuda.memory_allocated()
    s = L.Solver(allocator=alloc, **kw)
    try:
        held = torch.cuda.memory_allocated() - before
        print(f"\n[allocator] device bytes {s.device_bytes}, counted by torch {held}, blocks {alloc.live}",
              flush=True)
        assert held >= s.device_bytes and alloc.live > 0
        b = rhs_normal(s.ndofs, 3)
        x1, i1 = _solve(ref, b)
        x2, i2 = _solve(s, b)
        assert i1["iters"] == i2["iters"] and np.array_equal(x1, x2)
        # batched workspace through the allocator too
        bs = [torch.from_numpy(rhs_normal(s.ndofs, 10 + q)).cuda() for q in range(2)]
        xs = [torch.empty_like(v) for v in bs]
        L.ldgmg_solve_batch(s.handle, bs, xs)
        torch.cuda.synchronize()
        s.unload()
        assert alloc.live == 0
        assert torch.cuda.memory_allocated() - before <= 2 * 16 * s.ndofs   # only the test's own vectors
        s.upload()                                                          # back from the host tier
        x3, _ = _solve(s, b)
        assert np.array_equal(x1, x3)
    finally:
        s.close()
        ref.close()
    assert alloc.live == 0


@pytest.mark.parametrize("case", ["stokes-std", "stokes-stress-disc", "poisson-neumann"])
def test_singular_operator(case):
    from paper_2412_12506_amd import ldgmg as L
    from oracle import solver as osolver, stokes, ldg
    if case.startswith("stokes"):
        gamma = 0 if case == "stokes-std" else 1
        mu = None
        if case == "stokes-stress-disc":
            from ldg_inputs import mu_field
            mu = mu_field(2, 8, "disc", 0.25, 1e3)
        kw = dict(dim=2, n=8, p=2, system="stokes", gamma=gamma, mu=mu, smoother="sai", order="OO")
        krylov = "gmres"
        b = stokes_body_force(2, 8, 9, 5)
    else:
        kw = dict(dim=2, n=8, p=2, bc=["N"] * 4, smoother="sai", order="OI")
        krylov = "cg"
        b = rhs_normal(8 * 8 * 9, 5)
    lv, vc = osolver.build(**{k: v for k, v in kw.items()})
    if case.startswith("stokes"):
        k = stokes.pressure_kernel(lv[0])
    else:                                          # constant: the (0,0) Legendre mode of every element
        k = np.zeros((64, 9))
        k[:, 0] = 1.0
        k = k.reshape(-1)
        assert np.abs(lv[0].A @ k).max() < 1e-12 * abs(lv[0].A).max()
    khat = k / np.linalg.norm(k)
    s = L.Solver(precision="fp64", **kw)
    try:
        cnt, kv = L.ldgmg_kernel(s.handle, with_vectors=True)
        assert cnt == 1 and np.abs(kv[0] - khat).max() < 1e-14
        b0 = b - (b @ khat) * khat                  # consistent part
        bi = b0 + 0.3 * np.linalg.norm(b0) * khat   # with a kernel component
        x0, i0 = _solve(s, b0, krylov)
        xi, ii = _solve(s, bi, krylov)
        assert i0["converged"] and ii["converged"]
        # the inconsistent right-hand side is projected: same solution
        assert np.linalg.norm(xi - x0) <= 1e-9 * np.linalg.norm(x0)
        # zero mean of the kernel component: M-weighted (int p = 0 / int u = 0)
        if case.startswith("stokes"):
            bss = 9
            P = x0.reshape(64, 3, bss)[:, 2]
            Me = ldg.ElementMatrices(2, 2, 1.0 / 8).M
            kp = k.reshape(64, 3, bss)[:, 2]
            integral = sum(kp[e] @ Me @ P[e] for e in range(64))
        else:
            integral = k @ (lv[0].M.tocsr() @ x0)
        print(f"\n[{case}] iters {i0['iters']}/{ii['iters']}, int of kernel component {integral:.2e}", flush=True)
        assert abs(integral) <= 1e-12 * np.linalg.norm(x0) * np.linalg.norm(k)
        # against the oracle on the consistent right-hand side, modulo the kernel
        ref = osolver.solve(lv, vc, b0, krylov)
        proj = lambda v: v - (v @ khat) * khat
        rel = np.linalg.norm(proj(x0) - proj(ref.x)) / np.linalg.norm(proj(ref.x))
        assert rel <= 1e-8, rel
        # explicit consistency check
        L.ldgmg_rhs_check(s.handle, 1e-8)
        _solve(s, b0, krylov)
        with pytest.raises(L.LdgmgError) as ex:
            _solve(s, bi, krylov)
        assert ex.value.code == L.ESINGULAR
    finally:
        s.close()


def test_nonsingular_has_no_kernel():
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(dim=2, n=8, p=2, smoother="jacobi", precision="fp64")
    try:
        assert L.ldgmg_kernel(s.handle) == 0
    finally:
        s.close()


def test_batch_over_several_handles():
    from paper_2412_12506_amd import ldgmg as L
    a = L.Solver(dim=2, n=16, p=2, smoother="sai", precision="bf16s")
    c = L.Solver(dim=3, n=8, p=1, smoother="gs", precision="fp32")
    st = L.Solver(dim=2, n=8, p=1, system="stokes", gamma=1, smoother="sai", order="OO", precision="fp32")
    try:
        hs = [a.handle, c.handle, a.handle, c.handle, a.handle]
        bs = [torch.from_numpy(rhs_normal(L.ldgmg_sizes(h)[0], 30 + q)).cuda() for q, h in enumerate(hs)]
        xs = [torch.empty_like(v) for v in bs]
        infos = L.ldgmg_solve_batch(hs, bs, xs)
        torch.cuda.synchronize()
        for q, h in enumerate(hs):
            s = a if h == a.handle else c
            x1, one = _solve(s, bs[q].cpu().numpy())
            rel = np.linalg.norm(xs[q].cpu().numpy() - x1) / np.linalg.norm(x1)
            print(f"\n[multi-handle batch] rhs {q}: iters {infos[q]['iters']} / single {one['iters']}, "
                  f"rel diff {rel:.1e}", flush=True)
            # the batch takes its products in another grouping (multi-vector kernels)
            assert infos[q]["converged"] and abs(infos[q]["iters"] - one["iters"]) <= 1 and rel <= 1e-8
            assert infos[q]["vcycles"] == infos[q]["iters"]      # its own V-cycles, not the batch's
        # GMRES on Stokes handles, one after the other: bitwise the single solves
        b2 = [torch.from_numpy(stokes_body_force(2, 8, 4, 40 + q)).cuda() for q in range(2)]
        x2 = [torch.empty_like(v) for v in b2]
        inf2 = L.ldgmg_solve_batch([st.handle, st.handle], b2, x2, krylov="gmres")
        torch.cuda.synchronize()
        for q in range(2):
            x1, one = _solve(st, b2[q].cpu().numpy(), "gmres")
            assert inf2[q]["iters"] == one["iters"] and np.array_equal(x2[q].cpu().numpy(), x1)
    finally:
        for s in (a, c, st):
            s.close()
