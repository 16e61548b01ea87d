"""The SAI least-squares problems solved on the GPU (setup_device = 1:
batched FP64 normal equations with one refinement step on rocBLAS /
rocSOLVER, Section 2.3.3) against the host setup and the oracle:

  * every level's balanced SAI matrix B from the device setup agrees with the
    host setup's within 1e-11 max|B| (both solve the same problems; the host
    by block-sparse normal equations with refinement or Householder QR), and
    with the oracle's QR solution within 1e-11 max|B|; the operators A are
    bitwise equal (they do not depend on where B is solved);
  * the problems the device declined (if any) went to the host, and the
    device solved the rest;
  * a solve with the device-built hierarchy needs the iterations of the
    host-built one.
Setup times of both paths are printed (the serving engine's cache misses
pay them)."""
import numpy as np
import pytest

from ldg_inputs import rhs_normal
from tests.gpu_common import lib_kwargs, oracle_build, smoother_matrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    dict(id="p3d-p3-sai1", dim=3, n=6, p=3, smoother="sai"),
    dict(id="i3d-p2-sphere-sai1", dim=3, n=8, p=2, smoother="sai", mu=("sphere", 0.3, 1e4)),
    dict(id="p2d-p3-sai2", dim=2, n=8, p=3, smoother="sai", sai_level=2),
    dict(id="s2d-p2-stress-disc-sai1", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("disc", 0.25, 1e3)),
    dict(id="s2d-p2-unsteady-gas-in-water", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("box", 0.0, 2e-4), rho=("box", 0.0, 1e-3), delta=0.1 / 8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["id"])
def test_device_setup_matches_host_and_oracle(case):
    from paper_2412_12506_amd import ldgmg as L
    hs = L.Solver(host_only=True, **lib_kwargs(case, "fp64"))
    ds = L.Solver(host_only=True, setup_device=True, **lib_kwargs(case, "fp64"))
    lv, vc = oracle_build(case)
    try:
        dev_total = 0
        for l in range(hs.nlevels - 1):
            Bh = L.export_bsr(hs.handle, l, "S").tocsr()
            Bd = L.export_bsr(ds.handle, l, "S").tocsr()
            Bo = smoother_matrix(vc, l)
            scale = abs(Bh).max()
            dh = abs(Bd - Bh).max() / scale
            do = abs(Bd - Bo).max() / scale
            ndev, nqr, t = L.ldgmg_setup_stats_device(ds.handle, l)
            nu, _ = L.ldgmg_setup_stats(ds.handle, l)
            dev_total += ndev
            print(f"\n[{case['id']}] level {l}: {nu} unique problems, {ndev} on the device, {nqr} by host QR; "
                  f"|B_dev - B_host| {dh:.1e}, |B_dev - B_oracle| {do:.1e}", flush=True)
            assert dh <= 1e-11 and do <= 1e-11
            assert ndev + nqr <= nu
            Ah = L.export_bsr(hs.handle, l, "A")
            Ad = L.export_bsr(ds.handle, l, "A")
            assert (Ah != Ad).nnz == 0
        assert dev_total > 0
        th = sum(L.ldgmg_setup_stats_device(hs.handle, l)[2] for l in range(hs.nlevels - 1))
        td = sum(L.ldgmg_setup_stats_device(ds.handle, l)[2] for l in range(ds.nlevels - 1))
        print(f"[{case['id']}] SAI least-squares solves: host {th:.3f} s, device {td:.3f} s", flush=True)
        if case.get("system") != "stokes":
            ds.upload()
            hs.upload()
            b = torch.from_numpy(rhs_normal(ds.ndofs, 3)).cuda()
            x1, x2 = torch.empty_like(b), torch.empty_like(b)
            i1 = L.ldgmg_solve(hs.handle, b, x1, "cg", 1e-10, 200)
            i2 = L.ldgmg_solve(ds.handle, b, x2, "cg", 1e-10, 200)
            torch.cuda.synchronize()
            assert i1["converged"] and i1["iters"] == i2["iters"]
    finally:
        hs.close()
        ds.close()


def test_device_setup_time_large():
    """3D Poisson Q_3 on 32^3 and a box interface at 1e4 on 24^3 (923 distinct
    SAI problems on its fine level): setup times of both paths, and the fine
    B of both within 1e-11 max|B|."""
    from paper_2412_12506_amd import ldgmg as L
    from ldg_inputs import mu_box
    for kw in (dict(dim=3, n=32, p=3), dict(dim=3, n=24, p=3, mu=mu_box(3, 24, 1e4))):
        hs = L.Solver(host_only=True, smoother="sai", precision="fp32", **kw)
        ds = L.Solver(host_only=True, smoother="sai", precision="fp32", setup_device=True, **kw)
        try:
            Bh = L.export_bsr(hs.handle, 0, "S").tocsr()
            Bd = L.export_bsr(ds.handle, 0, "S").tocsr()
            d = abs(Bd - Bh).max() / abs(Bh).max()
            th = L.ldgmg_setup_stats_device(hs.handle, 0)[2]
            nd, nq, td = L.ldgmg_setup_stats_device(ds.handle, 0)
            nu, _ = L.ldgmg_setup_stats(ds.handle, 0)
            print(f"\n[setup {kw['n']}^3 p=3 {'box 1e4' if 'mu' in kw else 'Poisson'}] {nu} unique fine problems "
                  f"({nd} device, {nq} host QR); fine-level SAI solves: host {th:.3f} s, device {td:.3f} s; "
                  f"|dB| {d:.1e}", flush=True)
            assert d <= 1e-11
        finally:
            hs.close()
            ds.close()
