"""Host-side setup of the C-ABI library (no GPU: ldgmg_setup_host) against the
oracle: the operators A on every level, the smoother matrices (balanced SAI
B, block inverses), the colouring and the bottom pseudo-inverse.  The two
setups share no code; agreement is to rounding (A, S) or to the conditioning
limit (pseudo-inverse)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from tests.gpu_common import lib_kwargs, oracle_build, smoother_matrix

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2412_12506_amd", "libldgmg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libldgmg.so not built")

CASES = [
    dict(id="p2d-p2-gl-jacobi", dim=2, n=8, p=2, basis="gl_nodal", smoother="jacobi"),
    dict(id="p3d-p3-sai1", dim=3, n=4, p=3, smoother="sai"),
    dict(id="i2d-p2-disc-sai1", dim=2, n=16, p=2, smoother="sai", mu=("disc", 0.25, 1e3)),
    dict(id="i2d-p2-box-gs", dim=2, n=8, p=2, smoother="gs", mu=("box", 0.0, 1e4)),
    dict(id="p2d-p1-sai2", dim=2, n=8, p=1, smoother="sai", sai_level=2),
    dict(id="s2d-p2-stress-disc", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("disc", 0.25, 1e3)),
    dict(id="s2d-p1-std-jacobi", dim=2, n=8, p=1, system="stokes", gamma=0, smoother="jacobi"),
    dict(id="p2d-p2-neumann-x", dim=2, n=8, p=2, smoother="sai", bc=["N", "N", "D", "D"]),
    # bottoms of 400 and 675 unknowns: the eigensolver splits its work over threads
    dict(id="p2d-p3-n10-threaded-bottom", dim=2, n=10, p=3, smoother="jacobi", nthreads=4),
    dict(id="s2d-p2-n10-threaded-bottom", dim=2, n=10, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("disc", 0.25, 1e3), nthreads=3),
    # unsteady Stokes (eq:blockformunsteady, delta = 0.1 h): a gas bubble in water, stress form;
    # single phase, standard form, periodic, mu = 1e-2
    dict(id="s2d-p2-unsteady-gas-in-water", dim=2, n=8, p=2, system="stokes", gamma=1, smoother="sai",
         mu=("box", 0.0, 2e-4), rho=("box", 0.0, 1e-3), delta=0.1 / 8),
    dict(id="s2d-p1-unsteady-periodic-std", dim=2, n=8, p=1, system="stokes", gamma=0, smoother="gs",
         mu=("uniform", 0.0, 1e-2), delta=0.1 / 8, bc=["P"] * 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["id"])
def test_host_setup_matches_oracle(case):
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(host_only=True, **lib_kwargs(case, "fp64"))
    lv, vc = oracle_build(case)
    try:
        assert s.nlevels == len(lv)
        for l in range(s.nlevels):
            A = L.export_bsr(s.handle, l, "A").tocsr()
            Ao = lv[l].A.tocsr()
            assert abs(A - Ao).max() <= 1e-13 * abs(Ao).max(), ("A", l)
            if l < s.nlevels - 1:
                S = L.export_bsr(s.handle, l, "S").tocsr()
                So = smoother_matrix(vc, l)
                assert abs(S - So).max() <= 1e-11 * abs(So).max(), ("S", l)
                if case["smoother"] == "gs":
                    assert np.array_equal(L.ldgmg_export_colours(s.handle, l), vc.levels[l].sm.colours)
        P = L.ldgmg_export(s.handle, 0, "PINV")
        Po = vc.levels[-1].pinv
        Ab = vc.levels[-1].A.toarray()
        lam = np.abs(np.linalg.eigvalsh(Ab))
        kappa = lam.max() / lam[lam > 1e-12 * lam.max()].min()
        assert np.abs(P - Po).max() <= max(1e-12, 20 * kappa * 2.0 ** -52) * np.abs(Po).max()
        # Moore-Penrose identity A P A = A holds to rounding for either one
        assert np.abs(Ab @ P @ Ab - Ab).max() <= 1e-12 * np.abs(Ab).max()
    finally:
        s.close()


def test_sai_cache_counts():
    """Uniform 3D grid, constant viscosity: the exact cache leaves 216 distinct
    least-squares problems per level (6 classes per axis from the one-sided
    flux and the two boundaries) and fewer on grids too small for them."""
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(host_only=True, dim=3, n=16, p=1, smoother="sai", precision="fp64")
    try:
        counts = [L.ldgmg_setup_stats(s.handle, l)[0] for l in range(s.nlevels - 1)]
        assert counts[0] == 216 and counts[1] == 216 and counts[2] == 64
    finally:
        s.close()


def test_invalid_problems_are_rejected():
    from paper_2412_12506_amd import ldgmg as L
    for bad in (dict(dim=4, n=8, p=2), dict(dim=2, n=8, p=0), dict(dim=2, n=1, p=2),
                dict(dim=2, n=8, p=2, bc=["P", "D", "D", "D"]),
                dict(dim=2, n=4, p=2, mu=np.array([1.0] * 15 + [np.nan])),
                dict(dim=2, n=8, p=2, smoother="jacobi", precision="bf16s"),   # BF16 is for SAI only
                dict(dim=2, n=8, p=2, smoother="gs", precision="bf16s")):
        with pytest.raises((L.LdgmgError, ValueError)) as ei:
            s = L.Solver(host_only=True, **bad)
            s.close()
        if isinstance(ei.value, L.LdgmgError):
            assert ei.value.code == L.EINVAL


def test_fp32_products_need_fp32_or_bf16_storage():
    """ldgmg_fp32_products is refused for FP64 storage and accepted (before any
    upload) for FP32 and BF16S storage."""
    from paper_2412_12506_amd import ldgmg as L
    for prec, ok in (("fp64", False), ("fp32", True), ("bf16s", True)):
        s = L.Solver(host_only=True, dim=2, n=8, p=2, smoother="sai", precision=prec)
        try:
            if ok:
                L.ldgmg_fp32_products(s.handle, True)
                L.ldgmg_fp32_products(s.handle, False)
            else:
                with pytest.raises(L.LdgmgError) as ei:
                    L.ldgmg_fp32_products(s.handle, True)
                assert ei.value.code == L.EINVAL
                L.ldgmg_fp32_products(s.handle, False)       # switching off is always allowed
        finally:
            s.close()


def test_bottom_independent_of_thread_count():
    """The threaded eigensolver does the same arithmetic in the same order."""
    from paper_2412_12506_amd import ldgmg as L
    out = []
    for nt in (1, 2, 5):
        s = L.Solver(host_only=True, dim=2, n=10, p=3, smoother="jacobi", nthreads=nt)
        try:
            out.append(L.ldgmg_export(s.handle, s.nlevels - 1, "PINV"))
        finally:
            s.close()
    assert out[0].shape == (400, 400)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_upload_bytes_by_storage():
    """Pooled storage keeps the distinct blocks once plus a block id per slot."""
    from paper_2412_12506_amd import ldgmg as L
    got = {}
    for st in ("expanded", "pooled", "auto"):
        s = L.Solver(host_only=True, dim=3, n=8, p=3, smoother="sai", storage=st)
        try:
            got[st] = s.upload_bytes
            nnz_a = L.ldgmg_level_info(s.handle, 0)["nnzb_A"]
        finally:
            s.close()
    # the fine A alone: 8^3 rows of 7 (interior) FP32 64x64 blocks when expanded
    assert got["expanded"] > nnz_a * 64 * 64 * 4
    assert got["pooled"] < got["expanded"] / 4
    assert got["pooled"] <= got["auto"] <= got["expanded"]


def test_rebuild_smoother_matches_fresh_build():
    """A GS hierarchy rebuilt from a SAI one (operators, transfers and bottom
    kept) exports exactly what a fresh GS setup exports; another problem is
    refused."""
    from paper_2412_12506_amd import ldgmg as L
    from ldg_inputs import mu_box
    kw = dict(dim=2, n=8, p=2, mu=mu_box(2, 8, 1e4))
    sai = L.Solver(host_only=True, smoother="sai", **kw)
    fresh = L.Solver(host_only=True, smoother="gs", **kw)
    rebuilt = sai.resmoothed(smoother="gs", **kw)
    try:
        assert rebuilt.nlevels == fresh.nlevels
        for l in range(fresh.nlevels):
            for what in ("A",) + (("S",) if l + 1 < fresh.nlevels else ()):
                a, b = L.export_bsr(fresh.handle, l, what), L.export_bsr(rebuilt.handle, l, what)
                assert (a != b).nnz == 0, (l, what)
            if l + 1 < fresh.nlevels:
                assert np.array_equal(L.ldgmg_export_colours(fresh.handle, l), L.ldgmg_export_colours(rebuilt.handle, l))
        assert np.array_equal(L.ldgmg_export(fresh.handle, 0, "PINV"), L.ldgmg_export(rebuilt.handle, 0, "PINV"))
        with pytest.raises(L.LdgmgError) as ei:
            sai.resmoothed(smoother="gs", dim=2, n=8, p=2, mu=mu_box(2, 8, 1e3))
        assert ei.value.code == L.EINVAL
    finally:
        for s in (sai, fresh, rebuilt):
            s.close()


def test_host_setup_under_sanitizers(tmp_path):
    """The host setup code (host.cpp, dense.cpp: assembly, coarsening, SAI
    least squares, block inverses, threaded bottom eigensolver, smoother
    rebuild) built with AddressSanitizer and UndefinedBehaviorSanitizer and
    run on a spread of problems: no memory or undefined-behaviour error."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_2412_12506_amd", "csrc")
    exe = str(tmp_path / "host_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-march=x86-64-v3", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(root, "tests", "host_asan_driver.cpp"),
           os.path.join(csrc, "host.cpp"), os.path.join(csrc, "dense.cpp"), "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
