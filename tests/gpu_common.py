"""Shared helpers of the GPU parity tests: build the same problem in the HIP
library (through the C-ABI binding) and in the CPU oracle."""
import numpy as np
import scipy.sparse as sp

from ldg_inputs import mu_field, mu_box
from oracle import solver as osolver


def field_of(case, name="mu"):
    """Per-element field of a case: None, ("box", _, inner) (inner value inside
    (1/4,3/4)^d, 1 outside), ("uniform", _, value), or a ball / disc spec."""
    spec = case.get(name)
    if spec is None:
        return None
    kind, radius, contrast = spec
    if kind == "box":
        return mu_box(case["dim"], case["n"], contrast)
    if kind == "uniform":
        return np.full(case["n"] ** case["dim"], float(contrast))
    return mu_field(case["dim"], case["n"], kind, radius, contrast)


def mu_of(case):
    return field_of(case, "mu")


def lib_kwargs(case, precision):
    kw = {k: v for k, v in case.items() if k not in ("mu", "rho", "id", "krylov")}
    kw["mu"] = mu_of(case)
    if "rho" in case:
        kw["rho"] = field_of(case, "rho")
    kw["precision"] = precision
    return kw


_BUILT = {}


def oracle_build(case):
    """The oracle's hierarchy and V-cycle for a case, built once per process
    (several test modules and precisions share a case; callers only read it)."""
    kw = {k: v for k, v in case.items() if k not in ("mu", "rho", "id", "krylov", "nthreads")}
    key = repr(sorted((k, repr(v)) for k, v in case.items() if k not in ("id", "krylov", "nthreads")))
    if key not in _BUILT:
        kw["mu"] = mu_of(case)
        if "rho" in case:
            kw["rho"] = field_of(case, "rho")
        _BUILT[key] = osolver.build(**kw)
    return _BUILT[key]


def smoother_matrix(vc, level):
    s = vc.levels[level].sm
    if s.kind == "sai":
        return sp.csr_matrix(s.B)
    return sp.block_diag(list(s.Dinv), format="csr")


def rel_err_bound(y, ref, absref):
    """max |y - ref| / max |absref| (absref = |A||x| style magnitude)."""
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(absref)), 1e-300))


def round_fp32(M):
    """Entries of a sparse matrix rounded to FP32 (nearest even), kept in FP64."""
    M = sp.csr_matrix(M, copy=True)
    M.data = M.data.astype(np.float32).astype(np.float64)
    return M


def round_bf16(M):
    """Entries rounded as the library stores BF16 blocks: to nearest even in
    FP32, then to nearest even on the upper 16 bits of the FP32 word."""
    M = sp.csr_matrix(M, copy=True)
    u = M.data.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    M.data = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return M


def stored_vcycle(vc, prec):
    """The oracle's V-cycle with its matrices rounded as a precision mode stores
    them ("bf16s": operators in FP32, SAI matrices in BF16; the bottom
    pseudo-inverse stays FP64).  Arithmetic stays FP64, as in the library."""
    from oracle.vcycle import MGLevel, SmootherData, VCycle
    assert prec == "bf16s"
    levels = []
    for lv in vc.levels:
        A = round_fp32(lv.A)
        if lv.sm is None:
            levels.append(MGLevel(A, lv.bs, None, None, pinv=lv.pinv))
            continue
        assert lv.sm.kind == "sai"
        sd = SmootherData("sai", B=round_bf16(lv.sm.B))
        levels.append(MGLevel(A, lv.bs, lv.I, sd))
    return VCycle(levels, vc.order, vc.nu1, vc.nu2)


class F32Products:
    """A stored matrix whose products are taken in FP32: the entries (already
    rounded as stored) times the input rounded to FP32 to nearest, summed in
    FP32, returned as FP64.  The test-side model of ldgmg_fp32_products (the
    summation order differs from the matrix cores')."""

    def __init__(self, M):
        self.M32 = sp.csr_matrix(M, dtype=np.float32)
        self.shape = self.M32.shape

    def __matmul__(self, x):
        return (self.M32 @ np.asarray(x, dtype=np.float32)).astype(np.float64)

    @property
    def T(self):
        return F32Products(self.M32.T)


def fp32_products_vcycle(vc, prec):
    """The oracle's V-cycle with FP32 products in every operator and SAI apply
    above the bottom (matrices rounded as `prec` stores them: "fp32" or
    "bf16s"); transfers, vector updates and the bottom stay FP64."""
    from oracle.vcycle import MGLevel, SmootherData, VCycle
    assert prec in ("fp32", "bf16s")
    levels = []
    for lv in vc.levels:
        if lv.sm is None:
            levels.append(MGLevel(lv.A, lv.bs, None, None, pinv=lv.pinv))
            continue
        assert lv.sm.kind == "sai"
        B = round_bf16(lv.sm.B) if prec == "bf16s" else round_fp32(lv.sm.B)
        sd = SmootherData("sai", B=F32Products(B))
        levels.append(MGLevel(F32Products(round_fp32(lv.A)), lv.bs, lv.I, sd))
    return VCycle(levels, vc.order, vc.nu1, vc.nu2)
