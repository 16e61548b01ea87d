"""Shared helpers of the GPU parity tests: build the same problem in the HIP
library (through the C-ABI binding) and in the CPU oracle."""
import numpy as np
import scipy.sparse as sp

from ldg_inputs import mu_field, mu_box
from oracle import solver as osolver


def mu_of(case):
    spec = case.get("mu")
    if spec is None:
        return None
    kind, radius, contrast = spec
    if kind == "box":
        return mu_box(case["dim"], case["n"], contrast)
    return mu_field(case["dim"], case["n"], kind, radius, contrast)


def lib_kwargs(case, precision):
    kw = {k: v for k, v in case.items() if k not in ("mu", "id", "krylov")}
    kw["mu"] = mu_of(case)
    kw["precision"] = precision
    return kw


def oracle_build(case):
    kw = {k: v for k, v in case.items() if k not in ("mu", "id", "krylov", "nthreads")}
    kw["mu"] = mu_of(case)
    return osolver.build(**kw)


def smoother_matrix(vc, level):
    s = vc.levels[level].sm
    if s.kind == "sai":
        return sp.csr_matrix(s.B)
    return sp.block_diag(list(s.Dinv), format="csr")


def rel_err_bound(y, ref, absref):
    """max |y - ref| / max |absref| (absref = |A||x| style magnitude)."""
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(absref)), 1e-300))
