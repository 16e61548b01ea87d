"""The oracle's local rows / local SAI columns agree with its global assembly
(so they can stand in for it on grids too large to assemble whole)."""
import numpy as np
import pytest
import scipy.sparse as sp

from ldg_inputs import mu_field
from oracle import hierarchy, stokes, smoothers as sm
from oracle.local import LocalOperator


@pytest.mark.parametrize("case", [
    dict(dim=2, n=6, p=2, mu=("disc", 0.25, 1e3)),
    dict(dim=3, n=4, p=1, mu=("sphere", 0.3, 1e4)),
    dict(dim=2, n=5, p=2, system="stokes", gamma=1, mu=("disc", 0.25, 1e3)),
    dict(dim=2, n=4, p=1, system="stokes", gamma=0),
], ids=["disc2d", "sphere3d", "stokes-stress", "stokes-std"])
def test_local_rows_match_global(case):
    mu = None
    if "mu" in case:
        k, r, c = case["mu"]
        mu = mu_field(case["dim"], case["n"], k, r, c)
    system = case.get("system", "poisson")
    if system == "poisson":
        A = hierarchy.scalar_levels(case["dim"], case["n"], case["p"], mu=mu)[0].A.tocsr()
    else:
        A = stokes.stokes_levels(case["dim"], case["n"], case["p"], mu=mu, gamma=case["gamma"],
                                 cp=0.1)[0].A.tocsr()
    lo = LocalOperator(case["dim"], case["n"], case["p"], mu=mu, system=system,
                       gamma=case.get("gamma", 1))
    bs = lo.bs
    rng = np.random.default_rng(0)
    x = rng.standard_normal(A.shape[0])
    rows = list(range(lo.grid.ne))
    y = lo.apply_rows(rows, x).reshape(-1)
    assert np.abs(y - A @ x).max() <= 1e-12 * np.abs(A @ x).max() + 1e-12 * (abs(A) @ np.abs(x)).max()


def test_local_sai_column_matches_global():
    dim, n, p = 2, 8, 2
    mu = mu_field(dim, n, "disc", 0.25, 1e3)
    A = hierarchy.scalar_levels(dim, n, p, mu=mu)[0].A
    bs = (p + 1) ** dim
    B, _ = sm.sai(A, bs, 1, sm.balance_scalar(A, bs))
    B = sp.csr_matrix(B)
    lo = LocalOperator(dim, n, p, mu=mu)
    for i in (0, 27, 36, 63):
        col = lo.sai_column(i)
        for j, blk in col.items():
            ref = B[j * bs:(j + 1) * bs, i * bs:(i + 1) * bs].toarray()
            assert np.abs(blk - ref).max() <= 1e-10 * np.abs(ref).max() + 1e-14
