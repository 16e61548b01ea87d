"""Writes curved_iters.json: Krylov iteration counts of the oracle on the
curved-interface workloads at reduced grid sizes and on the 3D Poisson Q_3
workload at 12^3, all with seeded right-hand sides (seed 20241216).

  * sphere: 3D Q_2, viscosity 1e4 on elements whose centre lies inside the
    sphere r = 0.3 about the box centre (element-centre test), Legendre basis;
    SAI_1 OI and coloured Gauss-Seidel OI V-cycles in plain CG to 1e-10
    (at most 200 iterations), N(0,1) right-hand side;
  * disc: 2D stress-form Stokes Q_2, viscosity 1e3 inside the disc r = 0.25,
    velocity Dirichlet, balanced SAI_1 (zeta from tab:zeta) in left GMRES to
    ||V r|| <= 1e-10 ||V b|| (at most 100 iterations), OO and OI orderings,
    N(0,1) body force on the velocity coefficients;
  * poisson: 3D Q_3 on 12^3, SAI_1 OI, CG.

Calls only the oracle.  Run from the repository root:
python tests/golden/make_curved_iters.py (about 20 minutes on 8 cores)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from ldg_inputs import mu_field, rhs_normal, stokes_body_force  # noqa: E402
from oracle import solver as S  # noqa: E402

SEED = 20241216
out = []


def record(**kw):
    out.append(kw)
    print(kw, flush=True)


for n in (12, ):
    lv, vc = S.build(dim=3, n=n, p=3, smoother="sai", sai_level=1, order="OI")
    r = S.solve(lv, vc, rhs_normal(lv[0].A.shape[0], SEED), "cg", rtol=1e-10, maxit=200)
    record(kind="poisson", dim=3, n=n, p=3, smoother="sai", order="OI", krylov="cg",
           iters=int(r.iters), converged=bool(r.converged), eta=float(r.eta))
for n in (8, 12):
    mu = mu_field(3, n, "sphere", 0.3, 1e4)
    for smoother in ("sai", "gs"):
        lv, vc = S.build(dim=3, n=n, p=2, mu=mu, smoother=smoother, sai_level=1, order="OI")
        r = S.solve(lv, vc, rhs_normal(lv[0].A.shape[0], SEED), "cg", rtol=1e-10, maxit=200)
        record(kind="sphere", dim=3, n=n, p=2, contrast=1e4, radius=0.3, smoother=smoother, order="OI",
               krylov="cg", iters=int(r.iters), converged=bool(r.converged), eta=float(r.eta))
for n, orders in ((32, ("OO", "OI")), (64, ("OO",))):
    mu = mu_field(2, n, "disc", 0.25, 1e3)
    b = stokes_body_force(2, n, 9, SEED)
    for order in orders:
        lv, vc = S.build(dim=2, n=n, p=2, system="stokes", gamma=1, mu=mu, smoother="sai", sai_level=1,
                         order=order)
        r = S.solve(lv, vc, b, "gmres", rtol=1e-10, maxit=100)
        record(kind="disc", dim=2, n=n, p=2, contrast=1e3, radius=0.25, system="stokes", gamma=1,
               smoother="sai", order=order, krylov="gmres", iters=int(r.iters), converged=bool(r.converged),
               eta=float(r.eta))
json.dump({"source": "oracle V-cycles and Krylov solvers, seed 20241216", "cases": out},
          open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "curved_iters.json"), "w"), indent=1)
