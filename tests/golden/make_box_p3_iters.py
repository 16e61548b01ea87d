"""Writes box_p3_iters.json: CG iteration counts of the oracle's SAI_1 OI
V-cycle on the 3D box inclusion (Section 2.4.3 geometry, viscosity contrast
inside (1/4, 3/4)^3), Legendre Q_3, seeded N(0,1) right-hand side (seed
20241216), plain preconditioned CG to 1e-10, at most 200 iterations.

8^3 coarsens 8 -> 4 -> 2, every level aligned with the box; 12^3 coarsens
12 -> 6 -> 3, and on 6^3 the box faces cut through elements.  Calls only the
oracle.  Run from the repository root: python tests/golden/make_box_p3_iters.py
(about half an hour on 8 cores)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from ldg_inputs import mu_box, rhs_normal  # noqa: E402
from oracle import solver as S  # noqa: E402

out = []
for n, contrast in [(8, 1e4), (8, 1e3), (12, 1e3), (12, 1e4)]:
    lv, vc = S.build(dim=3, n=n, p=3, mu=mu_box(3, n, contrast), smoother="sai", sai_level=1, order="OI")
    b = rhs_normal(lv[0].A.shape[0], 20241216)
    r = S.solve(lv, vc, b, "cg", rtol=1e-10, maxit=200)
    out.append({"n": n, "p": 3, "contrast": contrast, "iters": int(r.iters), "converged": bool(r.converged),
                "eta": float(r.eta)})
    print(out[-1], flush=True)
json.dump({"source": "oracle SAI_1 OI V-cycle, plain CG, box inclusion (1/4,3/4)^3, seed 20241216",
           "cases": out}, open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "box_p3_iters.json"), "w"),
          indent=1)
