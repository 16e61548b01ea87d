"""Serving on the GPU: continuous batching of a seeded stream of mixed
requests (2D and 3D, Poisson and box interface, several degrees), with
hierarchies admitted by HBM budget and kept resident.

  * every request's result in the mix equals the same request solved alone
    (a fresh hierarchy, ldgmg_solve): the same CG iteration count and the
    solution within 1e-10 relative (batched and single solves differ only in
    the summation order of the inner products), each to a true FP64 relative
    residual <= 2e-10;
  * a request whose hierarchy does not fit beside one in use waits, and is
    admitted once that one's batch has ended (the idle hierarchy is evicted);
  * a problem larger than the whole budget is refused, not waited on.
"""
import numpy as np
import pytest

from ldg_inputs import Request, rhs_normal_device, serving_requests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GIB = 1 << 30


def _alone(results, precision):
    from paper_2412_12506_amd import ldgmg as L
    from paper_2412_12506_amd.serving import problem_kwargs
    by_key = {}
    for r in results:
        by_key.setdefault((r.key, r.smoother), []).append(r)
    worst = 0.0
    for (key, smoother), rs in by_key.items():
        s = L.Solver(**problem_kwargs(key, precision, smoother))
        try:
            for r in rs:
                b = rhs_normal_device(s.ndofs, r.seed_used)
                x = torch.empty_like(b)
                info = L.ldgmg_solve(s.handle, b, x, "cg", 1e-10, 200)
                torch.cuda.synchronize()
                assert info["converged"], key
                assert r.iters == info["iters"], (r.rid, key, r.iters, info["iters"])
                xa = x.cpu().numpy()
                err = np.linalg.norm(r.x - xa) / np.linalg.norm(xa)
                worst = max(worst, err)
                assert err <= 1e-10, (r.rid, key, err)
        finally:
            s.close()
    return worst


def _run(eng, reqs, **kw):
    res = eng.run(reqs, **kw)
    seed = {q.rid: q.seed for q in reqs}
    for r in res:
        r.seed_used = seed[r.rid]
    return res


def test_mix_equals_alone():
    from paper_2412_12506_amd.serving import ServingEngine, summarize
    reqs = serving_requests(count=40, rate=400.0, grids2d=(16, 32), grids3d=(8,), degrees=(1, 2),
                            contrasts=(1.0, 1e2, 1e4))
    eng = ServingEngine(hbm_budget=16 * GIB, workers=3, keep_solutions=True)
    try:
        res = _run(eng, reqs)
        st = summarize(res)
        print(f"\n[serving mix] {st}", flush=True)
        assert not eng.errors, eng.errors
        assert len(res) == len(reqs) and all(r.converged for r in res)
        assert all(r.rel_res_true <= 2e-10 for r in res)
        assert max(r.batch for r in res) >= 2          # requests were batched
        assert eng.peak_used <= eng.budget
        worst = _alone(res, eng.precision)
        print(f"[serving mix] alone vs mix worst relative difference {worst:.2e}", flush=True)
    finally:
        eng.close()


def test_admission_waits_for_memory():
    from paper_2412_12506_amd.serving import ServingEngine, problem_key
    big = [Request(i, 0.0, "interface", 3, 8, 2, 1e4, 900 + i) for i in range(3)]
    small = [Request(10 + i, 0.001, "poisson", 2, 32, 2, 1.0, 950 + i) for i in range(3)]
    eng = ServingEngine(hbm_budget=1, workers=2, keep_solutions=True)
    ka, kb = problem_key(big[0]), problem_key(small[0])
    eng.prebuild([ka, kb], threads=2)                  # exact device bytes from the host tier
    na, nb = eng._need_bytes(ka), eng._need_bytes(kb)
    eng.budget = max(na, nb) + min(na, nb) // 2       # one fits, not both
    try:
        res = _run(eng, big + small)
        assert not eng.errors, eng.errors
        assert all(r.converged for r in res)
        assert eng.peak_used <= eng.budget
        first = {}
        for k, t in eng.admissions:
            first.setdefault(k, t)
        assert set(first) == {ka, kb}
        kx, ky = sorted(first, key=first.get)           # admitted first, admitted second
        x_end = min(r.end for r in res if r.key == kx)
        # the second hierarchy was admitted only after the first one's batch had
        # ended, by evicting it
        assert first[ky] >= x_end, (first, x_end)
        assert eng.evictions and eng.evictions[0][0] == kx
        print(f"\n[serving memory] admissions {eng.admissions} evictions {eng.evictions}", flush=True)
        _alone(res, eng.precision)
    finally:
        eng.close()


def test_refuses_problem_over_budget():
    from paper_2412_12506_amd.serving import ServingEngine
    reqs = [Request(0, 0.0, "poisson", 2, 16, 1, 1.0, 5), Request(1, 0.0, "poisson", 2, 16, 1, 1.0, 6)]
    eng = ServingEngine(hbm_budget=1 << 16, workers=1)
    try:
        res = eng.run(reqs)
        assert len(res) == 2 and all(r.error and not r.converged for r in res)
        assert eng.used == 0
    finally:
        eng.close()


def test_continuous_batching_tiled_mix_equals_alone():
    """Hierarchies that the AUTO storage tiles (3D Q_2 on 32^3, 2D Q_3 on
    128^2: at least 16,384 block rows), requests arriving while batches run:
    each result equals the same request solved alone (same iterations,
    1e-10), and requests joined batches already in flight (a request started
    while another of its key was in flight, after a third had completed)."""
    from paper_2412_12506_amd import ldgmg as L
    from paper_2412_12506_amd.serving import ServingEngine, problem_kwargs, summarize
    reqs = [Request(i, 0.004 * i, "poisson" if i % 3 else "interface", 3 if i % 2 else 2, 32 if i % 2 else 128,
                    2 if i % 2 else 3, 1.0 if i % 3 else 1e2, 700 + i) for i in range(24)]
    eng = ServingEngine(hbm_budget=64 * GIB, workers=2, max_batch=4, keep_solutions=True)
    try:
        keys = {(q.dim, q.n, q.p, float(q.contrast)) for q in reqs}
        eng.prebuild(keys, threads=2)
        for k in keys:
            s = eng.entries[k].solver
            s.upload()
            st = L.ldgmg_level_storage(s.handle, 0)
            s.unload()
            print(f"\n[serving tiled] key {k}: fine-level storage {st}", flush=True)
            if k[3] == 1.0:
                assert st["tiled_A"] and st["tiled_S"], (k, st)
        res = _run(eng, reqs)
        print(f"\n[serving tiled] {summarize(res)}", flush=True)
        assert not eng.errors, eng.errors
        assert all(r.converged and r.rel_res_true <= 2e-10 for r in res)
        joined = 0
        for b in res:
            same = [r for r in res if r.key == b.key and r.rid != b.rid]
            if any(c.start < b.start < c.end for c in same) and any(a.end <= b.start for a in same):
                joined += 1
        print(f"[serving tiled] requests that joined a running batch: {joined}", flush=True)
        assert joined >= 1
        worst = _alone(res, eng.precision)
        print(f"[serving tiled] alone vs mix worst relative difference {worst:.2e}", flush=True)
    finally:
        eng.close()
