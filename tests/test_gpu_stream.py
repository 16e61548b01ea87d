"""Continuous batching in the library (ldgmg_solve_stream) and batches of up
to 16 right-hand sides:

  * right-hand sides handed over while others are in flight (a feeder that
    offers nothing at some stages and more later): every one is solved as by
    ldgmg_solve (iterations +-1, solution within 1e-8 relative, true FP64
    residual <= 2e-10), on tiled storage (the matrix-core path) and on the
    per-row vector kernels; the V-cycles reported per right-hand side equal
    its iterations;
  * 16 right-hand sides in one batched CG on tiled storage (one block row and
    16 vectors per 16-column tile): each as its single solve.
"""
import numpy as np
import pytest

from ldg_inputs import rhs_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _single(s, b):
    from paper_2412_12506_amd import ldgmg as L
    x = torch.empty_like(b)
    info = L.ldgmg_solve(s.handle, b, x, "cg", 1e-10, 200)
    torch.cuda.synchronize()
    return x, info


@pytest.mark.parametrize("storage", ["tiled", "pooled"])
def test_stream_admits_while_running(storage):
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(dim=3, n=16, p=2, smoother="sai", precision="bf16s", storage=storage)
    try:
        nrhs = 11
        bs = [torch.from_numpy(rhs_normal(s.ndofs, 500 + q)).cuda() for q in range(nrhs)]
        xs = [torch.empty_like(b) for b in bs]
        stage = [0]
        fed = []
        log = []
        # offer 3 at once, then one more every other stage while others are in
        # flight (with nothing in flight, nothing offered ends the call)
        def next_rhs():
            stage[0] += 1
            in_flight = len(fed) - sum(1 for e in log if e[0] == "out")
            if len(fed) < nrhs and (len(fed) < 3 or stage[0] % 2 == 0 or in_flight == 0):
                q = len(fed)
                fed.append(stage[0])
                log.append(("in", q, len(fed) - sum(1 for e in log if e[0] == "out")))
                return bs[q], xs[q], q
            return None

        infos = {}

        def on_done(tag, info):
            infos[tag] = info
            log.append(("out", tag))

        rc = L.ldgmg_solve_stream(s.handle, 4, next_rhs, on_done)
        torch.cuda.synchronize()
        assert rc == L.OK and len(infos) == nrhs
        # some right-hand side was admitted after another had completed, while others ran
        first_out = next(i for i, e in enumerate(log) if e[0] == "out")
        assert any(e[0] == "in" for e in log[first_out:])
        for q in range(nrhs):
            x1, one = _single(s, bs[q])
            rel = float(torch.linalg.norm(xs[q] - x1) / torch.linalg.norm(x1))
            print(f"\n[stream {storage}] rhs {q}: iters {infos[q]['iters']} single {one['iters']} rel {rel:.1e}",
                  flush=True)
            assert infos[q]["converged"] and infos[q]["rel_res_true"] <= 2e-10
            assert abs(infos[q]["iters"] - one["iters"]) <= 1 and rel <= 1e-8
            assert infos[q]["vcycles"] == infos[q]["iters"]
    finally:
        s.close()


def test_batch_of_16_on_tiled_storage():
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(dim=3, n=16, p=2, smoother="sai", precision="bf16s", storage="tiled")
    try:
        bs = [torch.from_numpy(rhs_normal(s.ndofs, 600 + q)).cuda() for q in range(16)]
        xs = [torch.empty_like(b) for b in bs]
        infos = L.ldgmg_solve_batch(s.handle, bs, xs)
        torch.cuda.synchronize()
        for q in range(16):
            x1, one = _single(s, bs[q])
            rel = float(torch.linalg.norm(xs[q] - x1) / torch.linalg.norm(x1))
            assert infos[q]["converged"] and abs(infos[q]["iters"] - one["iters"]) <= 1 and rel <= 1e-8, (q, rel)
        # a V-cycle batch of 16 equals 16 single V-cycles (FP64 products, same column sums)
        vb = [torch.empty_like(b) for b in bs]
        L.ldgmg_vcycle_batch(s.handle, bs, vb)
        for q in (0, 7, 15):
            v1 = torch.empty_like(bs[q])
            L.ldgmg_vcycle(s.handle, bs[q], v1)
            torch.cuda.synchronize()
            rel = float(torch.linalg.norm(vb[q] - v1) / torch.linalg.norm(v1))
            assert rel <= 1e-12, (q, rel)
    finally:
        s.close()
