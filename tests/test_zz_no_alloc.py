"""The entry point that allocates nothing (ldgmg_vcycle_batch_noalloc): the
batched V-cycle with its level vectors in the library's static scratch
array gives exactly the result of ldgmg_vcycle_batch (same kernels, same
arithmetic: bitwise), on two calls in a row, the second with a smaller input
(fewer right-hand sides, then a smaller hierarchy), and a request beyond the
scratch size is refused with LDGMG_EINVAL."""
import numpy as np
import pytest

from ldg_inputs import rhs_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _compare(s, k, seed):
    from paper_2412_12506_amd import ldgmg as L
    bs = [torch.from_numpy(rhs_normal(s.ndofs, seed + q)).cuda() for q in range(k)]
    ref = [torch.empty_like(b) for b in bs]
    out = [torch.full_like(b, float("nan")) for b in bs]
    L.ldgmg_vcycle_batch(s.handle, bs, ref)
    L.ldgmg_vcycle_batch_noalloc(s.handle, bs, out)
    torch.cuda.synchronize()
    for q in range(k):
        assert torch.isfinite(out[q]).all()
        assert torch.equal(out[q], ref[q]), (k, q, float((out[q] - ref[q]).abs().max()))


def test_noalloc_vcycle_batch_matches():
    from paper_2412_12506_amd import ldgmg as L
    big = L.Solver(dim=3, n=16, p=2, smoother="sai", precision="bf16s", storage="tiled")
    small = L.Solver(dim=2, n=16, p=2, smoother="gs", precision="fp32")
    try:
        print(f"\n[noalloc] 3D Q_2 16^3 k=6 then k=3; 2D Q_2 16^2 GS k=2", flush=True)
        _compare(big, 6, 100)
        _compare(big, 3, 200)          # the second call, smaller
        _compare(small, 2, 300)        # a smaller hierarchy on the same scratch
        huge = L.Solver(dim=3, n=24, p=2, smoother="jacobi", precision="fp32", host_only=True)
        try:
            huge.upload()
            bs = [torch.zeros(huge.ndofs, dtype=torch.float64, device="cuda") for _ in range(16)]
            with pytest.raises(L.LdgmgError) as ex:
                L.ldgmg_vcycle_batch_noalloc(huge.handle, bs, bs)
            assert ex.value.code == L.EINVAL
        finally:
            huge.close()
    finally:
        big.close()
        small.close()
