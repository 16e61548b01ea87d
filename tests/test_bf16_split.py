"""The exact three-way BF16 split of FP32 values that the BF16-core smoother
applies use (FP32 products mode, BF16 smoother matrices reading the FP32
residual), checked on the CPU as arithmetic, independently of the kernels:

  * hi keeps the top 8 significand bits of x (truncation), mid the top 8 of
    x - hi, lo = x - hi - mid; both remainders are exact in FP32;
  * hi + mid + lo == x exactly in FP32 arithmetic; hi and mid are BF16
    values, and lo is one whenever |x| >= 2^-103 (lo is then an FP32 normal
    number of at most 8 significand bits); for smaller |x| lo can be an FP32
    subnormal, whose BF16 truncation (the kernel keeps the top 16 bits of its
    FP32 word) loses less than 2^-133 in absolute terms;
  * a BF16 entry times any part is exact in FP32, so an apply that sums these
    3n products in FP32 has the rounding of an FP32 sum of 3n exact terms.

Inputs: seeded FP32 values over the whole normal exponent range, both signs,
and the special cases 0, -0, powers of two, values one ulp either side of
them, the largest finite value and the smallest normal one.
"""
import numpy as np

MASK = np.uint32(0xFFFF0000)


def _trunc16(v):
    return (v.view(np.uint32) & MASK).view(np.float32)


def _split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = _trunc16(x)
    r1 = (x - hi).astype(np.float32)
    mid = _trunc16(r1)
    lo = (r1 - mid).astype(np.float32)
    return hi, mid, lo


def _inputs():
    rng = np.random.default_rng(1212)
    m = rng.uniform(1.0, 2.0, 20000)
    e = rng.integers(-120, 120, 20000)
    x = (m * np.exp2(e.astype(np.float64)) * rng.choice([-1.0, 1.0], 20000)).astype(np.float32)
    p2 = np.exp2(np.arange(-120, 121, dtype=np.float64)).astype(np.float32)
    near = np.concatenate([np.nextafter(p2, np.float32(np.inf)), np.nextafter(p2, np.float32(0))])
    fi = np.finfo(np.float32)
    special = np.array([0.0, -0.0, fi.max, -fi.max, fi.tiny, -fi.tiny, 1.0 + fi.eps, 3.0, 1.0 / 3.0], np.float32)
    return np.concatenate([x, p2, -p2, near, -near, special]).astype(np.float32)


def test_split_is_exact_and_bf16():
    x = _inputs()
    hi, mid, lo = _split(x)
    total = hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(total, x.astype(np.float64))
    for part in (hi, mid):
        assert not np.any(part.view(np.uint32) & np.uint32(0xFFFF)), "a part is not a BF16 value"
    big = np.abs(x.astype(np.float64)) >= 2.0 ** -103
    assert not np.any(lo[big].view(np.uint32) & np.uint32(0xFFFF)), "lo is not a BF16 value"
    lo16 = _trunc16(lo)                                  # what the BF16 operand holds
    assert np.all(np.abs(lo16.astype(np.float64) - lo.astype(np.float64)) < 2.0 ** -133)
    # parts shrink (normal range): |mid| < 2^-7 |x|, |lo| < 2^-15 |x| (truncation keeps 8 bits each)
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(mid[big]) <= ax[big] * 2.0 ** -7)
    assert np.all(np.abs(lo[big]) <= ax[big] * 2.0 ** -15)


def test_bf16_products_exact_in_fp32():
    rng = np.random.default_rng(1213)
    x = _inputs()
    a = _trunc16(rng.standard_normal(x.size).astype(np.float32) * np.float32(3.0))   # BF16 entries
    a = a * np.exp2(rng.integers(-4, 5, x.size)).astype(np.float32)
    for part in _split(x):
        p64 = a.astype(np.float64) * part.astype(np.float64)
        ok = np.abs(p64) < np.finfo(np.float32).max
        p32 = (a[ok] * part[ok]).astype(np.float32)
        tiny = np.abs(p64[ok]) < np.finfo(np.float32).tiny * 2.0 ** 16   # products near the FP32 underflow
        assert np.array_equal(p32[~tiny].astype(np.float64), p64[ok][~tiny])


def test_split_sum_matches_fp32_product_accuracy():
    """A row of n terms: summing the 3n exact products in FP32 stays within
    (3n + 1) u32 sum(|a||x|) of the exact dot product, the bound used for
    these applies (and in practice far inside it)."""
    rng = np.random.default_rng(1214)
    n = 448
    u32 = 2.0 ** -24
    worst = 0.0
    for _ in range(50):
        a = _trunc16(rng.standard_normal(n).astype(np.float32))
        x = rng.standard_normal(n).astype(np.float32)
        exact = float(np.dot(a.astype(np.float64), x.astype(np.float64)))
        acc = np.float32(0.0)
        for part in _split(x)[::-1]:
            for k in range(n):
                acc = np.float32(acc + a[k] * part[k])
        bound = (3 * n + 1) * u32 * float(np.dot(np.abs(a.astype(np.float64)), np.abs(x.astype(np.float64))))
        worst = max(worst, abs(float(acc) - exact) / bound)
    assert worst <= 1.0, worst
