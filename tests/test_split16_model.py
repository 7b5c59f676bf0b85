"""The error model of the split FP16 products that the symmetric route's
FP32 substitutions use (a host model of the arithmetic, numpy only).

Each FP32 operand x is held as hi = fp16(x) and lo = fp16(x - hi); a product
is hi*hi + hi*lo + lo*hi with FP32 accumulation. With the operand scaled by
a power of two so that its largest magnitude lies in [1, 2), the pair keeps
x to within max(2^-22 |x|, 2^-25) (the second term is half the FP16
subnormal spacing, reached by small entries), and a 64-deep tile product
stays within a few 2^-22 of the exact product, far below the FP16 rounding
(2^-11) of the iterate that follows.
"""
import numpy as np


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = x.astype(np.float16)
    lo = (x - hi.astype(np.float32)).astype(np.float16)
    return hi, lo


def scale_of(amax):
    # the power of two that brings amax into [1, 2)
    _, e = np.frexp(amax)
    return np.ldexp(1.0, 1 - int(e))


def split_product(a, b):
    ah, al = split(a)
    bh, bl = split(b)
    f = lambda u, v: u.astype(np.float32) @ v.astype(np.float32)
    return f(al, bh) + f(ah, bl) + f(ah, bh)


def test_scale_brings_the_largest_magnitude_into_one_two():
    for amax in (1e-6, 0.3, 1.0, 1.5, 2.0, 37.0, 6.5e4, 3e9):
        sc = scale_of(amax)
        assert 1.0 <= sc * amax < 2.0
        assert np.log2(sc) == int(np.log2(sc))


def test_pair_holds_22_bits_in_the_normal_range():
    rng = np.random.default_rng(5)
    x = np.float32(2.0) ** rng.uniform(-3, 1, 20000).astype(np.float32) * rng.choice([-1, 1], 20000)
    hi, lo = split(x)
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -22 * np.abs(x) * 1.0001)
    # small entries: half the subnormal spacing
    y = np.float32(2.0) ** rng.uniform(-20, -3, 20000).astype(np.float32)
    yh, yl = split(y)
    erry = np.abs(y.astype(np.float64) - yh.astype(np.float64) - yl.astype(np.float64))
    assert np.all(erry <= np.maximum(2.0 ** -22 * y, 2.0 ** -25) * 1.0001)
    # hi alone would only hold 11 bits
    assert np.max(np.abs(x - hi.astype(np.float32)) / np.abs(x)) > 2.0 ** -13


def test_tile_product_error_far_below_fp16():
    rng = np.random.default_rng(6)
    for trial in range(4):
        a = rng.standard_normal((64, 64)) * 10.0 ** rng.uniform(-2, 3)
        b = np.tril(rng.standard_normal((64, 64)))   # a factor-like operand
        sa = scale_of(np.abs(a).max())
        c = split_product((sa * a).astype(np.float32), b.astype(np.float32)) / sa
        exact = a.astype(np.float32).astype(np.float64) @ b.astype(np.float32).astype(np.float64)
        rel = np.linalg.norm(c - exact) / np.linalg.norm(exact)
        assert rel < 2e-6, rel
        # one plain FP16 product is three orders worse
        c16 = (a * sa).astype(np.float16).astype(np.float32) @ b.astype(np.float16).astype(np.float32) / sa
        assert np.linalg.norm(c16 - exact) / np.linalg.norm(exact) > 100 * rel


def test_dropping_the_lo_terms_is_a_planted_mistake():
    # the check above would catch a product that kept only hi*hi
    rng = np.random.default_rng(7)
    a = rng.standard_normal((64, 64)).astype(np.float32)
    b = rng.standard_normal((64, 64)).astype(np.float32)
    sa, sb = scale_of(np.abs(a).max()), scale_of(np.abs(b).max())
    ah, _ = split(a * sa)
    bh, _ = split(b * sb)
    c = (ah.astype(np.float32) @ bh.astype(np.float32)) / (sa * sb)
    exact = a.astype(np.float64) @ b.astype(np.float64)
    assert np.linalg.norm(c - exact) / np.linalg.norm(exact) > 2e-6
