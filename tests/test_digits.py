"""The int8 form's digit arithmetic, checked on the CPU: balanced digits of
base 128 (|d| <= 64) or 256 recombine to the value; the three-product
(Karatsuba) recombination of a correlation term equals the plain product sum;
and no int32 accumulator can wrap for the largest operands over fewer than
2^17 terms.  These are the identities the matrix-core correlation relies on
(sec. 2, the correlation h evaluated exactly in integers)."""
import numpy as np


def bdigit(x, b):
    half = 1 << (b - 1)
    return ((x + half) & ((1 << b) - 1)) - half


def digits(x, b):
    d0 = bdigit(x, b)
    x1 = (x - d0) >> b
    d1 = bdigit(x1, b)
    d2 = (x1 - d1) >> b
    return d0, d1, d2


def test_balanced_digits_recombine():
    x = np.arange(0, 4 * 65535 + 1, dtype=np.int64)
    for b in (7, 8):
        d0, d1, d2 = digits(x, b)
        assert np.array_equal(d0 + (d1 << b) + (d2 << (2 * b)), x)
        half = 1 << (b - 1)
        assert d0.min() >= -half and d0.max() < half
        assert d1.min() >= -half and d1.max() < half
        # two digits hold exactly the values up to (2^(b-1)-1)(1 + 2^b)
        two = (d2 == 0)
        top = (half - 1) * (1 + (1 << b))
        assert two[: top + 1].all() and not two[top + 1:].any()
        # a box sum of uint16 pixels needs at most a third digit within int8
        assert d2.max() <= 127


def test_three_product_recombination_is_exact():
    rng = np.random.default_rng(7)
    X = rng.integers(0, 8128, size=(64, 300))
    Y = rng.integers(0, 8128, size=(64, 300))
    x0, x1, x2 = digits(X, 7)
    y0, y1, y2 = digits(Y, 7)
    assert not x2.any() and not y2.any()
    s0, s1 = x0 + x1, y0 + y1
    assert s0.min() >= -128 and s0.max() <= 127 and s1.min() >= -128 and s1.max() <= 127
    h00 = (x0 * y0).sum(axis=1)
    h11 = (x1 * y1).sum(axis=1)
    s = (s0 * s1).sum(axis=1)
    h = h00 + 128 * (s - h00 - h11) + 16384 * h11
    assert np.array_equal(h, (X * Y).sum(axis=1))


def test_four_product_recombination_is_exact():
    rng = np.random.default_rng(8)
    X = rng.integers(0, 32640, size=(64, 300))
    Y = rng.integers(0, 32640, size=(64, 300))
    x0, x1, _ = digits(X, 8)
    y0, y1, _ = digits(Y, 8)
    h = sum((xp * yq).sum(axis=1) << (8 * (p + q))
            for p, xp in enumerate((x0, x1)) for q, yq in enumerate((y0, y1)))
    assert np.array_equal(h, (X * Y).sum(axis=1))


def test_int32_accumulators_cannot_wrap():
    terms = (1 << 17) - 1          # fewer than 2^17 overlap terms per shift
    for largest in (128 * 128, 64 * 64, 128 * 128):   # sums, base-128 digits, base-256 digits
        assert largest * terms < (1 << 31)
