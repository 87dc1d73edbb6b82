"""Pins of the oracle's vectorised distance and weight functions.

sqdist_pairs must be D of every pair (D is pinned in test_oracle_pins.py);
weights must be the correctly rounded square root, which is checked here in
exact rational arithmetic, independently of any math library.
"""
from fractions import Fraction

import numpy as np

import oracle


def _pairs(rng, m, dim):
    kinds = [rng.random((m, dim)), rng.normal(0, 1e3, (m, dim)),
             rng.integers(-50, 50, (m, dim)).astype(np.float64),
             rng.random((m, dim)) * 1e-39]  # float32 denormals
    a = np.concatenate(kinds).astype(np.float32)
    b = np.concatenate([k[::-1] for k in kinds]).astype(np.float32)
    return a, b


def test_sqdist_pairs_is_sqdist_of_every_pair():
    rng = np.random.default_rng(3)
    for dim in (2, 3):
        a, b = _pairs(rng, 500, dim)
        got = oracle.sqdist_pairs(a, b)
        ref = np.array([oracle.sqdist(x, y) for x, y in zip(a, b)], np.float32)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_sqdist_pairs_exact_on_integers():
    rng = np.random.default_rng(4)
    a = rng.integers(-1000, 1000, (4000, 3))
    b = rng.integers(-1000, 1000, (4000, 3))
    exact = ((a - b) ** 2).sum(axis=1)  # < 2^24: exact in float32
    got = oracle.sqdist_pairs(a.astype(np.float32), b.astype(np.float32))
    assert np.array_equal(got, exact.astype(np.float32))


def _ulp_bracket_ok(x: np.float32, y: np.float32) -> bool:
    """y is the float32 nearest to sqrt(x) (ties to even) iff x lies between
    the squares of the midpoints to y's neighbours."""
    xf, yf = Fraction(float(x)), Fraction(float(y))
    up = Fraction(float(np.nextafter(y, np.float32(np.inf))))
    hi = ((yf + up) / 2) ** 2
    if y == 0:
        return xf < hi
    dn = Fraction(float(np.nextafter(y, np.float32(0))))
    lo = ((yf + dn) / 2) ** 2
    even = (int(np.float32(y).view(np.uint32)) & 1) == 0
    if lo < xf < hi:
        return True
    return even and (xf == lo or xf == hi)


def test_weights_are_correctly_rounded_square_roots():
    rng = np.random.default_rng(5)
    bits = np.concatenate([rng.integers(0, 0x7F800000, 3000, dtype=np.int64),
                           np.arange(0, 64), np.arange(0x00800000 - 32, 0x00800000 + 32),
                           np.arange(0x7F7FFFFF - 31, 0x7F7FFFFF + 1)]).astype(np.uint32)
    x = bits.view(np.float32)
    w = oracle.weights(x)
    for xi, wi in zip(x, w):
        assert _ulp_bracket_ok(xi, wi), (float(xi), float(wi))


def test_weights_of_perfect_squares_are_exact():
    k = np.arange(0, 4096, dtype=np.float32)
    assert np.array_equal(oracle.weights(k * k), k)
    assert oracle.weights(np.array([np.inf], np.float32))[0] == np.inf


def test_the_rounding_check_rejects_a_neighbouring_float():
    for x in (np.float32(2.0), np.float32(3.0e-40), np.float32(1.5e30), np.float32(7.0)):
        w = oracle.weights(np.array([x], np.float32))[0]
        assert _ulp_bracket_ok(x, w)
        assert not _ulp_bracket_ok(x, np.nextafter(w, np.float32(np.inf)))
        assert not _ulp_bracket_ok(x, np.nextafter(w, np.float32(0)))
