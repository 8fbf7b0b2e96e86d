"""Pins of the oracle's flight logarithm (the -ln(1 - u) of the exponential
flight distance) against the mathematics it computes: libm's log within one
ulp over the flight range, the exact values at 1 and at powers of two, and
the functional equation ln(ab) = ln a + ln b (not GPU)."""
import math

import numpy as np

from oracle import oracle as O


def _ulps(a, b):
    return abs(a - b) / math.ulp(b) if b != 0.0 else abs(a - b)


def test_log_within_one_ulp_of_libm():
    # Uniforms of the flight draws are multiples of 2^-53 in [0, 1), so the
    # argument 1 - u runs over (0, 1]: random values, values next to 1 (short
    # flights), tiny values (long flights) and the 53-bit grid near 2^-53.
    rng = np.random.default_rng(7)
    xs = np.concatenate([1.0 - rng.integers(0, 2**53, 40000) * 2.0**-53,
                         1.0 - np.arange(1, 4000) * 2.0**-53,
                         np.ldexp(rng.random(4000) + 0.5, -rng.integers(1, 53, 4000)),
                         np.arange(1, 2000) * 2.0**-53])
    d = np.array([_ulps(O.log(float(x)), math.log(float(x))) for x in xs if x > 0.0])
    assert d.max() <= 1.0, d.max()
    # Nearly always the same double as libm's (both are almost always the
    # correctly rounded value): a small error in a constant would show here.
    assert np.mean(d == 0.0) >= 0.9, np.mean(d == 0.0)


def test_log_exact_values():
    assert O.log(1.0) == 0.0
    for j in range(1, 60):
        # ln 2^-j = -j ln 2 (within one ulp: k ln 2 is a fused sum of two parts).
        assert _ulps(O.log(2.0**-j), -j * math.log(2.0)) <= 1.0, j
    # Both sides of the reduction's switch point sqrt(1/2).
    for x in (0.70710678118654746, 0.70710678118654757, 0.7071067811865476):
        assert _ulps(O.log(x), math.log(x)) <= 1.0, x


def test_log_functional_equation():
    rng = np.random.default_rng(3)
    a = rng.random(2000) * 0.99 + 0.005
    b = rng.random(2000) * 0.99 + 0.005
    for x, y in zip(a, b):
        lhs = O.log(float(x * y))
        rhs = O.log(float(x)) + O.log(float(y))
        # x*y is rounded (half an ulp, relative 2^-53 of the argument).
        assert abs(lhs - rhs) <= 4 * math.ulp(max(abs(lhs), 1e-300)) + 2.0**-52, (x, y)
