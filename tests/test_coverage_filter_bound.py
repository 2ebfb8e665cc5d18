"""The error bound behind the sampling walk's float32 coverage filter.

The walk evaluates each edge function e = tau * tbv - tav * tbu of float32
values as p = fl(tav * tbu), e = fl(fma(tau, tbv, -p)) and takes the sign of e
as exact when |e| > fl(fma(|p|, 2^-22, 2^-100)); otherwise the float64 test
decides.  These tests emulate that float32 arithmetic exactly (rationals,
rounded once to the nearest float32 with ties to even, subnormals included)
and check, on random, nearly cancelling, subnormal and exactly cancelling
inputs, that the filter never takes a sign that differs from the exact one
(an exactly zero edge function is never decided), and that it decides the
clear cases.
"""
from fractions import Fraction

import numpy as np

from oracle.exact import round_f32

TWO_M22 = Fraction(1, 2 ** 22)
TWO_M100 = Fraction(1, 2 ** 100)


def _f32(q):
    """Nearest float32 of a rational, overflow to infinity (None)."""
    try:
        return round_f32(q)
    except OverflowError:
        return None


def _filter(tau, tbv, tav, tbu):
    """The walk's decision: +1 or -1 when the float32 value is trusted, 0 when
    the float64 test must decide."""
    p = _f32(Fraction(tav) * Fraction(tbu))
    if p is None:
        return 0  # |p| = inf: the bound is infinite
    e = _f32(Fraction(tau) * Fraction(tbv) - p)
    if e is None:  # rounds past the largest float32: infinite with the exact sign
        return 1 if Fraction(tau) * Fraction(tbv) - p > 0 else -1
    t = _f32(abs(p) * TWO_M22 + TWO_M100)
    if t is None or not abs(e) > t:
        return 0
    return 1 if e > 0 else -1


def _exact(tau, tbv, tav, tbu):
    v = Fraction(tau) * Fraction(tbv) - Fraction(tav) * Fraction(tbu)
    return (v > 0) - (v < 0)


def _random_f32(rng, n, emin, emax):
    m = rng.uniform(1.0, 2.0, n)
    e = rng.integers(emin, emax + 1, n)
    s = rng.choice([-1.0, 1.0], n)
    return (s * np.ldexp(m, e)).astype(np.float32)


def _check(cases):
    decided = 0
    for tau, tbv, tav, tbu in cases:
        f = _filter(float(tau), float(tbv), float(tav), float(tbu))
        x = _exact(float(tau), float(tbv), float(tav), float(tbu))
        if f != 0:
            decided += 1
            assert f == x, (tau, tbv, tav, tbu, f, x)
    return decided


def test_random_magnitudes_are_decided_correctly():
    rng = np.random.default_rng(1)
    n = 3000
    cases = zip(*(_random_f32(rng, n, -40, 40) for _ in range(4)))
    assert _check(cases) > 0.99 * n


def _near_cancelling(seed, emin, emax, n=2000):
    """tbu within a few ulps of tau * tbv / tav: the exact value is a tiny
    difference of two products, where a one-ulp error flips the sign."""
    def step(q, k):  # q moved by k float32 ulps
        for _ in range(abs(k)):
            q = np.nextafter(q, np.float32(np.inf if k > 0 else -np.inf))
        return q

    rng = np.random.default_rng(seed)
    tau, tbv, tav = (_random_f32(rng, n, emin, emax) for _ in range(3))
    cases = []
    for a, b, c in zip(tau, tbv, tav):
        q = np.float32(np.float64(a) * np.float64(b) / np.float64(c))
        cases += [(a, b, c, step(q, k)) for k in range(-3, 4)]
    return cases


def test_nearly_cancelling_edges():
    _check(_near_cancelling(2, -20, 20))


def test_nearly_cancelling_below_the_normal_range():
    """The same with products of about 2^-140: they round to subnormals, an
    absolute error of at most 2^-150 each, so a float32 value that does not
    round to zero there still carries the exact sign (the bound's 2^-100 term
    is a margin on top of that)."""
    _check(_near_cancelling(5, -72, -68))


def test_subnormal_and_huge_products():
    rng = np.random.default_rng(3)
    n = 1500
    tiny = zip(*(_random_f32(rng, n, -75, -60) for _ in range(4)))
    _check(tiny)
    huge = zip(*(_random_f32(rng, n, 60, 66) for _ in range(4)))
    _check(huge)


def test_exactly_zero_edges_are_never_decided():
    """Points exactly on an edge line (small integers and dyadic scalings, so
    tau * tbv == tav * tbu holds exactly) go to the float64 test, where the
    tie rule decides them."""
    rng = np.random.default_rng(4)
    for _ in range(2000):
        a, b, k = (int(x) for x in rng.integers(1, 2 ** 11, 3))
        s = float(2.0 ** int(rng.integers(-80, 40)))
        tau, tbv, tav, tbu = (np.float32(a * k * s), np.float32(b), np.float32(a * s), np.float32(b * k))
        assert _exact(float(tau), float(tbv), float(tav), float(tbu)) == 0
        assert _filter(float(tau), float(tbv), float(tav), float(tbu)) == 0
