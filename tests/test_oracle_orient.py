"""Pins for the oracle's exact orientation predicate.

The oracle sums six error-free products as a floating-point expansion; these
tests check it against exact rational arithmetic (``fractions``) on inputs
where a dropped error term, a wrong sign or a transposed operand changes the
answer: k-ulp perturbations of collinear triples, magnitudes at both ends of
the input domain, and integer triples where the plain determinant is exact.
"""
import math
import random

import numpy as np
import pytest

import oracle
from tests.exact_ref import orient_q


def _ulp_walk(v: float, k: int) -> float:
    for _ in range(abs(k)):
        v = math.nextafter(v, math.inf if k > 0 else -math.inf)
    return v


def test_basic_signs():
    assert oracle.orient((0, 0), (1, 0), (0, 1)) == 1
    assert oracle.orient((0, 0), (0, 1), (1, 0)) == -1
    assert oracle.orient((0, 0), (1, 1), (2, 2)) == 0
    assert oracle.orient((1, 1), (1, 1), (3, 7)) == 0


def test_random_uniform_vs_fraction():
    rng = random.Random(12345)
    for _ in range(5000):
        pts = [(rng.random(), rng.random()) for _ in range(3)]
        assert oracle.orient(*pts) == orient_q(*pts)


def test_near_collinear_ulp_perturbations():
    """Points on the line through two doubles, moved by a few ulps: the plain
    determinant gets the sign wrong on many of these."""
    rng = random.Random(7)
    wrong_naive = 0
    for _ in range(4000):
        ax, ay = rng.uniform(-1, 1), rng.uniform(-1, 1)
        bx, by = rng.uniform(-1, 1), rng.uniform(-1, 1)
        t = rng.uniform(-2, 3)
        cx = ax + t * (bx - ax)
        cy = ay + t * (by - ay)
        cx = _ulp_walk(cx, rng.randint(-3, 3))
        cy = _ulp_walk(cy, rng.randint(-3, 3))
        a, b, c = (ax, ay), (bx, by), (cx, cy)
        exact = orient_q(a, b, c)
        assert oracle.orient(a, b, c) == exact
        naive = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
        if ((naive > 0) - (naive < 0)) != exact:
            wrong_naive += 1
    # the family is hard enough that plain floating point fails on it
    assert wrong_naive > 50


def test_extreme_magnitudes_of_domain():
    rng = random.Random(99)
    for _ in range(1500):
        e = rng.choice([-300, -299, -150, 0, 150, 299])
        s = math.ldexp(1.0, e)
        a = (rng.uniform(1, 2) * s, rng.uniform(1, 2) * s)
        b = (_ulp_walk(a[0], rng.randint(1, 4)), _ulp_walk(a[1], rng.randint(-4, 4)))
        c = (_ulp_walk(a[0], rng.randint(-4, 8)), _ulp_walk(a[1], rng.randint(-4, 8)))
        assert oracle.orient(a, b, c) == orient_q(a, b, c)
        # mixed scales: a huge and a tiny point
        d = (rng.uniform(-1, 1) * math.ldexp(1.0, 299), rng.uniform(-1, 1) * math.ldexp(1.0, 299))
        f = (rng.uniform(-1, 1) * math.ldexp(1.0, -299), rng.uniform(-1, 1) * math.ldexp(1.0, -299))
        assert oracle.orient(a, d, f) == orient_q(a, d, f)
        assert oracle.orient(f, a, d) == orient_q(f, a, d)


def test_integer_triples_match_plain_determinant():
    rng = np.random.default_rng(5)
    tri = rng.integers(-1000, 1000, size=(3000, 6)).astype(np.float64)
    for ax, ay, bx, by, cx, cy in tri:
        d = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)   # exact for these sizes
        assert oracle.orient((ax, ay), (bx, by), (cx, cy)) == int(d > 0) - int(d < 0)


def test_antisymmetry_and_cyclic_identities():
    rng = random.Random(3)
    for _ in range(2000):
        ax, ay = rng.uniform(-1, 1), rng.uniform(-1, 1)
        bx, by = _ulp_walk(ax, rng.randint(-5, 5)), _ulp_walk(ay, rng.randint(-5, 5))
        cx, cy = _ulp_walk(ax, rng.randint(-5, 5)), _ulp_walk(ay, rng.randint(-5, 5))
        a, b, c = (ax, ay), (bx, by), (cx, cy)
        o = oracle.orient(a, b, c)
        assert oracle.orient(b, c, a) == o
        assert oracle.orient(c, a, b) == o
        assert oracle.orient(b, a, c) == -o
        assert oracle.orient(a, c, b) == -o
        assert o == orient_q(a, b, c)


@pytest.mark.parametrize("bad,status", [
    ((float("nan"), 0.0), oracle.NONFINITE),
    ((float("inf"), 0.0), oracle.NONFINITE),
    ((1e-310, 0.0), oracle.RANGE),
    ((0.0, math.ldexp(1.0, 301)), oracle.RANGE),
])
def test_domain_validation(bad, status):
    pts = np.array([[0.0, 0.0], [1.0, 1.0], bad], dtype=np.float64)
    assert oracle.validate(pts) == status
    with pytest.raises(oracle.OracleError) as e:
        oracle.hull(pts)
    assert e.value.status == status


def test_domain_edges_are_accepted():
    lo, hi = math.ldexp(1.0, -300), math.ldexp(1.0, 300)
    pts = np.array([[0.0, -0.0], [lo, -hi], [-lo, hi]], dtype=np.float64)
    assert oracle.validate(pts) == oracle.OK
