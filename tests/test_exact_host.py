"""The library's exact predicates (exact.hpp), built for the host, against
exact rational arithmetic.  The same source is compiled for gfx950; the GPU
tests repeat these checks on the device."""
import math
import random
from fractions import Fraction

import pytest

from tests.exact_ref import orient_q
from tests.native import host_exact


def _walk(v, k):
    for _ in range(abs(k)):
        v = math.nextafter(v, math.inf if k > 0 else -math.inf)
    return v


def key_q(x, y, x0, y0) -> int:
    """floor(2^31 * phi) in exact rational arithmetic."""
    dx = Fraction(x) - Fraction(x0)
    dy = Fraction(y) - Fraction(y0)
    assert dy > 0 or (dy == 0 and dx > 0)
    s = dy / (abs(dx) + dy)
    phi = s if dx >= 0 else 2 - s
    return math.floor(phi * 2 ** 31)


@pytest.fixture(scope="module")
def L():
    return host_exact()


def test_orient_near_degenerate(L):
    rng = random.Random(17)
    for _ in range(3000):
        ax, ay, bx, by = (rng.uniform(-1, 1) for _ in range(4))
        t = rng.uniform(-2, 3)
        cx = _walk(ax + t * (bx - ax), rng.randint(-3, 3))
        cy = _walk(ay + t * (by - ay), rng.randint(-3, 3))
        want = orient_q((ax, ay), (bx, by), (cx, cy))
        assert L.hx_orient(ax, ay, bx, by, cx, cy) == want
        assert L.hx_orient_exact(ax, ay, bx, by, cx, cy) == want


def test_orient_domain_extremes(L):
    rng = random.Random(18)
    for _ in range(1500):
        e = rng.choice([-300, -200, 0, 200, 299])
        s = math.ldexp(1.0, e)
        a = (rng.uniform(1, 2) * s, rng.uniform(1, 2) * s)
        b = (_walk(a[0], rng.randint(1, 4)), _walk(a[1], rng.randint(-4, 4)))
        c = (_walk(a[0], rng.randint(-4, 8)), _walk(a[1], rng.randint(-4, 8)))
        assert L.hx_orient(*a, *b, *c) == orient_q(a, b, c)
        d = (rng.uniform(-1, 1) * math.ldexp(1.0, 299), rng.uniform(-1, 1) * math.ldexp(1.0, 299))
        f = (rng.uniform(-1, 1) * math.ldexp(1.0, -299), rng.uniform(-1, 1) * math.ldexp(1.0, -299))
        assert L.hx_orient(*a, *d, *f) == orient_q(a, d, f)


def test_key_random(L):
    rng = random.Random(19)
    for _ in range(4000):
        x0, y0 = rng.uniform(-1, 1), rng.uniform(-1, 1)
        x, y = rng.uniform(-2, 2), y0 + rng.random()
        if y == y0 and x <= x0:
            continue
        assert L.hx_angle_key(x, y, x0, y0) == key_q(x, y, x0, y0)


def test_key_exact_boundaries(L):
    """Points whose pseudo-angle is exactly k/2^31, and their ulp neighbours."""
    rng = random.Random(20)
    checked = 0
    for _ in range(1500):
        k = rng.randrange(1, 2 ** 32 - 1)
        if k < 2 ** 31:      # dx >= 0: dy/(dx+dy) = k/2^31
            dx, dy = float(2 ** 31 - k), float(k)
        else:                # dx < 0: (2|dx|+dy)/(|dx|+dy) = k/2^31
            a, b = 2 ** 32 - k, k - 2 ** 31     # |dx| * a = dy * b -> |dx| = b, dy = a
            dx, dy = -float(b), float(a)
        if dy == 0:
            continue
        scale = math.ldexp(1.0, rng.randint(-40, 40))
        x0, y0 = rng.choice([(0.0, 0.0), (3.0, -5.0), (0.5, 0.25)])
        x, y = x0 + dx * scale, y0 + dy * scale
        for px, py in [(x, y), (_walk(x, 1), y), (_walk(x, -1), y), (x, _walk(y, 1)),
                       (x, _walk(y, -1))]:
            if py < y0 or (py == y0 and px <= x0):
                continue
            assert L.hx_angle_key(px, py, x0, y0) == key_q(px, py, x0, y0)
            checked += 1
    assert checked > 5000


def test_key_integer_grid(L):
    for x in range(-12, 13):
        for y in range(0, 13):
            if y == 0 and x <= 0:
                continue
            assert L.hx_angle_key(float(x), float(y), 0.0, 0.0) == key_q(x, y, 0, 0)


def test_key_monotone_vs_orientation(L):
    """K(a) < K(b) implies a strictly before b in angle (adversarial pairs)."""
    rng = random.Random(21)
    x0, y0 = 0.1, 0.2
    for _ in range(3000):
        ax, ay = rng.uniform(-1, 1), y0 + rng.uniform(1e-3, 1)
        bx, by = _walk(ax, rng.randint(-3, 3)), _walk(ay, rng.randint(-3, 3))
        ka = L.hx_angle_key(ax, ay, x0, y0)
        kb = L.hx_angle_key(bx, by, x0, y0)
        o = orient_q((x0, y0), (ax, ay), (bx, by))
        if ka < kb:
            assert o > 0
        elif ka > kb:
            assert o < 0


def turn_q(px, py, cx, cy) -> int:
    """Full-turn pseudo-angle key of p - c in exact rational arithmetic."""
    dx = Fraction(px) - Fraction(cx)
    dy = Fraction(py) - Fraction(cy)
    assert dx != 0 or dy != 0
    if dx > 0 and dy >= 0:
        q, a, b = 0, dx, dy
    elif dx <= 0 and dy > 0:
        q, a, b = 1, dy, -dx
    elif dx < 0 and dy <= 0:
        q, a, b = 2, -dx, -dy
    else:
        q, a, b = 3, -dy, dx
    return q * 2 ** 30 + math.floor(b / (a + b) * 2 ** 30)


def test_turn_key_random_and_axes(L):
    rng = random.Random(22)
    for _ in range(4000):
        cx, cy = rng.uniform(-1, 1), rng.uniform(-1, 1)
        px, py = rng.uniform(-2, 2), rng.uniform(-2, 2)
        assert L.hx_turn_key(px, py, cx, cy) == turn_q(px, py, cx, cy)
    for px, py in [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]:
        assert L.hx_turn_key(float(px), float(py), 0.0, 0.0) == turn_q(px, py, 0, 0)


def test_turn_key_exact_boundaries_and_half_turn(L):
    rng = random.Random(23)
    checked = 0
    for _ in range(1500):
        k = rng.randrange(1, 2 ** 30)
        a, b = float(2 ** 30 - k), float(k)     # b/(a+b) = k/2^30 exactly
        q = rng.randrange(4)
        dx, dy = [(a, b), (-b, a), (-a, -b), (b, -a)][q]
        sc = math.ldexp(1.0, rng.randint(-30, 30))
        cx, cy = rng.choice([(0.0, 0.0), (0.5, -0.25), (3.0, 7.0)])
        px, py = cx + dx * sc, cy + dy * sc
        for qx, qy in [(px, py), (_walk(px, 1), py), (px, _walk(py, -1)), (_walk(px, -2), _walk(py, 1))]:
            if qx == cx and qy == cy:
                continue
            assert L.hx_turn_key(qx, qy, cx, cy) == turn_q(qx, qy, cx, cy)
            checked += 1
        # a half turn adds exactly 2^31 (mod 2^32)
        k1 = L.hx_turn_key(cx + dx, cy + dy, cx, cy)
        k2 = L.hx_turn_key(cx - dx, cy - dy, cx, cy)
        assert (k2 - k1) % 2 ** 32 == 2 ** 31
    assert checked > 5000
